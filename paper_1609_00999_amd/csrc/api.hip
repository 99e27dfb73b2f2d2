// api.hip -- host entry points of libmont that enqueue no device work:
// the section 3.1 precomputation, status text and launch-shape tuning.
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace {

// -P^-1 mod 2^32 by Newton's iteration x <- x (2 - P x): each step doubles the
// number of correct low bits, starting from 3 (P*P = 1 mod 8 for odd P).
uint32_t neg_inverse_2_32(uint32_t P) {
  uint32_t x = P;
  for (int i = 0; i < 4; i++) x *= 2u - P * x;
  return 0u - x;
}

}  // namespace

extern "C" const char* mont_strerror(mont_status status) {
  switch (status) {
    case MONT_OK: return "ok";
    case MONT_EINVAL: return "invalid argument";
    case MONT_ERANGE: return "size or index out of the supported range";
    case MONT_ENOROOT: return "modulus has no root of unity of the needed order";
    case MONT_ENOMEM: return "scratch or device memory too small";
    case MONT_EHIP: return "HIP runtime error";
    case MONT_ETIMEOUT: return "device-side wait timed out";
    default: return "unknown status";
  }
}

extern "C" mont_status mont_setup(uint32_t P, mont_params* out) {
  if (!out || P < 3 || (P & 1u) == 0 || P >= 0x80000000u) return MONT_EINVAL;
  mont_params p;
  p.P = P;
  p.Pprime = neg_inverse_2_32(P);
  uint64_t r1 = ((uint64_t)1 << 32) % P;
  p.R1 = (uint32_t)r1;
  p.R2 = (uint32_t)((r1 * r1) % P);
  uint32_t k = 0;
  for (uint32_t q = P - 1; (q & 1u) == 0; q >>= 1) k++;
  p.k = k;
  *out = p;
  return MONT_OK;
}

extern "C" mont_status mont_elem_tune_set(int op, int block, int vpt, int nontemporal) {
  if (op < 0 || op >= mont::OP_COUNT) return MONT_EINVAL;
  if ((block != 64 && block != 128 && block != 256 && block != 512) || (vpt != 1 && vpt != 2 && vpt != 4))
    return MONT_EINVAL;
  mont::elem_tune(op) = mont::ElemTune{block, vpt, nontemporal ? 1 : 0};
  return MONT_OK;
}

extern "C" mont_status mont_elem_tune_get(int op, int* block, int* vpt, int* nontemporal) {
  if (op < 0 || op >= mont::OP_COUNT || !block || !vpt || !nontemporal) return MONT_EINVAL;
  const mont::ElemTune& t = mont::elem_tune(op);
  *block = t.block;
  *vpt = t.vpt;
  *nontemporal = t.nt;
  return MONT_OK;
}
