// mont64.hip -- Algorithm 2 (arXiv:1609.00999, section 3.1) on 64-bit
// residues, R = 2^64, P < 2^63: elementwise conversions, products, chained
// mul-add and fixed-window powers on gfx950.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "mont64.h"

namespace mont {
namespace {

typedef uint64_t v2u64 __attribute__((ext_vector_type(2)));
typedef uint32_t v4u32 __attribute__((ext_vector_type(4)));

struct Mod64 {
  uint64_t P;
  uint64_t Pp;  // -P^-1 mod 2^64
};

// REDC of T = hi R + lo < R P: m = lo P' mod R, and T + m P has a zero low
// word, so its high word is hi + mulhi(m, P) + (lo != 0), which is below
// 2P < 2^64; one conditional subtraction (an unsigned min) makes it canonical.
__device__ __forceinline__ uint64_t redc64(uint64_t lo, uint64_t hi, Mod64 md) {
  const uint64_t m = lo * md.Pp;
  const uint64_t t = hi + __umul64hi(m, md.P) + (lo != 0 ? 1u : 0u);
  const uint64_t u = t - md.P;
  return u < t ? u : t;
}

__device__ __forceinline__ uint64_t mmul64(uint64_t a, uint64_t b, Mod64 md) {
  return redc64(a * b, __umul64hi(a, b), md);
}

__device__ __forceinline__ uint64_t madd64(uint64_t a, uint64_t b, uint64_t P) {
  const uint64_t s = a + b;   // < 2P < 2^64
  const uint64_t u = s - P;
  return u < s ? u : s;
}

// Left-to-right fixed 2-bit windows over 64 exponent bits, table {1, x, x^2,
// x^3} selected without branches: 2 + 31 x 3 = 95 REDC.
__device__ __forceinline__ uint64_t mpow64(uint64_t x, uint64_t e, Mod64 md, uint64_t one) {
  const uint64_t x2 = mmul64(x, x, md);
  const uint64_t x3 = mmul64(x2, x, md);
  auto pick = [&](uint32_t d) {
    const uint64_t lo = (d & 1u) ? x : one;
    const uint64_t hi = (d & 1u) ? x3 : x2;
    return (d & 2u) ? hi : lo;
  };
  uint64_t r = pick((uint32_t)(e >> 62));
#pragma unroll 1
  for (int s = 60; s >= 0; s -= 2) {
    r = mmul64(r, r, md);
    r = mmul64(r, r, md);
    r = mmul64(r, pick((uint32_t)(e >> s) & 3u), md);
  }
  return r;
}

enum Op64 { OP64_TO = 0, OP64_FROM = 1, OP64_MUL = 2, OP64_MULADD = 3, OP64_POW = 4 };

template <int OP>
__device__ __forceinline__ uint64_t apply64(uint64_t a, uint64_t b, uint64_t c, Mod64 md, uint64_t k) {
  if constexpr (OP == OP64_TO) return mmul64(a, k, md);          // k = R2
  else if constexpr (OP == OP64_FROM) return redc64(a, 0, md);
  else if constexpr (OP == OP64_MUL) return mmul64(a, b, md);
  else if constexpr (OP == OP64_MULADD) return madd64(mmul64(a, b, md), c, md.P);
  else return mpow64(a, b, md, k);                               // k = R1
}

constexpr int NIN(int op) { return op == OP64_MULADD ? 3 : (op == OP64_TO || op == OP64_FROM) ? 1 : 2; }

// A workgroup's BLOCK vectors per pass are read and written through raw
// buffer resources (their base address and size in scalar registers, a
// 32-bit offset per lane, non-temporal policy; past the size loads return
// zeros and stores are dropped), the form that streams fastest here.
constexpr int kBufWord3 = 0x00020000;   // resource word 3 on gfx9: 32-bit data format
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc64(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, kBufWord3);
}

// One 128-bit vector (two residues) per lane per pass, non-temporal, with a
// scalar path for the ragged tail or for operands that are not 16-byte
// aligned.
template <int OP, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_elem64(Mod64 md, uint64_t k, const uint64_t* a, const uint64_t* b,
                                                  const uint64_t* c, uint64_t* out, size_t n) {
  const size_t stride = (size_t)gridDim.x * BLOCK;
  const size_t tid = (size_t)blockIdx.x * BLOCK + threadIdx.x;
  uintptr_t bits = (uintptr_t)a | (uintptr_t)out;
  if (NIN(OP) >= 2) bits |= (uintptr_t)b;
  if (NIN(OP) >= 3) bits |= (uintptr_t)c;
  size_t head = 0;
  if ((bits & 15u) == 0) {
    const size_t nvec = n >> 1;
    const uint32_t off = threadIdx.x * 16u;
    for (size_t first = (size_t)blockIdx.x * BLOCK; first < nvec; first += stride) {
      const size_t left = nvec - first;
      const uint32_t bytes = (uint32_t)(left < (size_t)BLOCK ? left : (size_t)BLOCK) * 16u;
      const __amdgpu_buffer_rsrc_t ra = tile_rsrc64(a + 2 * first, bytes);
      const __amdgpu_buffer_rsrc_t rb = tile_rsrc64(NIN(OP) >= 2 ? b + 2 * first : a, bytes);
      const __amdgpu_buffer_rsrc_t rc = tile_rsrc64(NIN(OP) >= 3 ? c + 2 * first : a, bytes);
      const __amdgpu_buffer_rsrc_t ro = tile_rsrc64(out + 2 * first, bytes);
      const v2u64 x = __builtin_bit_cast(v2u64, __builtin_amdgcn_raw_buffer_load_b128(ra, (int)off, 0, 2));
      v2u64 y = x, z = x, r;
      if constexpr (NIN(OP) >= 2) y = __builtin_bit_cast(v2u64, __builtin_amdgcn_raw_buffer_load_b128(rb, (int)off, 0, 2));
      if constexpr (NIN(OP) >= 3) z = __builtin_bit_cast(v2u64, __builtin_amdgcn_raw_buffer_load_b128(rc, (int)off, 0, 2));
      r.x = apply64<OP>(x.x, y.x, z.x, md, k);
      r.y = apply64<OP>(x.y, y.y, z.y, md, k);
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4u32, r), ro, (int)off, 0, 2);
    }
    head = nvec << 1;
  }
  for (size_t i = head + tid; i < n; i += stride) {
    const uint64_t y = NIN(OP) >= 2 ? b[i] : 0;
    const uint64_t z = NIN(OP) >= 3 ? c[i] : 0;
    out[i] = apply64<OP>(a[i], y, z, md, k);
  }
}

bool params64_ok(const mont64_params* prm) {
  if (!prm) return false;
  const uint64_t P = prm->P;
  if (P < 3 || (P & 1u) == 0 || P >= ((uint64_t)1 << 63)) return false;
  if (P * prm->Pprime != ~(uint64_t)0) return false;   // P P' = -1 mod 2^64
  return prm->R1 < P && prm->R2 < P;
}

template <int OP>
mont_status launch64(const mont64_params* prm, uint64_t k, const uint64_t* a, const uint64_t* b, const uint64_t* c,
                     uint64_t* out, size_t n, void* stream) {
  if (!params64_ok(prm)) return MONT_EINVAL;
  if (n == 0) return MONT_OK;
  if (!a || !out || (NIN(OP) >= 2 && !b) || (NIN(OP) >= 3 && !c)) return MONT_EINVAL;
  // The streaming ops are HBM-bound: 64-thread groups, one vector per lane.
  // The power is ALU-bound: 256-thread groups.
  constexpr int BLOCK = OP == OP64_POW ? 256 : 64;
  size_t blocks = ((n + 1) / 2 + BLOCK - 1) / BLOCK;
  if (blocks < 1) blocks = 1;
  if (blocks > ((size_t)1 << 22)) blocks = (size_t)1 << 22;
  (void)hipGetLastError();
  const Mod64 md{prm->P, prm->Pprime};
  hipLaunchKernelGGL((k_elem64<OP, BLOCK>), dim3((unsigned)blocks), dim3(BLOCK), 0, as_stream(stream), md, k, a, b,
                     c, out, n);
  return last_launch_status();
}

}  // namespace
}  // namespace mont

using namespace mont;

extern "C" mont_status mont64_setup(uint64_t P, mont64_params* out) {
  if (!out || P < 3 || (P & 1u) == 0 || P >= ((uint64_t)1 << 63)) return MONT_EINVAL;
  // P^-1 mod 2^64 by Newton's iteration x <- x (2 - P x): P is its own
  // inverse mod 8, and each step doubles the number of correct low bits.
  uint64_t x = P;
  for (int i = 0; i < 5; i++) x *= 2 - P * x;
  typedef unsigned __int128 u128;
  const uint64_t R1 = (uint64_t)((((u128)1) << 64) % P);
  mont64_params p;
  p.P = P;
  p.Pprime = (uint64_t)0 - x;
  p.R1 = R1;
  p.R2 = (uint64_t)(((u128)R1 * R1) % P);
  uint32_t k = 0;
  for (uint64_t q = P - 1; (q & 1u) == 0; q >>= 1) k++;
  p.k = k;
  p.reserved = 0;
  *out = p;
  return MONT_OK;
}

extern "C" mont_status mont64_to(const mont64_params* prm, const uint64_t* d_in, uint64_t* d_out, size_t n,
                                 void* stream) {
  return launch64<OP64_TO>(prm, prm ? prm->R2 : 0, d_in, nullptr, nullptr, d_out, n, stream);
}

extern "C" mont_status mont64_from(const mont64_params* prm, const uint64_t* d_in, uint64_t* d_out, size_t n,
                                   void* stream) {
  return launch64<OP64_FROM>(prm, 0, d_in, nullptr, nullptr, d_out, n, stream);
}

extern "C" mont_status mont64_mul(const mont64_params* prm, const uint64_t* d_a, const uint64_t* d_b,
                                  uint64_t* d_out, size_t n, void* stream) {
  return launch64<OP64_MUL>(prm, 0, d_a, d_b, nullptr, d_out, n, stream);
}

extern "C" mont_status mont64_muladd(const mont64_params* prm, const uint64_t* d_a, const uint64_t* d_b,
                                     const uint64_t* d_c, uint64_t* d_out, size_t n, void* stream) {
  return launch64<OP64_MULADD>(prm, 0, d_a, d_b, d_c, d_out, n, stream);
}

extern "C" mont_status mont64_pow(const mont64_params* prm, const uint64_t* d_base, const uint64_t* d_exp,
                                  uint64_t* d_out, size_t n, void* stream) {
  return launch64<OP64_POW>(prm, prm ? prm->R1 : 0, d_base, d_exp, nullptr, d_out, n, stream);
}
