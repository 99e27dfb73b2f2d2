// crt.hip -- exact integer polynomial products from three products modulo
// 31-bit Fourier primes: reduction of uint32 coefficients to residues, and
// Garner's reconstruction with Montgomery products (arXiv:1609.00999,
// section 3.1, Algorithm 2).
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "modarith.hpp"
#include "mont_crt.h"

namespace mont {
namespace {

constexpr int CRT_BLOCK = 256;

// x mod P for any uint32 x and 2^30 < P < 2^31: x < 2^32 < 4P, so one
// conditional subtraction of 2P and one of P (each an unsigned min, since
// 2P < 2^32).
__device__ __forceinline__ uint32_t reduce_word(uint32_t x, uint32_t P) {
  uint32_t u = x - 2 * P;
  x = u < x ? u : x;
  u = x - P;
  return u < x ? u : x;
}

struct CrtDev {
  Mod m2, m3;
  uint32_t P1, P2, P3;
  uint32_t inv12, p1_mod3, inv123;
};

__global__ __launch_bounds__(CRT_BLOCK) void k_crt_reduce(uint32_t P1, uint32_t P2, uint32_t P3, const uint32_t* x,
                                                          size_t n, uint32_t* r0, uint32_t* r1, uint32_t* r2) {
  const size_t stride = (size_t)gridDim.x * CRT_BLOCK;
  const size_t tid = (size_t)blockIdx.x * CRT_BLOCK + threadIdx.x;
  size_t head = 0;
  if (((((uintptr_t)x) | ((uintptr_t)r0) | ((uintptr_t)r1) | ((uintptr_t)r2)) & 15u) == 0) {
    const size_t nvec = n >> 2;
    for (size_t i = tid; i < nvec; i += stride) {
      const v4u v = __builtin_nontemporal_load(reinterpret_cast<const v4u*>(x) + i);
      v4u a, b, c;
      a.x = reduce_word(v.x, P1); a.y = reduce_word(v.y, P1); a.z = reduce_word(v.z, P1); a.w = reduce_word(v.w, P1);
      b.x = reduce_word(v.x, P2); b.y = reduce_word(v.y, P2); b.z = reduce_word(v.z, P2); b.w = reduce_word(v.w, P2);
      c.x = reduce_word(v.x, P3); c.y = reduce_word(v.y, P3); c.z = reduce_word(v.z, P3); c.w = reduce_word(v.w, P3);
      reinterpret_cast<v4u*>(r0)[i] = a;
      reinterpret_cast<v4u*>(r1)[i] = b;
      reinterpret_cast<v4u*>(r2)[i] = c;
    }
    head = nvec << 2;
  }
  for (size_t i = head + tid; i < n; i += stride) {
    const uint32_t v = x[i];
    r0[i] = reduce_word(v, P1);
    r1[i] = reduce_word(v, P2);
    r2[i] = reduce_word(v, P3);
  }
}

// Garner: y2 = (r2 - r1) P1^-1 mod P2; y3 = (r3 - r1 - P1 y2) (P1 P2)^-1 mod
// P3; X = r1 + P1 (y2 + P2 y3) < P1 P2 P3 < 2^93.  Products with constants in
// Montgomery form return ordinary residues: REDC(x * cR) = x c mod P.
__device__ __forceinline__ void garner(uint32_t a1, uint32_t a2, uint32_t a3, const CrtDev& c, uint32_t& w0,
                                       uint32_t& w1, uint32_t& w2) {
  const uint32_t r1_2 = reduce_word(a1, c.P2);          // r1 < 2^31 < 2 P2
  const uint32_t y2 = mmul(msub(a2, r1_2, c.P2), c.inv12, c.m2);
  const uint32_t r1_3 = reduce_word(a1, c.P3);
  const uint32_t y2_3 = reduce_word(y2, c.P3);
  const uint32_t v = mmul(y2_3, c.p1_mod3, c.m3);       // P1 y2 mod P3
  const uint32_t y3 = mmul(msub(msub(a3, r1_3, c.P3), v, c.P3), c.inv123, c.m3);
  const uint64_t t = (uint64_t)y3 * c.P2 + y2;          // < P2 P3 < 2^62
  const uint64_t lo = (uint64_t)(uint32_t)t * c.P1 + a1;
  const uint64_t hi = (t >> 32) * c.P1 + (lo >> 32);
  w0 = (uint32_t)lo;
  w1 = (uint32_t)hi;
  w2 = (uint32_t)(hi >> 32);
}

__global__ __launch_bounds__(CRT_BLOCK) void k_crt_combine(CrtDev c, const uint32_t* r0, const uint32_t* r1,
                                                           const uint32_t* r2, size_t n, uint32_t* out) {
  const size_t stride = (size_t)gridDim.x * CRT_BLOCK;
  for (size_t i = (size_t)blockIdx.x * CRT_BLOCK + threadIdx.x; i < n; i += stride) {
    uint32_t w0, w1, w2;
    garner(r0[i], r1[i], r2[i], c, w0, w1, w2);
    out[3 * i] = w0;
    out[3 * i + 1] = w1;
    out[3 * i + 2] = w2;
  }
}

// Host: a^-1 mod m by the extended Euclidean algorithm (0 if none).
uint32_t inv_mod(uint64_t a, uint64_t m) {
  int64_t r0 = (int64_t)m, r1 = (int64_t)(a % m), s0 = 0, s1 = 1;
  while (r1 != 0) {
    const int64_t q = r0 / r1;
    int64_t t = r0 - q * r1; r0 = r1; r1 = t;
    t = s0 - q * s1; s0 = s1; s1 = t;
  }
  if (r0 != 1) return 0;
  return (uint32_t)(s0 < 0 ? s0 + (int64_t)m : s0);
}

uint32_t to_mont_host(uint64_t x, uint32_t P) { return (uint32_t)(((x % P) << 32) % P); }

bool crt_ok(const crt_params* p) {
  if (!p) return false;
  for (int j = 0; j < 3; j++) {
    if (p->P[j] <= (1u << 30) || p->P[j] >= (1u << 31) || p->m[j].P != p->P[j] || !params_ok(&p->m[j]))
      return false;
  }
  return true;
}

size_t blocks_for(size_t n, size_t per_lane) {
  size_t b = (n / per_lane + CRT_BLOCK - 1) / CRT_BLOCK;
  if (b < 1) b = 1;
  if (b > ((size_t)1 << 20)) b = (size_t)1 << 20;
  return b;
}

size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

}  // namespace
}  // namespace mont

using namespace mont;

extern "C" mont_status crt_setup(const uint32_t* primes, crt_params* out) {
  if (!primes || !out) return MONT_EINVAL;
  crt_params p{};
  for (int j = 0; j < 3; j++) {
    const uint32_t P = primes[j];
    if (P <= (1u << 30) || P >= (1u << 31) || (P & 1u) == 0) return MONT_EINVAL;
    if (mont_setup(P, &p.m[j]) != MONT_OK) return MONT_EINVAL;
    p.P[j] = P;
  }
  const uint64_t P1 = p.P[0], P2 = p.P[1], P3 = p.P[2];
  const uint32_t i12 = inv_mod(P1, P2);
  const uint32_t i123 = inv_mod((P1 % P3) * (P2 % P3) % P3, P3);
  if (i12 == 0 || i123 == 0 || inv_mod(P1, P3) == 0) return MONT_EINVAL;
  p.inv12 = to_mont_host(i12, p.P[1]);
  p.p1_mod3 = to_mont_host(P1, p.P[2]);
  p.inv123 = to_mont_host(i123, p.P[2]);
  p.reserved = 0;
  *out = p;
  return MONT_OK;
}

extern "C" mont_status crt_reduce(const crt_params* prm, const uint32_t* d_x, size_t n, uint32_t* d_r0,
                                  uint32_t* d_r1, uint32_t* d_r2, void* stream) {
  if (!crt_ok(prm)) return MONT_EINVAL;
  if (n == 0) return MONT_OK;
  if (!d_x || !d_r0 || !d_r1 || !d_r2) return MONT_EINVAL;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_crt_reduce, dim3((unsigned)blocks_for(n, 4)), dim3(CRT_BLOCK), 0, as_stream(stream),
                     prm->P[0], prm->P[1], prm->P[2], d_x, n, d_r0, d_r1, d_r2);
  return last_launch_status();
}

extern "C" mont_status crt_combine(const crt_params* prm, const uint32_t* d_r0, const uint32_t* d_r1,
                                   const uint32_t* d_r2, size_t n, uint32_t* d_out, void* stream) {
  if (!crt_ok(prm)) return MONT_EINVAL;
  if (n == 0) return MONT_OK;
  if (!d_r0 || !d_r1 || !d_r2 || !d_out) return MONT_EINVAL;
  CrtDev c;
  c.m2 = Mod{prm->m[1].P, prm->m[1].Pprime};
  c.m3 = Mod{prm->m[2].P, prm->m[2].Pprime};
  c.P1 = prm->P[0];
  c.P2 = prm->P[1];
  c.P3 = prm->P[2];
  c.inv12 = prm->inv12;
  c.p1_mod3 = prm->p1_mod3;
  c.inv123 = prm->inv123;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_crt_combine, dim3((unsigned)blocks_for(n, 1)), dim3(CRT_BLOCK), 0, as_stream(stream), c, d_r0,
                     d_r1, d_r2, n, d_out);
  return last_launch_status();
}

extern "C" size_t crt_polymul_scratch_bytes(uint32_t da, uint32_t db) {
  const uint64_t na = (uint64_t)da + 1, nb = (uint64_t)db + 1, nc = (uint64_t)da + db + 1;
  return 3 * (align16(4 * na) + align16(4 * nb) + align16(4 * nc)) + ntt_polymul_scratch_bytes(da, db);
}

extern "C" mont_status crt_polymul(const ntt_ctx* ctx, const int* prime_ids, const crt_params* prm,
                                   const uint32_t* d_a, uint32_t da, const uint32_t* d_b, uint32_t db, uint32_t* d_out,
                                   void* d_scratch, size_t scratch_bytes, void* stream) {
  if (!ctx || !prime_ids || !crt_ok(prm) || !d_a || !d_b || !d_out || !d_scratch) return MONT_EINVAL;
  if ((((uintptr_t)d_scratch) & 15u) != 0) return MONT_EINVAL;
  if ((uint64_t)(da < db ? da : db) + 1 > ((uint64_t)1 << 26)) return MONT_ERANGE;
  if ((uint64_t)da + db + 1 > ((uint64_t)1 << 31)) return MONT_ERANGE;
  for (int j = 0; j < 3; j++) {
    mont_params mp;
    const mont_status st = ntt_ctx_prime(ctx, prime_ids[j], &mp, nullptr, nullptr, nullptr, nullptr);
    if (st != MONT_OK) return st;
    if (mp.P != prm->P[j]) return MONT_EINVAL;
  }
  if (scratch_bytes < crt_polymul_scratch_bytes(da, db)) return MONT_ENOMEM;
  const size_t na = (size_t)da + 1, nb = (size_t)db + 1, nc = (size_t)da + db + 1;
  char* s = static_cast<char*>(d_scratch);
  uint32_t *ra[3], *rb[3], *rc[3];
  for (int j = 0; j < 3; j++) {
    ra[j] = reinterpret_cast<uint32_t*>(s); s += align16(4 * na);
    rb[j] = reinterpret_cast<uint32_t*>(s); s += align16(4 * nb);
    rc[j] = reinterpret_cast<uint32_t*>(s); s += align16(4 * nc);
  }
  const size_t nsb = ntt_polymul_scratch_bytes(da, db);
  void* nscratch = nsb ? static_cast<void*>(s) : nullptr;
  mont_status st = crt_reduce(prm, d_a, na, ra[0], ra[1], ra[2], stream);
  if (st == MONT_OK) st = crt_reduce(prm, d_b, nb, rb[0], rb[1], rb[2], stream);
  for (int j = 0; j < 3 && st == MONT_OK; j++)
    st = ntt_polymul(ctx, prime_ids[j], ra[j], da, rb[j], db, rc[j], nscratch, nsb, stream);
  if (st == MONT_OK) st = crt_combine(prm, rc[0], rc[1], rc[2], nc, d_out, stream);
  return st;
}
