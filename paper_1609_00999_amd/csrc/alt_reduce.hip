// alt_reduce.hip -- the paper's two other modular multiplications on the
// device, for comparison with Algorithm 2: Algorithm 3 (REDC for Fourier
// primes, on Montgomery residues) and Algorithm 1 (Barrett, on ordinary
// residues), elementwise and inside fixed 2-bit-window powers.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "modarith.hpp"

namespace mont {

namespace {
// Algorithm 3 of arXiv:1609.00999 (section 3.1): REDC for a Fourier prime
// P = c 2^k + 1 with 2k >= 32, so that K = c 2^k = P - 1 and K^2 = 0 mod R.
// With T = q1 R + r1:  q2 R + r2 = K r1,  q3 = floor(K r2 / R),  and
// T R^-1 = q1 - q2 + q3 (mod P) with the sum in (-(P-1), 2(P-1)).  For P
// above 2^30 the sum leaves the int32 range, so the sign-mask corrections of
// the paper are replaced by an explicit borrow: s = q1 + q3 < 2P fits in 32
// bits; d = s - q2 gets P added back on borrow, which leaves it in [0, 2P),
// and one conditional subtraction makes it canonical.
__device__ __forceinline__ uint32_t redc_fourier(uint64_t T, uint32_t P) {
  const uint32_t K = P - 1;
  const uint32_t q1 = (uint32_t)(T >> 32), r1 = (uint32_t)T;
  const uint64_t u = (uint64_t)r1 * K;
  const uint32_t q2 = (uint32_t)(u >> 32), r2 = (uint32_t)u;
  const uint32_t q3 = __umulhi(r2, K);
  const uint32_t s = q1 + q3;
  uint32_t d = s - q2;
  d = s < q2 ? d + P : d;                 // negative sum: add P back
  const uint32_t dm = d - P;
  return dm < d ? dm : d;
}

// Algorithm 1 (Barrett), on ordinary residues: with k the bit length of P and
// Pb = floor(2^(2k) / P),  m = floor(ab / 2^k),  q = floor(m Pb / 2^k),
// t = ab - qP in [0, 4P).  For a, b < P every factor fits in 32 bits:
// m < 2^k <= 2^31, Pb < 2^(k+1) <= 2^32 since P > 2^(k-1), and q <= ab/P < P,
// so each product is one 32x32->64 multiply.  The correction loop (at most
// three subtractions of P) is taken as one conditional subtraction of 2P and
// one of P, which gives the same result for every t < 4P.
__device__ __forceinline__ uint32_t barrett_mul(uint32_t a, uint32_t b, uint32_t P, uint32_t Pb, uint32_t k) {
  const uint64_t ab = (uint64_t)a * b;
  const uint32_t m = (uint32_t)(ab >> k);
  const uint32_t q = (uint32_t)(((uint64_t)m * Pb) >> k);
  const uint64_t t = ab - (uint64_t)q * P;             // [0, 4P), up to 33 bits
  const uint64_t d = t - 2 * (uint64_t)P;              // wraps iff t < 2P
  const uint32_t t1 = (int64_t)d < 0 ? (uint32_t)t : (uint32_t)d;   // [0, 2P)
  const uint32_t t2 = t1 - P;
  return t2 < t1 ? t2 : t1;
}


enum AltAlg { ALG_FOURIER = 0, ALG_BARRETT = 1 };

struct AltMod {
  uint32_t P;
  uint32_t k;     // Barrett: bit length of P
  uint32_t Pb;    // Barrett: floor(2^(2k) / P), below 2^32 for odd P
};

template <int ALG>
__device__ __forceinline__ uint32_t alt_mul(uint32_t a, uint32_t b, const AltMod& md) {
  if constexpr (ALG == ALG_FOURIER) return redc_fourier((uint64_t)a * b, md.P);
  else return barrett_mul(a, b, md.P, md.Pb, md.k);
}

// Same window schedule as mont_pow: table {1, x, x^2, x^3}, 15 windows.
template <int ALG>
__device__ __forceinline__ uint32_t alt_pow(uint32_t x, uint32_t e, const AltMod& md, uint32_t one) {
  const uint32_t x2 = alt_mul<ALG>(x, x, md);
  const uint32_t x3 = alt_mul<ALG>(x2, x, md);
  auto pick = [&](uint32_t d) {
    uint32_t lo = (d & 1u) ? x : one;
    uint32_t hi = (d & 1u) ? x3 : x2;
    return (d & 2u) ? hi : lo;
  };
  uint32_t r = pick(e >> 30);
#pragma unroll
  for (int s = 28; s >= 0; s -= 2) {
    r = alt_mul<ALG>(r, r, md);
    r = alt_mul<ALG>(r, r, md);
    r = alt_mul<ALG>(r, pick((e >> s) & 3u), md);
  }
  return r;
}

template <int ALG, bool POW>
__global__ __launch_bounds__(256) void k_alt(AltMod md, uint32_t one, const uint32_t* a, const uint32_t* b,
                                             uint32_t* out, size_t n) {
  const size_t nvec = n >> 2;
  const bool al = ((((uintptr_t)a) | ((uintptr_t)b) | ((uintptr_t)out)) & 15u) == 0;
  const size_t stride = (size_t)gridDim.x * 256;
  if (al) {
    const v4u* va = reinterpret_cast<const v4u*>(a);
    const v4u* vb = reinterpret_cast<const v4u*>(b);
    v4u* vo = reinterpret_cast<v4u*>(out);
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < nvec; i += stride) {
      const v4u x = __builtin_nontemporal_load(va + i), y = __builtin_nontemporal_load(vb + i);
      v4u r;
      if constexpr (POW) {
        r.x = alt_pow<ALG>(x.x, y.x, md, one);
        r.y = alt_pow<ALG>(x.y, y.y, md, one);
        r.z = alt_pow<ALG>(x.z, y.z, md, one);
        r.w = alt_pow<ALG>(x.w, y.w, md, one);
      } else {
        r.x = alt_mul<ALG>(x.x, y.x, md);
        r.y = alt_mul<ALG>(x.y, y.y, md);
        r.z = alt_mul<ALG>(x.z, y.z, md);
        r.w = alt_mul<ALG>(x.w, y.w, md);
      }
      __builtin_nontemporal_store(r, vo + i);
    }
  }
  for (size_t i = (al ? (nvec << 2) : 0) + (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
    out[i] = POW ? alt_pow<ALG>(a[i], b[i], md, one) : alt_mul<ALG>(a[i], b[i], md);
}

template <int ALG, bool POW>
mont_status launch_alt(const AltMod& md, uint32_t one, const uint32_t* a, const uint32_t* b, uint32_t* out,
                       size_t n, void* stream) {
  if (n == 0) return MONT_OK;
  if (!a || !b || !out) return MONT_EINVAL;
  (void)hipGetLastError();
  size_t blocks = (n / 4 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > ((size_t)1 << 20)) blocks = (size_t)1 << 20;
  hipLaunchKernelGGL((k_alt<ALG, POW>), dim3((unsigned)blocks), dim3(256), 0, as_stream(stream), md, one, a, b, out,
                     n);
  return last_launch_status();
}

bool fourier_ok(const mont_params* prm) { return params_ok(prm) && prm->k >= 16; }

bool barrett_setup(uint32_t P, AltMod& md) {
  if (P < 3 || (P & 1u) == 0 || P >= 0x80000000u) return false;
  uint32_t k = 0;
  while ((1u << k) <= P) k++;        // bit length: 2^(k-1) <= P < 2^k
  md.P = P;
  md.k = k;
  md.Pb = (uint32_t)((((uint64_t)1) << (2 * k)) / P);
  return true;
}

}  // namespace

}  // namespace mont

using namespace mont;

extern "C" mont_status mont_mul_fourier(const mont_params* prm, const uint32_t* d_a, const uint32_t* d_b,
                                        uint32_t* d_out, size_t n, void* stream) {
  if (!fourier_ok(prm)) return MONT_EINVAL;
  AltMod md{prm->P, 0, 0};
  return launch_alt<ALG_FOURIER, false>(md, 0, d_a, d_b, d_out, n, stream);
}

extern "C" mont_status mont_pow_fourier(const mont_params* prm, const uint32_t* d_base, const uint32_t* d_exp,
                                        uint32_t* d_out, size_t n, void* stream) {
  if (!fourier_ok(prm)) return MONT_EINVAL;
  AltMod md{prm->P, 0, 0};
  return launch_alt<ALG_FOURIER, true>(md, prm->R1, d_base, d_exp, d_out, n, stream);
}

extern "C" mont_status modmul_barrett(uint32_t P, const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_out, size_t n,
                                      void* stream) {
  AltMod md;
  if (!barrett_setup(P, md)) return MONT_EINVAL;
  return launch_alt<ALG_BARRETT, false>(md, 0, d_a, d_b, d_out, n, stream);
}

extern "C" mont_status modpow_barrett(uint32_t P, const uint32_t* d_base, const uint32_t* d_exp, uint32_t* d_out,
                                      size_t n, void* stream) {
  AltMod md;
  if (!barrett_setup(P, md)) return MONT_EINVAL;
  return launch_alt<ALG_BARRETT, true>(md, 1, d_base, d_exp, d_out, n, stream);
}
