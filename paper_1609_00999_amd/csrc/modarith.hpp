// modarith.hpp -- device-side modular arithmetic on 32-bit residues (gfx950).
//
// Montgomery reduction, Meng arXiv:1609.00999, section 3.1, Algorithm 2, with
// R = 2^32 and an odd modulus P < 2^31.  On a 64-wide wavefront every lane
// forms its own 64-bit product, so the SIMD gather of high and low halves
// that section 2 and section 3.2 spend shuffles on is not needed: the product
// T = a*b and the sum T + m*P come from v_mad_u64_u32, and the "short
// product" m = (T mod R)*P' mod R is one v_mul_lo_u32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mont {

typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Constants a kernel needs for one modulus (a subset of mont_params).
struct Mod {
  uint32_t P;   // odd modulus < 2^31
  uint32_t Pp;  // P' = -P^-1 mod 2^32
};

// Algorithm 2 applied to a 64-bit product T < R*P:
//   m = (T mod R) P' mod R;  t = (T + m P) / R  in [0, 2P);  t >= P ? t - P : t.
// T + mP < 2RP < 2^64, and its low word is zero by the choice of m, so the
// high word is exactly t.  The final comparison is an unsigned min: when
// t < P, t - P wraps above t.
__device__ __forceinline__ uint32_t redc(uint64_t T, Mod md) {
  uint32_t m = (uint32_t)T * md.Pp;
  uint64_t s = (uint64_t)m * md.P + T;
  uint32_t t = (uint32_t)(s >> 32);
  uint32_t u = t - md.P;
  return u < t ? u : t;
}

// Montgomery product of two residues: REDC(a*b) = a b R^-1 mod P.
__device__ __forceinline__ uint32_t mmul(uint32_t a, uint32_t b, Mod md) {
  return redc((uint64_t)a * b, md);
}

// (a + b) mod P for a, b in [0, P): the sum is below 2P < 2^32.
__device__ __forceinline__ uint32_t madd(uint32_t a, uint32_t b, uint32_t P) {
  uint32_t s = a + b;
  uint32_t u = s - P;
  return u < s ? u : s;
}

// (a - b) mod P for a, b in [0, P): on borrow the difference wraps above
// 2^32 - P and adding P brings it back into [0, P).
__device__ __forceinline__ uint32_t msub(uint32_t a, uint32_t b, uint32_t P) {
  uint32_t d = a - b;
  uint32_t u = d + P;
  return u < d ? u : d;
}

}  // namespace mont
