/*
 * mont64.h -- C ABI of libmont for 64-bit residues (the paper's 64-bit
 * modular integer type, section 4) on AMD Instinct MI355X (gfx950).
 *
 * Montgomery's reduction as in section 3.1 and Algorithm 2 of Meng,
 * arXiv:1609.00999, with R = 2^64 and an odd modulus P < 2^63:
 *   - precomputation: P' = -P^-1 mod 2^64 (R*R^-1 - P*P' = 1);
 *   - residue of x: x*R mod P;
 *   - REDC(T) for T = a*b < R*P (a 128-bit product): m = (T mod R)*P' mod R,
 *     t = (T + m*P)/R in [0, 2P), then one conditional subtraction of P.
 * A gfx950 lane has 32x32->64 multiplies only, so each 64x64->128 product
 * is assembled from four of them; t is the high 64-bit word of T + m*P,
 * whose low word is zero, plus the carry out of that low word (T mod R != 0).
 *
 * Conventions are those of mont.h: d_* are device pointers owned by the
 * caller, element arrays are contiguous uint64, `stream` is a hipStream_t
 * passed as void*, calls are asynchronous, n == 0 enqueues nothing, in-place
 * operation is allowed, and every function returns a mont_status.
 */
#ifndef MONT64_H
#define MONT64_H

#include "mont.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mont64_params {
  uint64_t P;        /* odd modulus, 3 <= P < 2^63                         */
  uint64_t Pprime;   /* P' = -P^-1 mod 2^64                                */
  uint64_t R1;       /* 2^64 mod P, the residue of 1                       */
  uint64_t R2;       /* 2^128 mod P; REDC(x*R2) is the residue of x        */
  uint32_t k;        /* largest k with 2^k dividing P-1                    */
  uint32_t reserved; /* zero                                               */
} mont64_params;

/* Section 3.1 precomputation for R = 2^64.  MONT_EINVAL if P is even,
 * P < 3, P >= 2^63, or out is NULL. */
MONT_API mont_status mont64_setup(uint64_t P, mont64_params* out);

/* d_out[i] = residue of d_in[i] (any uint64): REDC(d_in[i] * R2). */
MONT_API mont_status mont64_to(const mont64_params* prm, const uint64_t* d_in, uint64_t* d_out, size_t n,
                               void* stream);

/* d_out[i] = d_in[i] * R^-1 mod P (any uint64): REDC(d_in[i]). */
MONT_API mont_status mont64_from(const mont64_params* prm, const uint64_t* d_in, uint64_t* d_out, size_t n,
                                 void* stream);

/* d_out[i] = REDC(d_a[i] * d_b[i]); operands are residues in [0, P). */
MONT_API mont_status mont64_mul(const mont64_params* prm, const uint64_t* d_a, const uint64_t* d_b,
                                uint64_t* d_out, size_t n, void* stream);

/* d_out[i] = (REDC(d_a[i] * d_b[i]) + d_c[i]) mod P; operands in [0, P);
 * d_out may equal d_c. */
MONT_API mont_status mont64_muladd(const mont64_params* prm, const uint64_t* d_a, const uint64_t* d_b,
                                   const uint64_t* d_c, uint64_t* d_out, size_t n, void* stream);

/* d_out[i] = residue of x^e, x the value the residue d_base[i] represents,
 * e = d_exp[i] (any uint64; 0^0 = 1), by fixed 2-bit windows: 95 REDC per
 * element whatever the exponent. */
MONT_API mont_status mont64_pow(const mont64_params* prm, const uint64_t* d_base, const uint64_t* d_exp,
                                uint64_t* d_out, size_t n, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MONT64_H */
