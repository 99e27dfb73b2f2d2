/*
 * mont_crt.h -- C ABI of libmont's exact integer polynomial products: three
 * products modulo 31-bit Fourier primes (mont_ntt.h) joined by the Chinese
 * remainder theorem, on AMD Instinct MI355X (gfx950).
 *
 * The paper's word-size modular arithmetic serves computer algebra,
 * polynomial arithmetic and modular FFT libraries (arXiv:1609.00999, sections
 * 1 and 5); products whose coefficients outgrow one word are built from
 * several word-size primes, the multi-modular route.  For uint32 coefficients and
 * min(da, db) + 1 <= 2^26, every coefficient of the integer product is below
 * 2^64 (min(da, db) + 1) <= 2^90 < P1 P2 P3, so the three residues determine
 * it.  The reconstruction is Garner's mixed-radix form
 *   X = r1 + P1 (y2 + P2 y3),  y2 = (r2 - r1) P1^-1 mod P2,
 *   y3 = (r3 - r1 - P1 y2) (P1 P2)^-1 mod P3,
 * whose modular products are Montgomery products (section 3.1, Algorithm 2,
 * R = 2^32) against constants kept in Montgomery form.
 *
 * Conventions are those of mont.h (device pointers d_*, caller-owned,
 * asynchronous on `stream`, validation before anything is enqueued).
 * Integers wider than 32 bits are stored as three little-endian uint32 limbs
 * per element, element i at words 3i, 3i+1, 3i+2.
 */
#ifndef MONT_CRT_H
#define MONT_CRT_H

#include "mont.h"
#include "mont_ntt.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct crt_params {
  uint32_t P[3];       /* distinct primes, 2^30 < P < 2^31                      */
  mont_params m[3];    /* section 3.1 constants of each prime                   */
  uint32_t inv12;      /* Montgomery form mod P2 of P1^-1 mod P2                */
  uint32_t p1_mod3;    /* Montgomery form mod P3 of P1 mod P3                   */
  uint32_t inv123;     /* Montgomery form mod P3 of (P1 P2)^-1 mod P3           */
  uint32_t reserved;   /* zero                                                  */
} crt_params;

/* Constants for the primes (host array of 3).  MONT_EINVAL unless the three
 * are odd, pairwise coprime and in (2^30, 2^31); that they are prime is the
 * caller's promise, as for ntt_ctx_create. */
MONT_API mont_status crt_setup(const uint32_t* primes, crt_params* out);

/* d_r0[i], d_r1[i], d_r2[i] = d_x[i] mod P1, P2, P3 for any uint32 d_x[i]
 * (ordinary residues, ready for ntt_polymul).  Outputs may not overlap the
 * input or each other. */
MONT_API mont_status crt_reduce(const crt_params* prm, const uint32_t* d_x, size_t n, uint32_t* d_r0, uint32_t* d_r1,
                                uint32_t* d_r2, void* stream);

/* d_out (3n words) = the integers X in [0, P1 P2 P3) with X = d_r0[i] mod P1,
 * d_r1[i] mod P2, d_r2[i] mod P3; residues must be canonical. */
MONT_API mont_status crt_combine(const crt_params* prm, const uint32_t* d_r0, const uint32_t* d_r1,
                                 const uint32_t* d_r2, size_t n, uint32_t* d_out, void* stream);

/*
 * crt_polymul -- the exact integer product c = a b of polynomials with uint32
 * coefficients: d_out receives da+db+1 coefficients of 3 limbs each.
 * prime_ids name the context's primes in the order of prm->P (checked).  The
 * steps are one crt_reduce per operand, three ntt_polymul and one
 * crt_combine, all on `stream`.  d_scratch (16-byte aligned) must hold
 * crt_polymul_scratch_bytes(da, db) bytes.  Errors: those of ntt_polymul, and
 * MONT_ERANGE when min(da, db) + 1 > 2^26 (exactness bound above).
 */
MONT_API size_t crt_polymul_scratch_bytes(uint32_t da, uint32_t db);
MONT_API mont_status crt_polymul(const ntt_ctx* ctx, const int* prime_ids, const crt_params* prm, const uint32_t* d_a,
                                 uint32_t da, const uint32_t* d_b, uint32_t db, uint32_t* d_out, void* d_scratch,
                                 size_t scratch_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* MONT_CRT_H */
