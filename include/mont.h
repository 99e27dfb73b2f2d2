/*
 * mont.h -- C ABI of libmont: Montgomery modular arithmetic on 32-bit
 * residues for AMD Instinct MI355X (gfx950).
 *
 * The arithmetic is Montgomery's reduction as stated in Meng, "Automatic
 * Generation of Vectorized Montgomery Algorithm" (arXiv:1609.00999), section
 * 3.1 and Algorithm 2, with R = 2^32:
 *   - precomputation: P' with R*R^-1 - P*P' = 1, i.e. P' = -P^-1 mod 2^32;
 *   - residue representation: x_bar = x*R mod P;
 *   - REDC(a_bar, b_bar): T = a_bar*b_bar, m = (T mod R)*P' mod R,
 *     t = (T + m*P)/R, then one conditional subtraction of P.  The result is
 *     a_bar*b_bar*R^-1 mod P, canonical in [0, P), provided a_bar*b_bar < R*P.
 *
 * Conventions for every entry point below:
 *   - Pointers named d_* are DEVICE pointers (memory on the current HIP
 *     device); every other pointer is a HOST pointer.  The caller owns all of
 *     them.  Element arrays are contiguous uint32.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every device operation is asynchronous on that stream: results are valid
 *     once the stream has been synchronized.  Host-side validation happens
 *     before anything is enqueued; on error nothing is enqueued.
 *   - In-place operation (d_out equal to an input pointer) is allowed for the
 *     elementwise calls.  Partially overlapping arrays are not.
 *   - n == 0 is valid and enqueues nothing.  A NULL device pointer with
 *     n > 0 returns MONT_EINVAL.
 *   - No function throws; each returns a mont_status.  HIP runtime failures
 *     (launch errors) are reported as MONT_EHIP.
 *   - Operands outside [0, P) for mont_mul, mont_muladd and mont_pow give a
 *     deterministic but unspecified value (Algorithm 2 needs a_bar*b_bar < RP).
 *     The checked mode is mont_check_range below, enqueued on the same
 *     stream before the call.
 */
#ifndef MONT_H
#define MONT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define MONT_API __attribute__((visibility("default")))
#else
#define MONT_API
#endif

typedef int mont_status;
#define MONT_OK 0
#define MONT_EINVAL (-1)   /* bad argument: modulus, size, pointer, id      */
#define MONT_ERANGE (-2)   /* a size or index exceeds what the call supports */
#define MONT_ENOROOT (-3)  /* 2^k does not divide P-1 for the needed length  */
#define MONT_ENOMEM (-4)   /* scratch or device memory too small / exhausted */
#define MONT_EHIP (-5)     /* HIP runtime error                              */
#define MONT_ETIMEOUT (-6) /* a bounded device-side wait gave up             */

/*
 * Per-modulus constants (section 3.1, Montgomery precomputation).  Plain
 * data: the caller owns it and may copy it freely.
 */
typedef struct mont_params {
  uint32_t P;      /* odd modulus, 3 <= P < 2^31                          */
  uint32_t Pprime; /* P' = -P^-1 mod 2^32, so that R*R^-1 - P*P' = 1     */
  uint32_t R1;     /* R mod P, the residue of 1                           */
  uint32_t R2;     /* R^2 mod P; REDC(x*R2) is the residue of x           */
  uint32_t k;      /* largest k with 2^k dividing P-1                     */
} mont_params;

/* Human-readable text for a status code (static storage, never NULL). */
MONT_API const char* mont_strerror(mont_status status);

/*
 * mont_setup -- section 3.1 precomputation for modulus P with R = 2^32.
 * Fills *out.  Returns MONT_EINVAL if out is NULL, P is even, P < 3 or
 * P >= 2^31 (t < 2P must fit in 32 bits).  Odd composite P is accepted:
 * REDC needs only gcd(P, R) = 1.  Host only; enqueues nothing.
 */
MONT_API mont_status mont_setup(uint32_t P, mont_params* out);

/*
 * mont_to -- residues: d_out[i] = d_in[i]*R mod P, computed as
 * REDC(d_in[i], R2).  Accepts every uint32 input (d_in[i]*R2 < R*P holds for
 * any 32-bit d_in[i]).  prm is a host pointer to constants from mont_setup.
 */
MONT_API mont_status mont_to(const mont_params* prm, const uint32_t* d_in, uint32_t* d_out, size_t n, void* stream);

/*
 * mont_from -- back from residues: d_out[i] = d_in[i]*R^-1 mod P, computed as
 * REDC(d_in[i], 1).  Accepts every uint32 input; output in [0, P).
 */
MONT_API mont_status mont_from(const mont_params* prm, const uint32_t* d_in, uint32_t* d_out, size_t n, void* stream);

/*
 * mont_mul -- Algorithm 2 elementwise: d_out[i] = REDC(d_a[i], d_b[i]) =
 * d_a[i]*d_b[i]*R^-1 mod P.  Operands are residues in [0, P).
 */
MONT_API mont_status mont_mul(const mont_params* prm, const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_out,
                     size_t n, void* stream);

/*
 * mont_muladd -- d_out[i] = (REDC(d_a[i], d_b[i]) + d_c[i]) mod P: a Montgomery
 * product followed by an ordinary modular addition, which the residue
 * representation leaves unchanged (section 3.1).  Operands in [0, P).
 * d_out may equal d_c (accumulate in place).
 */
MONT_API mont_status mont_muladd(const mont_params* prm, const uint32_t* d_a, const uint32_t* d_b, const uint32_t* d_c,
                        uint32_t* d_out, size_t n, void* stream);

/*
 * mont_pow -- d_out[i] = d_base[i]^d_exp[i] in the residue system: d_base[i]
 * is a residue in [0, P), d_exp[i] an ordinary 32-bit exponent, and the result
 * is the residue of a^e (0^0 gives the residue of 1).  Every step is a REDC
 * product of residues, which keeps long chains of products in residue form
 * as section 3.1 recommends.
 */
MONT_API mont_status mont_pow(const mont_params* prm, const uint32_t* d_base, const uint32_t* d_exp, uint32_t* d_out,
                     size_t n, void* stream);

/*
 * mont_modmul -- d_out[i] = d_a[i] * d_b[i] mod P for ORDINARY values (any
 * uint32, not residues): the to / mul / from pipeline of section 3.1 in one
 * pass, with two Montgomery products instead of four: REDC(d_b[i] * R2) is
 * the residue of d_b[i], and REDC(d_a[i] * that) = d_a[i] d_b[i] mod P
 * (the product stays below R P for every uint32 operand).  Canonical output;
 * in place allowed.
 */
MONT_API mont_status mont_modmul(const mont_params* prm, const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_out,
                                 size_t n, void* stream);

/*
 * mont_check_range -- checked mode of the operand contract above: if any
 * d_x[i] >= P for i < n, stores MONT_ERANGE into the device word *d_status;
 * otherwise it does not write *d_status at all.  A status word the caller has
 * zeroed therefore accumulates over any number of checks (on one stream or
 * several), and the caller reads it after synchronizing.  P is any nonzero
 * bound (the modulus for residues and coefficients).  d_status must be a
 * 4-byte aligned device pointer.  Reads n words from HBM; not needed on the
 * fast path.  Errors: MONT_EINVAL (P == 0, NULL or misaligned pointer),
 * MONT_EHIP.
 */
MONT_API mont_status mont_check_range(uint32_t P, const uint32_t* d_x, size_t n, int32_t* d_status, void* stream);

/*
 * The paper's other two modular multiplications, for comparison with
 * Algorithm 2 (section 3.1).
 *
 * mont_mul_fourier / mont_pow_fourier -- Algorithm 3 (REDC for a Fourier
 * prime P = c 2^k + 1 with 2k >= 32, i.e. prm->k >= 16): with K = c 2^k = P-1
 * and T = a*b = q1 R + r1, K r1 = q2 R + r2 and q3 = floor(K r2 / R), the
 * result is q1 - q2 + q3 reduced into [0, P).  The paper's corrections use an
 * arithmetic shift of a signed 32-bit sum in (-(P-1), 2(P-1)), which
 * overflows once P > 2^30; these kernels take the sign from an explicit
 * borrow instead, so they are exact for every 31-bit Fourier prime.  Same
 * operands, results and contracts as mont_mul / mont_pow (residues in and
 * out).  MONT_EINVAL if prm->k < 16.
 */
MONT_API mont_status mont_mul_fourier(const mont_params* prm, const uint32_t* d_a, const uint32_t* d_b,
                                      uint32_t* d_out, size_t n, void* stream);
MONT_API mont_status mont_pow_fourier(const mont_params* prm, const uint32_t* d_base, const uint32_t* d_exp,
                                      uint32_t* d_out, size_t n, void* stream);

/*
 * modmul_barrett / modpow_barrett -- Algorithm 1 (Barrett) on ORDINARY
 * residues (no Montgomery form): d_out[i] = d_a[i]*d_b[i] mod P, respectively
 * d_base[i]^d_exp[i] mod P (0^0 = 1).  With k the bit length of P and
 * P' = floor(2^(2k) / P): m = floor(ab / 2^k), q = floor(m P' / 2^k),
 * t = ab - qP < 4P, at most three subtractions.  Odd 3 <= P < 2^31; operands
 * in [0, P).  MONT_EINVAL for an invalid P.
 */
MONT_API mont_status modmul_barrett(uint32_t P, const uint32_t* d_a, const uint32_t* d_b, uint32_t* d_out, size_t n,
                                    void* stream);
MONT_API mont_status modpow_barrett(uint32_t P, const uint32_t* d_base, const uint32_t* d_exp, uint32_t* d_out,
                                    size_t n, void* stream);

/*
 * Batches of vectors.  One descriptor per vector: device pointers a, b, out
 * (n residues each, out may equal a or b), and the vector's own modulus P
 * with P' = -P^-1 mod 2^32 as mont_setup returns them.
 */
typedef struct mont_vec_desc {
  const uint32_t* a;
  const uint32_t* b;
  uint32_t* out;
  uint64_t n;
  uint32_t P, Pprime;
} mont_vec_desc;

typedef struct mont_batch mont_batch;

/* mont_batch_reserve -- a reusable batch object for up to max_vectors
 * vectors (device descriptor array plus pinned staging). */
MONT_API mont_status mont_batch_reserve(int max_vectors, mont_batch** out);

/*
 * mont_batch_update -- loads `count` host descriptors.  Up to 16 are kept on
 * the host and passed to the kernel in its launch arguments; more are
 * uploaded asynchronously on `stream` (launches that use them go on the same
 * stream, after this call).  Blocks only until the previous upload has left
 * the staging buffer.  Errors: MONT_EINVAL (bad modulus pair, NULL pointer
 * with n > 0), MONT_ERANGE (count above the reserved capacity), MONT_EHIP.
 */
MONT_API mont_status mont_batch_update(mont_batch* b, const mont_vec_desc* descs, int count, void* stream);

/*
 * mont_batch_mul -- Algorithm 2 elementwise over every vector of the batch in
 * ONE launch: out_i[j] = REDC(a_i[j] * b_i[j]) modulo P_i.  The work is cut
 * into tiles of 4096 residues that never straddle two vectors, one workgroup
 * per tile.  Operands are residues in [0, P_i).
 */
MONT_API mont_status mont_batch_mul(const mont_batch* b, void* stream);

/* Frees the batch object (synchronizes the device first). */
MONT_API mont_status mont_batch_destroy(mont_batch* b);

/*
 * Launch-shape tuning of the streaming elementwise kernels (used by the
 * autotuner).  op: 0 = to, 1 = from, 2 = mul, 3 = muladd, 4 = pow, 5 = modmul.  block is
 * 64, 128, 256 or 512 threads, vpt 1, 2 or 4 128-bit vectors per thread, nontemporal
 * 0 or 1.  Settings are process-wide and take effect on the next call; they
 * never change results.  Returns MONT_EINVAL for values outside those sets.
 */
MONT_API mont_status mont_elem_tune_set(int op, int block, int vpt, int nontemporal);
MONT_API mont_status mont_elem_tune_get(int op, int* block, int* vpt, int* nontemporal);

#ifdef __cplusplus
}
#endif

#endif /* MONT_H */
