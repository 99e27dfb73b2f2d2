/*
 * oracle.c -- plain, slow, obviously correct CPU oracle for Montgomery
 * modular arithmetic and modular polynomial products.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * bench's CPU-baseline leg may load this file's library.  It shares no code,
 * header, table or constant generator with the GPU library, and it never uses
 * Montgomery reduction: every result is computed from its plain definition
 * with 64-bit products and the C remainder operator.
 *
 * Notation follows Meng, "Automatic Generation of Vectorized Montgomery
 * Algorithm" (arXiv:1609.00999):
 *   - section 3.1, Montgomery algorithm: R coprime to P with R > P, and the
 *     precomputed pair R^-1, P' with 0 < R^-1 < P, 0 < P' < R and
 *     R*R^-1 - P*P' = 1;
 *   - the residue of i is  i_bar = i*R mod P;
 *   - REDC(a_bar, b_bar) is a_bar*b_bar*R^-1 mod P (Algorithm 2), so the
 *     oracle's Montgomery product is that expression evaluated directly.
 * R is 2^r with 1 <= r <= 32; the library's R is 2^32.
 *
 * Functions operate on one contiguous range; the Python wrapper splits large
 * arrays over host threads.
 */
#include <stddef.h>
#include <stdint.h>

/* ------------------------------------------------------------------ */
/* Scalar helpers.                                                     */
/* ------------------------------------------------------------------ */

/* x*y mod m by definition (64-bit product, remainder). */
static uint32_t mulmod(uint32_t x, uint32_t y, uint32_t m) {
  return (uint32_t)(((uint64_t)x * (uint64_t)y) % m);
}

/* x^e mod m by plain left-to-right square-and-multiply. */
static uint32_t powmod(uint32_t x, uint64_t e, uint32_t m) {
  uint32_t r = 1 % m;
  x %= m;
  for (int bit = 63; bit >= 0; bit--) {
    r = mulmod(r, r, m);
    if ((e >> bit) & 1u) r = mulmod(r, x, m);
  }
  return r;
}

/* Inverse of a modulo m (m >= 2) by the extended Euclidean algorithm, as the
 * Montgomery precomputation in section 3.1 prescribes.  Returns 0 when
 * gcd(a, m) != 1.  Works for m up to 2^32. */
static uint64_t inverse_mod(uint64_t a, uint64_t m) {
  int64_t r0 = (int64_t)m, r1 = (int64_t)(a % m);
  int64_t s0 = 0, s1 = 1;
  while (r1 != 0) {
    int64_t q = r0 / r1, t;
    t = r0 - q * r1; r0 = r1; r1 = t;
    t = s0 - q * s1; s0 = s1; s1 = t;
  }
  if (r0 != 1) return 0;
  if (s0 < 0) s0 += (int64_t)m;
  return (uint64_t)s0;
}

/* ------------------------------------------------------------------ */
/* Montgomery precomputation (section 3.1).                            */
/* ------------------------------------------------------------------ */

/*
 * orc_setup: for odd P >= 3 and R = 2^r (1 <= r <= 32, P < R) fill
 *   out[0] = P'   with R*R^-1 - P*P' = 1, 0 < P' < R
 *   out[1] = R mod P          (the residue of 1)
 *   out[2] = R^2 mod P
 *   out[3] = R^-1 mod P       (0 < R^-1 < P)
 *   out[4] = largest k with 2^k dividing P - 1
 * Returns 0 on success, -1 if P is even, P < 3, r is out of range, P >= R,
 * or gcd(R, P) != 1.
 */
int orc_setup(uint32_t P, int r, uint32_t out[5]) {
  if (r < 1 || r > 32 || P < 3 || (P & 1u) == 0) return -1;
  uint64_t R = (uint64_t)1 << r;
  if ((uint64_t)P >= R) return -1;
  uint64_t Rmod = R % P;
  uint64_t Rinv = inverse_mod(Rmod, P);
  if (Rinv == 0) return -1;
  /* R*R^-1 - 1 is a multiple of P; the quotient is P' (section 3.1). */
  uint64_t RRinv = R * Rinv; /* < 2^32 * 2^31 */
  uint64_t Pp = (RRinv - 1) / P;
  out[0] = (uint32_t)Pp;
  out[1] = (uint32_t)Rmod;
  out[2] = (uint32_t)((Rmod * Rmod) % P);
  out[3] = (uint32_t)Rinv;
  uint32_t k = 0, q = P - 1;
  while ((q & 1u) == 0) { q >>= 1; k++; }
  out[4] = k;
  return 0;
}

/* ------------------------------------------------------------------ */
/* Elementwise operations on residues (section 3.1).                   */
/* ------------------------------------------------------------------ */

/* Residue of a: a*R mod P, R = 2^r.  Defined for every uint32 a. */
void orc_to(uint32_t P, int r, const uint32_t* in, uint32_t* out, size_t n) {
  for (size_t i = 0; i < n; i++) {
    uint64_t aR = (uint64_t)(in[i] % P) << r;   /* (a mod P) * 2^r < 2^63 */
    out[i] = (uint32_t)(aR % P);
  }
}

/* Back from a residue: x*R^-1 mod P.  Defined for every uint32 x. */
void orc_from(uint32_t P, uint32_t Rinv, const uint32_t* in, uint32_t* out, size_t n) {
  for (size_t i = 0; i < n; i++) out[i] = mulmod(in[i] % P, Rinv, P);
}

/* Montgomery product a_bar*b_bar*R^-1 mod P (the value Algorithm 2 returns). */
void orc_mul(uint32_t P, uint32_t Rinv, const uint32_t* a, const uint32_t* b, uint32_t* out, size_t n) {
  for (size_t i = 0; i < n; i++) out[i] = mulmod(mulmod(a[i], b[i], P), Rinv, P);
}

/* (a_bar*b_bar*R^-1 + c_bar) mod P: the residue representation leaves
 * modular addition unchanged (section 3.1). */
void orc_muladd(uint32_t P, uint32_t Rinv, const uint32_t* a, const uint32_t* b, const uint32_t* c,
                uint32_t* out, size_t n) {
  for (size_t i = 0; i < n; i++) {
    uint64_t prod = mulmod(mulmod(a[i], b[i], P), Rinv, P);
    out[i] = (uint32_t)((prod + (uint64_t)(c[i] % P)) % P);
  }
}

/* Powers in the residue system: base_bar is a residue, the exponent is an
 * ordinary uint32.  The result is the residue of a^e where a is the value
 * base_bar represents; 0^0 is taken as 1. */
void orc_pow(uint32_t P, int r, uint32_t Rinv, const uint32_t* base, const uint32_t* e, uint32_t* out,
             size_t n) {
  for (size_t i = 0; i < n; i++) {
    uint32_t a = mulmod(base[i] % P, Rinv, P);
    uint32_t v = powmod(a, e[i], P);
    out[i] = (uint32_t)(((uint64_t)v << r) % P);
  }
}

/* ------------------------------------------------------------------ */
/* Polynomial products modulo P.                                       */
/* ------------------------------------------------------------------ */

/* c_k = sum_{i+j=k} a_i b_j mod P for k = 0..da+db (schoolbook). */
void orc_polymul_schoolbook(uint32_t P, const uint32_t* a, uint32_t da, const uint32_t* b, uint32_t db,
                            uint32_t* c) {
  for (uint64_t k = 0; k <= (uint64_t)da + db; k++) c[k] = 0;
  for (uint32_t i = 0; i <= da; i++) {
    uint32_t ai = a[i] % P;
    for (uint32_t j = 0; j <= db; j++) {
      uint64_t s = (uint64_t)c[i + j] + mulmod(ai, b[j], P);
      c[i + j] = (uint32_t)(s % P);
    }
  }
}

/* Value of a(x) = sum a_i x^i at x mod P (Horner's rule). */
uint32_t orc_horner(uint32_t P, const uint32_t* a, uint32_t d, uint32_t x) {
  uint32_t acc = 0;
  for (int64_t i = d; i >= 0; i--) acc = (uint32_t)(((uint64_t)mulmod(acc, x, P) + a[i] % P) % P);
  return acc;
}

/* Smallest primitive root modulo the prime P: the least g >= 2 with
 * g^((P-1)/q) != 1 for every prime q dividing P-1.  Returns 0 if none is
 * found below P (P not prime). */
uint32_t orc_primitive_root(uint32_t P) {
  uint32_t q[32];
  int nq = 0;
  uint32_t m = P - 1;
  for (uint32_t f = 2; (uint64_t)f * f <= m; f++) {
    if (m % f == 0) {
      q[nq++] = f;
      while (m % f == 0) m /= f;
    }
  }
  if (m > 1) q[nq++] = m;
  for (uint32_t g = 2; g < P; g++) {
    int ok = 1;
    for (int i = 0; i < nq && ok; i++)
      if (powmod(g, (P - 1) / q[i], P) == 1) ok = 0;
    if (ok) return g;
  }
  return 0;
}

/* Textbook iterative number-theoretic transform of length N = 2^logn over
 * Z_P, in place: bit-reversal permutation, then Cooley-Tukey butterflies
 * with root w (an element of order N).  Output A_k = sum_j a_j w^(jk). */
static void plain_ntt(uint32_t P, uint32_t* A, uint32_t logn, uint32_t w) {
  uint64_t N = (uint64_t)1 << logn;
  for (uint64_t i = 0, j = 0; i < N; i++) {
    if (i < j) { uint32_t t = A[i]; A[i] = A[j]; A[j] = t; }
    uint64_t bit = N >> 1;
    while (bit && (j & bit)) { j ^= bit; bit >>= 1; }
    j |= bit;
  }
  for (uint64_t len = 2; len <= N; len <<= 1) {
    uint32_t wlen = powmod(w, N / len, P);
    for (uint64_t i = 0; i < N; i += len) {
      uint32_t wj = 1;
      for (uint64_t j = 0; j < len / 2; j++) {
        uint32_t u = A[i + j];
        uint32_t v = mulmod(A[i + j + len / 2], wj, P);
        A[i + j] = (uint32_t)(((uint64_t)u + v) % P);
        A[i + j + len / 2] = (uint32_t)(((uint64_t)u + P - v) % P);
        wj = mulmod(wj, wlen, P);
      }
    }
  }
}

/* Forward transform exposed for invariant checks; w must have order 2^logn. */
void orc_ntt(uint32_t P, uint32_t* A, uint32_t logn, uint32_t w) { plain_ntt(P, A, logn, w); }

/*
 * Polynomial product through the plain transform: N = smallest power of two
 * >= da+db+1, root w = g^((P-1)/N) with g the smallest primitive root (passed
 * in by the caller, computed by orc_primitive_root), inverse transform with
 * w^-1 and scaling by N^-1.  work must hold 2N uint32.  Returns 0, or -1 if
 * 2^k with k = v2(P-1) is smaller than N.
 */
int orc_polymul_ntt(uint32_t P, uint32_t g, const uint32_t* a, uint32_t da, const uint32_t* b, uint32_t db,
                    uint32_t* c, uint32_t* work) {
  uint64_t need = (uint64_t)da + db + 1;
  uint32_t logn = 0;
  while (((uint64_t)1 << logn) < need) logn++;
  uint64_t N = (uint64_t)1 << logn;
  if ((P - 1) % N != 0) return -1;
  uint32_t* A = work;
  uint32_t* B = work + N;
  for (uint64_t i = 0; i < N; i++) {
    A[i] = i <= da ? a[i] % P : 0;
    B[i] = i <= db ? b[i] % P : 0;
  }
  uint32_t w = powmod(g, (P - 1) / N, P);
  plain_ntt(P, A, logn, w);
  plain_ntt(P, B, logn, w);
  for (uint64_t i = 0; i < N; i++) A[i] = mulmod(A[i], B[i], P);
  uint32_t winv = powmod(w, P - 2, P);
  plain_ntt(P, A, logn, winv);
  uint32_t ninv = powmod((uint32_t)(N % P), P - 2, P);
  for (uint64_t k = 0; k < need; k++) c[k] = mulmod(A[k], ninv, P);
  return 0;
}

/* Ordinary modular product a*b mod P and power a^e mod P (no residue
 * representation): the results Algorithm 1 (Barrett) must reproduce. */
void orc_modmul(uint32_t P, const uint32_t* a, const uint32_t* b, uint32_t* out, size_t n) {
  for (size_t i = 0; i < n; i++) out[i] = mulmod(a[i] % P, b[i] % P, P);
}

void orc_modpow(uint32_t P, const uint32_t* base, const uint32_t* e, uint32_t* out, size_t n) {
  for (size_t i = 0; i < n; i++) out[i] = powmod(base[i], e[i], P);
}
