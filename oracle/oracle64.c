/*
 * oracle64.c -- plain CPU oracle for Montgomery arithmetic on 64-bit
 * residues (the paper's 64-bit modular integer type, section 4), and for the
 * Chinese-remainder reconstruction of integer polynomial products.
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: it shares nothing with the GPU
 * library, never uses Montgomery reduction, and computes every result from
 * its plain definition with 128-bit products and the C remainder operator.
 *
 * Section 3.1 with R = 2^r, 1 <= r <= 64: R^-1 and P' with
 * R*R^-1 - P*P' = 1, 0 < R^-1 < P, 0 < P' < R; the residue of i is i*R mod P,
 * and the Montgomery product of residues is a*b*R^-1 mod P.
 */
#include <stddef.h>
#include <stdint.h>

typedef unsigned __int128 u128;
typedef __int128 i128;

static uint64_t mulmod64(uint64_t x, uint64_t y, uint64_t m) { return (uint64_t)(((u128)x * y) % m); }

static uint64_t powmod64(uint64_t x, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  x %= m;
  for (int bit = 63; bit >= 0; bit--) {
    r = mulmod64(r, r, m);
    if ((e >> bit) & 1u) r = mulmod64(r, x, m);
  }
  return r;
}

/* Inverse of a modulo m by the extended Euclidean algorithm in 128-bit
 * signed arithmetic; 0 when gcd(a, m) != 1. */
static uint64_t inverse_mod64(uint64_t a, uint64_t m) {
  i128 r0 = (i128)m, r1 = (i128)(a % m);
  i128 s0 = 0, s1 = 1;
  while (r1 != 0) {
    i128 q = r0 / r1, t;
    t = r0 - q * r1; r0 = r1; r1 = t;
    t = s0 - q * s1; s0 = s1; s1 = t;
  }
  if (r0 != 1) return 0;
  if (s0 < 0) s0 += (i128)m;
  return (uint64_t)s0;
}

/* (1 << r) mod P for r <= 64, through 128 bits. */
static uint64_t pow2_mod(int r, uint64_t P) { return (uint64_t)((((u128)1) << r) % P); }

/*
 * orc64_setup: odd P >= 3, R = 2^r with 1 <= r <= 64 and P < R:
 *   out[0] = P'  (R*R^-1 - P*P' = 1),  out[1] = R mod P,  out[2] = R^2 mod P,
 *   out[3] = R^-1 mod P,  out[4] = largest k with 2^k dividing P - 1.
 * Returns -1 on an invalid modulus.
 */
int orc64_setup(uint64_t P, int r, uint64_t out[5]) {
  if (r < 1 || r > 64 || P < 3 || (P & 1u) == 0) return -1;
  if (r < 64 && P >= ((uint64_t)1 << r)) return -1;
  uint64_t Rmod = pow2_mod(r, P);
  uint64_t Rinv = inverse_mod64(Rmod, P);
  if (Rinv == 0) return -1;
  u128 RRinv = (((u128)1) << r) * Rinv;  /* < 2^64 * 2^64 */
  out[0] = (uint64_t)((RRinv - 1) / P);
  out[1] = Rmod;
  out[2] = mulmod64(Rmod, Rmod, P);
  out[3] = Rinv;
  uint64_t k = 0, q = P - 1;
  while ((q & 1u) == 0) { q >>= 1; k++; }
  out[4] = k;
  return 0;
}

/* Residue a*R mod P of every uint64 a. */
void orc64_to(uint64_t P, int r, const uint64_t* in, uint64_t* out, size_t n) {
  uint64_t Rmod = pow2_mod(r, P);
  for (size_t i = 0; i < n; i++) out[i] = mulmod64(in[i] % P, Rmod, P);
}

/* x*R^-1 mod P of every uint64 x. */
void orc64_from(uint64_t P, uint64_t Rinv, const uint64_t* in, uint64_t* out, size_t n) {
  for (size_t i = 0; i < n; i++) out[i] = mulmod64(in[i] % P, Rinv, P);
}

/* Montgomery product a*b*R^-1 mod P. */
void orc64_mul(uint64_t P, uint64_t Rinv, const uint64_t* a, const uint64_t* b, uint64_t* out, size_t n) {
  for (size_t i = 0; i < n; i++) out[i] = mulmod64(mulmod64(a[i], b[i], P), Rinv, P);
}

/* (a*b*R^-1 + c) mod P. */
void orc64_muladd(uint64_t P, uint64_t Rinv, const uint64_t* a, const uint64_t* b, const uint64_t* c,
                  uint64_t* out, size_t n) {
  for (size_t i = 0; i < n; i++) {
    uint64_t p = mulmod64(mulmod64(a[i], b[i], P), Rinv, P);
    out[i] = (uint64_t)(((u128)p + (c[i] % P)) % P);
  }
}

/* Residue of x^e where x is the value the residue base represents (0^0 = 1). */
void orc64_pow(uint64_t P, int r, uint64_t Rinv, const uint64_t* base, const uint64_t* e, uint64_t* out,
               size_t n) {
  uint64_t Rmod = pow2_mod(r, P);
  for (size_t i = 0; i < n; i++) {
    uint64_t x = mulmod64(base[i], Rinv, P);
    out[i] = mulmod64(powmod64(x, e[i], P), Rmod, P);
  }
}

/*
 * orc_crt: the unique integer X with 0 <= X < P_0 * ... * P_{np-1} and
 * X = r_j mod P_j for every j, for each of n residue tuples, written as
 * `limbs` little-endian 32-bit words (the product of the moduli must be below
 * 2^(32 limbs)).  Residue j of element i is res[j*n + i].  Computed from the
 * textbook formula X = sum_j r_j M_j (M_j^-1 mod P_j) mod M with M = prod P_j,
 * M_j = M / P_j, in 32-bit-limb schoolbook arithmetic.  Supports np <= 6
 * moduli below 2^32.  Returns -1 on bad arguments.
 */
#define CRT_MAXW 8
static void big_mul_small(uint32_t* x, int w, uint32_t s) {
  uint64_t carry = 0;
  for (int i = 0; i < w; i++) {
    uint64_t t = (uint64_t)x[i] * s + carry;
    x[i] = (uint32_t)t;
    carry = t >> 32;
  }
}
static void big_add(uint32_t* x, const uint32_t* y, int w) {
  uint64_t carry = 0;
  for (int i = 0; i < w; i++) {
    uint64_t t = (uint64_t)x[i] + y[i] + carry;
    x[i] = (uint32_t)t;
    carry = t >> 32;
  }
}
static int big_ge(const uint32_t* x, const uint32_t* y, int w) {
  for (int i = w - 1; i >= 0; i--) {
    if (x[i] != y[i]) return x[i] > y[i];
  }
  return 1;
}
static void big_sub(uint32_t* x, const uint32_t* y, int w) {
  int64_t borrow = 0;
  for (int i = 0; i < w; i++) {
    int64_t t = (int64_t)x[i] - y[i] - borrow;
    borrow = t < 0;
    x[i] = (uint32_t)(t + (borrow ? ((int64_t)1 << 32) : 0));
  }
}

int orc_crt(const uint32_t* primes, int np, const uint32_t* res, size_t n, uint32_t* out, int limbs) {
  if (np < 1 || np > 6 || limbs < 1 || limbs > CRT_MAXW) return -1;
  uint32_t M[CRT_MAXW + 1] = {1};
  for (int j = 0; j < np; j++) big_mul_small(M, CRT_MAXW + 1, primes[j]);
  for (int i = limbs; i <= CRT_MAXW; i++)
    if (M[i] != 0) return -1;                 /* M must fit in `limbs` words */
  uint32_t Mj[6][CRT_MAXW + 1];
  uint32_t inv[6];
  for (int j = 0; j < np; j++) {
    for (int i = 0; i <= CRT_MAXW; i++) Mj[j][i] = (i == 0);
    uint64_t mj_mod = 1;
    for (int l = 0; l < np; l++)
      if (l != j) {
        big_mul_small(Mj[j], CRT_MAXW + 1, primes[l]);
        mj_mod = (mj_mod * (primes[l] % primes[j])) % primes[j];
      }
    inv[j] = (uint32_t)inverse_mod64(mj_mod, primes[j]);
    if (inv[j] == 0) return -1;
  }
  for (size_t i = 0; i < n; i++) {
    uint32_t acc[CRT_MAXW + 1] = {0};
    for (int j = 0; j < np; j++) {
      uint32_t term[CRT_MAXW + 1];
      for (int l = 0; l <= CRT_MAXW; l++) term[l] = Mj[j][l];
      big_mul_small(term, CRT_MAXW + 1, (uint32_t)(((uint64_t)res[(size_t)j * n + i] * inv[j]) % primes[j]));
      big_add(acc, term, CRT_MAXW + 1);
    }
    while (big_ge(acc, M, CRT_MAXW + 1)) big_sub(acc, M, CRT_MAXW + 1);
    for (int l = 0; l < limbs; l++) out[i * (size_t)limbs + l] = acc[l];
  }
  return 0;
}
