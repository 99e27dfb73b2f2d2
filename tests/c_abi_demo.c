/*
 * c_abi_demo.c -- libmont used from plain C through its headers only: no
 * Python, no torch.  Built by tests/test_c_abi.py with gcc against
 * include/*.h, linked with libmont.so, the HIP runtime and the CPU oracle
 * (test infrastructure).
 *
 *   c_abi_demo host   -- host-only calls: section 3.1 precomputation, the CRT
 *                        constants and error statuses (no GPU needed);
 *   c_abi_demo device -- device buffers from hipMalloc: conversion, product
 *                        and mul-add chains, a polynomial product, 64-bit
 *                        products, vector batches and reusable plans (small
 *                        enough for the launch arguments and not), each
 *                        compared with the oracle.
 * Prints one line per check and exits 0 only if all pass.
 */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mont.h"
#include "mont64.h"
#include "mont_crt.h"
#include "mont_ntt.h"

/* oracle (liboracle.so) */
int orc_setup(uint32_t P, int r, uint32_t out[5]);
void orc_mul(uint32_t P, uint32_t Rinv, const uint32_t* a, const uint32_t* b, uint32_t* out, size_t n);
void orc_muladd(uint32_t P, uint32_t Rinv, const uint32_t* a, const uint32_t* b, const uint32_t* c, uint32_t* out,
                size_t n);
void orc_polymul_schoolbook(uint32_t P, const uint32_t* a, uint32_t da, const uint32_t* b, uint32_t db, uint32_t* c);
int orc64_setup(uint64_t P, int r, uint64_t out[5]);
void orc64_mul(uint64_t P, uint64_t Rinv, const uint64_t* a, const uint64_t* b, uint64_t* out, size_t n);

static int failures = 0;

static void check(int ok, const char* what) {
  printf("%s %s\n", ok ? "ok  " : "FAIL", what);
  if (!ok) failures++;
}

/* xorshift64: the demo's own input generator */
static uint64_t rs = 88172645463325252ull;
static uint64_t next64(void) {
  rs ^= rs << 13;
  rs ^= rs >> 7;
  rs ^= rs << 17;
  return rs;
}

static int host_checks(void) {
  mont_params p;
  uint32_t ref[5];
  check(mont_setup(998244353u, &p) == MONT_OK && orc_setup(998244353u, 32, ref) == 0 && p.Pprime == ref[0] &&
            p.R1 == ref[1] && p.R2 == ref[2] && p.k == ref[4],
        "mont_setup(998244353) matches the oracle");
  check(p.P * p.Pprime == 0xFFFFFFFFu, "P P' = -1 mod 2^32");
  check(mont_setup(4u, &p) == MONT_EINVAL && mont_setup(0x80000001u, &p) == MONT_EINVAL, "even / too large P");
  check(strlen(mont_strerror(MONT_ENOROOT)) > 0, "mont_strerror");
  mont64_params q;
  uint64_t ref64[5];
  check(mont64_setup(9223372036854775783ull, &q) == MONT_OK && orc64_setup(9223372036854775783ull, 64, ref64) == 0 &&
            q.Pprime == ref64[0] && q.R1 == ref64[1] && q.R2 == ref64[2],
        "mont64_setup(2^63 - 25) matches the oracle");
  crt_params c;
  const uint32_t primes[3] = {2013265921u, 1811939329u, 2113929217u};
  check(crt_setup(primes, &c) == MONT_OK && c.P[2] == primes[2], "crt_setup");
  const uint32_t bad[3] = {2013265921u, 2013265921u, 2113929217u};
  check(crt_setup(bad, &c) == MONT_EINVAL, "crt_setup rejects a repeated prime");
  check(mont_mul(&p, NULL, NULL, NULL, 0, NULL) == MONT_OK, "n = 0 enqueues nothing");
  check(ntt_polymul_scratch_bytes(100, 100) == 0 && ntt_polymul_scratch_bytes(10000, 10000) == ((size_t)8 << 15),
        "ntt_polymul_scratch_bytes");
  check(ntt_scratch_bytes(NULL, NULL, 0) == 0, "ntt_scratch_bytes without a context");
  check(ntt_polymul_batch(NULL, NULL, 0, NULL, NULL, NULL, 0, NULL) == MONT_EINVAL, "ntt_polymul_batch validation");
  return failures;
}

#define HIP_OK(x)                                              \
  do {                                                         \
    if ((x) != hipSuccess) {                                   \
      printf("FAIL hip call %s\n", #x);                         \
      return 1;                                                \
    }                                                          \
  } while (0)

static int device_checks(void) {
  const uint32_t P = 2013265921u;
  const size_t n = 100003;
  mont_params p;
  uint32_t ref[5];
  if (mont_setup(P, &p) != MONT_OK || orc_setup(P, 32, ref) != 0) return 1;
  uint32_t *ha = malloc(4 * n), *hb = malloc(4 * n), *hc = malloc(4 * n), *hout = malloc(4 * n),
           *want = malloc(4 * n);
  for (size_t i = 0; i < n; i++) {
    ha[i] = (uint32_t)(next64() % P);
    hb[i] = (uint32_t)(next64() % P);
    hc[i] = (uint32_t)(next64() % P);
  }
  uint32_t *da, *db, *dc, *dout;
  HIP_OK(hipMalloc((void**)&da, 4 * n));
  HIP_OK(hipMalloc((void**)&db, 4 * n));
  HIP_OK(hipMalloc((void**)&dc, 4 * n));
  HIP_OK(hipMalloc((void**)&dout, 4 * n));
  HIP_OK(hipMemcpy(da, ha, 4 * n, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(db, hb, 4 * n, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(dc, hc, 4 * n, hipMemcpyHostToDevice));
  hipStream_t s;
  HIP_OK(hipStreamCreate(&s));

  /* a*b mod P through residues: to, to, mul, from */
  check(mont_to(&p, da, dout, n, s) == MONT_OK && mont_to(&p, db, dc, n, s) == MONT_OK &&
            mont_mul(&p, dout, dc, dout, n, s) == MONT_OK && mont_from(&p, dout, dout, n, s) == MONT_OK,
        "enqueue to/to/mul/from");
  HIP_OK(hipMemcpyAsync(hout, dout, 4 * n, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  int ok = 1;
  for (size_t i = 0; i < n && ok; i++) ok = hout[i] == (uint32_t)(((uint64_t)ha[i] * hb[i]) % P);
  check(ok, "from(mul(to a, to b)) = a b mod P for 100003 pairs");

  /* mul-add on residues, in place on c */
  HIP_OK(hipMemcpy(dc, hc, 4 * n, hipMemcpyHostToDevice));
  check(mont_muladd(&p, da, db, dc, dc, n, s) == MONT_OK, "enqueue mul-add");
  HIP_OK(hipMemcpyAsync(hout, dc, 4 * n, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  orc_muladd(P, ref[3], ha, hb, hc, want, n);
  check(memcmp(hout, want, 4 * n) == 0, "mont_muladd matches the oracle");

  /* a polynomial product of degrees 3000 and 2000 */
  ntt_ctx* ctx = NULL;
  const uint32_t pr[1] = {P};
  check(ntt_ctx_create(pr, 1, 16, &ctx) == MONT_OK, "ntt_ctx_create");
  const uint32_t dA = 3000, dB = 2000;
  check(ntt_polymul(ctx, 0, da, dA, db, dB, dout, NULL, 0, s) == MONT_OK, "enqueue ntt_polymul");
  HIP_OK(hipMemcpyAsync(hout, dout, 4 * (dA + dB + 1), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  orc_polymul_schoolbook(P, ha, dA, hb, dB, want);
  check(memcmp(hout, want, 4 * (dA + dB + 1)) == 0, "ntt_polymul matches the schoolbook product");
  check(ntt_polymul(ctx, 0, da, 20000, db, 20000, dout, NULL, 0, s) == MONT_ENOMEM, "missing scratch: ENOMEM");
  ntt_ctx_destroy(ctx);

  /* 64-bit residues */
  const uint64_t Q = 9223372036854775783ull;
  const size_t m = 50001;
  mont64_params q;
  uint64_t r64[5];
  if (mont64_setup(Q, &q) != MONT_OK || orc64_setup(Q, 64, r64) != 0) return 1;
  uint64_t *xa = malloc(8 * m), *xb = malloc(8 * m), *xo = malloc(8 * m), *xw = malloc(8 * m);
  for (size_t i = 0; i < m; i++) {
    xa[i] = next64() % Q;
    xb[i] = next64() % Q;
  }
  uint64_t *ya, *yb;
  HIP_OK(hipMalloc((void**)&ya, 8 * m));
  HIP_OK(hipMalloc((void**)&yb, 8 * m));
  HIP_OK(hipMemcpy(ya, xa, 8 * m, hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(yb, xb, 8 * m, hipMemcpyHostToDevice));
  check(mont64_mul(&q, ya, yb, ya, m, s) == MONT_OK, "enqueue mont64_mul");
  HIP_OK(hipMemcpyAsync(xo, ya, 8 * m, hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  orc64_mul(Q, r64[3], xa, xb, xw, m);
  check(memcmp(xo, xw, 8 * m) == 0, "mont64_mul matches the oracle");

  /* vector batches: 3 vectors (descriptors passed in the launch), then 20
   * (descriptors uploaded), each a prefix of its own 4000-word segment */
  mont_batch* vb = NULL;
  check(mont_batch_reserve(20, &vb) == MONT_OK, "mont_batch_reserve");
  for (int round = 0; round < 2; round++) {
    const int cnt = round == 0 ? 3 : 20;
    const size_t seg = 4000;
    mont_vec_desc vd[20];
    for (int i = 0; i < cnt; i++) {
      vd[i].a = da + i * seg;
      vd[i].b = db + i * seg;
      vd[i].out = dout + i * seg;
      vd[i].n = 1 + next64() % seg;
      vd[i].P = p.P;
      vd[i].Pprime = p.Pprime;
    }
    ok = mont_batch_update(vb, vd, cnt, s) == MONT_OK && mont_batch_mul(vb, s) == MONT_OK;
    HIP_OK(hipMemcpyAsync(hout, dout, 4 * n, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (int i = 0; i < cnt && ok; i++) {
      orc_mul(P, ref[3], ha + i * seg, hb + i * seg, want, vd[i].n);
      ok = memcmp(hout + i * seg, want, 4 * vd[i].n) == 0;
    }
    check(ok, round == 0 ? "mont_batch_mul, 3 vectors (descriptors in the launch)"
                         : "mont_batch_mul, 20 vectors (descriptors uploaded)");
  }
  check(mont_batch_destroy(vb) == MONT_OK, "mont_batch_destroy");

  /* a reusable plan: 2 products (lists passed in the launch), then 6 (lists
   * uploaded); operands and results packed in one input and one output buffer */
  ntt_ctx* c2 = NULL;
  ntt_plan* pl = NULL;
  void* dscr = NULL;
  const size_t scr_cap = 1 << 20;
  check(ntt_ctx_create(pr, 1, 16, &c2) == MONT_OK && ntt_plan_reserve(c2, 8, 4096, &pl) == MONT_OK,
        "ntt_plan_reserve");
  HIP_OK(hipMalloc(&dscr, scr_cap));
  for (int round = 0; round < 2; round++) {
    const int cnt = round == 0 ? 2 : 6;
    polymul_desc pd[6];
    uint64_t cpos = 0;
    for (int i = 0; i < cnt; i++) {
      pd[i].prime_id = 0;
      pd[i].da = (uint32_t)(next64() % 2000);
      pd[i].db = (uint32_t)(next64() % 2000);
      pd[i].reserved = 0;
      pd[i].a_off = (uint64_t)i * 5000;
      pd[i].b_off = (uint64_t)i * 5000 + 2500;
      pd[i].c_off = cpos;
      cpos += pd[i].da + pd[i].db + 1;
    }
    size_t sb = 0;
    ok = ntt_plan_update(pl, pd, cnt, 0, s) == MONT_OK && ntt_plan_info(pl, &sb, NULL, NULL, NULL, NULL) == MONT_OK &&
         sb <= scr_cap && ntt_plan_execute(pl, da, dout, dscr, sb, 0, 0, s) == MONT_OK &&
         ntt_plan_status(pl, dscr, s) == MONT_OK;
    HIP_OK(hipMemcpyAsync(hout, dout, 4 * cpos, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (int i = 0; i < cnt && ok; i++) {
      orc_polymul_schoolbook(P, ha + pd[i].a_off, pd[i].da, ha + pd[i].b_off, pd[i].db, want);
      ok = memcmp(hout + pd[i].c_off, want, 4 * (pd[i].da + pd[i].db + 1)) == 0;
    }
    check(ok, round == 0 ? "ntt_plan_execute, 2 products (lists in the launch)"
                         : "ntt_plan_execute, 6 products (lists uploaded)");
  }
  {
    int th = 0, rl = 0, gm = 0;
    ok = ntt_plan_shape(pl, &th, &rl, &gm) == MONT_OK && (th == 256 || th == 512 || th == 1024) &&
         (rl == 3 || rl == 4) && gm >= 1;
    check(ok, "ntt_plan_shape");
  }
  check(ntt_plan_destroy(pl) == MONT_OK, "ntt_plan_destroy");

  /* a one-call batch: six products whose descriptors sit in device memory
   * and are planned there; degrees 8200 x 8200 (length just above 2^14) take
   * the split path and its fix-up */
  {
    const uint32_t degs[6][2] = {{8200, 8200}, {3000, 2000}, {1, 0}, {0, 0}, {9000, 7000}, {500, 1999}};
    polymul_desc bd[6];
    uint64_t apos = 0, cpos = 0;
    for (int i = 0; i < 6; i++) {
      bd[i].prime_id = 0;
      bd[i].da = degs[i][0];
      bd[i].db = degs[i][1];
      bd[i].reserved = 0;
      bd[i].a_off = apos;
      apos += bd[i].da + 1;
      bd[i].b_off = apos;
      apos += bd[i].db + 1;
      bd[i].c_off = cpos;
      cpos += bd[i].da + bd[i].db + 1;
    }
    const size_t sb = ntt_scratch_bytes(c2, bd, 6);
    check(sb > 0 && ntt_scratch_bytes(c2, bd, -1) == 0, "ntt_scratch_bytes");
    void* bscr = NULL;
    polymul_desc* ddesc = NULL;
    HIP_OK(hipMalloc(&bscr, sb));
    HIP_OK(hipMalloc((void**)&ddesc, sizeof(bd)));
    HIP_OK(hipMemcpy(ddesc, bd, sizeof(bd), hipMemcpyHostToDevice));
    ok = ntt_polymul_batch(c2, ddesc, 6, da, dout, bscr, sb, s) == MONT_OK && ntt_batch_status(bscr, s) == MONT_OK;
    HIP_OK(hipMemcpyAsync(hout, dout, 4 * cpos, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (int i = 0; i < 6 && ok; i++) {
      orc_polymul_schoolbook(P, ha + bd[i].a_off, bd[i].da, ha + bd[i].b_off, bd[i].db, want);
      ok = memcmp(hout + bd[i].c_off, want, 4 * (bd[i].da + bd[i].db + 1)) == 0;
    }
    check(ok, "ntt_polymul_batch, 6 products planned on the device");
    check(ntt_polymul_batch(c2, ddesc, 6, da, dout, bscr, sb - 4, s) == MONT_OK &&
              ntt_batch_status(bscr, s) == MONT_ENOMEM,
          "scratch below ntt_scratch_bytes: MONT_ENOMEM from the planning kernel");
    check(ntt_polymul_batch(c2, ddesc, 6, da, dout, bscr, 64, s) == MONT_ENOMEM,
          "scratch below the fixed layout: MONT_ENOMEM on the host");
    HIP_OK(hipFree(bscr));
    HIP_OK(hipFree(ddesc));
  }
  ntt_ctx_destroy(c2);
  HIP_OK(hipFree(dscr));

  HIP_OK(hipFree(ya));
  HIP_OK(hipFree(yb));
  HIP_OK(hipFree(da));
  HIP_OK(hipFree(db));
  HIP_OK(hipFree(dc));
  HIP_OK(hipFree(dout));
  HIP_OK(hipStreamDestroy(s));
  free(ha); free(hb); free(hc); free(hout); free(want);
  free(xa); free(xb); free(xo); free(xw);
  return failures;
}

int main(int argc, char** argv) {
  if (argc < 2) {
    fprintf(stderr, "usage: %s host|device\n", argv[0]);
    return 2;
  }
  int bad = strcmp(argv[1], "host") == 0 ? host_checks() : device_checks();
  printf("%d failures\n", bad);
  return bad == 0 ? 0 : 1;
}
