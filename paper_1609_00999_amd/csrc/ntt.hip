// ntt.hip -- radix-2 number-theoretic transforms and polynomial products
// modulo word-size Fourier primes, with Montgomery-form twiddles.
//
// The butterflies apply REDC (arXiv:1609.00999, section 3.1, Algorithm 2) to
// an ordinary residue times a twiddle kept in Montgomery form, w_bar = w R mod
// P, so REDC(x * w_bar) = x w mod P and the data never leave the ordinary
// representation.  P = c 2^k + 1 (a Fourier prime) has roots of unity of
// every order 2^n <= 2^k, which the transforms need.
//
// Transform layout (no permutation pass anywhere):
//   forward  = decimation in frequency (Gentleman-Sande), natural order in,
//              bit-reversed order out: stages h = N/2, ..., 1 with
//              (x, y) -> (x + y, (x - y) w_{2h}^i);
//   inverse  = decimation in time (Cooley-Tukey), bit-reversed in, natural
//              out: stages h = 1, ..., N/2 with
//              (x, y) -> (x + y w_{2h}^-i, x - y w_{2h}^-i).
// Twiddle tables hold w_{2h}^i at index h + i (h = 2^s, 0 <= i < h), so any
// stage of any length N <= Nmax reads a contiguous run.
//
// Lengths up to 2^13 are done by one workgroup in LDS.  Longer transforms
// (N = 2^n, n = n1 + 13) take two passes over HBM: a column pass over tiles
// of 2^n1 rows x C adjacent columns (the first n1 stages, rows strided by
// 2^13 in memory) and a row pass over contiguous blocks of 2^13 (the last 13
// stages).  A polynomial product fuses the forward row pass of both operands,
// the pointwise product and the first 13 inverse stages into one row task.
// In row blocks and in column tiles of lengths 2^14..2^23 the first register
// round reads its groups from HBM and the last writes them back, so the
// blocks are not staged through LDS on the way in or out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <random>
#include <vector>

#include "internal.hpp"
#include "modarith.hpp"
#include "mont_ntt.h"

namespace mont {

constexpr int kRowLog = 13;            // row block = small-product limit: 2^13 residues
constexpr int kLdsWords = 1 << 14;     // 64 KiB of LDS per workgroup
// Longest transform: 2^23.  Every multi-pass length 2^14 .. 2^23 has
// compile-time column rounds; longer column tiles would hold fewer than eight
// adjacent columns (2^(27-n) of them), whose strided rows read HBM poorly.
constexpr int kMaxLog = 23;

// Per-prime device constants.
struct PrimeDev {
  uint32_t P, Pp, R1, R2;
  uint32_t logmax;          // tables cover lengths up to 2^logmax
  uint32_t pad[3];
  const uint32_t* twf;      // twf[h + i] = residue of w_{2h}^i
  const uint32_t* twi;      // twi[h + i] = residue of w_{2h}^-i
  uint32_t s1[32];          // s1[n] = R N^-1 mod P  (REDC(x s1) = x / N)
  uint32_t s2[32];          // s2[n] = R^2 N^-1 mod P (REDC(x s2) = x R / N)
};

// One product in a batch plan.  Its transform length 2^n is normally the
// least power of two >= da + db + 1; a plan may also force a shorter length,
// and then the product is the cyclic convolution of that length (the
// coefficients of a b reduced modulo x^(2^n) - 1).  It stores nout =
// min(da + db + 1, 2^n) coefficients at c_off in the output buffer, or in the
// plan's scratch when to_scr is set.
struct ProdDev {
  uint32_t prime_id, n, da, db;
  uint64_t a_off, b_off, c_off, scr_off;
  uint32_t lc;              // log2 of the columns per column tile
  uint32_t ntiles;          // column tiles per operand
  uint32_t nblocks;         // row blocks (2^(n - 13))
  uint32_t nout;            // coefficients stored
  uint32_t to_scr;          // 1: c_off is an offset into the scratch buffer
  uint32_t tft;             // 0, or log2 N of the product whose truncated-transform block this is (below)
  uint32_t pad[2];
};

// Fix-up of a product computed in two parts, after the persistent launch.
// Both kinds start from the cyclic part r = c mod (x^h - 1) in the output
// (c[k] holds c_k + c_(h+k)), with h = 2^(n-1) and m = da + db + 1 - h.
//  FIX_SPLIT: t is the product of the top m coefficients of a and b, and
//    c[k] -= t[m-1+k], c[h+k] = t[m-1+k] for k < m.
//  FIX_TFT: t is the truncated-transform block of length s (below), the
//    cyclic product that gives u = c mod (x^s - w^s) as u_k = t_k w^-k, and
//    q_k = (sum_i r_(k+is) w^(is) - u_k) / 2, c[k] -= q_k, c[h+k] = q_k for k < m.
enum FixKind : uint32_t { FIX_SPLIT = 0, FIX_TFT = 1 };
struct FixDev {
  uint64_t c_off;           // product output, in the output buffer
  uint64_t t_off;           // top product or block output, in the scratch buffer
  uint32_t m, h, P;
  uint32_t chunk0;          // first of its ceil(m / kFixChunk) chunks in the fix-up launch
  uint32_t kind;            // FixKind
  uint32_t prime_id;        // FIX_TFT: the prime (tables, Montgomery constants)
  uint32_t s_log;           // FIX_TFT: log2 of the block length s
  uint32_t pad;
};
constexpr uint32_t kFixChunk = 1024;
// A reusable plan uploads products, fix-ups and tasks back to back in one block.
static_assert(sizeof(ProdDev) % 16 == 0 && sizeof(FixDev) % 16 == 0, "records keep the block 16-byte aligned");

enum TaskKind : uint32_t { T_SMALL = 0, T_COLF_A = 1, T_COLF_B = 2, T_ROW = 3, T_COLI = 4 };

// Scratch header used by the persistent kernel (words).
constexpr int kHdrWords = 64;          // [0] queue head, [1] status
constexpr uint32_t kStatusTimeout = 1;
// A batch planned on the device (ntt_polymul_batch) also keeps in its header
// the task count, the fix-up chunk count, a planning error (a negative
// mont_status, 0 if none), the scratch words the plan needs (64-bit) and the
// word offset of the table of each fix-up chunk's record (64-bit).
constexpr int kHdrNtasks = 2, kHdrNchunks = 3, kHdrError = 4, kHdrWordsNeeded = 6, kHdrOwner = 8;
constexpr uint32_t kStatusPlanError = 2;

// ---------------------------------------------------------------------------
// Product shapes, shared by the host planner and the device planner.
// ---------------------------------------------------------------------------

__host__ __device__ inline int ceil_log2(uint64_t x) {
  int n = 0;
  while (((uint64_t)1 << n) < x) n++;
  return n;
}

// Column-tile width for a multi-pass length 2^n: as many adjacent columns as
// fit 2^14 residues of LDS, at most the 2^13 columns there are.
__host__ __device__ inline int col_lc(int n) { return 14 - (n - kRowLog) < kRowLog ? 14 - (n - kRowLog) : kRowLog; }

// Splitting a product whose length L = da + db + 1 is just above h = N/2.
// With both operands shorter than h, the cyclic product of length h gives
// c_k + c_(h+k), and the top m = L - h coefficients of a and b (a[h-db ..
// da], b[h-da .. db]) have a product whose coefficients m-1 .. 2m-2 are
// c_h .. c_(L-1).  The split is taken when the top product's length 2^nt
// (>= 2m - 1) is at most N/4: the pair then costs at most 3/4 of the
// butterflies of the length-N product.  (With 2^nt = N/2 it would save only
// one stage in log2 N, not worth a second product and the fix-up.)  Only
// multi-pass products are split: a product of length <= 2^13 is one task
// whose cost is mostly its fixed overhead.
__host__ __device__ inline bool split_rule(uint32_t da, uint32_t db, int n, uint32_t& m, int& nt) {
  if (n <= kRowLog) return false;
  const uint64_t h = 1ull << (n - 1);
  if ((uint64_t)da + 1 > h || (uint64_t)db + 1 > h) return false;
  m = (uint32_t)((uint64_t)da + db + 1 - h);
  nt = ceil_log2(2ull * m - 1);
  return nt <= n - 2;
}

// The two-block truncated transform (the truncated Fourier transform of the
// paper's references, cut to two blocks).  A product of length L = da+db+1
// in (N/2, N] is fixed by its residues modulo coprime factors of x^N - 1
// whose degrees sum to at least L: here x^h - 1 (h = N/2, the cyclic part
// above) and x^s - w^s with w = w_N and s = N/4 or N/8, whose roots are odd
// powers of w.  The second residue is a cyclic product of length s of the
// folded and twisted operands a'_r = w^r sum_i a_(r+is) w^(is) (likewise b'),
// since a(w y) mod (y^s - 1) has exactly those coefficients; the fix-up
// untwists it and joins both residues (Chinese remainders: (x^h - 1) =
// -2 mod (x^s - w^s)).  For a product with N/16 < m <= N/4 (m = L - h) the
// pair costs transforms of h + s points instead of N, and beats the split's
// top product (>= 2m points).  Lengths from 2^18 keep the block at 2^15
// points or more, where the column tiles read their first round from HBM
// (the fold and twist happen in that load).
constexpr int kTftMinLog = 18;

__host__ __device__ inline bool tft_rule(uint32_t da, uint32_t db, int n, uint32_t& m, int& ls) {
  if (n < kTftMinLog) return false;
  const uint64_t N = 1ull << n, h = N >> 1;
  if ((uint64_t)da + 1 > h || (uint64_t)db + 1 > h) return false;
  const uint64_t mm = (uint64_t)da + db + 1 - h;
  if (mm <= N / 16 || mm > N / 4) return false;
  m = (uint32_t)mm;
  ls = mm <= N / 8 ? n - 3 : n - 2;
  return true;
}

__host__ __device__ inline uint32_t product_tasks(int n) {
  if (n <= kRowLog) return 1;
  const uint32_t ntiles = 1u << (kRowLog - col_lc(n));
  return 3 * ntiles + (1u << (n - kRowLog));
}

// One internal product ("slot") of a one-call batch: slot 2i is product i,
// or its cyclic part when the split rule takes it; slot 2i + 1 is the top
// part of a split product and unused otherwise.
struct SlotShape {
  int err;                  // nonzero: the product's descriptor is invalid (a mont_status)
  bool used;
  bool split;               // the product is computed in two parts (both slots describe it)
  bool tft;                 // ... as a cyclic part and a truncated-transform block (else a top product)
  bool block;               // this slot is the truncated-transform block
  int nfull;                // log2 N of the whole product
  int n;                    // log2 of the slot's transform length
  uint32_t da, db;          // the slot's operand degrees
  uint64_t a_off, b_off;    // the slot's operand offsets in the input
  uint32_t nout;            // coefficients the slot stores
  uint32_t m, h;            // split products: top coefficients and half length
};

__host__ __device__ inline SlotShape slot_shape(const polymul_desc& d, int part, uint32_t nprimes,
                                                const uint32_t* logmax) {
  SlotShape sh = {};
  if (d.prime_id >= nprimes || d.reserved != 0) {
    sh.err = MONT_EINVAL;
    return sh;
  }
  const uint64_t L = (uint64_t)d.da + d.db + 1;
  if (L > ((uint64_t)1 << 31)) {
    sh.err = MONT_ERANGE;
    return sh;
  }
  const int n = ceil_log2(L);
  if ((uint32_t)n > logmax[d.prime_id]) {
    sh.err = MONT_ENOROOT;
    return sh;
  }
  uint32_t m = 0;
  int nt = 0;
  sh.nfull = n;
  sh.tft = tft_rule(d.da, d.db, n, m, nt);
  sh.split = sh.tft || split_rule(d.da, d.db, n, m, nt);
  if (!sh.split) {
    sh.used = part == 0;
    sh.n = n;
    sh.da = d.da;
    sh.db = d.db;
    sh.a_off = d.a_off;
    sh.b_off = d.b_off;
    sh.nout = (uint32_t)L;
    return sh;
  }
  const uint32_t h = 1u << (n - 1);
  sh.used = true;
  sh.m = m;
  sh.h = h;
  if (part == 0) {              // cyclic part of length h, straight into the output
    sh.n = n - 1;
    sh.da = d.da;
    sh.db = d.db;
    sh.a_off = d.a_off;
    sh.b_off = d.b_off;
    sh.nout = h;
  } else if (sh.tft) {          // block of length 2^nt: folds and twists the whole operands
    sh.block = true;
    sh.n = nt;
    sh.da = d.da;
    sh.db = d.db;
    sh.a_off = d.a_off;
    sh.b_off = d.b_off;
    sh.nout = m;
  } else {                      // top part, into scratch
    sh.n = nt;
    sh.da = m - 1;
    sh.db = m - 1;
    sh.a_off = d.a_off + (h - d.db);
    sh.b_off = d.b_off + (h - d.da);
    sh.nout = 2 * m - 1;
  }
  return sh;
}

// REDC operations a slot executes: three transforms of (N/2) log2 N
// butterflies, N pointwise products and db + 1 scalings of b; a block also
// folds (one product per operand coefficient beyond its length) and twists
// (one per point, both operands).
__host__ __device__ inline uint64_t slot_redc(const SlotShape& sh) {
  const uint64_t N = 1ull << sh.n;
  uint64_t r = 3 * (N / 2) * (uint64_t)sh.n + N + (sh.block ? N : (uint64_t)sh.db + 1);
  if (sh.block) {
    r += 2 * N;
    r += sh.da + 1 > N ? sh.da + 1 - N : 0;
    r += sh.db + 1 > N ? sh.db + 1 - N : 0;
  }
  return r;
}

// Butterflies of a slot's three transforms whose twiddle is 1, which the
// kernels run without a product (transforms of 2^rm-point register rounds):
// those of stages t < r in the round holding stages 0 .. r-1, 2^n / 2^(t+1)
// per stage and transform.  A multi-pass slot has that round in its row
// pass (the last forward round of both operands and the first inverse round,
// of the 13-stage row: r = 13 / ceil(13 / rm)); a one-task slot in its last
// forward round (r = n / ceil(n / rm), both operands) and its first inverse
// round (one more when rm does not divide the rounds evenly).
__host__ __device__ inline uint64_t unit_bfly(int n, int rm) {
  if (n <= 0) return 0;
  const uint64_t N = 1ull << n;
  const int lr = n > kRowLog ? kRowLog : n;
  const int nr = (lr + rm - 1) / rm;
  const int r_small = lr / nr, r_large = r_small + (lr % nr ? 1 : 0);
  const uint64_t fwd = N - (N >> r_small);
  if (n > kRowLog) return 3 * fwd;
  return 2 * fwd + (N - (N >> r_large));
}

// REDC operations of a product's fix-up, counted on its second slot: a
// block's untwist, the fold of the cyclic part and the halving, per fixed
// coefficient.
__host__ __device__ inline uint64_t fix_redc(const SlotShape& sh) {
  return sh.block ? (uint64_t)sh.m * ((sh.h >> sh.n) + 1) : 0;
}

// Scratch words a slot's data take: the two length-N transforms of a
// multi-pass product, then a top part's output (16-byte aligned).
__host__ __device__ inline uint64_t slot_words(const SlotShape& sh, int part) {
  if (!sh.used) return 0;
  uint64_t w = sh.n > kRowLog ? (2ull << sh.n) : 0;
  if (sh.split && part == 1) w += (sh.nout + 3u) & ~3u;
  return w;
}

// Fix-up chunks of a product, counted on its top slot.
__host__ __device__ inline uint32_t slot_chunks(const SlotShape& sh, int part) {
  return sh.split && part == 1 ? (sh.m + kFixChunk - 1) / kFixChunk : 0u;
}


namespace {

__device__ __forceinline__ Mod mod_of(const PrimeDev& pr) { return Mod{pr.P, pr.Pp}; }

// LDS word addressing.  Every access to a workgroup's LDS buffer goes through
// lds_at(i), which XORs the low six bits of the word index with 9 (r mod 8),
// r its 64-word row (a bijection inside each row).  With 64 banks this
// spreads the strided accesses of the low-stage rounds (lanes 8 or 16 words
// apart, or groups of 8 or 16 lanes 64+ words apart) over the banks: the
// worst wave access is 2-way instead of 16-way, the mean 1.2-way.
constexpr bool kSwizzle = true;
// The key 9 k = (k << 3) | k of row bits k = (i >> 6) & 7 is linear over
// GF(2) in i, so lds_at(x ^ y) = lds_at(x) ^ lds_at(y): the address of a
// group element yb | s (s in bits that are zero in yb) is lds_at(yb) ^ lds_at(s).
__host__ __device__ constexpr uint32_t lds_at(uint32_t i) {
  if constexpr (kSwizzle) {
    const uint32_t k = (i >> 6) & 7u;
    return i ^ ((k << 3) | k);
  }
  else return i;
}

// ---------------------------------------------------------------------------
// LDS stages.  X is viewed as rows x C columns (C = 2^lc, element (k, c) at
// X[k*C + c]); the transform runs along rows, independently per column.  The
// global index of element (k, c) is colbase + c + k*S with S = 2^rs, so the
// stage with row half-distance 2^s has global half-size h = 2^(s+rs) and
// twiddle index h + (i mod h) = 2^(s+rs) + colbase + c + ((k mod 2^s) << rs).
//
// Stages are done R at a time in registers (a radix-2^R round): a lane loads
// the 2^R residues whose rows differ only in bits s_lo .. s_lo+R-1, applies
// the R radix-2 stages to them, and stores them back, so LDS is read and
// written once per round instead of once per stage, and one barrier ends the
// round.  Inside a group the twiddle of stage s_lo+t depends only on the low
// t bits of the element's position in the group, so a round loads 2^R - 1
// twiddles per group instead of R 2^(R-1).
// ---------------------------------------------------------------------------


// Twiddle tables are reached through pointers stored in device memory, so the
// compiler cannot tell their address space; reading them as global memory
// keeps the loads off the FLAT path (whose counter is shared with LDS).
typedef const __attribute__((address_space(1))) uint32_t* gptr_u32;
__device__ __forceinline__ uint32_t ldg(const uint32_t* p, uint32_t i) {
  return ((gptr_u32)p)[i];
}

// Raw buffer loads (CDNA buffer instructions): a 128-bit resource in scalar
// registers holds a base address and a size in bytes; each lane supplies a
// 32-bit byte offset, and a constant part of the offset may ride in a scalar
// register.  A load at or past the size returns 0 (the range check of raw,
// unstrided buffers on the lane's offset), which gives a first round's zero
// padding beyond the operand without a compare, and each address costs one
// 32-bit add instead of a 64-bit address pair.  The base must be uniform
// across the workgroup; it is read from the first lane.
constexpr int kBufWord3 = 0x00020000;   // resource word 3 on gfx9: 32-bit data format
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const uint32_t* p, uint32_t bytes) {
  const uint64_t a = (uint64_t)(uintptr_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  return __builtin_amdgcn_make_buffer_rsrc((void*)(uintptr_t)(((uint64_t)hi << 32) | lo), 0, (int)bytes, kBufWord3);
}
// Size of a first round's source: words 0 .. dvalid (all of the 32-bit range
// when dvalid is the "no bound" value).
__device__ __forceinline__ uint32_t src_bytes(uint32_t dvalid) {
  return dvalid >= 0x3FFFFFFFu ? 0xFFFFFFFFu : (dvalid + 1) << 2;
}
__device__ __forceinline__ uint32_t buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff = 0) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
}

// The lane's index in the workgroup as the task bodies use it.  The empty asm
// makes each read opaque, so what a task derives from it (group bases, LDS
// addresses) is computed inside the persistent task loop rather than hoisted
// out of it and held in registers across every task variant, which pushed
// the persistent kernel past its register budget into spills.
__device__ __forceinline__ uint32_t task_tid() {
  uint32_t t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// Stores whose data another workgroup reads later in the same persistent
// launch are agent-scope atomic stores (global_store ... sc1): they are
// written through to the device coherence point, so a consumer on another
// XCD sees them once they have completed, and no L2 write-back is needed
// when the task is published.
template <bool COH>
__device__ __forceinline__ void st_out(uint32_t* p, uint32_t v) {
  if constexpr (COH) __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else *p = v;
}

// Lower output of the forward (decimation-in-frequency) butterfly,
// (x - y) w mod P for x, y in [0, P) and w a twiddle in Montgomery form.
// With wn = P - w, x w + y wn = (x - y) w mod P and the sum is below P^2 < R P,
// Algorithm 2's precondition, so REDC takes it directly: two v_mad_u64_u32
// replace the subtraction, the add of P and the product.
__device__ __forceinline__ uint32_t bfly_lo(uint32_t x, uint32_t y, uint32_t w, uint32_t wn, Mod md) {
  return redc((uint64_t)x * w + (uint64_t)y * wn, md);
}

// The R radix-2 stages of one register round on a group of 2^R residues.
// Stage t pairs elements 2^t apart; its twiddle for pair (j, j + 2^t) is
// w[2^t - 1 + (j mod 2^t)] (wn holds P - w for the forward butterfly).
//
// UNIT: the group is one whose twiddles for j mod 2^t = 0 are w^0 = 1 (the
// round holding stages 0 .. R-1 of a block that starts at twiddle offset 0:
// rows, and whole transforms in one workgroup).  Those butterflies add and
// subtract without a product: REDC(y R) = y exactly, so the results are the
// same residues.  They are half of stage 0, a quarter of stage 1, and so on:
// N (1 - 2^-R) of a transform's (N/2) log2 N butterflies.
template <int R, bool UNIT = false>
__device__ __forceinline__ void dif_stages(uint32_t* v, const uint32_t* w, const uint32_t* wn, Mod md) {
  constexpr int E = 1 << R;
#pragma unroll
  for (int t = R - 1; t >= 0; t--) {
    const int d = 1 << t;
#pragma unroll
    for (int j = 0; j < E; j++) {
      if (j & d) continue;
      const uint32_t x = v[j], y = v[j + d];
      v[j] = madd(x, y, md.P);
      if (UNIT && (j & (d - 1)) == 0) v[j + d] = msub(x, y, md.P);
      else v[j + d] = bfly_lo(x, y, w[d - 1 + (j & (d - 1))], wn[d - 1 + (j & (d - 1))], md);
    }
  }
}

template <int R, bool UNIT = false>
__device__ __forceinline__ void dit_stages(uint32_t* v, const uint32_t* w, Mod md) {
  constexpr int E = 1 << R;
#pragma unroll
  for (int t = 0; t < R; t++) {
    const int d = 1 << t;
#pragma unroll
    for (int j = 0; j < E; j++) {
      if (j & d) continue;
      const uint32_t x = v[j];
      const uint32_t y = UNIT && (j & (d - 1)) == 0 ? v[j + d] : mmul(v[j + d], w[d - 1 + (j & (d - 1))], md);
      v[j] = madd(x, y, md.P);
      v[j + d] = msub(x, y, md.P);
    }
  }
}

template <int NT, int NA, int R, bool INV, bool UNIT>
__device__ __forceinline__ void lds_round_body(uint32_t* X, int off, uint32_t M, int s_lo, int lc, int rs,
                                               uint32_t colbase, const uint32_t* tw, Mod md) {
  constexpr int E = 1 << R;
  const int a_lo = s_lo + lc;                      // LDS address bit of stage s_lo
  const uint32_t lomask = (1u << a_lo) - 1;
  const uint32_t ngroups = M >> R;
  for (uint32_t g = task_tid(); g < ngroups; g += NT) {
    const uint32_t base = ((g & ~lomask) << R) | (g & lomask);   // zero in bits a_lo .. a_lo+R-1
    const uint32_t c = base & ((1u << lc) - 1);
    const uint32_t kb = base >> lc;
    const uint32_t t0 = colbase + c + ((kb & ((1u << s_lo) - 1)) << rs);
    uint32_t w[E - 1];
#pragma unroll
    for (int t = 0; t < R; t++)
#pragma unroll
      for (int jj = 0; jj < (1 << t); jj++)
        w[(1 << t) - 1 + jj] = ldg(tw, (1u << (s_lo + t + rs)) + t0 + ((uint32_t)jj << (s_lo + rs)));
    uint32_t wn[E - 1];
    if constexpr (!INV) {
#pragma unroll
      for (int k = 0; k < E - 1; k++) wn[k] = md.P - w[k];
    }
#pragma unroll
    for (int a = 0; a < NA; a++) {
      const uint32_t pb = lds_at((uint32_t)(a * off) + base);
      uint32_t v[E];
#pragma unroll
      for (int j = 0; j < E; j++) v[j] = X[pb ^ lds_at((uint32_t)j << a_lo)];
      if constexpr (!INV) dif_stages<R, UNIT>(v, w, wn, md);
      else dit_stages<R, UNIT>(v, w, md);
#pragma unroll
      for (int j = 0; j < E; j++) X[pb ^ lds_at((uint32_t)j << a_lo)] = v[j];
    }
  }
  __syncthreads();
}

// A round over stages s_lo .. s_lo + R - 1.  The round holding stage 0 of
// blocks whose twiddles start at offset 0 (one column, offset 0) skips the
// products by twiddle 1.
template <int NT, int NA, int R, bool INV>
__device__ __forceinline__ void lds_round(uint32_t* X, int off, uint32_t M, int s_lo, int lc, int rs,
                                          uint32_t colbase, const uint32_t* tw, Mod md) {
  if (s_lo == 0 && lc == 0 && colbase == 0) lds_round_body<NT, NA, R, INV, true>(X, off, M, 0, 0, rs, 0u, tw, md);
  else lds_round_body<NT, NA, R, INV, false>(X, off, M, s_lo, lc, rs, colbase, tw, md);
}

template <int NT, int NA, bool INV, int RM>
__device__ __forceinline__ void lds_round_r(int r, uint32_t* X, int off, uint32_t M, int s_lo, int lc, int rs,
                                            uint32_t colbase, const uint32_t* tw, Mod md) {
  switch (r) {
    case 1: lds_round<NT, NA, 1, INV>(X, off, M, s_lo, lc, rs, colbase, tw, md); break;
    case 2: lds_round<NT, NA, 2, INV>(X, off, M, s_lo, lc, rs, colbase, tw, md); break;
    case 3: lds_round<NT, NA, 3, INV>(X, off, M, s_lo, lc, rs, colbase, tw, md); break;
    default:
      if constexpr (RM >= 4) lds_round<NT, NA, 4, INV>(X, off, M, s_lo, lc, rs, colbase, tw, md);
      break;
  }
}

// Round sizes for lr stages: ceil(lr / RM) rounds of at most RM stages, as
// even as possible, the larger ones first.
template <int RM>
__device__ __forceinline__ int round_size(int lr, int idx) {
  const int nr = (lr + RM - 1) / RM;
  const int base = lr / nr, extra = lr % nr;
  return base + (idx < extra ? 1 : 0);
}

// Forward (decimation in frequency): stages lr-1 .. 0, rounds from the top.
template <int NT, int NA, int RM>
__device__ __forceinline__ void lds_dif(uint32_t* X, int off, int lr, int lc, int rs, uint32_t colbase, const uint32_t* tw,
                        Mod md) {
  const uint32_t M = 1u << (lr + lc);
  int s_hi = lr;
  for (int idx = 0; s_hi > 0; idx++) {
    const int r = round_size<RM>(lr, idx);
    s_hi -= r;
    lds_round_r<NT, NA, false, RM>(r, X, off, M, s_hi, lc, rs, colbase, tw, md);
  }
}

// Inverse (decimation in time): stages 0 .. lr-1, rounds from the bottom.
template <int NT, int RM>
__device__ __forceinline__ void lds_dit(uint32_t* X, int lr, int lc, int rs, uint32_t colbase, const uint32_t* tw, Mod md) {
  const uint32_t M = 1u << (lr + lc);
  int s_lo = 0;
  for (int idx = 0; s_lo < lr; idx++) {
    const int r = round_size<RM>(lr, idx);
    lds_round_r<NT, 1, true, RM>(r, X, 0, M, s_lo, lc, rs, colbase, tw, md);
    s_lo += r;
  }
}

// ---------------------------------------------------------------------------
// The row pass of long transforms always covers LR = 13 stages of a
// contiguous 2^13 block, so its rounds are generated at compile time: the
// round geometry (first stage, group stride) is a constant, and the LDS
// address of a group's j-th element needs at most one operation:
//   * first stage >= 9: the swizzle touches only bits the stride never
//     reaches, so lds_at(yb + j 2^s) = lds_at(yb) + j 2^s;
//   * the group lies inside one 64-word row (first stage + R <= 6): the row
//     key is shared, so lds_at(yb + j 2^s) = lds_at(yb) ^ (j 2^s);
//   * otherwise, by the linearity of the key, lds_at(yb) ^ lds_at(j 2^s) with
//     the second term a compile-time constant.
// The inverse uses the forward's round sizes in reverse order, so its first
// rounds also fall in the cheap cases.
// ---------------------------------------------------------------------------

template <int LR, int RM>
constexpr int fixed_nrounds() { return (LR + RM - 1) / RM; }

template <int LR, int RM>
constexpr int fixed_rsize(int idx) {
  return LR / fixed_nrounds<LR, RM>() + (idx < LR % fixed_nrounds<LR, RM>() ? 1 : 0);
}

// First stage of forward round idx (rounds from the top).
template <int LR, int RM>
constexpr int fixed_dif_slo(int idx) {
  int s = LR;
  for (int i = 0; i <= idx; i++) s -= fixed_rsize<LR, RM>(i);
  return s;
}

// Size and first stage of inverse round idx (sizes mirrored, from the bottom).
template <int LR, int RM>
constexpr int fixed_dit_rsize(int idx) { return fixed_rsize<LR, RM>(fixed_nrounds<LR, RM>() - 1 - idx); }

template <int LR, int RM>
constexpr int fixed_dit_slo(int idx) {
  int s = 0;
  for (int i = 0; i < idx; i++) s += fixed_dit_rsize<LR, RM>(i);
  return s;
}

template <int A_LO, int R, int J>
__device__ __forceinline__ uint32_t group_addr(uint32_t yb, uint32_t pb) {
  constexpr uint32_t step = (uint32_t)J << A_LO;
  if constexpr (A_LO >= 9) return pb + step;
  else if constexpr (A_LO + R <= 6) return pb ^ step;
  else {
    constexpr uint32_t cs = lds_at(step);
    return pb ^ cs;
  }
}

template <int A_LO, int R, int J>
__device__ __forceinline__ void fill_group_addr(uint32_t* ad, uint32_t yb, uint32_t pb) {
  if constexpr (J < (1 << R)) {
    ad[J] = group_addr<A_LO, R, J>(yb, pb);
    fill_group_addr<A_LO, R, J + 1>(ad, yb, pb);
  }
}

// Global operands of a column tile whose first and last rounds read and
// write global memory directly.  Element (k, c) of the tile is global index
// colbase + c + k 2^RS.
struct ColIO {
  const uint32_t* src;   // first round: residues, zero beyond index dvalid
  uint32_t dvalid;
  uint32_t scale;        // first round: nonzero multiplies by REDC(x * scale)
  uint32_t* dst;         // last round: stores only indices < nout
  uint32_t nout;
  // A truncated-transform block (forward tiles): the first round loads
  // w^r sum_i src[r + i s] w^(is) instead of src[r], with s the tile's
  // transform length and w = w_N of the whole product.
  const uint32_t* twist; // nullptr: plain load; else entry r holds w^r (Montgomery form)
  uint32_t fold_s;       // s
  uint32_t z[3];         // w^(is) for i = 1, 2, 3 (Montgomery form; 0 where unused)
};

// One round with compile-time geometry: rows of 2^LC columns (LC = 0 for the
// row pass), transform length 2^LR along rows, global row stride 2^RS.  GIN:
// the group is loaded from io.src instead of LDS; GOUT: it is stored to
// io.dst (coherent stores if COH) instead of LDS.  With both, the round does
// not touch LDS.
template <int NT, int NA, int R, bool INV, int LR, int LC, int RS, int S_LO, bool GIN = false, bool GOUT = false,
          bool COH = false>
__device__ __forceinline__ void lds_round_fixed(uint32_t* X, int off, uint32_t colbase, const uint32_t* tw,
                                                Mod md, ColIO io = ColIO{}) {
  static_assert(NA == 1 || !(GIN || GOUT), "global rounds take one operand");
  static_assert(LC > 0 || RS == 0, "LC = 0 is the row pass (unit twiddles in its stage-0 round)");
  constexpr int E = 1 << R;
  constexpr int A_LO = S_LO + LC;
  constexpr uint32_t lomask = (1u << A_LO) - 1;
  constexpr uint32_t ngroups = (1u << (LR + LC)) >> R;
  constexpr int GS = S_LO + RS;
  if constexpr (GIN && ngroups == 2 * NT) {
    // A round that loads from HBM with two groups per lane (the first round
    // of a column tile): the lane issues both groups' data loads before any
    // arithmetic, so it waits on HBM once per round instead of once per
    // group.  (The group loop below cannot overlap them: its start, the lane
    // index, is opaque to the compiler.)  The second group's twiddles are
    // loaded after the first group's arithmetic (they come from the
    // cache-resident tables), which keeps the round within the register
    // budget.  Truncated-transform blocks take the loop.
    if (!io.twist) {
      const uint32_t tid = task_tid();
      const __amdgpu_buffer_rsrc_t rs = buf_rsrc(io.src, src_bytes(io.dvalid));
      const __amdgpu_buffer_rsrc_t rt = buf_rsrc(tw, 0xFFFFFFFFu);
      uint32_t v[2][E], gi0[2], base[2], c[2];
#pragma unroll
      for (int q = 0; q < 2; q++) {
        const uint32_t g = tid + (uint32_t)q * NT;
        base[q] = ((g & ~lomask) << R) | (g & lomask);
        c[q] = base[q] & ((1u << LC) - 1);
        gi0[q] = colbase + c[q] + ((base[q] >> LC) << RS);
#pragma unroll
        for (int j = 0; j < E; j++) v[q][j] = buf_ld(rs, (gi0[q] + ((uint32_t)j << GS)) << 2);
      }
#pragma unroll
      for (int q = 0; q < 2; q++) {
        // keeps the scheduler from hoisting the second group's twiddle loads
        // above the first group's arithmetic
        __builtin_amdgcn_sched_barrier(0);
        const uint32_t t0 = (colbase + c[q] + (((base[q] >> LC) & ((1u << S_LO) - 1)) << RS)) << 2;
        uint32_t w[E - 1];
#pragma unroll
        for (int t = 0; t < R; t++)
#pragma unroll
          for (int jj = 0; jj < (1 << t); jj++)
            w[(1 << t) - 1 + jj] = buf_ld(rt, t0, ((1u << (S_LO + t + RS)) + ((uint32_t)jj << (S_LO + RS))) << 2);
        if (io.scale) {
#pragma unroll
          for (int j = 0; j < E; j++) v[q][j] = mmul(v[q][j], io.scale, md);
        }
        if constexpr (!INV) {
          uint32_t wn[E - 1];
#pragma unroll
          for (int k = 0; k < E - 1; k++) wn[k] = md.P - w[k];
          dif_stages<R>(v[q], w, wn, md);
        } else {
          dit_stages<R>(v[q], w, md);
        }
        if constexpr (GOUT) {
#pragma unroll
          for (int j = 0; j < E; j++) {
            const uint32_t gi = gi0[q] + ((uint32_t)j << GS);
            if (gi < io.nout) st_out<COH>(io.dst + gi, v[q][j]);
          }
        } else {
          uint32_t ad[E];
          fill_group_addr<A_LO, R, 0>(ad, base[q], lds_at(base[q]));
#pragma unroll
          for (int j = 0; j < E; j++) X[ad[j]] = v[q][j];
        }
      }
      __syncthreads();
      return;
    }
  }
  const __amdgpu_buffer_rsrc_t rt = buf_rsrc(tw, 0xFFFFFFFFu);
  const __amdgpu_buffer_rsrc_t rs = buf_rsrc(GIN ? io.src : tw, GIN ? src_bytes(io.dvalid) : 0u);
  for (uint32_t g = task_tid(); g < ngroups; g += NT) {
    const uint32_t base = ((g & ~lomask) << R) | (g & lomask);
    const uint32_t c = base & ((1u << LC) - 1);
    const uint32_t t0 = (colbase + c + (((base >> LC) & ((1u << S_LO) - 1)) << RS)) << 2;
    uint32_t w[E - 1];
#pragma unroll
    for (int t = 0; t < R; t++)
#pragma unroll
      for (int jj = 0; jj < (1 << t); jj++)
        w[(1 << t) - 1 + jj] = buf_ld(rt, t0, ((1u << (S_LO + t + RS)) + ((uint32_t)jj << (S_LO + RS))) << 2);
    uint32_t wn[E - 1];
    if constexpr (!INV) {
#pragma unroll
      for (int k = 0; k < E - 1; k++) wn[k] = md.P - w[k];
    }
#pragma unroll
    for (int a = 0; a < NA; a++) {
      const uint32_t yb = (uint32_t)(a * off) + base;
      const uint32_t pb = lds_at(yb);
      uint32_t v[E];
      uint32_t ad[E];
      fill_group_addr<A_LO, R, 0>(ad, yb, pb);
      // global index of the group's element j
      const uint32_t gi0 = colbase + c + ((base >> LC) << RS);
      if constexpr (GIN) {
        if (io.twist) {
          // fold modulo x^s - w^s (operands are shorter than 4s), then twist
#pragma unroll
          for (int j = 0; j < E; j++) {
            const uint32_t gi = gi0 + ((uint32_t)j << GS);
            uint32_t acc = gi <= io.dvalid ? io.src[gi] : 0u;
#pragma unroll
            for (int i = 1; i < 4; i++) {
              const uint32_t gk = gi + (uint32_t)i * io.fold_s;
              if (gk <= io.dvalid) acc = madd(acc, mmul(io.src[gk], io.z[i - 1], md), md.P);
            }
            v[j] = mmul(acc, ldg(io.twist, gi), md);
          }
        } else {
#pragma unroll
          for (int j = 0; j < E; j++) v[j] = buf_ld(rs, (gi0 + ((uint32_t)j << GS)) << 2);
        }
        if (io.scale) {
#pragma unroll
          for (int j = 0; j < E; j++) v[j] = mmul(v[j], io.scale, md);
        }
      } else {
#pragma unroll
        for (int j = 0; j < E; j++) v[j] = X[ad[j]];
      }
      // LC = 0 is the row pass, whose blocks start at twiddle offset 0
      // (colbase = 0): its round holding stage 0 skips the unit twiddles
      if constexpr (!INV) dif_stages<R, S_LO == 0 && LC == 0>(v, w, wn, md);
      else dit_stages<R, S_LO == 0 && LC == 0>(v, w, md);
      if constexpr (GOUT) {
#pragma unroll
        for (int j = 0; j < E; j++) {
          const uint32_t gi = gi0 + ((uint32_t)j << GS);
          if (gi < io.nout) st_out<COH>(io.dst + gi, v[j]);
        }
      } else {
#pragma unroll
        for (int j = 0; j < E; j++) X[ad[j]] = v[j];
      }
    }
  }
  __syncthreads();
}

// Forward rounds IDX .. END-1 (all of them by default).  GIO: round 0 loads
// from and round END-1 stores to global memory (ColIO).
template <int NT, int NA, int RM, int LR, int LC, int RS, int IDX = 0, int END = fixed_nrounds<LR, RM>(),
          bool GIO = false, bool COH = false>
__device__ __forceinline__ void fixed_dif(uint32_t* X, int off, uint32_t colbase, const uint32_t* tw, Mod md,
                                          ColIO io = ColIO{}) {
  if constexpr (IDX < END) {
    lds_round_fixed<NT, NA, fixed_rsize<LR, RM>(IDX), false, LR, LC, RS, fixed_dif_slo<LR, RM>(IDX), GIO && IDX == 0,
                    GIO && IDX == END - 1, COH>(X, off, colbase, tw, md, io);
    fixed_dif<NT, NA, RM, LR, LC, RS, IDX + 1, END, GIO, COH>(X, off, colbase, tw, md, io);
  }
}

// Inverse rounds IDX .. END-1 (all of them by default), GIO as above.
template <int NT, int RM, int LR, int LC, int RS, int IDX = 0, int END = fixed_nrounds<LR, RM>(), bool GIO = false,
          bool COH = false>
__device__ __forceinline__ void fixed_dit(uint32_t* X, uint32_t colbase, const uint32_t* tw, Mod md,
                                          ColIO io = ColIO{}) {
  if constexpr (IDX < END) {
    lds_round_fixed<NT, 1, fixed_dit_rsize<LR, RM>(IDX), true, LR, LC, RS, fixed_dit_slo<LR, RM>(IDX), GIO && IDX == 0,
                    GIO && IDX == END - 1, COH>(X, 0, colbase, tw, md, io);
    fixed_dit<NT, RM, LR, LC, RS, IDX + 1, END, GIO, COH>(X, colbase, tw, md, io);
  }
}

// The first forward round of a row-block product reads both blocks straight
// from global memory and the last inverse round writes the product straight
// back, instead of staging the blocks through LDS.  Both rounds cover the top
// stages (first stage S_LO >= 9), where a group's residues lie 2^S_LO apart:
// lane g of a wave takes group base g, so each of the 2^R loads or stores of
// a wave covers 64 adjacent words, and the LDS address of element j is
// lds_at(base) + j 2^S_LO (the swizzle leaves bits >= 9 alone).
template <int NT, int R, int S_LO>
__device__ __forceinline__ void row_round_in(uint32_t* X, uint32_t L, const uint32_t* gA, const uint32_t* gB,
                                             const uint32_t* tw, Mod md) {
  static_assert(S_LO >= 9, "the group stride must be above the swizzled bits");
  constexpr int E = 1 << R;
  constexpr uint32_t lomask = (1u << S_LO) - 1;
  const __amdgpu_buffer_rsrc_t rt = buf_rsrc(tw, 0xFFFFFFFFu);
  const __amdgpu_buffer_rsrc_t ra = buf_rsrc(gA, 0xFFFFFFFFu);
  const __amdgpu_buffer_rsrc_t rb = buf_rsrc(gB, 0xFFFFFFFFu);
  for (uint32_t g = task_tid(); g < ((1u << kRowLog) >> R); g += NT) {
    const uint32_t base = ((g & ~lomask) << R) | (g & lomask);
    const uint32_t t0 = (base & lomask) << 2;
    uint32_t w[E - 1], wn[E - 1];
#pragma unroll
    for (int t = 0; t < R; t++)
#pragma unroll
      for (int jj = 0; jj < (1 << t); jj++)
        w[(1 << t) - 1 + jj] = buf_ld(rt, t0, ((1u << (S_LO + t)) + ((uint32_t)jj << S_LO)) << 2);
#pragma unroll
    for (int k = 0; k < E - 1; k++) wn[k] = md.P - w[k];
#pragma unroll
    for (int a = 0; a < 2; a++) {
      uint32_t v[E];
#pragma unroll
      for (int j = 0; j < E; j++) v[j] = buf_ld(a == 0 ? ra : rb, base << 2, ((uint32_t)j << S_LO) << 2);
      dif_stages<R>(v, w, wn, md);
      const uint32_t pb = lds_at((uint32_t)a * L + base);
#pragma unroll
      for (int j = 0; j < E; j++) X[pb + ((uint32_t)j << S_LO)] = v[j];
    }
  }
  __syncthreads();
}

template <int NT, int R, int S_LO, bool COH>
__device__ __forceinline__ void row_round_out(const uint32_t* X, uint32_t* gA, const uint32_t* tw, Mod md) {
  static_assert(S_LO >= 9, "the group stride must be above the swizzled bits");
  constexpr int E = 1 << R;
  constexpr uint32_t lomask = (1u << S_LO) - 1;
  const __amdgpu_buffer_rsrc_t rt = buf_rsrc(tw, 0xFFFFFFFFu);
  for (uint32_t g = task_tid(); g < ((1u << kRowLog) >> R); g += NT) {
    const uint32_t base = ((g & ~lomask) << R) | (g & lomask);
    const uint32_t t0 = (base & lomask) << 2;
    uint32_t w[E - 1];
#pragma unroll
    for (int t = 0; t < R; t++)
#pragma unroll
      for (int jj = 0; jj < (1 << t); jj++)
        w[(1 << t) - 1 + jj] = buf_ld(rt, t0, ((1u << (S_LO + t)) + ((uint32_t)jj << S_LO)) << 2);
    const uint32_t pb = lds_at(base);
    uint32_t v[E];
#pragma unroll
    for (int j = 0; j < E; j++) v[j] = X[pb + ((uint32_t)j << S_LO)];
    dit_stages<R>(v, w, md);
#pragma unroll
    for (int j = 0; j < E; j++) st_out<COH>(gA + base + ((uint32_t)j << S_LO), v[j]);
  }
}

// The middle of a row-block product: the last forward round of both blocks,
// their pointwise product and the first inverse round.  The forward's last
// round and the inverse's first cover the same stages 0 .. R-1 on the same
// groups of 2^R adjacent residues, and for those stages the twiddles are the
// same for every group, so the three steps run on registers: LDS is read and
// written once for them instead of three times, and two barriers go away.
// A (L words) is at X[lds_at(0 ..)], B at X[lds_at(L ..)]; the product
// replaces A.  A group lies inside one 64-word LDS row (R <= 6), where the
// swizzle is the same for all its words.
template <int NT, int R>
__device__ __forceinline__ void row_round_fused(uint32_t* X, uint32_t L, const uint32_t* twf, const uint32_t* twi,
                                                Mod md) {
  static_assert(R <= 6, "group must lie inside one LDS row");
  constexpr int E = 1 << R;
  uint32_t wf[E - 1], wfn[E - 1], wi[E - 1];
#pragma unroll
  for (int k = 0; k < E - 1; k++) {
    // entry k = 2^t - 1 + jj of stage t sits at table index 2^t + jj = k + 1
    wf[k] = ldg(twf, (uint32_t)k + 1);
    wi[k] = ldg(twi, (uint32_t)k + 1);
    wfn[k] = md.P - wf[k];
  }
  for (uint32_t g = task_tid(); g < (L >> R); g += NT) {
    const uint32_t pa = lds_at(g << R), pb = lds_at(L + (g << R));
    uint32_t va[E], vb[E];
#pragma unroll
    for (int j = 0; j < E; j++) {
      va[j] = X[pa ^ (uint32_t)j];
      vb[j] = X[pb ^ (uint32_t)j];
    }
    dif_stages<R, true>(va, wf, wfn, md);
    dif_stages<R, true>(vb, wf, wfn, md);
#pragma unroll
    for (int j = 0; j < E; j++) va[j] = mmul(va[j], vb[j], md);
    dit_stages<R, true>(va, wi, md);
#pragma unroll
    for (int j = 0; j < E; j++) X[pa ^ (uint32_t)j] = va[j];
  }
  __syncthreads();
}

// Column tiles of a length-2^N transform: 2^(N-13) rows x 2^col_lc(N) columns.

constexpr int col_lc_c(int n) { return 13 < 14 - (n - 13) ? 13 : 14 - (n - 13); }

// For 14 <= N <= 23 the column rounds are generated at compile time, the
// first reading the tile from global memory and the last writing it there;
// up to N = 17 a single round does both and the tile never passes through LDS.
template <int NT, int RM, int N, bool GIO, bool COH>
__device__ __forceinline__ void col_dif_fixed(uint32_t* X, uint32_t colbase, const uint32_t* tw, Mod md,
                                              ColIO io = ColIO{}) {
  fixed_dif<NT, 1, RM, N - 13, col_lc_c(N), 13, 0, fixed_nrounds<N - 13, RM>(), GIO, COH>(X, 0, colbase, tw, md, io);
}

template <int NT, int RM, int N, bool GIO, bool COH>
__device__ __forceinline__ void col_dit_fixed(uint32_t* X, uint32_t colbase, const uint32_t* tw, Mod md,
                                              ColIO io = ColIO{}) {
  fixed_dit<NT, RM, N - 13, col_lc_c(N), 13, 0, fixed_nrounds<N - 13, RM>(), GIO, COH>(X, colbase, tw, md, io);
}

// Whole column tile (load, stages, store) with HBM first and last rounds, for
// 2^15..2^23; false, doing nothing, for the others.  A 2^14 tile (two rows of
// 2^13) is a single radix-2 round whose sixteen groups per lane would each
// wait on HBM in turn; it is staged through LDS with wide loads instead.
template <int NT, int RM, bool INV, bool COH>
__device__ __forceinline__ bool col_fixed(int n, uint32_t* X, uint32_t colbase, const uint32_t* tw, Mod md, ColIO io) {
  switch (n) {
#define MONT_COL(NN)                                                               \
  case NN:                                                                         \
    if constexpr (INV) col_dit_fixed<NT, RM, NN, true, COH>(X, colbase, tw, md, io); \
    else col_dif_fixed<NT, RM, NN, true, COH>(X, colbase, tw, md, io);              \
    return true;
    MONT_COL(15) MONT_COL(16) MONT_COL(17) MONT_COL(18)
    MONT_COL(19) MONT_COL(20) MONT_COL(21) MONT_COL(22) MONT_COL(23)
#undef MONT_COL
    default: return false;
  }
}

// Column stages on an LDS tile for the one length col_fixed leaves out,
// 2^14 (two rows of 2^13): compile-time rounds.  Contexts cap transforms at
// 2^kMaxLog = 2^23, so no other length reaches this point.
template <int NT, int RM, bool INV>
__device__ __forceinline__ void col_stages(uint32_t* X, uint32_t colbase, const uint32_t* tw, Mod md) {
  if constexpr (INV) col_dit_fixed<NT, RM, 14, false, false>(X, colbase, tw, md);
  else col_dif_fixed<NT, RM, 14, false, false>(X, colbase, tw, md);
}


// ---------------------------------------------------------------------------
// Task bodies.  Every thread of the workgroup calls them (they contain
// barriers); X is the workgroup's LDS buffer of kLdsWords words.
// ---------------------------------------------------------------------------

// Whole product with N = 2^n <= 2^13: zero-padded loads, b scaled by R/N on
// load, forward transforms of both, pointwise REDC (which removes one R and
// leaves a b / N), inverse transform, store of the da + db + 1 coefficients.
template <int NT, int RM>
__device__ __forceinline__ void exec_small_poly(const PrimeDev& pr, int n, const uint32_t* a, uint32_t da, const uint32_t* b,
                                uint32_t db, uint32_t* out, uint32_t nout, uint32_t* X) {
  const Mod md = mod_of(pr);
  const uint32_t N = 1u << n;
  const uint32_t sc = pr.s2[n];
  for (uint32_t e = task_tid(); e < N; e += NT) {
    X[lds_at(e)] = e <= da ? a[e] : 0u;
    X[lds_at(N + e)] = e <= db ? mmul(b[e], sc, md) : 0u;
  }
  __syncthreads();
  if (n > 0) lds_dif<NT, 2, RM>(X, (int)N, n, 0, 0, 0, pr.twf, md);
  for (uint32_t e = task_tid(); e < N; e += NT) X[lds_at(e)] = mmul(X[lds_at(e)], X[lds_at(N + e)], md);
  __syncthreads();
  if (n > 0) lds_dit<NT, RM>(X, n, 0, 0, 0, pr.twi, md);
  for (uint32_t e = task_tid(); e < nout; e += NT) out[e] = X[lds_at(e)];
  __syncthreads();
}

// Forward column pass, tile t: rows k < 2^n1, columns t*C + c; the input is
// zero beyond index dvalid; scale != 0 multiplies by REDC(x * scale) on load.
// A truncated-transform block (tft = log2 N of the whole product, 0 for a
// plain product; lengths 2^15 and up) folds and twists its operand in the
// first round's loads.
template <int NT, int RM, bool COH>
__device__ __forceinline__ void exec_col_dif(const PrimeDev& pr, int n, int lc, uint32_t t, const uint32_t* src, uint32_t dvalid,
                             uint32_t scale, uint32_t* dst, uint32_t* X, uint32_t tft = 0) {
  const Mod md = mod_of(pr);
  const int n1 = n - kRowLog;
  const uint32_t colbase = t << lc;
  const uint32_t cnt = 1u << (n1 + lc);
  const uint32_t cmask = (1u << lc) - 1;
  ColIO io = ColIO{src, dvalid, scale, dst, 0xFFFFFFFFu};
  if (tft) {
    const uint32_t half = 1u << (tft - 1);        // w^r for r < N/2 sits at table entry N/2 + r
    io.twist = pr.twf + half;
    io.fold_s = 1u << n;
#pragma unroll
    for (int i = 1; i < 4; i++) io.z[i - 1] = (uint32_t)i << n < half ? ldg(pr.twf, half + ((uint32_t)i << n)) : 0u;
  }
  if (col_fixed<NT, RM, false, COH>(n, X, colbase, pr.twf, md, io)) return;
  if (lc >= 2 && ((uintptr_t)src & 15u) == 0) {
    // rows of C >= 4 adjacent residues: 128-bit loads where all four are
    // inside the operand, element loads on the (at most one) straddling chunk
    for (uint32_t e4 = task_tid(); e4 < (cnt >> 2); e4 += NT) {
      const uint32_t e = e4 << 2;
      const uint32_t i = colbase + (e & cmask) + ((e >> lc) << kRowLog);
      v4u v;
      if (i + 3 <= dvalid) {
        v = *reinterpret_cast<const v4u*>(src + i);
      } else {
        v.x = i <= dvalid ? src[i] : 0u;
        v.y = i + 1 <= dvalid ? src[i + 1] : 0u;
        v.z = i + 2 <= dvalid ? src[i + 2] : 0u;
        v.w = 0u;
      }
      if (scale) {
        v.x = mmul(v.x, scale, md);
        v.y = mmul(v.y, scale, md);
        v.z = mmul(v.z, scale, md);
        v.w = mmul(v.w, scale, md);
      }
      X[lds_at(e)] = v.x;
      X[lds_at(e + 1)] = v.y;
      X[lds_at(e + 2)] = v.z;
      X[lds_at(e + 3)] = v.w;
    }
  } else {
    for (uint32_t e = task_tid(); e < cnt; e += NT) {
      const uint32_t i = colbase + (e & cmask) + ((e >> lc) << kRowLog);
      uint32_t v = i <= dvalid ? src[i] : 0u;
      if (scale) v = mmul(v, scale, md);
      X[lds_at(e)] = v;
    }
  }
  __syncthreads();
  col_stages<NT, RM, false>(X, colbase, pr.twf, md);
  for (uint32_t e = task_tid(); e < cnt; e += NT) {
    const uint32_t i = colbase + (e & cmask) + ((e >> lc) << kRowLog);
    st_out<COH>(dst + i, X[lds_at(e)]);
  }
  __syncthreads();
}

// Inverse column pass, tile t: the last n1 inverse stages; stores only
// indices < nout.
template <int NT, int RM>
__device__ __forceinline__ void exec_col_dit(const PrimeDev& pr, int n, int lc, uint32_t t, const uint32_t* src, uint32_t* dst,
                             uint32_t nout, uint32_t* X) {
  const Mod md = mod_of(pr);
  const int n1 = n - kRowLog;
  const uint32_t colbase = t << lc;
  const uint32_t cnt = 1u << (n1 + lc);
  const uint32_t cmask = (1u << lc) - 1;
  if (col_fixed<NT, RM, true, false>(n, X, colbase, pr.twi, md, ColIO{src, 0xFFFFFFFFu, 0u, dst, nout})) return;
  if (lc >= 2 && ((uintptr_t)src & 15u) == 0) {
    // rows of C >= 4 adjacent residues: 128-bit loads
    for (uint32_t e4 = task_tid(); e4 < (cnt >> 2); e4 += NT) {
      const uint32_t e = e4 << 2;
      const uint32_t i = colbase + (e & cmask) + ((e >> lc) << kRowLog);
      const v4u v = *reinterpret_cast<const v4u*>(src + i);
      X[lds_at(e)] = v.x;
      X[lds_at(e + 1)] = v.y;
      X[lds_at(e + 2)] = v.z;
      X[lds_at(e + 3)] = v.w;
    }
  } else {
    for (uint32_t e = task_tid(); e < cnt; e += NT) {
      const uint32_t i = colbase + (e & cmask) + ((e >> lc) << kRowLog);
      X[lds_at(e)] = src[i];
    }
  }
  __syncthreads();
  col_stages<NT, RM, true>(X, colbase, pr.twi, md);
  for (uint32_t e = task_tid(); e < cnt; e += NT) {
    const uint32_t i = colbase + (e & cmask) + ((e >> lc) << kRowLog);
    if (i < nout) dst[i] = X[lds_at(e)];
  }
  __syncthreads();
}

enum RowMode { ROW_POLY = 0, ROW_FWD = 1, ROW_INV = 2 };

// Row pass over one contiguous block of 2^lr residues (block offsets are
// multiples of 2^lr, so the twiddle index needs no column term).
//   ROW_POLY: forward stages on A and B, A = REDC(A B), inverse stages on A;
//   ROW_FWD:  forward stages on A;
//   ROW_INV:  A scaled by REDC(x * prescale) on load, inverse stages on A.
template <int NT, int RM, bool COH>
__device__ __forceinline__ void exec_row(const PrimeDev& pr, int lr, int mode, uint32_t* gA, const uint32_t* gB,
                         uint32_t prescale, uint32_t* X) {
  const Mod md = mod_of(pr);
  const uint32_t L = 1u << lr;
  if (mode == ROW_POLY && lr == kRowLog) {
    // compile-time rounds: the first reads global memory, the last forward
    // round, the pointwise product and the first inverse round run fused, the
    // last writes global memory
    constexpr int nr = fixed_nrounds<kRowLog, RM>();
    static_assert(nr >= 3, "first, middle and last rounds must be distinct");
    row_round_in<NT, fixed_rsize<kRowLog, RM>(0), fixed_dif_slo<kRowLog, RM>(0)>(X, L, gA, gB, pr.twf, md);
    fixed_dif<NT, 2, RM, kRowLog, 0, 0, 1, nr - 1>(X, (int)L, 0u, pr.twf, md);
    row_round_fused<NT, fixed_rsize<kRowLog, RM>(nr - 1)>(X, L, pr.twf, pr.twi, md);
    fixed_dit<NT, RM, kRowLog, 0, 0, 1, nr - 1>(X, 0u, pr.twi, md);
    row_round_out<NT, fixed_dit_rsize<kRowLog, RM>(nr - 1), fixed_dit_slo<kRowLog, RM>(nr - 1), COH>(X, gA, pr.twi, md);
    __syncthreads();
    return;
  }
  if (mode == ROW_POLY && lr >= 2 && (((uintptr_t)gA | (uintptr_t)gB) & 15u) == 0) {
    // 128-bit loads of both blocks
    const v4u* a4 = reinterpret_cast<const v4u*>(gA);
    const v4u* b4 = reinterpret_cast<const v4u*>(gB);
    for (uint32_t e4 = task_tid(); e4 < (L >> 2); e4 += NT) {
      const v4u va = a4[e4], vb = b4[e4];
      const uint32_t e = e4 << 2;
      X[lds_at(e)] = va.x;
      X[lds_at(e + 1)] = va.y;
      X[lds_at(e + 2)] = va.z;
      X[lds_at(e + 3)] = va.w;
      X[lds_at(L + e)] = vb.x;
      X[lds_at(L + e + 1)] = vb.y;
      X[lds_at(L + e + 2)] = vb.z;
      X[lds_at(L + e + 3)] = vb.w;
    }
  } else {
    for (uint32_t e = task_tid(); e < L; e += NT) {
      uint32_t v = gA[e];
      if (mode == ROW_INV && prescale) v = mmul(v, prescale, md);
      X[lds_at(e)] = v;
      if (mode == ROW_POLY) X[lds_at(L + e)] = gB[e];
    }
  }
  __syncthreads();
  if (lr > 0) {
    if (mode == ROW_POLY) lds_dif<NT, 2, RM>(X, (int)L, lr, 0, 0, 0, pr.twf, md);
    else if (mode == ROW_FWD) lds_dif<NT, 1, RM>(X, 0, lr, 0, 0, 0, pr.twf, md);
  }
  if (mode == ROW_POLY) {
    for (uint32_t e = task_tid(); e < L; e += NT) X[lds_at(e)] = mmul(X[lds_at(e)], X[lds_at(L + e)], md);
    __syncthreads();
  }
  if (mode != ROW_FWD && lr == kRowLog) fixed_dit<NT, RM, kRowLog, 0, 0>(X, 0u, pr.twi, md);
  else if (mode != ROW_FWD && lr > 0) lds_dit<NT, RM>(X, lr, 0, 0, 0, pr.twi, md);
  for (uint32_t e = task_tid(); e < L; e += NT) st_out<COH>(gA + e, X[lds_at(e)]);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------


// Plain launches: one task per workgroup, the task index is blockIdx.x.
struct DirectArgs {
  const PrimeDev* primes;
  uint32_t prime_id, kind, n, lc;
  const uint32_t* a;
  const uint32_t* b;
  uint32_t* out;
  uint32_t* scr;        // 2N words for the multi-pass product
  uint32_t da, db;
  uint32_t ntiles;
  uint32_t prescale;
};

enum DirectKind : uint32_t {
  D_SMALL_POLY = 0,  // grid 1
  D_COLF = 1,        // grid 2 ntiles: tiles of a, then of b (scaled)
  D_ROW_POLY = 2,    // grid nblocks
  D_COLI = 3,        // grid ntiles
  D_FWD_SMALL = 4,   // in place on out, grid 1
  D_INV_SMALL = 5,   // in place on out, grid 1, prescale = s1[n]
  D_COLF_INPLACE = 6,
  D_ROW_FWD = 7,
  D_ROW_INV = 8,
  D_COLI_INPLACE = 9,
};

template <int NT, int RM>
__global__ __launch_bounds__(NT, NT >= 1024 ? 4 : NT / 128) void k_ntt_direct(DirectArgs g) {
  __shared__ uint32_t X[kLdsWords];
  const PrimeDev& pr = g.primes[g.prime_id];
  const uint32_t bid = blockIdx.x;
  const uint32_t N = 1u << g.n;
  const uint32_t S = 1u << kRowLog;
  switch (g.kind) {
    case D_SMALL_POLY: exec_small_poly<NT, RM>(pr, g.n, g.a, g.da, g.b, g.db, g.out, g.da + g.db + 1, X); break;
    case D_COLF:
      if (bid < g.ntiles) exec_col_dif<NT, RM, false>(pr, g.n, g.lc, bid, g.a, g.da, 0u, g.scr, X);
      else exec_col_dif<NT, RM, false>(pr, g.n, g.lc, bid - g.ntiles, g.b, g.db, pr.s2[g.n], g.scr + N, X);
      break;
    case D_ROW_POLY: exec_row<NT, RM, false>(pr, kRowLog, ROW_POLY, g.scr + bid * S, g.scr + N + bid * S, 0u, X); break;
    case D_COLI: exec_col_dit<NT, RM>(pr, g.n, g.lc, bid, g.scr, g.out, g.da + g.db + 1, X); break;
    case D_FWD_SMALL: exec_row<NT, RM, false>(pr, g.n, ROW_FWD, g.out, nullptr, 0u, X); break;
    case D_INV_SMALL: exec_row<NT, RM, false>(pr, g.n, ROW_INV, g.out, nullptr, g.prescale, X); break;
    case D_COLF_INPLACE: exec_col_dif<NT, RM, false>(pr, g.n, g.lc, bid, g.out, N - 1, 0u, g.out, X); break;
    case D_ROW_FWD: exec_row<NT, RM, false>(pr, kRowLog, ROW_FWD, g.out + bid * S, nullptr, 0u, X); break;
    case D_ROW_INV: exec_row<NT, RM, false>(pr, kRowLog, ROW_INV, g.out + bid * S, nullptr, g.prescale, X); break;
    default: exec_col_dit<NT, RM>(pr, g.n, g.lc, bid, g.out, g.out, N, X); break;
  }
}

// Persistent batch kernel: workgroups take task indices from a counter in
// the scratch header; a task's prerequisites always sit earlier in the list,
// so every wait is on a task some running workgroup already holds.  Waits are
// bounded by spin_limit sleeps; on expiry the status word is set, the task is
// skipped, and so are all later waits, so the grid always drains.
// A small plan (a serving loop's batch) travels in the launch arguments, so
// its execution needs no upload before the launch.
constexpr uint32_t kInlineProds = 4;
constexpr uint32_t kInlineTasks = 384;

struct PlanArgs {
  const PrimeDev* primes;
  const ProdDev* prods;
  const uint2* tasks;       // (product, kind << 28 | index)
  uint32_t ntasks;
  uint32_t nprods;
  const uint32_t* in;
  uint32_t* out;
  uint32_t* scr;            // header, two counters per product, then product scratch
  uint32_t spin_limit;
  uint32_t inl;             // 1: products and tasks are the copies below, not prods / tasks
  uint32_t dyn;             // 1: planned on the device; the task count is in the scratch header
  ProdDev inl_prods[kInlineProds];
  uint2 inl_tasks[kInlineTasks];
};

// Spin (lane 0 only) until *ctr >= need.  The loop reads the counter with
// relaxed agent-scope loads, which go past the non-coherent caches without
// invalidating them; one acquire fence after success makes the producers'
// data visible (it invalidates this CU's L1 and this XCD's L2 once).
__device__ __forceinline__ bool wait_count(uint32_t* ctr, uint32_t need, uint32_t* status, uint32_t spin_limit) {
  uint32_t it = 0;
  while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
    if (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
    if (++it > spin_limit) {
      __hip_atomic_store(status, kStatusTimeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(4);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

// s_waitcnt with vmcnt = 0 and the other counters at their maximum (gfx9
// encoding: vmcnt[3:0], expcnt[6:4], lgkmcnt[11:8], vmcnt_hi[15:14]): the
// wave's outstanding global stores have been acknowledged by L2.
constexpr int kWaitVmcnt0 = 0x0F70;

template <int NT, int RM>
__global__ __launch_bounds__(NT, NT >= 1024 ? 4 : NT / 128) void k_ntt_persistent(PlanArgs g) {
  __shared__ uint32_t X[kLdsWords];
  __shared__ uint32_t s_task, s_go;
  uint32_t* head = g.scr;
  uint32_t* status = g.scr + 1;
  uint32_t* cnt_col = g.scr + kHdrWords;
  uint32_t* cnt_row = cnt_col + g.nprods;
  const uint32_t S = 1u << kRowLog;
  // written by the planning kernel before this launch (zero after a planning error)
  const uint32_t ntasks = g.dyn ? g.scr[kHdrNtasks] : g.ntasks;
  if (threadIdx.x == 0) s_task = __hip_atomic_fetch_add(head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    __syncthreads();
    // uniform across the workgroup: keeps the task's fields and pointers in
    // scalar registers
    const uint32_t ti = __builtin_amdgcn_readfirstlane(s_task);
    if (ti >= ntasks) break;
    // Reserve the next task now: its index is needed only when this task
    // ends, so the atomic's round trip overlaps the work.  A workgroup holds
    // at most one reserved task beside its running one, and the lowest
    // unfinished task is always a running one (a reserved task's workgroup
    // is busy with a lower one), so every wait still ends.
    uint32_t next = 0;
    if (threadIdx.x == 0) next = __hip_atomic_fetch_add(head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint2 tk = g.inl ? g.inl_tasks[ti] : g.tasks[ti];
    const uint32_t p = tk.x;
    const uint32_t kind = tk.y >> 28;
    const uint32_t idx = tk.y & 0x0FFFFFFFu;
    const ProdDev pd = g.inl ? g.inl_prods[p] : g.prods[p];
    const PrimeDev& pr = g.primes[pd.prime_id];
    const uint32_t N = 1u << pd.n;
    uint32_t* scr = g.scr + pd.scr_off;
    if (threadIdx.x == 0) {
      bool go = true;
      if (kind == T_ROW) go = wait_count(cnt_col + p, 2 * pd.ntiles, status, g.spin_limit);
      else if (kind == T_COLI) go = wait_count(cnt_row + p, pd.nblocks, status, g.spin_limit);
      s_go = go ? 1u : 0u;
    }
    __syncthreads();
    if (s_go) {
      switch (kind) {
        case T_SMALL:
          exec_small_poly<NT, RM>(pr, pd.n, g.in + pd.a_off, pd.da, g.in + pd.b_off, pd.db,
                                  (pd.to_scr ? g.scr : g.out) + pd.c_off, pd.nout, X);
          break;
        case T_COLF_A: exec_col_dif<NT, RM, true>(pr, pd.n, pd.lc, idx, g.in + pd.a_off, pd.da, 0u, scr, X, pd.tft); break;
        case T_COLF_B:
          exec_col_dif<NT, RM, true>(pr, pd.n, pd.lc, idx, g.in + pd.b_off, pd.db, pr.s2[pd.n], scr + N, X, pd.tft);
          break;
        case T_ROW: exec_row<NT, RM, true>(pr, kRowLog, ROW_POLY, scr + idx * S, scr + N + idx * S, 0u, X); break;
        default:
          exec_col_dit<NT, RM>(pr, pd.n, pd.lc, idx, scr, (pd.to_scr ? g.scr : g.out) + pd.c_off, pd.nout, X);
          break;
      }
      if (kind != T_SMALL && kind != T_COLI) {
        // Publish: every wave waits until its coherent stores have completed,
        // the workgroup meets, and one lane bumps the product's counter.
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        __syncthreads();
        if (threadIdx.x == 0) {
          uint32_t* ctr = kind == T_ROW ? cnt_row + p : cnt_col + p;
          __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) s_task = next;
  }
}

// Fix-ups of split products, after the persistent launch, in chunks of
// kFixChunk coefficients so that a long product's fix-up is spread over the
// device (a workgroup takes chunks; the fix-up of a chunk is found by binary
// search on the chunks' first indices).  The cyclic part left c[k] = c_k +
// c_(h+k); the top product t gives c_(h+k) = t[m-1+k].
// owner, when given, holds the record of every chunk, so a chunk's loads
// wait on two dependent reads instead of the search's dozen.  A plan made
// once on the host passes its own table; a batch planned on the device
// passes dyn (its scratch header, which holds the chunk count and where the
// planner put the table; its records of unsplit products have m = 0 and own
// no chunk).
__global__ __launch_bounds__(256) void k_split_fix(const PrimeDev* primes, const FixDev* fx, uint32_t nfix,
                                                   uint32_t nchunks, uint32_t* out, const uint32_t* scr,
                                                   const uint32_t* dyn, const uint32_t* owner) {
  if (dyn) {
    nchunks = dyn[kHdrNchunks];
    owner = dyn + ((uint64_t)dyn[kHdrOwner] | ((uint64_t)dyn[kHdrOwner + 1] << 32));
  }
  for (uint32_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    uint32_t lo = 0, hi = nfix;                  // fx[lo].chunk0 <= c < fx[hi].chunk0
    if (owner) {
      lo = owner[c];
    } else {
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (fx[mid].chunk0 <= c) lo = mid;
        else hi = mid;
      }
    }
    const FixDev d = fx[lo];
    uint32_t* cc = out + d.c_off;
    const uint32_t k0 = (c - d.chunk0) * kFixChunk;
    const uint32_t k1 = min(d.m, k0 + kFixChunk);
    if (d.kind == FIX_TFT) {
      // Block output t (m words) and cyclic part r = cc[0 .. h).  Indices k
      // < m <= s are rewritten; the fold reads r at k + i s >= s only.
      const PrimeDev& pr = primes[d.prime_id];
      const Mod md{pr.P, pr.Pp};
      const uint32_t sl = d.s_log, nf = d.h >> sl;           // 2 or 4 terms fold r modulo x^s - w^s
      const uint32_t* t = scr + d.t_off;
      uint32_t z[3];
#pragma unroll
      for (int i = 1; i < 4; i++) z[i - 1] = (uint32_t)i < nf ? ldg(pr.twf, d.h + ((uint32_t)i << sl)) : 0u;
      const uint32_t half = (pr.R1 & 1u ? pr.R1 + pr.P : pr.R1) >> 1;    // R / 2 mod P: REDC(x half) = x / 2
      // Each lane takes four coefficients of the chunk and issues all their
      // loads before any arithmetic, so the loads' latencies overlap.
      constexpr int kPer = kFixChunk / 256;
      uint32_t tv[kPer], wv[kPer], rv[kPer][4];
#pragma unroll
      for (int j = 0; j < kPer; j++) {
        const uint32_t k = k0 + threadIdx.x + 256u * j;
        const bool in = k < k1;
        tv[j] = in ? t[k] : 0u;
        wv[j] = in ? ldg(pr.twi, d.h + k) : 0u;
#pragma unroll
        for (uint32_t i = 0; i < 4; i++) rv[j][i] = in && i < nf ? cc[k + (i << sl)] : 0u;
      }
#pragma unroll
      for (int j = 0; j < kPer; j++) {
        const uint32_t k = k0 + threadIdx.x + 256u * j;
        if (k >= k1) continue;
        const uint32_t u = mmul(tv[j], wv[j], md);                     // t_k w^-k
        uint32_t f = rv[j][0];
#pragma unroll
        for (uint32_t i = 1; i < 4; i++)
          if (i < nf) f = madd(f, mmul(rv[j][i], z[i - 1], md), md.P);
        const uint32_t q = mmul(msub(f, u, md.P), half, md);
        cc[k] = msub(rv[j][0], q, md.P);
        cc[d.h + k] = q;
      }
    } else {
      const uint32_t* t = scr + d.t_off + (d.m - 1);
      for (uint32_t k = k0 + threadIdx.x; k < k1; k += 256) {
        const uint32_t hv = t[k];
        cc[k] = msub(cc[k], hv, d.P);
        cc[d.h + k] = hv;
      }
    }
  }
}

// Zero the scratch header and counters (a kernel, not a memset, so that the
// sequence can be captured in a graph).
__global__ void k_fill_zero(uint32_t* p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// Batch planning on the device (ntt_polymul_batch).  The descriptors are in
// device memory; one workgroup turns them into the same records the host
// planner makes (products, fix-ups, phase-ordered tasks) inside the caller's
// scratch, so one call needs no host round trip and no upload, and a
// captured graph replays with whatever descriptors the buffer then holds.
//
// Scratch layout (words): header | 2 counters x 2 count slots | ProdDev x 2
// count | FixDev x count | tasks | data (64-word aligned) | chunk table,
// where data holds, slot by slot, the two length-N transforms of each
// multi-pass slot and the output of each top part, and the chunk table the
// record of each fix-up chunk.  The task list is in phase order: forward column
// tiles, the first half of the single-task slots, row blocks, the other
// half, inverse column tiles, each phase longest transform first and the
// slots of one length prime by prime (the host planner's phase order; within
// one prime and length, slots take their ranks in the order their lanes reach
// a shared counter).
// ---------------------------------------------------------------------------

constexpr int kPlanThreads = 512;
constexpr int kPlanWaves = kPlanThreads / 64;
constexpr int kPlanBuckets = kMaxLog + 1;

struct BatchLayout {
  uint64_t cnt, prods, fixes, tasks;   // word offsets
};

__host__ __device__ inline BatchLayout batch_layout(uint32_t count) {
  BatchLayout l;
  l.cnt = kHdrWords;
  l.prods = (l.cnt + 4ull * count + 63) & ~63ull;
  l.fixes = l.prods + (sizeof(ProdDev) / 4) * 2ull * count;
  l.tasks = l.fixes + (sizeof(FixDev) / 4) * (uint64_t)count;
  return l;
}

__host__ __device__ inline uint64_t batch_data_offset(const BatchLayout& l, uint64_t ntasks) {
  return (l.tasks + 2 * ntasks + 63) & ~63ull;
}

// Exclusive prefix sum over the workgroup (every thread calls it); *total
// receives the sum.  Waves scan with lane shuffles, then add the totals of
// the waves before them.
__device__ __forceinline__ uint64_t plan_scan(uint64_t v, uint64_t* s_wsum, uint64_t* total) {
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
  uint64_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x += y;
  }
  if (lane == 63) s_wsum[wave] = x;
  __syncthreads();
  uint64_t before = 0, all = 0;
  for (int w = 0; w < kPlanWaves; w++) {
    if (w < (int)wave) before += s_wsum[w];
    all += s_wsum[w];
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

__global__ __launch_bounds__(kPlanThreads) void k_batch_plan(const PrimeDev* primes, uint32_t nprimes,
                                                              const polymul_desc* descs, uint32_t count,
                                                              uint32_t* scr, uint64_t scr_words) {
  __shared__ uint32_t s_logmax[64];
  __shared__ uint32_t s_cnt[kPlanBuckets];          // slots per transform length
  __shared__ unsigned long long s_words, s_chunks;
  __shared__ int s_err;
  __shared__ uint32_t s_base[kPlanBuckets];         // first task of the length's slots in their phase
  __shared__ uint32_t s_rowb[kPlanBuckets], s_colib[kPlanBuckets];   // same, row blocks and inverse tiles
  // per (length, prime): slots, then the first rank of the group within
  // its length (primes in order), and the ranks handed out so far
  __shared__ uint32_t s_bp[kPlanBuckets * 64], s_bpr[kPlanBuckets * 64];
  // the multi-pass slots of the current chunk of slots: slot, first forward
  // tile, first inverse tile and first row block task, tiles, blocks (their
  // tasks are written by the whole workgroup)
  __shared__ uint32_t s_eslot[kPlanThreads], s_ef0[kPlanThreads], s_ei0[kPlanThreads], s_er0[kPlanThreads];
  __shared__ uint32_t s_ent[kPlanThreads], s_enb[kPlanThreads];
  // the split products of the current chunk of slots: first fix-up chunk,
  // chunks, record (their entries of the chunk table)
  __shared__ uint32_t s_fc0[kPlanThreads], s_fcn[kPlanThreads], s_fid[kPlanThreads];
  __shared__ uint64_t s_wsum[kPlanWaves];
  __shared__ uint32_t s_C, s_R, s_half;
  __shared__ uint64_t s_data, s_chk, s_own;
  const uint32_t tid = threadIdx.x;
  const uint32_t lane = tid & 63u, wave = tid >> 6;
  const uint32_t nslots = 2 * count;
  for (uint32_t i = tid; i < 64; i += kPlanThreads) s_logmax[i] = i < nprimes ? primes[i].logmax : 0u;
  for (uint32_t i = tid; i < (uint32_t)kPlanBuckets * 64; i += kPlanThreads) {
    s_bp[i] = 0;
    s_bpr[i] = 0;
  }
  if (tid == 0) {
    s_words = 0;
    s_chunks = 0;
    s_err = 0;
  }
  __syncthreads();
  // Pass 1: validate, count slots per length, sum data words and chunks.
  // Each wave sums its lanes first and makes one shared atomic per total
  // (every lane adding to one shared word serialized thousands of atomics).
  for (uint32_t base = 0; base < nslots; base += kPlanThreads) {
    const uint32_t slot = base + tid;
    unsigned long long words = 0, chunks = 0;
    if (slot < nslots) {
      const int part = (int)(slot & 1u);
      const polymul_desc d = descs[slot >> 1];
      const SlotShape sh = slot_shape(d, part, nprimes, s_logmax);
      if (sh.err) atomicCAS(&s_err, 0, sh.err);
      else if (sh.used) {
        atomicAdd(&s_bp[sh.n * 64 + d.prime_id], 1u);
        words = slot_words(sh, part);
        chunks = slot_chunks(sh, part);
      }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      words += __shfl_xor(words, d, 64);
      chunks += __shfl_xor(chunks, d, 64);
    }
    if (lane == 0) {
      atomicAdd(&s_words, words);
      atomicAdd(&s_chunks, chunks);
    }
  }
  __syncthreads();
  // Slots per length, and each (length, prime) group's first rank: within
  // a length the slots go prime by prime, so that tasks that run together
  // read one prime's twiddle tables.
  if (tid < (uint32_t)kPlanBuckets) {
    uint32_t acc = 0;
    for (uint32_t p = 0; p < 64; p++) {
      const uint32_t c = s_bp[tid * 64 + p];
      s_bp[tid * 64 + p] = acc;
      acc += c;
    }
    s_cnt[tid] = acc;
  }
  __syncthreads();
  const BatchLayout lay = batch_layout(count);
  if (tid == 0) {
    // task bases per length, longest first within each phase
    uint32_t C = 0, S = 0, R = 0, I = 0;
    for (int n = kMaxLog; n >= 0; n--) {
      if (n > kRowLog) {
        const uint32_t nt = 1u << (kRowLog - col_lc(n)), nb = 1u << (n - kRowLog);
        s_base[n] = C;
        s_rowb[n] = R;
        s_colib[n] = I;
        C += s_cnt[n] * 2 * nt;
        R += s_cnt[n] * nb;
        I += s_cnt[n] * nt;
      } else {
        s_base[n] = S;
        S += s_cnt[n];
      }
    }
    const uint32_t half = S / 2;
    for (int n = kRowLog + 1; n <= kMaxLog; n++) {
      // forward tiles, then (after half the single tasks) the rows, then
      // (after the rest) the inverse tiles
      s_rowb[n] += C + half;
      s_colib[n] += C + S + R;
    }
    s_C = C;
    s_R = R;
    s_half = half;
    const uint64_t ntasks = (uint64_t)C + S + R + I;
    // the chunk table follows the data
    const uint64_t own = batch_data_offset(lay, ntasks) + s_words;
    const uint64_t need = own + s_chunks;
    int err = s_err;
    if (!err && need > scr_words) err = MONT_ENOMEM;
    if (!err && ntasks > 0xFFFFFFFFull) err = MONT_ERANGE;
    s_err = err;
    scr[0] = 0;
    scr[1] = err ? kStatusPlanError : 0u;
    scr[kHdrNtasks] = err ? 0u : (uint32_t)ntasks;
    scr[kHdrNchunks] = err ? 0u : (uint32_t)s_chunks;
    scr[kHdrError] = (uint32_t)err;
    scr[kHdrWordsNeeded] = (uint32_t)need;
    scr[kHdrWordsNeeded + 1] = (uint32_t)(need >> 32);
    scr[kHdrOwner] = (uint32_t)own;
    scr[kHdrOwner + 1] = (uint32_t)(own >> 32);
    s_data = batch_data_offset(lay, ntasks);
    s_chk = 0;
    s_own = own;
  }
  __syncthreads();
  if (s_err) return;                                 // uniform: every thread leaves
  for (uint64_t i = tid; i < 4ull * count; i += kPlanThreads) scr[lay.cnt + i] = 0u;
  ProdDev* prods = reinterpret_cast<ProdDev*>(scr + lay.prods);
  FixDev* fixes = reinterpret_cast<FixDev*>(scr + lay.fixes);
  uint2* tasks = reinterpret_cast<uint2*>(scr + lay.tasks);
  uint32_t* owner = scr + s_own;
  const uint32_t C = s_C, R = s_R, half = s_half;
  // Pass 2: ranks within each length (by prime), data offsets and fix-up
  // chunks by prefix sums, then the records and the tasks.
  for (uint32_t base = 0; base < nslots; base += kPlanThreads) {
    const uint32_t slot = base + tid;
    const int part = (int)(slot & 1u);
    SlotShape sh = {};
    const polymul_desc d = slot < nslots ? descs[slot >> 1] : polymul_desc{};
    if (slot < nslots) sh = slot_shape(d, part, nprimes, s_logmax);
    const uint32_t b = sh.used ? (uint32_t)sh.n : 0xFFu;
    uint64_t wtot = 0, ctot = 0, etot = 0, ftot = 0;
    const uint64_t woff = plan_scan(slot_words(sh, part), s_wsum, &wtot);
    const uint64_t coff = plan_scan(slot < nslots && part == 1 ? slot_chunks(sh, part) : 0u, s_wsum, &ctot);
    const uint32_t ei = (uint32_t)plan_scan(sh.used && sh.n > kRowLog ? 1u : 0u, s_wsum, &etot);
    const uint32_t fi = (uint32_t)plan_scan(sh.split && part == 1 ? 1u : 0u, s_wsum, &ftot);
    if (slot < nslots) {
      // rank within the length: the (length, prime) group's first rank plus
      // the order of arrival within the group (any order of the slots of one
      // phase keeps every prerequisite ahead of its dependants, and the
      // results do not depend on it)
      const uint32_t rank = sh.used ? s_bp[b * 64 + d.prime_id] + atomicAdd(&s_bpr[b * 64 + d.prime_id], 1u) : 0u;
      const uint64_t dat = s_data + woff;
      const uint32_t chunk0 = (uint32_t)(s_chk + coff);
      if (sh.used) {
        ProdDev pd = {};
        pd.prime_id = d.prime_id;
        pd.n = (uint32_t)sh.n;
        pd.da = sh.da;
        pd.db = sh.db;
        pd.a_off = sh.a_off;
        pd.b_off = sh.b_off;
        pd.nout = sh.nout;
        pd.to_scr = sh.split && part == 1 ? 1u : 0u;
        pd.tft = sh.block ? (uint32_t)sh.nfull : 0u;
        pd.c_off = pd.to_scr ? dat + (sh.n > kRowLog ? (2ull << sh.n) : 0ull) : d.c_off;
        uint32_t nt = 0, nb = 0;
        if (sh.n > kRowLog) {
          pd.lc = (uint32_t)col_lc(sh.n);
          nt = pd.ntiles = 1u << (kRowLog - pd.lc);
          nb = pd.nblocks = 1u << (sh.n - kRowLog);
          pd.scr_off = dat;
        }
        prods[slot] = pd;
        if (sh.n <= kRowLog) {
          const uint32_t q = s_base[b] + rank;
          const uint32_t at = q < half ? C + q : C + R + q;
          tasks[at] = make_uint2(slot, (uint32_t)T_SMALL << 28);
        } else {
          // its tasks are written below, by the whole workgroup
          s_eslot[ei] = slot;
          s_ef0[ei] = s_base[b] + rank * 2 * nt;
          s_ei0[ei] = s_colib[b] + rank * nt;
          s_er0[ei] = s_rowb[b] + rank * nb;
          s_ent[ei] = nt;
          s_enb[ei] = nb;
        }
      }
      // one fix-up record per product: the top slot writes a split product's,
      // slot 2i an unsplit one's (m = 0, never selected)
      if (sh.split && part == 1) {
        FixDev f = {};
        f.c_off = d.c_off;
        f.t_off = dat + (sh.n > kRowLog ? (2ull << sh.n) : 0ull);
        f.m = sh.m;
        f.h = sh.h;
        f.P = primes[d.prime_id].P;
        f.chunk0 = chunk0;
        f.kind = sh.block ? FIX_TFT : FIX_SPLIT;
        f.prime_id = d.prime_id;
        f.s_log = (uint32_t)sh.n;
        fixes[slot >> 1] = f;
        s_fc0[fi] = chunk0;
        s_fcn[fi] = slot_chunks(sh, part);
        s_fid[fi] = slot >> 1;
      } else if (!sh.split && part == 0) {
        FixDev f = {};
        f.chunk0 = chunk0;
        fixes[slot >> 1] = f;
      }
    }
    __syncthreads();
    // The chunk's multi-pass tasks (3 ntiles + nblocks per slot): a wave
    // per slot, its lanes on consecutive tasks, so every store of a wave
    // covers 64 adjacent records.  (One lane per slot writing a 2^21
    // product's 640 tasks took most of the planning time.)
    for (uint32_t e = wave; e < (uint32_t)etot; e += kPlanWaves) {
      const uint32_t sl = s_eslot[e], nt = s_ent[e], nb = s_enb[e];
      const uint32_t f0 = s_ef0[e], i0 = s_ei0[e], r0 = s_er0[e];
      for (uint32_t q = lane; q < 2 * nt; q += 64)
        tasks[f0 + q] = make_uint2(sl, ((q < nt ? (uint32_t)T_COLF_A : (uint32_t)T_COLF_B) << 28) |
                                           (q < nt ? q : q - nt));
      for (uint32_t q = lane; q < nt; q += 64) tasks[i0 + q] = make_uint2(sl, ((uint32_t)T_COLI << 28) | q);
      for (uint32_t q = lane; q < nb; q += 64) tasks[r0 + q] = make_uint2(sl, ((uint32_t)T_ROW << 28) | q);
    }
    for (uint32_t e = wave; e < (uint32_t)ftot; e += kPlanWaves) {
      const uint32_t c0 = s_fc0[e], nc = s_fcn[e], id = s_fid[e];
      for (uint32_t q = lane; q < nc; q += 64) owner[c0 + q] = id;
    }
    if (tid == 0) {
      s_data += wtot;
      s_chk += ctot;
    }
    __syncthreads();
  }
}

// Twiddle generation.  pw[b] = residue of w^(2^b) by repeated squaring of
// the residue of w (one lane), then every table entry is a product of those.
__global__ void k_tw_pows(uint32_t P, uint32_t Pp, uint32_t R2, uint32_t w, uint32_t L, uint32_t* pw) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const Mod md{P, Pp};
    uint32_t x = mmul(w, R2, md);
    for (uint32_t b = 0; b < L; b++) {
      pw[b] = x;
      x = mmul(x, x, md);
    }
  }
}

__global__ void k_tw_fill(uint32_t P, uint32_t Pp, uint32_t R1, uint32_t L, const uint32_t* pw, uint32_t* twf,
                          uint32_t* twi) {
  const Mod md{P, Pp};
  const uint32_t Nmax = 1u << L;
  for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < Nmax; x += gridDim.x * blockDim.x) {
    if (x == 0) {
      twf[0] = 0u;
      twi[0] = 0u;
      continue;
    }
    const uint32_t s = 31u - __builtin_clz(x);          // h = 2^s
    const uint32_t i = x - (1u << s);
    const uint32_t ef = i << (L - 1 - s);               // w_{2h}^i = w^(i Nmax / 2h)
    const uint32_t ei = (Nmax - ef) & (Nmax - 1);       // w^-e = w^(Nmax - e)
    uint32_t f = R1, v = R1;
    for (uint32_t b = 0; b < L; b++) {
      if ((ef >> b) & 1u) f = mmul(f, pw[b], md);
      if ((ei >> b) & 1u) v = mmul(v, pw[b], md);
    }
    twf[x] = f;
    twi[x] = v;
  }
}

// ---------------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------------

uint32_t powmod_host(uint64_t x, uint64_t e, uint32_t P) {
  uint64_t r = 1 % P;
  x %= P;
  while (e) {
    if (e & 1) r = r * x % P;
    x = x * x % P;
    e >>= 1;
  }
  return (uint32_t)r;
}

// Smallest primitive root of prime P (0 if P is not prime).
uint32_t primitive_root_host(uint32_t P) {
  std::vector<uint32_t> qs;
  uint32_t m = P - 1;
  for (uint32_t f = 2; (uint64_t)f * f <= m; f++)
    if (m % f == 0) {
      qs.push_back(f);
      while (m % f == 0) m /= f;
    }
  if (m > 1) qs.push_back(m);
  for (uint32_t g = 2; g < P; g++) {
    bool ok = true;
    for (uint32_t q : qs)
      if (powmod_host(g, (P - 1) / q, P) == 1) {
        ok = false;
        break;
      }
    if (ok) return g;
  }
  return 0;
}

bool is_prime_host(uint32_t P) {
  if (P < 2) return false;
  for (uint32_t f = 2; (uint64_t)f * f <= P; f++)
    if (P % f == 0) return false;
  return true;
}


}  // namespace

}  // namespace mont

using namespace mont;

// Scratch of the allocation-free product (ntt_polymul_noalloc): the two
// length-N transforms of one product of N <= 2^21, 16 MiB, one copy on every
// device the library runs on, held until the process ends.  In host code the
// array's name is only a host-side stand-in; its device address is looked
// up once per device with hipGetSymbolAddress (noalloc_scratch_on) and only
// that address is used.
constexpr int kNoAllocLog = 21;
static __device__ __align__(256) uint32_t noalloc_scratch[(size_t)2 << kNoAllocLog];

namespace {

constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
uint32_t* g_noalloc_ptr[kNoAllocDevices] = {};

// Device address of noalloc_scratch on `device`, which must be current.
mont_status noalloc_scratch_on(int device, uint32_t** out) {
  *out = nullptr;
  if (device < 0 || device >= kNoAllocDevices) return MONT_EHIP;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)) != hipSuccess || !p) return MONT_EHIP;
    g_noalloc_ptr[device] = static_cast<uint32_t*>(p);
  }
  *out = g_noalloc_ptr[device];
  return MONT_OK;
}

}  // namespace

namespace mont {
// Launch shape of the transform kernels: threads per workgroup, the largest
// radix-2^R round, and the persistent grid as a multiple of the resident
// workgroups.
struct NttTune {
  int threads;
  int radix_log;
  int grid_mult;
};
}  // namespace mont

struct ntt_ctx {
  int device = 0;
  int log2_nmax = 0;
  std::vector<mont_params> params;
  std::vector<uint32_t> roots;      // w of order 2^logmax_p (ordinary residue)
  std::vector<uint32_t> logmax;
  std::vector<uint32_t*> twf, twi;  // device pointers into tw_mem
  PrimeDev* d_primes = nullptr;
  uint32_t* tw_mem = nullptr;
  uint32_t* noalloc_scr = nullptr;  // this device's noalloc_scratch (nullptr if the lookup failed)
};

struct ntt_plan {
  const ntt_ctx* ctx = nullptr;
  int count = 0;
  uint32_t ntasks = 0;
  uint64_t scratch_words = 0;
  uint64_t in_words = 0, out_words = 0;
  ProdDev* d_prods = nullptr;
  uint2* d_tasks = nullptr;
  uint32_t nfix = 0;        // split products (count above counts their two parts)
  uint32_t nchunks = 0;     // fix-up chunks
  uint64_t redc = 0;        // REDC one execution performs
  FixDev* d_fix = nullptr;
  uint32_t* d_owner = nullptr;  // plans made once: the fix-up record of each chunk
  int default_grid = 0;
  // Reusable plans (ntt_plan_reserve): one device block and one pinned
  // staging block of the same capacity.  An update packs its products, fix-ups
  // and tasks back to back into staging and uploads them with one copy;
  // d_prods, d_fix and d_tasks then point into the device block.  `staged`
  // marks the last upload from staging.
  bool reusable = false;
  int cap_prods = 0;        // caller's products; internal capacity is twice that
  uint32_t cap_tasks = 0;
  void* d_block = nullptr;
  void* h_block = nullptr;
  hipEvent_t staged = nullptr;
  bool staged_pending = false;
  // A reusable plan of at most kInlineProds internal products, kInlineTasks
  // tasks and no fix-ups keeps them here and passes them in the launch.
  bool inl = false;
  ProdDev inl_prods[kInlineProds];
  uint2 inl_tasks[kInlineTasks];
  NttTune shape = {512, 4, 1};  // launch shape, chosen when the plan is (re)planned
  // host time of the last ntt_plan_update, microseconds: planning, waiting
  // for the previous upload to leave staging, the upload call, in all
  uint32_t upd_us[4] = {0, 0, 0, 0};
};

namespace {

mont_status hip_ok(hipError_t e) { return e == hipSuccess ? MONT_OK : MONT_EHIP; }

// Launch shapes: the process-wide default, and per transform length
// (threads == 0: no entry, the default applies).  Read when a launch is
// enqueued, and for a plan when it is (re)planned.
NttTune g_ntt_tune = {512, 4, 1};
NttTune g_ntt_len[kMaxLog + 1] = {};

NttTune shape_for(int n) {
  const NttTune& e = g_ntt_len[n < 0 ? 0 : (n > kMaxLog ? kMaxLog : n)];
  return e.threads ? e : g_ntt_tune;
}

bool shape_ok(int threads, int radix_log, int grid_mult) {
  return (threads == 256 || threads == 512 || threads == 1024) && (radix_log == 3 || radix_log == 4) &&
         (grid_mult == 1 || grid_mult == 2 || grid_mult == 4);
}

// A plan's launch shape.  A plan with at least 90 % of its butterflies
// (2^n n per product of length 2^n) at one transform length takes that
// length's shape (a batch of one length, like most of a serving loop's);
// any other takes the default, which the tuner picks on a batch of uneven
// lengths (on MI355X the two differ: 1024-thread workgroups win on batches
// of one length, 512-thread ones on the uneven 2048-product batch).
NttTune plan_shape(const std::vector<ProdDev>& prods) {
  double work[kMaxLog + 1] = {}, total = 0;
  for (const ProdDev& pd : prods) {
    const double w = std::ldexp((double)pd.n + 1, (int)pd.n);
    work[pd.n] += w;
    total += w;
  }
  int best = 0;
  for (int n = 1; n <= kMaxLog; n++)
    if (work[n] > work[best]) best = n;
  return total > 0 && work[best] >= 0.9 * total ? shape_for(best) : g_ntt_tune;
}

// Butterflies with a unit twiddle that a plan's products skip at radix 2^rm.
uint64_t plan_unit_bfly(const std::vector<ProdDev>& prods, int rm) {
  uint64_t u = 0;
  for (const ProdDev& pd : prods) u += unit_bfly((int)pd.n, rm);
  return u;
}

template <int NT, int RM>
void launch_direct_v(const DirectArgs& g, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL((k_ntt_direct<NT, RM>), dim3(grid), dim3(NT), 0, s, g);
}

template <int NT, int RM>
void launch_persistent_v(const PlanArgs& g, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL((k_ntt_persistent<NT, RM>), dim3(grid), dim3(NT), 0, s, g);
}

template <int NT, int RM>
int occupancy_v() {
  int per_cu = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_ntt_persistent<NT, RM>, NT, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return per_cu;
}

#define MONT_NTT_VARIANTS(X) X(256, 3) X(256, 4) X(512, 3) X(512, 4) X(1024, 3) X(1024, 4)

// Plain launches take the shape of their transform length.
void launch_direct(const DirectArgs& g, uint32_t grid, hipStream_t s) {
  const NttTune sh = shape_for((int)g.n);
#define MONT_V(T, R)                                                      \
  if (sh.threads == T && sh.radix_log == R) {                             \
    launch_direct_v<T, R>(g, grid, s);                                    \
    return;                                                               \
  }
  MONT_NTT_VARIANTS(MONT_V)
#undef MONT_V
  launch_direct_v<512, 4>(g, grid, s);
}

void launch_persistent(const PlanArgs& g, uint32_t grid, hipStream_t s, const NttTune& sh) {
#define MONT_V(T, R)                                                      \
  if (sh.threads == T && sh.radix_log == R) {                             \
    launch_persistent_v<T, R>(g, grid, s);                                \
    return;                                                               \
  }
  MONT_NTT_VARIANTS(MONT_V)
#undef MONT_V
  launch_persistent_v<512, 4>(g, grid, s);
}

// Resident persistent workgroups for the current launch shape.
// Resident workgroups of each launch shape on each device, computed once:
// the occupancy query costs more host time than a launch, and a serving loop
// asks for the grid on every update and execution.
constexpr int kGridDevices = 64;
std::atomic<int> g_grid_cache[kGridDevices][6];

int persistent_grid(const NttTune& sh) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  int v = 0, per_cu = 1;
#define MONT_V(T, R)                                                    \
  if (sh.threads == T && sh.radix_log == R) break;                     \
  v++;
  do {
    MONT_NTT_VARIANTS(MONT_V)
  } while (0);
#undef MONT_V
  if (v > 5) v = 3;                                   // unknown shape: the 512 x 4 default
  std::atomic<int>* slot = dev >= 0 && dev < kGridDevices ? &g_grid_cache[dev][v] : nullptr;
  int resident = slot ? slot->load(std::memory_order_relaxed) : 0;
  if (resident <= 0) {
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
#define MONT_V(T, R) \
  if (sh.threads == T && sh.radix_log == R) per_cu = occupancy_v<T, R>();
    MONT_NTT_VARIANTS(MONT_V)
#undef MONT_V
    resident = cus * per_cu;
    if (slot) slot->store(resident, std::memory_order_relaxed);
  }
  return resident * sh.grid_mult;
}

bool prime_ok(const ntt_ctx* ctx, int prime_id) {
  return ctx && prime_id >= 0 && prime_id < (int)ctx->params.size();
}

DirectArgs direct_base(const ntt_ctx* ctx, int prime_id, int n) {
  DirectArgs g;
  std::memset(&g, 0, sizeof(g));
  g.primes = ctx->d_primes;
  g.prime_id = (uint32_t)prime_id;
  g.n = (uint32_t)n;
  if (n > kRowLog) {
    g.lc = (uint32_t)col_lc(n);
    g.ntiles = 1u << (kRowLog - g.lc);
  }
  return g;
}

}  // namespace

extern "C" mont_status ntt_tune_set(int threads, int radix_log, int grid_mult) {
  if (!shape_ok(threads, radix_log, grid_mult)) return MONT_EINVAL;
  g_ntt_tune = NttTune{threads, radix_log, grid_mult};
  return MONT_OK;
}

extern "C" mont_status ntt_tune_set_length(int log2n, int threads, int radix_log, int grid_mult) {
  if (log2n < 0 || log2n > kMaxLog) return MONT_EINVAL;
  if (threads == 0) {
    g_ntt_len[log2n] = NttTune{0, 0, 0};
    return MONT_OK;
  }
  if (!shape_ok(threads, radix_log, grid_mult)) return MONT_EINVAL;
  g_ntt_len[log2n] = NttTune{threads, radix_log, grid_mult};
  return MONT_OK;
}

extern "C" mont_status ntt_tune_get_length(int log2n, int* threads, int* radix_log, int* grid_mult) {
  if (log2n < 0 || log2n > kMaxLog || !threads || !radix_log || !grid_mult) return MONT_EINVAL;
  const NttTune sh = shape_for(log2n);
  *threads = sh.threads;
  *radix_log = sh.radix_log;
  *grid_mult = sh.grid_mult;
  return MONT_OK;
}

extern "C" mont_status ntt_tune_get(int* threads, int* radix_log, int* grid_mult) {
  if (!threads || !radix_log || !grid_mult) return MONT_EINVAL;
  *threads = g_ntt_tune.threads;
  *radix_log = g_ntt_tune.radix_log;
  *grid_mult = g_ntt_tune.grid_mult;
  return MONT_OK;
}

extern "C" mont_status ntt_ctx_create(const uint32_t* primes, int nprimes, int log2_nmax, ntt_ctx** out) {
  if (!out || !primes || nprimes <= 0 || nprimes > 64 || log2_nmax < 1 || log2_nmax > kMaxLog) return MONT_EINVAL;
  *out = nullptr;
  ntt_ctx* ctx = new (std::nothrow) ntt_ctx;
  if (!ctx) return MONT_ENOMEM;
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    return MONT_EHIP;
  }
  ctx->log2_nmax = log2_nmax;
  uint64_t total = 0;
  for (int i = 0; i < nprimes; i++) {
    mont_params prm;
    if (mont_setup(primes[i], &prm) != MONT_OK || !is_prime_host(primes[i])) {
      delete ctx;
      return MONT_EINVAL;
    }
    uint32_t L = std::min<uint32_t>((uint32_t)log2_nmax, prm.k);
    ctx->params.push_back(prm);
    ctx->logmax.push_back(L);
    uint32_t g = primitive_root_host(prm.P);
    ctx->roots.push_back(powmod_host(g, (prm.P - 1) >> L, prm.P));
    total += 2ull << L;
  }
  total += 32ull * nprimes;  // per-prime power tables
  if (hipMalloc(&ctx->tw_mem, total * 4) != hipSuccess) {
    delete ctx;
    return MONT_ENOMEM;
  }
  if (hipMalloc(&ctx->d_primes, sizeof(PrimeDev) * nprimes) != hipSuccess) {
    (void)hipFree(ctx->tw_mem);
    delete ctx;
    return MONT_ENOMEM;
  }
  std::vector<PrimeDev> hp(nprimes);
  uint32_t* cur = ctx->tw_mem;
  uint32_t* pw = ctx->tw_mem + (total - 32ull * nprimes);
  mont_status st = MONT_OK;
  for (int i = 0; i < nprimes && st == MONT_OK; i++) {
    const mont_params& prm = ctx->params[i];
    uint32_t L = ctx->logmax[i];
    PrimeDev& d = hp[i];
    std::memset(&d, 0, sizeof(d));
    d.P = prm.P;
    d.Pp = prm.Pprime;
    d.R1 = prm.R1;
    d.R2 = prm.R2;
    d.logmax = L;
    uint32_t* f = cur;
    uint32_t* v = cur + (1u << L);
    cur += 2ull << L;
    d.twf = f;
    d.twi = v;
    ctx->twf.push_back(f);
    ctx->twi.push_back(v);
    for (uint32_t n = 0; n <= L; n++) {
      // N^-1 = P - (P-1)/N because N (P-1)/N = P - 1 = -1 (mod P)
      uint64_t ninv = prm.P - ((prm.P - 1) >> n);
      d.s1[n] = (uint32_t)((uint64_t)prm.R1 * ninv % prm.P);
      d.s2[n] = (uint32_t)((uint64_t)prm.R2 * ninv % prm.P);
    }
    hipLaunchKernelGGL(k_tw_pows, dim3(1), dim3(64), 0, 0, prm.P, prm.Pprime, prm.R2, ctx->roots[i], L, pw + 32 * i);
    uint32_t blocks = std::max(1u, std::min(4096u, (1u << L) / 256));
    hipLaunchKernelGGL(k_tw_fill, dim3(blocks), dim3(256), 0, 0, prm.P, prm.Pprime, prm.R1, L, pw + 32 * i, f, v);
    st = last_launch_status();
  }
  if (st == MONT_OK) st = hip_ok(hipMemcpy(ctx->d_primes, hp.data(), sizeof(PrimeDev) * nprimes,
                                           hipMemcpyHostToDevice));
  if (st == MONT_OK) st = hip_ok(hipDeviceSynchronize());
  if (st != MONT_OK) {
    (void)hipFree(ctx->tw_mem);
    (void)hipFree(ctx->d_primes);
    delete ctx;
    return st;
  }
  // the allocation-free product's scratch on this device; a failed lookup
  // only disables that entry point (it then returns MONT_EHIP)
  if (noalloc_scratch_on(ctx->device, &ctx->noalloc_scr) != MONT_OK) ctx->noalloc_scr = nullptr;
  *out = ctx;
  return MONT_OK;
}

extern "C" mont_status ntt_ctx_destroy(ntt_ctx* ctx) {
  if (!ctx) return MONT_EINVAL;
  (void)hipDeviceSynchronize();
  (void)hipFree(ctx->tw_mem);
  (void)hipFree(ctx->d_primes);
  delete ctx;
  return MONT_OK;
}

extern "C" mont_status ntt_ctx_prime(const ntt_ctx* ctx, int prime_id, mont_params* prm, uint32_t* root,
                                     uint32_t* log2_max, const uint32_t** d_twf, const uint32_t** d_twi) {
  if (!prime_ok(ctx, prime_id)) return MONT_EINVAL;
  if (prm) *prm = ctx->params[prime_id];
  if (root) *root = ctx->roots[prime_id];
  if (log2_max) *log2_max = ctx->logmax[prime_id];
  if (d_twf) *d_twf = ctx->twf[prime_id];
  if (d_twi) *d_twi = ctx->twi[prime_id];
  return MONT_OK;
}

extern "C" mont_status ntt_ctx_read_twiddles(const ntt_ctx* ctx, int prime_id, uint32_t* h_fwd, uint32_t* h_inv) {
  if (!prime_ok(ctx, prime_id) || !h_fwd || !h_inv) return MONT_EINVAL;
  size_t bytes = (size_t)4 << ctx->logmax[prime_id];
  if (hipMemcpy(h_fwd, ctx->twf[prime_id], bytes, hipMemcpyDeviceToHost) != hipSuccess) return MONT_EHIP;
  if (hipMemcpy(h_inv, ctx->twi[prime_id], bytes, hipMemcpyDeviceToHost) != hipSuccess) return MONT_EHIP;
  return MONT_OK;
}

extern "C" mont_status ntt_forward(const ntt_ctx* ctx, int prime_id, uint32_t* d_x, uint32_t log2n, void* stream) {
  if (!prime_ok(ctx, prime_id) || !d_x) return MONT_EINVAL;
  if (log2n > ctx->logmax[prime_id]) return MONT_ENOROOT;
  hipStream_t s = as_stream(stream);
  (void)hipGetLastError();
  int n = (int)log2n;
  DirectArgs g = direct_base(ctx, prime_id, n);
  g.out = d_x;
  if (n <= kRowLog) {
    g.kind = D_FWD_SMALL;
    launch_direct(g, 1, s);
  } else {
    g.kind = D_COLF_INPLACE;
    launch_direct(g, g.ntiles, s);
    g.kind = D_ROW_FWD;
    launch_direct(g, 1u << (n - kRowLog), s);
  }
  return last_launch_status();
}

extern "C" mont_status ntt_inverse(const ntt_ctx* ctx, int prime_id, uint32_t* d_x, uint32_t log2n, void* stream) {
  if (!prime_ok(ctx, prime_id) || !d_x) return MONT_EINVAL;
  if (log2n > ctx->logmax[prime_id]) return MONT_ENOROOT;
  hipStream_t s = as_stream(stream);
  (void)hipGetLastError();
  int n = (int)log2n;
  const mont_params& prm = ctx->params[prime_id];
  uint64_t ninv = prm.P - ((prm.P - 1) >> n);
  DirectArgs g = direct_base(ctx, prime_id, n);
  g.out = d_x;
  g.prescale = (uint32_t)((uint64_t)prm.R1 * ninv % prm.P);
  if (n <= kRowLog) {
    g.kind = D_INV_SMALL;
    launch_direct(g, 1, s);
  } else {
    g.kind = D_ROW_INV;
    launch_direct(g, 1u << (n - kRowLog), s);
    g.kind = D_COLI_INPLACE;
    launch_direct(g, g.ntiles, s);
  }
  return last_launch_status();
}

extern "C" size_t ntt_polymul_scratch_bytes(uint32_t da, uint32_t db) {
  int n = ceil_log2((uint64_t)da + db + 1);
  return n <= kRowLog ? 0 : (size_t)8 << n;
}

namespace {

// The plain-launch product on scratch scr (2N words when N > 2^13), after
// the caller's validation.
mont_status polymul_launch(const ntt_ctx* ctx, int prime_id, int n, const uint32_t* d_a, uint32_t da,
                           const uint32_t* d_b, uint32_t db, uint32_t* d_out, uint32_t* scr, hipStream_t s) {
  (void)hipGetLastError();
  DirectArgs g = direct_base(ctx, prime_id, n);
  g.a = d_a;
  g.b = d_b;
  g.da = da;
  g.db = db;
  g.out = d_out;
  g.scr = scr;
  if (n <= kRowLog) {
    g.kind = D_SMALL_POLY;
    launch_direct(g, 1, s);
  } else {
    g.kind = D_COLF;
    launch_direct(g, 2 * g.ntiles, s);
    g.kind = D_ROW_POLY;
    launch_direct(g, 1u << (n - kRowLog), s);
    g.kind = D_COLI;
    launch_direct(g, g.ntiles, s);
  }
  return last_launch_status();
}

}  // namespace

extern "C" mont_status ntt_polymul(const ntt_ctx* ctx, int prime_id, const uint32_t* d_a, uint32_t da,
                                   const uint32_t* d_b, uint32_t db, uint32_t* d_out, void* d_scratch,
                                   size_t scratch_bytes, void* stream) {
  if (!prime_ok(ctx, prime_id) || !d_a || !d_b || !d_out) return MONT_EINVAL;
  if ((uint64_t)da + db + 1 > ((uint64_t)1 << 31)) return MONT_ERANGE;
  int n = ceil_log2((uint64_t)da + db + 1);
  if ((uint32_t)n > ctx->logmax[prime_id]) return MONT_ENOROOT;
  size_t need = ntt_polymul_scratch_bytes(da, db);
  if (need && (!d_scratch || scratch_bytes < need)) return MONT_ENOMEM;
  if (need && !aligned16(d_scratch)) return MONT_EINVAL;
  return polymul_launch(ctx, prime_id, n, d_a, da, d_b, db, d_out, static_cast<uint32_t*>(d_scratch),
                        as_stream(stream));
}

extern "C" mont_status ntt_polymul_noalloc(const ntt_ctx* ctx, int prime_id, const uint32_t* d_a, uint32_t da,
                                           const uint32_t* d_b, uint32_t db, uint32_t* d_out, void* stream) {
  if (!prime_ok(ctx, prime_id) || !d_a || !d_b || !d_out) return MONT_EINVAL;
  if ((uint64_t)da + db + 1 > ((uint64_t)1 << 31)) return MONT_ERANGE;
  const int n = ceil_log2((uint64_t)da + db + 1);
  if ((uint32_t)n > ctx->logmax[prime_id]) return MONT_ENOROOT;
  if (n > kNoAllocLog) return MONT_ENOMEM;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return MONT_EHIP;
  if (dev != ctx->device) return MONT_EINVAL;
  if (!ctx->noalloc_scr) return MONT_EHIP;
  return polymul_launch(ctx, prime_id, n, d_a, da, d_b, db, d_out, ctx->noalloc_scr, as_stream(stream));
}

// ---------------------------------------------------------------------------
// Batch plans.
// ---------------------------------------------------------------------------

namespace {

// Groups of multi-pass products in the task pipeline of a plan.
constexpr int kPipeGroups = 8;
// Batches with fewer multi-pass products than this are ordered phase by phase
// (the software pipeline pays only when many products overlap; a serving
// loop's batches of a few dozen products finish sooner without it).
constexpr size_t kPipeMinProducts = 128;

size_t product_task_total(const std::vector<ProdDev>& prods) {
  size_t t = 0;
  for (const ProdDev& pd : prods) t += pd.n > (uint32_t)kRowLog ? 3 * pd.ntiles + pd.nblocks : 1;
  return t;
}

// Host side of planning: internal products (a product the split rule takes
// becomes its cyclic part and its top part), the ordered task list, the
// fix-up list and the scratch layout: header, two counters per internal
// product, then 2N words per multi-pass product and the top parts' outputs.
mont_status build_plan(const ntt_ctx* ctx, const polymul_desc* descs, int count, uint32_t order_seed,
                       std::vector<ProdDev>& prods, std::vector<uint2>& tasks, std::vector<FixDev>& fixes,
                       uint32_t& nchunks, uint64_t& scr_words, uint64_t& in_words, uint64_t& out_words,
                       uint64_t& redc) {
  nchunks = 0;
  redc = 0;
  prods.clear();
  prods.reserve(2 * (size_t)count);
  fixes.clear();
  tasks.clear();
  std::vector<uint2> small;
  in_words = 0;
  out_words = 0;
  std::vector<uint32_t> top_words;                 // per fix-up: words of its second part's output
  const uint32_t nprimes = (uint32_t)ctx->params.size();
  for (int p = 0; p < count; p++) {
    const polymul_desc& d = descs[p];
    const SlotShape s0 = slot_shape(d, 0, nprimes, ctx->logmax.data());
    if (s0.err) return s0.err;
    const uint64_t nout = (uint64_t)d.da + d.db + 1;
    in_words = std::max<uint64_t>(in_words, std::max(d.a_off + d.da + 1, d.b_off + d.db + 1));
    out_words = std::max<uint64_t>(out_words, d.c_off + nout);
    for (int part = 0; part < 2; part++) {
      const SlotShape sh = part == 0 ? s0 : slot_shape(d, 1, nprimes, ctx->logmax.data());
      if (!sh.used) continue;
      ProdDev pd;
      std::memset(&pd, 0, sizeof(pd));
      pd.prime_id = d.prime_id;
      pd.n = (uint32_t)sh.n;
      pd.da = sh.da;
      pd.db = sh.db;
      pd.a_off = sh.a_off;
      pd.b_off = sh.b_off;
      pd.c_off = d.c_off;                          // second parts: set with the scratch layout
      pd.nout = sh.nout;
      pd.to_scr = part == 1 ? 1u : 0u;
      pd.tft = sh.block ? (uint32_t)sh.nfull : 0u;
      prods.push_back(pd);
      redc += slot_redc(sh) + fix_redc(sh);
      if (part == 1) {
        FixDev f;
        std::memset(&f, 0, sizeof(f));
        f.c_off = d.c_off;
        f.t_off = 0;                               // set with the scratch layout
        f.m = sh.m;
        f.h = sh.h;
        f.P = ctx->params[d.prime_id].P;
        f.chunk0 = nchunks;
        f.kind = sh.block ? FIX_TFT : FIX_SPLIT;
        f.prime_id = d.prime_id;
        f.s_log = (uint32_t)sh.n;
        nchunks += (sh.m + kFixChunk - 1) / kFixChunk;
        fixes.push_back(f);
        top_words.push_back(sh.nout);
      }
    }
  }
  const int np = (int)prods.size();
  uint64_t scr = kHdrWords + 2ull * np;
  scr = (scr + 63) & ~63ull;
  for (int p = 0, f = 0; p < np; p++) {
    ProdDev& pd = prods[p];
    if (pd.n > (uint32_t)kRowLog) {
      pd.lc = (uint32_t)col_lc((int)pd.n);
      pd.ntiles = 1u << (kRowLog - pd.lc);
      pd.nblocks = 1u << (pd.n - kRowLog);
      pd.scr_off = scr;
      scr += 2ull << pd.n;
    }
    if (pd.to_scr) {
      pd.c_off = scr;
      fixes[f].t_off = scr;
      scr += (top_words[f] + 3) & ~3u;
      f++;
    }
  }
  for (int p = 0; p < np; p++)
    if (prods[p].n <= (uint32_t)kRowLog) small.push_back(make_uint2((uint32_t)p, T_SMALL << 28));
  std::vector<int> big;
  for (int p = 0; p < np; p++)
    if (prods[p].n > (uint32_t)kRowLog) big.push_back(p);
  // longest first; products of one length by prime, so that tasks that run
  // together share one prime's twiddle tables in the caches
  std::stable_sort(big.begin(), big.end(), [&](int x, int y) {
    return prods[x].n != prods[y].n ? prods[x].n > prods[y].n : prods[x].prime_id < prods[y].prime_id;
  });
  std::stable_sort(small.begin(), small.end(), [&](uint2 x, uint2 y) { return prods[x.x].n > prods[y.x].n; });
  tasks.reserve(product_task_total(prods));
  if (big.size() < kPipeMinProducts) {
    // Phase order: every forward column tile (longest products first), half
    // the single-task products, every row block, the other half, every
    // inverse column tile.  A batch of a few multi-pass products finishes
    // soonest this way: its longest product's tasks are not spread out behind
    // other products' tasks.
    std::vector<uint2> colf, row, coli;
    for (int p : big) {
      const ProdDev& pd = prods[p];
      for (uint32_t t = 0; t < pd.ntiles; t++) colf.push_back(make_uint2((uint32_t)p, (T_COLF_A << 28) | t));
      for (uint32_t t = 0; t < pd.ntiles; t++) colf.push_back(make_uint2((uint32_t)p, (T_COLF_B << 28) | t));
      for (uint32_t j = 0; j < pd.nblocks; j++) row.push_back(make_uint2((uint32_t)p, (T_ROW << 28) | j));
      for (uint32_t t = 0; t < pd.ntiles; t++) coli.push_back(make_uint2((uint32_t)p, (T_COLI << 28) | t));
    }
    if (order_seed != 0) {
      // Any order within a phase keeps prerequisites earlier in the list.
      std::mt19937_64 rng(order_seed);
      std::shuffle(colf.begin(), colf.end(), rng);
      std::shuffle(small.begin(), small.end(), rng);
      std::shuffle(row.begin(), row.end(), rng);
      std::shuffle(coli.begin(), coli.end(), rng);
    }
    const size_t half = small.size() / 2;
    tasks.insert(tasks.end(), colf.begin(), colf.end());
    tasks.insert(tasks.end(), small.begin(), small.begin() + half);
    tasks.insert(tasks.end(), row.begin(), row.end());
    tasks.insert(tasks.end(), small.begin() + half, small.end());
    tasks.insert(tasks.end(), coli.begin(), coli.end());
    scr_words = scr;
    return MONT_OK;
  }
  // Many multi-pass products: longest first, cut into kPipeGroups groups of
  // about equal work.  The list is a software pipeline over the groups: block
  // b interleaves the row blocks of group b-1 (bound by the vector ALU) with
  // the forward column tiles of group b and the inverse column tiles of group
  // b-2 (bound by memory latency), so the two workgroups of a CU tend to hold
  // tasks of both kinds.  Every prerequisite still precedes its dependants:
  // the forward tiles of a group come in an earlier block than its rows, and
  // its rows in an earlier block than its inverse tiles.
  double total = 0;
  for (int p : big) total += std::ldexp(1.0, (int)prods[p].n) * prods[p].n;
  const int ng = kPipeGroups;
  std::vector<std::vector<uint2>> colf_g(ng), row_g(ng), coli_g(ng);
  double acc = 0;
  for (int p : big) {
    const ProdDev& pd = prods[p];
    const int g = std::min(ng - 1, (int)(acc / total * ng));
    acc += std::ldexp(1.0, (int)pd.n) * pd.n;
    for (uint32_t t = 0; t < pd.ntiles; t++) colf_g[g].push_back(make_uint2((uint32_t)p, (T_COLF_A << 28) | t));
    for (uint32_t t = 0; t < pd.ntiles; t++) colf_g[g].push_back(make_uint2((uint32_t)p, (T_COLF_B << 28) | t));
    for (uint32_t j = 0; j < pd.nblocks; j++) row_g[g].push_back(make_uint2((uint32_t)p, (T_ROW << 28) | j));
    for (uint32_t t = 0; t < pd.ntiles; t++) coli_g[g].push_back(make_uint2((uint32_t)p, (T_COLI << 28) | t));
  }
  // Single-task products are spread over the blocks.
  const int nblk = ng + 2;
  std::vector<std::vector<uint2>> small_b(nblk);
  for (size_t i = 0; i < small.size(); i++) small_b[i * nblk / small.size()].push_back(small[i]);
  if (order_seed != 0) {
    // Any order within a list keeps prerequisites earlier in the whole list.
    std::mt19937_64 rng(order_seed);
    for (int g = 0; g < ng; g++) {
      std::shuffle(colf_g[g].begin(), colf_g[g].end(), rng);
      std::shuffle(row_g[g].begin(), row_g[g].end(), rng);
      std::shuffle(coli_g[g].begin(), coli_g[g].end(), rng);
    }
    for (auto& v : small_b) std::shuffle(v.begin(), v.end(), rng);
  }
  // Block b (0 .. ng+1) holds the forward tiles of group b, the rows of group
  // b-1, the inverse tiles of group b-2 and a share of the single tasks,
  // merged in proportion to their lengths.
  for (int b = 0; b < nblk; b++) {
    const std::vector<uint2>* parts[4] = {b < ng ? &colf_g[b] : nullptr,
                                          b >= 1 && b - 1 < ng ? &row_g[b - 1] : nullptr,
                                          b >= 2 && b - 2 < ng ? &coli_g[b - 2] : nullptr, &small_b[b]};
    size_t pos[4] = {0, 0, 0, 0}, len[4];
    size_t left = 0;
    for (int i = 0; i < 4; i++) left += (len[i] = parts[i] ? parts[i]->size() : 0);
    while (left > 0) {
      int pick = -1;
      double best = 2.0;
      for (int i = 0; i < 4; i++) {
        if (pos[i] >= len[i]) continue;
        const double f = (pos[i] + 0.5) / (double)len[i];
        if (f < best) best = f, pick = i;
      }
      tasks.push_back((*parts[pick])[pos[pick]++]);
      left--;
    }
  }
  scr_words = scr;
  return MONT_OK;
}

void free_plan(ntt_plan* plan) {
  if (plan->reusable) {
    (void)hipFree(plan->d_block);
    if (plan->h_block) (void)hipHostFree(plan->h_block);
  } else {
    (void)hipFree(plan->d_prods);
    (void)hipFree(plan->d_tasks);
    (void)hipFree(plan->d_fix);
    (void)hipFree(plan->d_owner);
  }
  if (plan->staged) (void)hipEventDestroy(plan->staged);
  delete plan;
}

// Bytes of a reusable plan's block: 2 max_products product descriptors (a
// split product has two parts), max_products fix-ups, max_tasks tasks.
size_t plan_block_bytes(int max_products, uint32_t max_tasks) {
  return sizeof(ProdDev) * 2 * (size_t)max_products + sizeof(FixDev) * (size_t)max_products +
         sizeof(uint2) * (size_t)max_tasks;
}

}  // namespace

extern "C" mont_status ntt_plan_create(const ntt_ctx* ctx, const polymul_desc* descs, int count, uint32_t order_seed,
                                       ntt_plan** out) {
  if (!ctx || !out || count < 0 || (count > 0 && !descs)) return MONT_EINVAL;
  *out = nullptr;
  std::vector<ProdDev> prods;
  std::vector<uint2> tasks;
  std::vector<FixDev> fixes;
  uint64_t scr = 0, in_words = 0, out_words = 0;
  uint32_t nchunks = 0;
  uint64_t redc = 0;
  mont_status st = build_plan(ctx, descs, count, order_seed, prods, tasks, fixes, nchunks, scr, in_words, out_words,
                              redc);
  if (st != MONT_OK) return st;
  ntt_plan* plan = new (std::nothrow) ntt_plan;
  if (!plan) return MONT_ENOMEM;
  plan->ctx = ctx;
  plan->count = (int)prods.size();
  plan->ntasks = (uint32_t)tasks.size();
  plan->nfix = (uint32_t)fixes.size();
  plan->nchunks = nchunks;
  plan->scratch_words = scr;
  plan->in_words = in_words;
  plan->out_words = out_words;
  std::vector<uint32_t> owner(nchunks);
  for (size_t i = 0; i < fixes.size(); i++) {
    const uint32_t c1 = fixes[i].chunk0 + (fixes[i].m + kFixChunk - 1) / kFixChunk;
    for (uint32_t c = fixes[i].chunk0; c < c1; c++) owner[c] = (uint32_t)i;
  }
  if (!prods.empty()) {
    if (hipMalloc(&plan->d_prods, sizeof(ProdDev) * prods.size()) != hipSuccess ||
        hipMalloc(&plan->d_tasks, sizeof(uint2) * std::max<size_t>(1, tasks.size())) != hipSuccess ||
        (!fixes.empty() && hipMalloc(&plan->d_fix, sizeof(FixDev) * fixes.size()) != hipSuccess) ||
        (nchunks && hipMalloc(&plan->d_owner, sizeof(uint32_t) * nchunks) != hipSuccess)) {
      free_plan(plan);
      return MONT_ENOMEM;
    }
    if (hipMemcpy(plan->d_prods, prods.data(), sizeof(ProdDev) * prods.size(), hipMemcpyHostToDevice) != hipSuccess ||
        (tasks.size() && hipMemcpy(plan->d_tasks, tasks.data(), sizeof(uint2) * tasks.size(),
                                   hipMemcpyHostToDevice) != hipSuccess) ||
        (fixes.size() && hipMemcpy(plan->d_fix, fixes.data(), sizeof(FixDev) * fixes.size(),
                                   hipMemcpyHostToDevice) != hipSuccess) ||
        (nchunks && hipMemcpy(plan->d_owner, owner.data(), sizeof(uint32_t) * nchunks, hipMemcpyHostToDevice) !=
                        hipSuccess)) {
      free_plan(plan);
      return MONT_EHIP;
    }
  }
  plan->shape = plan_shape(prods);
  plan->redc = redc - plan_unit_bfly(prods, plan->shape.radix_log);
  plan->default_grid = persistent_grid(plan->shape);
  *out = plan;
  return MONT_OK;
}

extern "C" mont_status ntt_plan_reserve(const ntt_ctx* ctx, int max_products, uint32_t max_tasks, ntt_plan** out) {
  if (!ctx || !out || max_products < 1 || max_tasks < 1) return MONT_EINVAL;
  *out = nullptr;
  ntt_plan* plan = new (std::nothrow) ntt_plan;
  if (!plan) return MONT_ENOMEM;
  plan->ctx = ctx;
  plan->reusable = true;
  plan->cap_prods = max_products;
  plan->cap_tasks = max_tasks;
  const size_t bytes = plan_block_bytes(max_products, max_tasks);
  if (hipMalloc(&plan->d_block, bytes) != hipSuccess ||
      hipHostMalloc(&plan->h_block, bytes, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&plan->staged, hipEventDisableTiming) != hipSuccess) {
    free_plan(plan);
    return MONT_ENOMEM;
  }
  plan->shape = g_ntt_tune;
  plan->default_grid = persistent_grid(plan->shape);
  *out = plan;
  return MONT_OK;
}

extern "C" mont_status ntt_plan_update(ntt_plan* plan, const polymul_desc* descs, int count, uint32_t order_seed,
                                       void* stream) {
  if (!plan || !plan->reusable || count < 0 || (count > 0 && !descs)) return MONT_EINVAL;
  if (count > plan->cap_prods) return MONT_ERANGE;
  using clock = std::chrono::steady_clock;
  const auto us_since = [](clock::time_point t) {
    return (uint32_t)std::chrono::duration_cast<std::chrono::microseconds>(clock::now() - t).count();
  };
  const clock::time_point t0 = clock::now();
  std::vector<ProdDev> prods;
  std::vector<uint2> tasks;
  std::vector<FixDev> fixes;
  uint64_t scr = 0, in_words = 0, out_words = 0;
  uint32_t nchunks = 0;
  uint64_t redc = 0;
  mont_status st = build_plan(plan->ctx, descs, count, order_seed, prods, tasks, fixes, nchunks, scr, in_words,
                              out_words, redc);
  if (st != MONT_OK) return st;
  if (tasks.size() > plan->cap_tasks) return MONT_ERANGE;
  plan->upd_us[0] = us_since(t0);
  // The previous upload must have finished reading the staging buffers.
  const clock::time_point t1 = clock::now();
  if (plan->staged_pending && hipEventSynchronize(plan->staged) != hipSuccess) return MONT_EHIP;
  plan->staged_pending = false;
  plan->upd_us[1] = us_since(t1);
  plan->upd_us[2] = 0;
  hipStream_t s = as_stream(stream);
  plan->inl = !prods.empty() && prods.size() <= kInlineProds && tasks.size() <= kInlineTasks && fixes.empty();
  if (plan->inl) {
    // small enough for the launch arguments: nothing to upload
    std::copy(prods.begin(), prods.end(), plan->inl_prods);
    std::copy(tasks.begin(), tasks.end(), plan->inl_tasks);
  } else if (!prods.empty()) {
    // products, fix-ups, tasks back to back (every record size is a multiple
    // of 8 bytes), one upload
    const size_t bp = sizeof(ProdDev) * prods.size(), bf = sizeof(FixDev) * fixes.size(),
                 bt = sizeof(uint2) * tasks.size();
    char* h = static_cast<char*>(plan->h_block);
    char* d = static_cast<char*>(plan->d_block);
    std::memcpy(h, prods.data(), bp);
    if (bf) std::memcpy(h + bp, fixes.data(), bf);
    if (bt) std::memcpy(h + bp + bf, tasks.data(), bt);
    const clock::time_point t2 = clock::now();
    if (hipMemcpyAsync(d, h, bp + bf + bt, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipEventRecord(plan->staged, s) != hipSuccess)
      return MONT_EHIP;
    plan->upd_us[2] = us_since(t2);
    plan->staged_pending = true;
    plan->d_prods = reinterpret_cast<ProdDev*>(d);
    plan->d_fix = reinterpret_cast<FixDev*>(d + bp);
    plan->d_tasks = reinterpret_cast<uint2*>(d + bp + bf);
  }
  plan->count = (int)prods.size();
  plan->ntasks = (uint32_t)tasks.size();
  plan->nfix = (uint32_t)fixes.size();
  plan->nchunks = nchunks;
  plan->scratch_words = scr;
  plan->in_words = in_words;
  plan->out_words = out_words;
  plan->shape = plan_shape(prods);
  plan->redc = redc - plan_unit_bfly(prods, plan->shape.radix_log);
  plan->default_grid = persistent_grid(plan->shape);
  plan->upd_us[3] = us_since(t0);
  return MONT_OK;
}

extern "C" mont_status ntt_plan_update_times(const ntt_plan* plan, uint32_t* us) {
  if (!plan || !us) return MONT_EINVAL;
  for (int i = 0; i < 4; i++) us[i] = plan->upd_us[i];
  return MONT_OK;
}

extern "C" uint32_t ntt_plan_task_count(uint32_t da, uint32_t db) {
  polymul_desc d;
  std::memset(&d, 0, sizeof(d));
  d.da = da;
  d.db = db;
  const uint32_t any_length = 31;                   // the rules do not depend on the prime
  uint32_t t = 0;
  for (int part = 0; part < 2; part++) {
    const SlotShape sh = slot_shape(d, part, 1, &any_length);
    if (sh.err) return 0;
    if (sh.used) t += product_tasks(sh.n);
  }
  return t;
}

extern "C" mont_status ntt_plan_info(const ntt_plan* plan, size_t* scratch_bytes, uint32_t* ntasks,
                                     uint64_t* in_words, uint64_t* out_words, int* default_grid) {
  if (!plan) return MONT_EINVAL;
  if (scratch_bytes) *scratch_bytes = (size_t)plan->scratch_words * 4;
  if (ntasks) *ntasks = plan->ntasks;
  if (in_words) *in_words = plan->in_words;
  if (out_words) *out_words = plan->out_words;
  if (default_grid) *default_grid = persistent_grid(plan->shape);
  return MONT_OK;
}

extern "C" mont_status ntt_plan_work(const ntt_plan* plan, uint64_t* redc, uint32_t* split_products) {
  if (!plan) return MONT_EINVAL;
  if (redc) *redc = plan->redc;
  if (split_products) *split_products = plan->nfix;
  return MONT_OK;
}

extern "C" mont_status ntt_plan_shape(const ntt_plan* plan, int* threads, int* radix_log, int* grid_mult) {
  if (!plan) return MONT_EINVAL;
  if (threads) *threads = plan->shape.threads;
  if (radix_log) *radix_log = plan->shape.radix_log;
  if (grid_mult) *grid_mult = plan->shape.grid_mult;
  return MONT_OK;
}

extern "C" mont_status ntt_plan_execute(const ntt_plan* plan, const uint32_t* d_in, uint32_t* d_out, void* d_scratch,
                                        size_t scratch_bytes, int grid, uint32_t spin_limit, void* stream) {
  if (!plan) return MONT_EINVAL;
  if (plan->count == 0) return MONT_OK;
  if (!d_in || !d_out || !d_scratch) return MONT_EINVAL;
  if (scratch_bytes < plan->scratch_words * 4) return MONT_ENOMEM;
  if (grid < 0 || !aligned16(d_scratch)) return MONT_EINVAL;
  hipStream_t s = as_stream(stream);
  (void)hipGetLastError();
  uint32_t* scr = static_cast<uint32_t*>(d_scratch);
  uint32_t nz = (uint32_t)(kHdrWords + 2ull * plan->count);
  hipLaunchKernelGGL(k_fill_zero, dim3(std::min(1024u, (nz + 255) / 256)), dim3(256), 0, s, scr, nz);
  PlanArgs g;
  // every scalar field zero (the inline arrays that follow are filled below
  // only as far as they are used)
  std::memset(&g, 0, offsetof(PlanArgs, inl_prods));
  g.primes = plan->ctx->d_primes;
  g.prods = plan->d_prods;
  g.tasks = plan->d_tasks;
  g.inl = plan->inl ? 1u : 0u;
  if (plan->inl) {
    std::copy(plan->inl_prods, plan->inl_prods + plan->count, g.inl_prods);
    std::copy(plan->inl_tasks, plan->inl_tasks + plan->ntasks, g.inl_tasks);
  }
  g.ntasks = plan->ntasks;
  g.nprods = (uint32_t)plan->count;
  g.in = d_in;
  g.out = d_out;
  g.scr = scr;
  g.spin_limit = spin_limit ? spin_limit : (1u << 24);
  uint32_t gsz = grid > 0 ? (uint32_t)grid : (uint32_t)persistent_grid(plan->shape);
  gsz = std::max(1u, std::min(gsz, plan->ntasks));
  launch_persistent(g, gsz, s, plan->shape);
  if (plan->nfix > 0)
    // one workgroup per chunk; a reusable plan has no owner table and each
    // chunk searches the records
    hipLaunchKernelGGL(k_split_fix, dim3(plan->nchunks), dim3(256), 0, s, plan->ctx->d_primes,
                       plan->d_fix, plan->nfix, plan->nchunks, d_out, static_cast<const uint32_t*>(scr), nullptr,
                       plan->d_owner);
  return last_launch_status();
}

extern "C" mont_status ntt_plan_status(const ntt_plan* plan, const void* d_scratch, void* stream) {
  if (!plan || !d_scratch) return MONT_EINVAL;
  if (plan->count == 0) return MONT_OK;
  hipStream_t s = as_stream(stream);
  uint32_t st = 0;
  if (hipMemcpyAsync(&st, static_cast<const uint32_t*>(d_scratch) + 1, 4, hipMemcpyDeviceToHost, s) != hipSuccess)
    return MONT_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return MONT_EHIP;
  return st == 0 ? MONT_OK : MONT_ETIMEOUT;
}

extern "C" mont_status ntt_plan_status_async(const ntt_plan* plan, const void* d_scratch, uint32_t* h_status,
                                             void* stream) {
  if (!plan || !d_scratch || !h_status) return MONT_EINVAL;
  if (plan->count == 0) {
    *h_status = 0;
    return MONT_OK;
  }
  if (hipMemcpyAsync(h_status, static_cast<const uint32_t*>(d_scratch) + 1, 4, hipMemcpyDeviceToHost,
                     as_stream(stream)) != hipSuccess)
    return MONT_EHIP;
  return MONT_OK;
}

// ---------------------------------------------------------------------------
// One-call batches planned on the device.
// ---------------------------------------------------------------------------

extern "C" size_t ntt_scratch_bytes(const ntt_ctx* ctx, const polymul_desc* descs, int count) {
  if (!ctx || count < 0 || (count > 0 && !descs)) return 0;
  const uint32_t np = (uint32_t)ctx->params.size();
  uint64_t ntasks = 0, words = 0, chunks = 0;
  for (int i = 0; i < count; i++)
    for (int part = 0; part < 2; part++) {
      const SlotShape sh = slot_shape(descs[i], part, np, ctx->logmax.data());
      if (sh.err) return 0;
      if (!sh.used) continue;
      ntasks += product_tasks(sh.n);
      words += slot_words(sh, part);
      chunks += slot_chunks(sh, part);
    }
  // header, records and tasks | data | the fix-up chunks' record table
  return (size_t)(batch_data_offset(batch_layout((uint32_t)count), ntasks) + words + chunks) * 4;
}

extern "C" mont_status ntt_polymul_batch(const ntt_ctx* ctx, const polymul_desc* d_descs, int count,
                                         const uint32_t* d_in, uint32_t* d_out, void* d_scratch, size_t scratch_bytes,
                                         void* stream) {
  if (!ctx || count < 0 || !d_scratch || (count > 0 && (!d_descs || !d_in || !d_out))) return MONT_EINVAL;
  if (!aligned16(d_scratch) || ((uintptr_t)d_descs & 7u) != 0) return MONT_EINVAL;
  const BatchLayout lay = batch_layout((uint32_t)count);
  if (scratch_bytes / 4 < batch_data_offset(lay, 0)) return MONT_ENOMEM;
  hipStream_t s = as_stream(stream);
  (void)hipGetLastError();
  uint32_t* scr = static_cast<uint32_t*>(d_scratch);
  hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(kPlanThreads), 0, s, ctx->d_primes, (uint32_t)ctx->params.size(),
                     d_descs, (uint32_t)count, scr, (uint64_t)(scratch_bytes / 4));
  if (count == 0) return last_launch_status();
  PlanArgs g;
  std::memset(&g, 0, sizeof(g));
  g.primes = ctx->d_primes;
  g.prods = reinterpret_cast<const ProdDev*>(scr + lay.prods);
  g.tasks = reinterpret_cast<const uint2*>(scr + lay.tasks);
  g.nprods = 2u * (uint32_t)count;
  g.in = d_in;
  g.out = d_out;
  g.scr = scr;
  g.spin_limit = 1u << 24;
  g.dyn = 1;
  // the descriptors are on the device: the default shape (not a per-length one)
  launch_persistent(g, (uint32_t)persistent_grid(g_ntt_tune), s, g_ntt_tune);
  // the chunk count is known only on the device: a grid that covers the
  // chunks of most batches at one workgroup each, striding beyond
  hipLaunchKernelGGL(k_split_fix, dim3(32768), dim3(256), 0, s, ctx->d_primes,
                     reinterpret_cast<const FixDev*>(scr + lay.fixes), (uint32_t)count, 0u, d_out,
                     static_cast<const uint32_t*>(scr), scr, nullptr);
  return last_launch_status();
}

extern "C" mont_status ntt_batch_status(const void* d_scratch, void* stream) {
  if (!d_scratch) return MONT_EINVAL;
  hipStream_t s = as_stream(stream);
  uint32_t hdr[8];
  if (hipMemcpyAsync(hdr, d_scratch, sizeof(hdr), hipMemcpyDeviceToHost, s) != hipSuccess) return MONT_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return MONT_EHIP;
  if (hdr[kHdrError] != 0) return (mont_status)(int32_t)hdr[kHdrError];
  return hdr[1] == 0 ? MONT_OK : MONT_ETIMEOUT;
}

extern "C" mont_status ntt_plan_destroy(ntt_plan* plan) {
  if (!plan) return MONT_EINVAL;
  (void)hipDeviceSynchronize();
  free_plan(plan);
  return MONT_OK;
}
