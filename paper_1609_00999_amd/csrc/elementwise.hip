// elementwise.hip -- streaming Montgomery kernels: residue conversion,
// products, fused product-plus-sum and powers over device arrays.
//
// Each lane applies Algorithm 2 (arXiv:1609.00999, section 3.1) to four
// residues fetched with one 128-bit load; a wavefront therefore covers 256
// contiguous residues per load instruction, and the kernels are bound by HBM
// bandwidth (mont_pow excepted, which is bound by the vector ALU).
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "modarith.hpp"

namespace mont {

namespace {

// The vector kernel addresses each workgroup tile through raw buffer
// resources (CDNA buffer instructions): a resource in scalar registers holds
// the tile's first address and its size in bytes, each lane one 32-bit
// offset.  Loads past the size return 0 and stores past it are dropped (the
// range check of raw, unstrided buffers), so the array's last, partial tile
// needs no per-lane compare, and an address costs no 64-bit arithmetic.  NT:
// the non-temporal cache policy (streamed data, read or written once).
constexpr int kBufWord3 = 0x00020000;   // resource word 3 on gfx9: 32-bit data format
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, kBufWord3);
}
template <bool NT>
__device__ __forceinline__ v4u ld(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, NT ? 2 : 0);
}
template <bool NT>
__device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t off, v4u v) {
  __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)off, 0, NT ? 2 : 0);
}

// x^e in the residue system by fixed 2-bit windows, most significant first.
// The window table {1, x, x^2, x^3} is indexed with selects, so every lane
// runs the same instruction stream whatever its exponent: 2 table products,
// then 15 windows of two squarings and one product (47 REDC per power).
__device__ __forceinline__ uint32_t pow_win2(uint32_t x, uint32_t e, Mod md, uint32_t one) {
  uint32_t x2 = mmul(x, x, md);
  uint32_t x3 = mmul(x2, x, md);
  auto pick = [&](uint32_t d) {
    uint32_t lo = (d & 1u) ? x : one;
    uint32_t hi = (d & 1u) ? x3 : x2;
    return (d & 2u) ? hi : lo;
  };
  uint32_t r = pick(e >> 30);
#pragma unroll
  for (int s = 28; s >= 0; s -= 2) {
    r = mmul(r, r, md);
    r = mmul(r, r, md);
    r = mmul(r, pick((e >> s) & 3u), md);
  }
  return r;
}

// REDC without its final subtraction: for T < R P, t = (T + m P) / R lies in
// [0, 2P).  When 4P < R, operands in [0, 2P) keep T < 4P^2 < R P, so a chain
// of such products stays in [0, 2P) and one conditional subtraction at its
// end makes the result canonical.  Three instructions instead of five.
__device__ __forceinline__ uint32_t mmul_lazy(uint32_t a, uint32_t b, Mod md) {
  const uint64_t T = (uint64_t)a * b;
  const uint32_t m = (uint32_t)T * md.Pp;
  return (uint32_t)(((uint64_t)m * md.P + T) >> 32);
}

// pow_win2 for P < 2^30 with lazy products: the window table and the running
// power stay in [0, 2P) and are reduced once at the end.
__device__ __forceinline__ uint32_t pow_win2_lazy(uint32_t x, uint32_t e, Mod md, uint32_t one) {
  uint32_t x2 = mmul_lazy(x, x, md);
  uint32_t x3 = mmul_lazy(x2, x, md);
  auto pick = [&](uint32_t d) {
    uint32_t lo = (d & 1u) ? x : one;
    uint32_t hi = (d & 1u) ? x3 : x2;
    return (d & 2u) ? hi : lo;
  };
  uint32_t r = pick(e >> 30);
#pragma unroll
  for (int s = 28; s >= 0; s -= 2) {
    r = mmul_lazy(r, r, md);
    r = mmul_lazy(r, r, md);
    r = mmul_lazy(r, pick((e >> s) & 3u), md);
  }
  const uint32_t u = r - md.P;
  return u < r ? u : r;
}

// Operation for the lazy power; shares OP_POW's launch shape.
constexpr int OP_POW_LAZY = OP_COUNT;

// Scalar operation applied per element.
template <int OP>
__device__ __forceinline__ uint32_t elem_op(uint32_t a, uint32_t b, uint32_t c, Mod md, uint32_t kc) {
  if constexpr (OP == OP_TO) return mmul(a, kc, md);             // REDC(a * R^2 mod P)
  else if constexpr (OP == OP_FROM) return redc((uint64_t)a, md); // REDC(a * 1)
  else if constexpr (OP == OP_MUL) return mmul(a, b, md);
  else if constexpr (OP == OP_MULADD) return madd(mmul(a, b, md), c, md.P);
  else if constexpr (OP == OP_POW_LAZY) return pow_win2_lazy(a, b, md, kc);
  // a b mod P of ordinary values: REDC(b R2) = b R mod P, then
  // REDC(a * bR) = a b; a * bR < 2^32 P = R P for every uint32 a, b.
  else if constexpr (OP == OP_MODMUL) return mmul(a, mmul(b, kc, md), md);   // kc = R^2 mod P
  else return pow_win2(a, b, md, kc);                             // kc = residue of 1
}

template <int OP>
constexpr int n_inputs() { return OP == OP_TO || OP == OP_FROM ? 1 : (OP == OP_MULADD ? 3 : 2); }

// Vector kernel: element i of every array is read once and the result
// written once.  Workgroup w handles vectors [w*BLOCK*VPT, (w+1)*BLOCK*VPT),
// lane l vector w*BLOCK*VPT + j*BLOCK + l for j < VPT (coalesced per j),
// through buffer resources sized to the tile's vectors inside the array;
// the grid strides over workgroup tiles when nvec exceeds it.  The last
// n - 4*nvec (< 4) elements are done by the first lanes of workgroup 0.
template <int OP, int BLOCK, int VPT, bool NT>
__global__ __launch_bounds__(BLOCK) void k_elem_v4(Mod md, uint32_t kc, const uint32_t* a,
                                                   const uint32_t* b,
                                                   const uint32_t* c, uint32_t* out,
                                                   size_t n) {
  constexpr int NIN = n_inputs<OP>();
  const size_t nvec = n >> 2;
  const size_t ntile = (nvec + (size_t)BLOCK * VPT - 1) / ((size_t)BLOCK * VPT);
  for (size_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const size_t first = tile * ((size_t)BLOCK * VPT);             // first vector of the tile
    const size_t left = nvec - first;
    const uint32_t bytes = (uint32_t)(left < (size_t)BLOCK * VPT ? left : (size_t)BLOCK * VPT) * 16u;
    const __amdgpu_buffer_rsrc_t ra = tile_rsrc(a + 4 * first, bytes);
    const __amdgpu_buffer_rsrc_t rb = tile_rsrc(NIN >= 2 ? b + 4 * first : a, bytes);
    const __amdgpu_buffer_rsrc_t rc = tile_rsrc(NIN >= 3 ? c + 4 * first : a, bytes);
    const __amdgpu_buffer_rsrc_t ro = tile_rsrc(out + 4 * first, bytes);
    v4u x[VPT], y[VPT], z[VPT];
#pragma unroll
    for (int j = 0; j < VPT; j++) {
      const uint32_t off = (threadIdx.x + (uint32_t)j * BLOCK) * 16u;
      x[j] = ld<NT>(ra, off);
      if constexpr (NIN >= 2) y[j] = ld<NT>(rb, off);
      if constexpr (NIN >= 3) z[j] = ld<NT>(rc, off);
    }
#pragma unroll
    for (int j = 0; j < VPT; j++) {
      const uint32_t off = (threadIdx.x + (uint32_t)j * BLOCK) * 16u;
      {
        v4u r;
        if constexpr (NIN == 1) {
          r.x = elem_op<OP>(x[j].x, 0, 0, md, kc);
          r.y = elem_op<OP>(x[j].y, 0, 0, md, kc);
          r.z = elem_op<OP>(x[j].z, 0, 0, md, kc);
          r.w = elem_op<OP>(x[j].w, 0, 0, md, kc);
        } else if constexpr (NIN == 2) {
          r.x = elem_op<OP>(x[j].x, y[j].x, 0, md, kc);
          r.y = elem_op<OP>(x[j].y, y[j].y, 0, md, kc);
          r.z = elem_op<OP>(x[j].z, y[j].z, 0, md, kc);
          r.w = elem_op<OP>(x[j].w, y[j].w, 0, md, kc);
        } else {
          r.x = elem_op<OP>(x[j].x, y[j].x, z[j].x, md, kc);
          r.y = elem_op<OP>(x[j].y, y[j].y, z[j].y, md, kc);
          r.z = elem_op<OP>(x[j].z, y[j].z, z[j].z, md, kc);
          r.w = elem_op<OP>(x[j].w, y[j].w, z[j].w, md, kc);
        }
        st<NT>(ro, off, r);
      }
    }
  }
  if (blockIdx.x == 0) {
    const size_t i = (nvec << 2) + threadIdx.x;
    if (i < n) {
      uint32_t ea = a[i];
      uint32_t eb = NIN >= 2 ? b[i] : 0u;
      uint32_t ec = NIN >= 3 ? c[i] : 0u;
      out[i] = elem_op<OP>(ea, eb, ec, md, kc);
    }
  }
}

// Scalar fallback for arrays that are not 16-byte aligned.
template <int OP>
__global__ __launch_bounds__(256) void k_elem_scalar(Mod md, uint32_t kc, const uint32_t* a, const uint32_t* b,
                                                     const uint32_t* c, uint32_t* out, size_t n) {
  constexpr int NIN = n_inputs<OP>();
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
    uint32_t ea = a[i];
    uint32_t eb = NIN >= 2 ? b[i] : 0u;
    uint32_t ec = NIN >= 3 ? c[i] : 0u;
    out[i] = elem_op<OP>(ea, eb, ec, md, kc);
  }
}

constexpr size_t kMaxGrid = (size_t)1 << 20;

template <int OP, int BLOCK, int VPT, bool NT>
void launch_v4(Mod md, uint32_t kc, const uint32_t* a, const uint32_t* b, const uint32_t* c, uint32_t* out,
               size_t n, hipStream_t s) {
  size_t nvec = n >> 2;
  size_t ntile = (nvec + (size_t)BLOCK * VPT - 1) / ((size_t)BLOCK * VPT);
  size_t grid = ntile < kMaxGrid ? ntile : kMaxGrid;
  if (grid == 0) grid = 1;
  hipLaunchKernelGGL((k_elem_v4<OP, BLOCK, VPT, NT>), dim3((unsigned)grid), dim3(BLOCK), 0, s, md, kc, a, b, c,
                     out, n);
}

template <int OP>
void dispatch(const ElemTune& t, Mod md, uint32_t kc, const uint32_t* a, const uint32_t* b, const uint32_t* c,
              uint32_t* out, size_t n, hipStream_t s) {
  bool al = aligned16(a) && aligned16(out) && (b == nullptr || aligned16(b)) && (c == nullptr || aligned16(c));
  if (!al) {
    size_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL((k_elem_scalar<OP>), dim3((unsigned)blocks), dim3(256), 0, s, md, kc, a, b, c, out, n);
    return;
  }
#define MONT_CASE(B, V, N)                                        \
  if (t.block == B && t.vpt == V && (t.nt != 0) == N) {           \
    launch_v4<OP, B, V, N>(md, kc, a, b, c, out, n, s);           \
    return;                                                       \
  }
  MONT_CASE(64, 1, true) MONT_CASE(64, 2, true) MONT_CASE(64, 4, true)
  MONT_CASE(128, 1, true) MONT_CASE(128, 2, true) MONT_CASE(128, 4, true)
  MONT_CASE(256, 1, true) MONT_CASE(256, 2, true) MONT_CASE(256, 4, true)
  MONT_CASE(512, 1, true) MONT_CASE(512, 2, true) MONT_CASE(512, 4, true)
  MONT_CASE(64, 1, false) MONT_CASE(64, 2, false) MONT_CASE(64, 4, false)
  MONT_CASE(128, 1, false) MONT_CASE(128, 2, false) MONT_CASE(128, 4, false)
  MONT_CASE(256, 1, false) MONT_CASE(256, 2, false) MONT_CASE(256, 4, false)
  MONT_CASE(512, 1, false) MONT_CASE(512, 2, false) MONT_CASE(512, 4, false)
#undef MONT_CASE
  launch_v4<OP, 256, 1, true>(md, kc, a, b, c, out, n, s);
}

ElemTune g_tune[OP_COUNT] = {
    {256, 1, 1}, {256, 1, 1}, {256, 1, 1}, {256, 1, 1}, {256, 1, 1}, {64, 1, 1},
};

mont_status run(int op, const mont_params* prm, const uint32_t* a, const uint32_t* b, const uint32_t* c,
                uint32_t* out, size_t n, void* stream) {
  if (!params_ok(prm)) return MONT_EINVAL;
  if (n == 0) return MONT_OK;
  if (!a || !out) return MONT_EINVAL;
  if ((op == OP_MUL || op == OP_MULADD || op == OP_POW || op == OP_MODMUL) && !b) return MONT_EINVAL;
  if (op == OP_MULADD && !c) return MONT_EINVAL;
  Mod md{prm->P, prm->Pprime};
  hipStream_t s = as_stream(stream);
  (void)hipGetLastError();
  const ElemTune& t = g_tune[op];
  switch (op) {
    case OP_TO: dispatch<OP_TO>(t, md, prm->R2, a, nullptr, nullptr, out, n, s); break;
    case OP_FROM: dispatch<OP_FROM>(t, md, 0, a, nullptr, nullptr, out, n, s); break;
    case OP_MUL: dispatch<OP_MUL>(t, md, 0, a, b, nullptr, out, n, s); break;
    case OP_MULADD: dispatch<OP_MULADD>(t, md, 0, a, b, c, out, n, s); break;
    case OP_MODMUL: dispatch<OP_MODMUL>(t, md, prm->R2, a, b, nullptr, out, n, s); break;
    default:
      if (prm->P < (1u << 30)) dispatch<OP_POW_LAZY>(t, md, prm->R1, a, b, nullptr, out, n, s);
      else dispatch<OP_POW>(t, md, prm->R1, a, b, nullptr, out, n, s);
      break;
  }
  return last_launch_status();
}

}  // namespace

ElemTune& elem_tune(int op) { return g_tune[op]; }

}  // namespace mont

using namespace mont;

extern "C" mont_status mont_to(const mont_params* prm, const uint32_t* d_in, uint32_t* d_out, size_t n,
                               void* stream) {
  return run(OP_TO, prm, d_in, nullptr, nullptr, d_out, n, stream);
}

extern "C" mont_status mont_from(const mont_params* prm, const uint32_t* d_in, uint32_t* d_out, size_t n,
                                 void* stream) {
  return run(OP_FROM, prm, d_in, nullptr, nullptr, d_out, n, stream);
}

extern "C" mont_status mont_mul(const mont_params* prm, const uint32_t* d_a, const uint32_t* d_b,
                                uint32_t* d_out, size_t n, void* stream) {
  return run(OP_MUL, prm, d_a, d_b, nullptr, d_out, n, stream);
}

extern "C" mont_status mont_muladd(const mont_params* prm, const uint32_t* d_a, const uint32_t* d_b,
                                   const uint32_t* d_c, uint32_t* d_out, size_t n, void* stream) {
  return run(OP_MULADD, prm, d_a, d_b, d_c, d_out, n, stream);
}

extern "C" mont_status mont_pow(const mont_params* prm, const uint32_t* d_base, const uint32_t* d_exp,
                                uint32_t* d_out, size_t n, void* stream) {
  return run(OP_POW, prm, d_base, d_exp, nullptr, d_out, n, stream);
}

extern "C" mont_status mont_modmul(const mont_params* prm, const uint32_t* d_a, const uint32_t* d_b,
                                   uint32_t* d_out, size_t n, void* stream) {
  return run(OP_MODMUL, prm, d_a, d_b, nullptr, d_out, n, stream);
}
