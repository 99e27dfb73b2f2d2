// elementwise.hip -- streaming Montgomery kernels: residue conversion,
// products, fused product-plus-sum and powers over device arrays.
//
// Each lane applies Algorithm 2 (arXiv:1609.00999, section 3.1) to four
// residues fetched with one 128-bit load; a wavefront therefore covers 256
// contiguous residues per load instruction, and the kernels are bound by HBM
// bandwidth (mont_pow excepted, which is bound by the vector ALU).
#include <hip/hip_runtime.h>

#include <new>

#include "internal.hpp"
#include "modarith.hpp"

namespace mont {

namespace {

__device__ __forceinline__ bool aligned16_dev(const void* p) { return ((uintptr_t)p & 15u) == 0; }

template <bool NT>
__device__ __forceinline__ v4u ld(const v4u* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT>
__device__ __forceinline__ void st(v4u* p, v4u v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
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

// Scalar operation applied per element.
template <int OP>
__device__ __forceinline__ uint32_t elem_op(uint32_t a, uint32_t b, uint32_t c, Mod md, uint32_t kc) {
  if constexpr (OP == OP_TO) return mmul(a, kc, md);             // REDC(a * R^2 mod P)
  else if constexpr (OP == OP_FROM) return redc((uint64_t)a, md); // REDC(a * 1)
  else if constexpr (OP == OP_MUL) return mmul(a, b, md);
  else if constexpr (OP == OP_MULADD) return madd(mmul(a, b, md), c, md.P);
  else return pow_win2(a, b, md, kc);                             // kc = residue of 1
}

template <int OP>
constexpr int n_inputs() { return OP == OP_TO || OP == OP_FROM ? 1 : (OP == OP_MULADD ? 3 : 2); }

// Vector kernel: element i of every array is read once and the result
// written once.  Workgroup w handles vectors [w*BLOCK*VPT, (w+1)*BLOCK*VPT),
// lane l vector w*BLOCK*VPT + j*BLOCK + l for j < VPT (coalesced per j);
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
  const v4u* va = reinterpret_cast<const v4u*>(a);
  const v4u* vb = reinterpret_cast<const v4u*>(b);
  const v4u* vc = reinterpret_cast<const v4u*>(c);
  v4u* vo = reinterpret_cast<v4u*>(out);
  for (size_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const size_t base = tile * ((size_t)BLOCK * VPT) + threadIdx.x;
    v4u x[VPT], y[VPT], z[VPT];
#pragma unroll
    for (int j = 0; j < VPT; j++) {
      const size_t i = base + (size_t)j * BLOCK;
      if (i < nvec) {
        x[j] = ld<NT>(va + i);
        if constexpr (NIN >= 2) y[j] = ld<NT>(vb + i);
        if constexpr (NIN >= 3) z[j] = ld<NT>(vc + i);
      }
    }
#pragma unroll
    for (int j = 0; j < VPT; j++) {
      const size_t i = base + (size_t)j * BLOCK;
      if (i < nvec) {
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
        st<NT>(vo + i, r);
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
  MONT_CASE(256, 1, true) MONT_CASE(256, 2, true) MONT_CASE(256, 4, true)
  MONT_CASE(512, 1, true) MONT_CASE(512, 2, true) MONT_CASE(512, 4, true)
  MONT_CASE(256, 1, false) MONT_CASE(256, 2, false) MONT_CASE(256, 4, false)
  MONT_CASE(512, 1, false) MONT_CASE(512, 2, false) MONT_CASE(512, 4, false)
#undef MONT_CASE
  launch_v4<OP, 256, 1, true>(md, kc, a, b, c, out, n, s);
}

ElemTune g_tune[OP_COUNT] = {
    {256, 1, 1}, {256, 1, 1}, {256, 1, 1}, {256, 1, 1}, {256, 1, 1},
};

mont_status run(int op, const mont_params* prm, const uint32_t* a, const uint32_t* b, const uint32_t* c,
                uint32_t* out, size_t n, void* stream) {
  if (!params_ok(prm)) return MONT_EINVAL;
  if (n == 0) return MONT_OK;
  if (!a || !out) return MONT_EINVAL;
  if ((op == OP_MUL || op == OP_MULADD || op == OP_POW) && !b) return MONT_EINVAL;
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
    default: dispatch<OP_POW>(t, md, prm->R1, a, b, nullptr, out, n, s); break;
  }
  return last_launch_status();
}

// ---------------------------------------------------------------------------
// Batches of vectors of uneven lengths, each with its own modulus, in one
// persistent launch.  The flattened work is cut into tiles of kBatchTile
// residues that never straddle two vectors: vector v owns tiles
// [tile_begin[v], tile_begin[v+1]).  A workgroup finds its tile's vector by
// binary search and streams that tile with 128-bit accesses when the
// vector's arrays are 16-byte aligned.
// ---------------------------------------------------------------------------

constexpr int kBatchThreads = 256;
constexpr uint32_t kBatchTile = 4096;   // residues per tile: 4 per lane, 4 rounds

struct VecDev {
  const uint32_t* a;
  const uint32_t* b;
  uint32_t* out;
  uint64_t n;
  uint64_t tile_begin;
  uint32_t P, Pp;
};

__global__ __launch_bounds__(kBatchThreads) void k_batch_mul(const VecDev* vecs, uint32_t nvec, uint64_t ntiles) {
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    uint32_t lo = 0, hi = nvec - 1;             // last v with tile_begin[v] <= t
    while (lo < hi) {
      const uint32_t mid = (lo + hi + 1) >> 1;
      if (vecs[mid].tile_begin <= t) lo = mid;
      else hi = mid - 1;
    }
    const VecDev v = vecs[lo];
    const Mod md{v.P, v.Pp};
    const uint64_t e0 = (t - v.tile_begin) * kBatchTile;
    const uint64_t e1 = e0 + kBatchTile < v.n ? e0 + kBatchTile : v.n;
    const bool al = aligned16_dev(v.a) && aligned16_dev(v.b) && aligned16_dev(v.out);
    if (al && e1 - e0 == kBatchTile) {
      const v4u* va = reinterpret_cast<const v4u*>(v.a + e0);
      const v4u* vb = reinterpret_cast<const v4u*>(v.b + e0);
      v4u* vo = reinterpret_cast<v4u*>(v.out + e0);
      v4u x[4], y[4];
#pragma unroll
      for (int j = 0; j < 4; j++) {
        x[j] = __builtin_nontemporal_load(va + j * kBatchThreads + threadIdx.x);
        y[j] = __builtin_nontemporal_load(vb + j * kBatchThreads + threadIdx.x);
      }
#pragma unroll
      for (int j = 0; j < 4; j++) {
        v4u r;
        r.x = mmul(x[j].x, y[j].x, md);
        r.y = mmul(x[j].y, y[j].y, md);
        r.z = mmul(x[j].z, y[j].z, md);
        r.w = mmul(x[j].w, y[j].w, md);
        __builtin_nontemporal_store(r, vo + j * kBatchThreads + threadIdx.x);
      }
    } else {
      for (uint64_t e = e0 + threadIdx.x; e < e1; e += kBatchThreads) v.out[e] = mmul(v.a[e], v.b[e], md);
    }
  }
}

}  // namespace

ElemTune& elem_tune(int op) { return g_tune[op]; }

}  // namespace mont

using namespace mont;

struct mont_batch {
  int cap = 0;
  int count = 0;
  uint64_t ntiles = 0;
  VecDev* d_vecs = nullptr;
  VecDev* h_vecs = nullptr;       // pinned staging
  hipEvent_t staged = nullptr;
  bool staged_pending = false;
  int grid = 0;
};

namespace {

void free_batch(mont_batch* b) {
  (void)hipFree(b->d_vecs);
  if (b->h_vecs) (void)hipHostFree(b->h_vecs);
  if (b->staged) (void)hipEventDestroy(b->staged);
  delete b;
}

}  // namespace

extern "C" mont_status mont_batch_reserve(int max_vectors, mont_batch** out) {
  if (!out || max_vectors < 1) return MONT_EINVAL;
  *out = nullptr;
  mont_batch* b = new (std::nothrow) mont_batch;
  if (!b) return MONT_ENOMEM;
  b->cap = max_vectors;
  if (hipMalloc(&b->d_vecs, sizeof(VecDev) * max_vectors) != hipSuccess ||
      hipHostMalloc((void**)&b->h_vecs, sizeof(VecDev) * max_vectors, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess) {
    free_batch(b);
    return MONT_ENOMEM;
  }
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  b->grid = cus * 8;
  *out = b;
  return MONT_OK;
}

extern "C" mont_status mont_batch_update(mont_batch* b, const mont_vec_desc* descs, int count, void* stream) {
  if (!b || count < 0 || (count > 0 && !descs)) return MONT_EINVAL;
  if (count > b->cap) return MONT_ERANGE;
  for (int i = 0; i < count; i++) {
    const mont_vec_desc& d = descs[i];
    mont_params prm{d.P, d.Pprime, 0, 0, 0};
    if (!params_ok(&prm)) return MONT_EINVAL;
    if (d.n > 0 && (!d.a || !d.b || !d.out)) return MONT_EINVAL;
  }
  if (b->staged_pending && hipEventSynchronize(b->staged) != hipSuccess) return MONT_EHIP;
  b->staged_pending = false;
  uint64_t tiles = 0;
  for (int i = 0; i < count; i++) {
    const mont_vec_desc& d = descs[i];
    VecDev& v = b->h_vecs[i];
    v.a = d.a;
    v.b = d.b;
    v.out = d.out;
    v.n = d.n;
    v.tile_begin = tiles;
    v.P = d.P;
    v.Pp = d.Pprime;
    tiles += (d.n + kBatchTile - 1) / kBatchTile;
  }
  b->count = count;
  b->ntiles = tiles;
  if (count > 0) {
    hipStream_t s = as_stream(stream);
    if (hipMemcpyAsync(b->d_vecs, b->h_vecs, sizeof(VecDev) * count, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipEventRecord(b->staged, s) != hipSuccess)
      return MONT_EHIP;
    b->staged_pending = true;
  }
  return MONT_OK;
}

extern "C" mont_status mont_batch_mul(const mont_batch* b, void* stream) {
  if (!b) return MONT_EINVAL;
  if (b->count == 0 || b->ntiles == 0) return MONT_OK;
  (void)hipGetLastError();
  uint64_t grid = b->ntiles < (uint64_t)b->grid ? b->ntiles : (uint64_t)b->grid;
  hipLaunchKernelGGL(k_batch_mul, dim3((unsigned)grid), dim3(kBatchThreads), 0, as_stream(stream), b->d_vecs,
                     (uint32_t)b->count, b->ntiles);
  return last_launch_status();
}

extern "C" mont_status mont_batch_destroy(mont_batch* b) {
  if (!b) return MONT_EINVAL;
  (void)hipDeviceSynchronize();
  free_batch(b);
  return MONT_OK;
}

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
