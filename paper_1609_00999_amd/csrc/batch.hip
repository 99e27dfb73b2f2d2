// batch.hip -- Montgomery products over a batch of vectors of uneven
// lengths, each with its own modulus, in one launch (Algorithm 2 of
// arXiv:1609.00999, section 3.1, elementwise).
#include <hip/hip_runtime.h>

#include <new>

#include "internal.hpp"
#include "modarith.hpp"

namespace mont {

namespace {

__device__ __forceinline__ bool aligned16_dev(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// ---------------------------------------------------------------------------
// Batches of vectors of uneven lengths, each with its own modulus, in one
// launch.  The flattened work is cut into tiles of kBatchTile residues that
// never straddle two vectors: vector v owns tiles [tile_begin[v],
// tile_begin[v+1]).  One workgroup takes one tile (workgroups stride over the
// tiles only beyond 2^20 of them), finds the tile's vector by binary search
// and streams it with 128-bit accesses when the vector's arrays are 16-byte
// aligned.
// ---------------------------------------------------------------------------

constexpr int kBatchThreads = 256;
constexpr int kBatchVpt = 4;            // 128-bit vectors per lane per tile
constexpr uint32_t kBatchTile = 4u * kBatchThreads * kBatchVpt;   // residues per tile

struct VecDev {
  const uint32_t* a;
  const uint32_t* b;
  uint32_t* out;
  uint64_t n;
  uint64_t tile_begin;
  uint32_t P, Pp;
};

// One tile: kBatchTile residues of vector v starting at its tile t.
__device__ __forceinline__ void batch_tile(const VecDev& v, uint64_t t) {
  const Mod md{v.P, v.Pp};
  const uint64_t e0 = (t - v.tile_begin) * kBatchTile;
  const uint64_t e1 = e0 + kBatchTile < v.n ? e0 + kBatchTile : v.n;
  const bool al = aligned16_dev(v.a) && aligned16_dev(v.b) && aligned16_dev(v.out);
  if (al && e1 - e0 == kBatchTile) {
    const v4u* va = reinterpret_cast<const v4u*>(v.a + e0);
    const v4u* vb = reinterpret_cast<const v4u*>(v.b + e0);
    v4u* vo = reinterpret_cast<v4u*>(v.out + e0);
    v4u x[kBatchVpt], y[kBatchVpt];
#pragma unroll
    for (int j = 0; j < kBatchVpt; j++) {
      x[j] = __builtin_nontemporal_load(va + j * kBatchThreads + threadIdx.x);
      y[j] = __builtin_nontemporal_load(vb + j * kBatchThreads + threadIdx.x);
    }
#pragma unroll
    for (int j = 0; j < kBatchVpt; j++) {
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

// Last v < nvec with begin[v] <= t (begin[0] = 0 <= t).
template <typename BEGIN>
__device__ __forceinline__ uint32_t tile_owner(BEGIN begin, uint32_t nvec, uint64_t t) {
  uint32_t lo = 0, hi = nvec - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (begin[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// tile_begin[v] repeats vecs[v].tile_begin in a contiguous array, so the
// binary search touches a few cache lines instead of one descriptor each.
__global__ __launch_bounds__(kBatchThreads) void k_batch_mul(const VecDev* vecs, const uint64_t* tile_begin,
                                                             uint32_t nvec, uint64_t ntiles) {
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const VecDev v = vecs[tile_owner(tile_begin, nvec, t)];
    batch_tile(v, t);
  }
}

// Small batches pass their descriptors by value in the kernel arguments, so
// a launch needs no upload before it: a serving loop's batches hold one or
// two vectors, and the host-to-device copy of their descriptors cost more
// latency than the products.
constexpr int kInlineVecs = 16;
struct InlineVecs {
  VecDev v[kInlineVecs];
  uint32_t nvec;
};

struct InlineBegin {
  const InlineVecs& iv;
  __device__ uint64_t operator[](uint32_t i) const { return iv.v[i].tile_begin; }
};

__global__ __launch_bounds__(kBatchThreads) void k_batch_mul_inline(InlineVecs iv, uint64_t ntiles) {
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint32_t o = tile_owner(InlineBegin{iv}, iv.nvec, t);
    batch_tile(iv.v[o], t);
  }
}

}  // namespace

}  // namespace mont

using namespace mont;

// The descriptors and the contiguous array of the vectors' first tiles share
// one device block (and one pinned staging block), so an update is one copy:
// count VecDev records, then count uint64 tile starts.
struct mont_batch {
  int cap = 0;
  int count = 0;
  uint64_t ntiles = 0;
  void* d_block = nullptr;
  void* h_block = nullptr;        // pinned staging
  hipEvent_t staged = nullptr;
  bool staged_pending = false;
  int grid = 0;
  InlineVecs inl;                 // the descriptors of a batch of at most kInlineVecs vectors
};
static_assert(sizeof(VecDev) % 8 == 0, "the tile starts follow the descriptors 8-byte aligned");

namespace {

void free_batch(mont_batch* b) {
  (void)hipFree(b->d_block);
  if (b->h_block) (void)hipHostFree(b->h_block);
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
  const size_t bytes = (sizeof(VecDev) + sizeof(uint64_t)) * (size_t)max_vectors;
  if (hipMalloc(&b->d_block, bytes) != hipSuccess ||
      hipHostMalloc(&b->h_block, bytes, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess) {
    free_batch(b);
    return MONT_ENOMEM;
  }
  // One workgroup per tile (the launch shape that streams best), striding
  // over tiles only beyond 2^20 of them.
  b->grid = 1 << 20;
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
  VecDev* hv = static_cast<VecDev*>(b->h_block);
  uint64_t* hbeg = reinterpret_cast<uint64_t*>(hv + count);
  uint64_t tiles = 0;
  for (int i = 0; i < count; i++) {
    const mont_vec_desc& d = descs[i];
    VecDev& v = hv[i];
    v.a = d.a;
    v.b = d.b;
    v.out = d.out;
    v.n = d.n;
    v.tile_begin = tiles;
    hbeg[i] = tiles;
    v.P = d.P;
    v.Pp = d.Pprime;
    tiles += (d.n + kBatchTile - 1) / kBatchTile;
  }
  b->count = count;
  b->ntiles = tiles;
  if (count > 0 && count <= kInlineVecs) {
    // launched with the descriptors by value: nothing to upload
    for (int i = 0; i < count; i++) b->inl.v[i] = hv[i];
    b->inl.nvec = (uint32_t)count;
    return MONT_OK;
  }
  if (count > 0) {
    hipStream_t s = as_stream(stream);
    if (hipMemcpyAsync(b->d_block, b->h_block, (sizeof(VecDev) + sizeof(uint64_t)) * count, hipMemcpyHostToDevice,
                       s) != hipSuccess ||
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
  if (b->count <= kInlineVecs) {
    hipLaunchKernelGGL(k_batch_mul_inline, dim3((unsigned)grid), dim3(kBatchThreads), 0, as_stream(stream), b->inl,
                       b->ntiles);
    return last_launch_status();
  }
  const VecDev* dv = static_cast<const VecDev*>(b->d_block);
  hipLaunchKernelGGL(k_batch_mul, dim3((unsigned)grid), dim3(kBatchThreads), 0, as_stream(stream), dv,
                     reinterpret_cast<const uint64_t*>(dv + b->count), (uint32_t)b->count, b->ntiles);
  return last_launch_status();
}

extern "C" mont_status mont_batch_destroy(mont_batch* b) {
  if (!b) return MONT_EINVAL;
  (void)hipDeviceSynchronize();
  free_batch(b);
  return MONT_OK;
}

