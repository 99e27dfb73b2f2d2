// check.hip -- device-side operand range check, the checked mode of the
// operand contract: Algorithm 2 (arXiv:1609.00999, section 3.1) needs
// a_bar*b_bar < R P, which the library guarantees by requiring operands in
// [0, P).  The check reads the operand once more from HBM and flags any
// element >= P; it is a debugging aid, not part of the timed path.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "modarith.hpp"

namespace mont {
namespace {

constexpr int CHECK_BLOCK = 256;

__global__ __launch_bounds__(CHECK_BLOCK) void k_check_range(uint32_t P, const uint32_t* x, size_t n,
                                                             int32_t* status) {
  const size_t stride = (size_t)gridDim.x * CHECK_BLOCK;
  const size_t tid = (size_t)blockIdx.x * CHECK_BLOCK + threadIdx.x;
  bool bad = false;
  size_t head = 0;
  if ((((uintptr_t)x) & 15u) == 0) {
    const size_t nvec = n >> 2;
    const v4u* vx = reinterpret_cast<const v4u*>(x);
    for (size_t i = tid; i < nvec; i += stride) {
      const v4u v = __builtin_nontemporal_load(vx + i);
      bad |= (v.x >= P) | (v.y >= P) | (v.z >= P) | (v.w >= P);
    }
    head = nvec << 2;
  }
  for (size_t i = head + tid; i < n; i += stride) bad |= x[i] >= P;
  // Every offending lane stores the same value; the store is a vector
  // (per-lane) global store, so its order against other lanes is irrelevant.
  if (bad) __hip_atomic_store(status, (int32_t)MONT_ERANGE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace
}  // namespace mont

using namespace mont;

extern "C" mont_status mont_check_range(uint32_t P, const uint32_t* d_x, size_t n, int32_t* d_status, void* stream) {
  if (P == 0 || !d_status) return MONT_EINVAL;
  if (n == 0) return MONT_OK;
  if (!d_x) return MONT_EINVAL;
  if ((((uintptr_t)d_status) & 3u) != 0) return MONT_EINVAL;
  (void)hipGetLastError();
  size_t blocks = (n / 4 + CHECK_BLOCK - 1) / CHECK_BLOCK;
  if (blocks < 1) blocks = 1;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_check_range, dim3((unsigned)blocks), dim3(CHECK_BLOCK), 0, as_stream(stream), P, d_x, n,
                     d_status);
  return last_launch_status();
}
