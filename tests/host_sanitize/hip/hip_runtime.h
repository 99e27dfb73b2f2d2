// Host-only stand-in for <hip/hip_runtime.h>, for sanitizer builds of
// libmont's host code on a machine without a GPU (tests/host_sanitize).
//
// "Device" memory is host memory from malloc, copies are memcpy (so the
// address sanitizer checks both ranges of every copy), events and streams
// are inert handles, and a kernel launch runs the kernel on the host, one
// workgroup and one lane at a time.  That emulation is exact only for
// kernels without barriers, cross-lane operations or shared memory, which
// is what the harnesses launch.
#pragma once

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
struct hip_stub_idx {
  unsigned x = 0, y = 0, z = 0;
};
inline hip_stub_idx threadIdx, blockIdx, blockDim, gridDim;

typedef int hipError_t;
#define hipSuccess 0
#define hipErrorOutOfMemory 2
typedef struct hip_stub_stream* hipStream_t;
typedef struct hip_stub_event {
  int recorded;
}* hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToHost, hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice };
#define hipHostMallocDefault 0u
#define hipEventDisableTiming 2u

// counters the harness reads
inline long hip_stub_live_allocs = 0;
inline long hip_stub_copies = 0;
inline long hip_stub_launches = 0;

inline hipError_t hipMalloc(void** p, size_t n) {
  *p = malloc(n ? n : 1);
  if (!*p) return hipErrorOutOfMemory;
  hip_stub_live_allocs++;
  return hipSuccess;
}
template <typename T>
inline hipError_t hipMalloc(T** p, size_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), n);
}
inline hipError_t hipFree(void* p) {
  if (p) hip_stub_live_allocs--;
  free(p);
  return hipSuccess;
}
inline hipError_t hipHostMalloc(void** p, size_t n, unsigned) { return hipMalloc(p, n); }
inline hipError_t hipHostFree(void* p) { return hipFree(p); }
inline hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
  memcpy(dst, src, n);
  hip_stub_copies++;
  return hipSuccess;
}
inline hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind k) {
  return hipMemcpyAsync(dst, src, n, k, nullptr);
}
inline hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = new hip_stub_event{0};
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  e->recorded = 1;
  return hipSuccess;
}
inline hipError_t hipEventSynchronize(hipEvent_t e) { return e->recorded ? hipSuccess : 1; }
inline hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
inline hipError_t hipGetLastError() { return hipSuccess; }
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }

#define hipLaunchKernelGGL(K, G, B, SHM, S, ...)                             \
  do {                                                                      \
    const dim3 hip_stub_g = (G), hip_stub_b = (B);                          \
    hip_stub_launches++;                                                    \
    gridDim.x = hip_stub_g.x;                                               \
    blockDim.x = hip_stub_b.x;                                              \
    for (unsigned hip_stub_i = 0; hip_stub_i < hip_stub_g.x; hip_stub_i++)  \
      for (unsigned hip_stub_t = 0; hip_stub_t < hip_stub_b.x; hip_stub_t++) { \
        blockIdx.x = hip_stub_i;                                            \
        threadIdx.x = hip_stub_t;                                           \
        K(__VA_ARGS__);                                                     \
      }                                                                     \
  } while (0)
