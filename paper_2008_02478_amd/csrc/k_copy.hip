// A plain streaming copy: the HBM read + write rate the device reaches on a
// trivially bandwidth-bound kernel, against which the field passes' byte
// rates are compared (alongside the 8 TB/s data-sheet figure).  Each thread
// moves UNROLL 16-byte vectors per step, all loads issued before the stores,
// so that enough bytes are in flight per CU.
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace demag {

constexpr int COPY_THREADS = 256;
constexpr int COPY_UNROLL = 4;
typedef float vec4 __attribute__((ext_vector_type(4)));   // 16 bytes, a native vector for the nontemporal builtins

__global__ void __launch_bounds__(COPY_THREADS) k_stream_copy(const vec4* __restrict__ src,
                                                              vec4* __restrict__ dst, size_t n) {
  const size_t step = (size_t)gridDim.x * COPY_THREADS * COPY_UNROLL;
  size_t i = (size_t)blockIdx.x * COPY_THREADS * COPY_UNROLL + threadIdx.x;
  for (; i + (COPY_UNROLL - 1) * COPY_THREADS < n; i += step) {
    vec4 v[COPY_UNROLL];
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) v[u] = __builtin_nontemporal_load(src + i + u * COPY_THREADS);
#pragma unroll
    for (int u = 0; u < COPY_UNROLL; ++u) __builtin_nontemporal_store(v[u], dst + i + u * COPY_THREADS);
  }
  // the ragged end: this thread's remaining vectors of its last step
  for (int u = 0; u < COPY_UNROLL; ++u)
    if (i + u * COPY_THREADS < n) dst[i + u * COPY_THREADS] = src[i + u * COPY_THREADS];
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t n = bytes / sizeof(vec4);
  if (n == 0) return hipSuccess;
  size_t blocks = (n + (size_t)COPY_THREADS * COPY_UNROLL - 1) / ((size_t)COPY_THREADS * COPY_UNROLL);
  if (blocks > 4096) blocks = 4096;   // 16 workgroups per CU, grid-stride beyond
  hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(COPY_THREADS), 0, s,
                     static_cast<const vec4*>(src), static_cast<vec4*>(dst), n);
  return hipGetLastError();
}

}  // namespace demag
