// Workgroup sums in a fixed order (the same result on every run).
#pragma once
#include <hip/hip_runtime.h>

namespace demag {

// Sum of v over the workgroup, returned on thread 0 (0 on the others): a
// butterfly over each wavefront, then the wavefronts' sums in order.  red
// holds one entry per wavefront and is written only after a barrier, so
// consecutive calls may share it.  Every thread of the workgroup must call.
template <typename Tv>
__device__ __forceinline__ Tv block_sum(Tv v, Tv* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  Tv s = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

}  // namespace demag
