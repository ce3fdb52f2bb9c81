// Fixed-order combination of per-sub-lane sums in the reduction kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace epic {

// Adds the NV values of the sub-lanes of each pixel of a 256-thread block in
// sub-lane order; the result is valid in sub-lane 0.  red: [NV][256].
template <int NV>
__device__ __forceinline__ void combine_sublanes(double (&s)[NV], int sub, int ppb, int j, int lp,
                                                 double* red) {
  if (sub == 1) return;
#pragma unroll
  for (int u = 0; u < NV; ++u) red[u * 256 + threadIdx.x] = s[u];
  __syncthreads();
  if (j == 0) {
#pragma unroll
    for (int u = 0; u < NV; ++u) {
      double t = red[u * 256 + lp];
      for (int q = 1; q < sub; ++q) t += red[u * 256 + q * ppb + lp];
      s[u] = t;
    }
  }
}

}  // namespace epic
