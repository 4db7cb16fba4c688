// dm_modes.hpp -- power of each probe mode, sum over pixels of |P_k|^2, the
// quantity behind the paper's rule for the number of probe modes (Section
// II: add modes in trial runs while each one carries at least 1% of the
// total intensity).
#pragma once
#include <hip/hip_runtime.h>

#include "dm_kernels.hpp"

namespace dmk {

// one block of 256 threads per mode; FP64 sum in a fixed order
__global__ __launch_bounds__(256) void k_mode_sums(const float2* __restrict__ P, int FF,
                                                   double* __restrict__ out) {
  __shared__ double red[256];
  const float2* __restrict__ Pk = P + (size_t)blockIdx.x * FF;
  double acc = 0.0;
  for (int p = threadIdx.x; p < FF; p += 256) acc += (double)cabs2(Pk[p]);
  acc = block_sum_d(acc, red);
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

}  // namespace dmk
