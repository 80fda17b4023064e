// Fixed-order block reductions for 256-thread blocks (four wave64s).
// The result depends only on the inputs and their positions, never on
// scheduling, so every reduction in the library is reproducible run to run.
#pragma once

#include <hip/hip_runtime.h>

namespace fi {

template <int NC>
__device__ __forceinline__ void block_sum(double (&v)[NC], double* lds /* >= 4 * NC */) {
  // within each wave64: tree over lane offsets 32, 16, ..., 1
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] += __shfl_down(v[c], off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int c = 0; c < NC; ++c) lds[wave * NC + c] = v[c];
  }
  __syncthreads();
  // every thread gets the total of the four waves, summed in wave order
#pragma unroll
  for (int c = 0; c < NC; ++c) v[c] = ((lds[c] + lds[NC + c]) + lds[2 * NC + c]) + lds[3 * NC + c];
  __syncthreads();
}

}  // namespace fi
