// Fixed-order block reductions (block_sum: 256-thread blocks, four wave64s).
// The result depends only on the inputs and their positions, never on
// scheduling, so every reduction in the library is reproducible run to run.
#pragma once

#include <hip/hip_runtime.h>

namespace fi {

// Sum over a block of NW wave64s; every thread receives the total. Waves
// are combined in wave order. lds must hold NW * NC doubles.
template <int NC, int NW>
__device__ __forceinline__ void block_sum_w(double (&v)[NC], double* lds) {
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
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double t = lds[c];
#pragma unroll
    for (int w = 1; w < NW; ++w) t += lds[w * NC + c];
    v[c] = t;
  }
  __syncthreads();
}

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
