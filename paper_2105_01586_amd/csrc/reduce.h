// Fixed-order block reductions (block_sum: 256-thread blocks, four wave64s;
// block_sum_once: DPP within waves, one barrier).
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

// Sum over the 64 lanes of a wave, every lane receiving the same bits: DPP
// swaps within each 16-lane row (neighbours, pairs, half-row and row
// mirrors; each step adds two equal partial sums, in either order), then the
// four row sums in row order.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int lo2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  const int hi2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi2, lo2);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

template <int NC>
__device__ __forceinline__ void wave_sum(double (&v)[NC]) {
#pragma unroll
  for (int c = 0; c < NC; ++c) v[c] += dpp_move<0xB1>(v[c]);   // lanes i, i ^ 1
#pragma unroll
  for (int c = 0; c < NC; ++c) v[c] += dpp_move<0x4E>(v[c]);   // lanes i, i ^ 2
#pragma unroll
  for (int c = 0; c < NC; ++c) v[c] += dpp_move<0x141>(v[c]);  // half-row mirror
#pragma unroll
  for (int c = 0; c < NC; ++c) v[c] += dpp_move<0x140>(v[c]);  // row mirror
#pragma unroll
  for (int c = 0; c < NC; ++c)
    v[c] = ((read_lane(v[c], 0) + read_lane(v[c], 16)) + read_lane(v[c], 32)) +
           read_lane(v[c], 48);
}

// Sum over a block of NW waves, every thread receiving the total (waves in
// wave order). One barrier; lds (NW * NC doubles) must not be written again
// before every thread has read it.
template <int NC, int NW>
__device__ __forceinline__ void block_sum_once(double (&v)[NC], double* lds) {
  wave_sum<NC>(v);
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
}

}  // namespace fi
