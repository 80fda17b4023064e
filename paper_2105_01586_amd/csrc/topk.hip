// Global top-k mask growth: choose the k non-mask pixels with the largest
// pointwise error e_i = (u_i - f_i)^2 (Section 3's error map), ties broken by
// the lower linear index, returned in ascending index order.
//
// Radix select finds the k-th largest key in four passes of 16-bit digits
// (integer histograms, so counts are exact); pixels above that key are all
// taken, and among pixels equal to it the lowest indices fill the rest. A
// prefix sum over the selection flags writes the result in index order.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

#include "internal.h"

namespace fi {

namespace {

constexpr int kDigitBits = 16;
constexpr int kBins = 1 << kDigitBits;

// Monotone map from double to uint64 (larger double -> larger key).
__device__ __forceinline__ uint64_t order_key(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ void k_mark_mask(int m, const int32_t* __restrict__ pix, uint8_t* __restrict__ is_mask) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) is_mask[pix[j]] = 1;
}

__global__ void k_zero_u8(int64_t n, uint8_t* __restrict__ a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

__global__ void k_zero_i32(int64_t n, int32_t* __restrict__ a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

// Histogram of digit `shift` over candidates whose bits above it equal `prefix`.
__global__ __launch_bounds__(kBlock) void k_hist(int64_t P, const double* __restrict__ e,
                                                 const uint8_t* __restrict__ is_mask, int shift,
                                                 uint64_t prefix, uint64_t hi_mask,
                                                 int32_t* __restrict__ hist) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < P;
       i += (int64_t)gridDim.x * kBlock) {
    if (is_mask[i]) continue;
    const uint64_t k = order_key(e[i]);
    if ((k & hi_mask) != prefix) continue;
    atomicAdd(&hist[(k >> shift) & (kBins - 1)], 1);
  }
}

__global__ __launch_bounds__(kBlock) void k_flags(int64_t P, const double* __restrict__ e,
                                                  const uint8_t* __restrict__ is_mask,
                                                  uint64_t tau, int32_t* __restrict__ gt,
                                                  int32_t* __restrict__ eq) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < P) {
    const uint64_t k = order_key(e[i]);
    const int cand = !is_mask[i];
    gt[i] = cand && k > tau;
    eq[i] = cand && k == tau;
  }
  if (i == P) { gt[P] = 0; eq[P] = 0; }
}

__global__ __launch_bounds__(kBlock) void k_select(int64_t P, const int32_t* __restrict__ gt,
                                                   const int32_t* __restrict__ eq,
                                                   const int32_t* __restrict__ eq_rank,
                                                   int32_t need, int32_t* __restrict__ sel) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < P) sel[i] = gt[i] || (eq[i] && eq_rank[i] < need);
  if (i == P) sel[P] = 0;
}

__global__ __launch_bounds__(kBlock) void k_scatter(int64_t P, const int32_t* __restrict__ sel,
                                                    const int32_t* __restrict__ pos,
                                                    int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < P && sel[i]) out[pos[i]] = (int32_t)i;
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int topk_new_pixels(fi_mesh* M, const double* e, int64_t k, int32_t* out) {
  if (k == 0) return FI_OK;
  hipStream_t st = M->ctx->stream;
  const int64_t P = M->P;
  // workspace: is_mask (P bytes, rounded), hist, gt, eq, rank, sel, pos
  const size_t mask_bytes = ((size_t)P + 255) & ~(size_t)255;
  const size_t tmp_ints = (size_t)scan_tmp_ints(P + 1);
  const size_t need =
      mask_bytes + sizeof(int32_t) * ((size_t)kBins + 5 * (size_t)(P + 1) + tmp_ints);
  if ((int64_t)need > M->topk_bytes) {
    void* p = nullptr;
    int rc = device_alloc(M, &p, need);
    if (rc) return rc;
    M->d_topk = p;
    M->topk_bytes = (int64_t)need;
  }
  uint8_t* is_mask = (uint8_t*)M->d_topk;
  int32_t* hist = (int32_t*)((char*)M->d_topk + mask_bytes);
  int32_t* gt = hist + kBins;
  int32_t* eq = gt + (P + 1);
  int32_t* rank = eq + (P + 1);
  int32_t* sel = rank + (P + 1);
  int32_t* pos = sel + (P + 1);
  int32_t* scan_tmp = pos + (P + 1);

  hipLaunchKernelGGL(k_zero_u8, dim3(blocks(P)), dim3(kBlock), 0, st, P, is_mask);
  hipLaunchKernelGGL(k_mark_mask, dim3(blocks(M->m)), dim3(kBlock), 0, st, (int)M->m,
                     M->d_mask_pix, is_mask);
  FI_HIP_TRY(hipGetLastError());

  std::vector<int32_t> h(kBins);
  uint64_t prefix = 0, hi_mask = 0;
  int64_t remaining = k;  // rank (1-based, from the top) still to locate
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 64 - kDigitBits * (pass + 1);
    hipLaunchKernelGGL(k_zero_i32, dim3(blocks(kBins)), dim3(kBlock), 0, st, (int64_t)kBins, hist);
    int g = (int)std::min<int64_t>(blocks(P), 2048);
    hipLaunchKernelGGL(k_hist, dim3(g), dim3(kBlock), 0, st, P, e, is_mask, shift, prefix, hi_mask,
                       hist);
    FI_HIP_TRY(hipGetLastError());
    FI_HIP_TRY(hipMemcpyAsync(h.data(), hist, sizeof(int32_t) * kBins, hipMemcpyDeviceToHost, st));
    FI_HIP_TRY(hipStreamSynchronize(st));
    int64_t acc = 0;
    int d = kBins - 1;
    for (; d >= 0; --d) {
      if (acc + h[d] >= remaining) break;
      acc += h[d];
    }
    if (d < 0) return fail(FI_E_INVALID, "top-k: fewer candidates than requested");
    remaining -= acc;
    prefix |= (uint64_t)d << shift;
    hi_mask |= (uint64_t)(kBins - 1) << shift;
  }
  const uint64_t tau = prefix;  // the k-th largest key; `remaining` ties are needed
  hipLaunchKernelGGL(k_flags, dim3(blocks(P + 1)), dim3(kBlock), 0, st, P, e, is_mask, tau, gt, eq);
  FI_HIP_TRY(hipGetLastError());
  int rc = scan_exclusive(st, eq, rank, P + 1, scan_tmp);
  if (rc) return rc;
  hipLaunchKernelGGL(k_select, dim3(blocks(P + 1)), dim3(kBlock), 0, st, P, gt, eq, rank,
                     (int32_t)remaining, sel);
  FI_HIP_TRY(hipGetLastError());
  rc = scan_exclusive(st, sel, pos, P + 1, scan_tmp);
  if (rc) return rc;
  hipLaunchKernelGGL(k_scatter, dim3(blocks(P)), dim3(kBlock), 0, st, P, sel, pos, out);
  FI_HIP_TRY(hipGetLastError());
  FI_HIP_TRY(hipStreamSynchronize(st));
  return FI_OK;
}

}  // namespace fi
