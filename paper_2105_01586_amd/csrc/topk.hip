// Error-driven mask growth (Section 3's error map e_i = (u_i - f_i)^2):
// - global top-k: the k non-mask pixels with the largest e_i, ties broken by
//   the lower linear index, returned in ascending index order;
// - the paper's per-triangle step: the k triangles of largest total error
//   (ties: lower triangle index) that still own an empty pixel, each giving
//   its empty pixel of largest e_i (ties: lower index).
//
// Radix select finds the k-th largest key in four passes of 16-bit digits
// (integer histograms, so counts are exact); pixels above that key are all
// taken, and among pixels equal to it the lowest indices fill the rest. A
// prefix sum over the selection flags writes the result in index order.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <mutex>
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

__global__ void k_excl_no_best(int64_t T, const int32_t* __restrict__ best,
                               uint8_t* __restrict__ excl) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < T) excl[t] = best[t] < 0;
}

__global__ void k_flag_best(int64_t k, const int32_t* __restrict__ sel_tri,
                            const int32_t* __restrict__ best, int32_t* __restrict__ flag) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < k) flag[best[sel_tri[j]]] = 1;
}

// Workspace of a selection over n keys (device, from the mesh).
struct SelectSpace {
  uint8_t* excl;  // n bytes (rounded to 256)
  int32_t *hist, *gt, *eq, *rank, *sel, *pos, *scan_tmp;
};

size_t select_space_bytes(int64_t n) {
  const size_t excl_bytes = ((size_t)n + 255) & ~(size_t)255;
  const size_t tmp_ints = (size_t)scan_tmp_ints(n + 1);
  return excl_bytes + sizeof(int32_t) * ((size_t)kBins + 5 * (size_t)(n + 1) + tmp_ints);
}

// Lays the workspace of a selection over n keys out from `base`
// (select_space_bytes(n) bytes, 256-byte aligned).
void select_space_carve(void* base, int64_t n, SelectSpace& W) {
  const size_t excl_bytes = ((size_t)n + 255) & ~(size_t)255;
  W.excl = (uint8_t*)base;
  W.hist = (int32_t*)((char*)base + excl_bytes);
  W.gt = W.hist + kBins;
  W.eq = W.gt + (n + 1);
  W.rank = W.eq + (n + 1);
  W.sel = W.rank + (n + 1);
  W.pos = W.sel + (n + 1);
  W.scan_tmp = W.pos + (n + 1);
}

int select_space(fi_mesh* M, int64_t n, SelectSpace& W) {
  const size_t need = select_space_bytes(n);
  if ((int64_t)need > M->topk_bytes) {
    void* p = nullptr;
    int rc = device_alloc(M, &p, need);
    if (rc) return rc;
    M->d_topk = p;
    M->topk_bytes = (int64_t)need;
  }
  select_space_carve(M->d_topk, n, W);
  return FI_OK;
}

// The k entries of largest key among those not excluded (ties: lower index),
// written in ascending index order to out. With fewer than k candidates,
// *taken < k of them (all) are written.
// h: host memory for one histogram (kBins ints).
int select_topk(hipStream_t st, int64_t n, const double* key, SelectSpace& W, int64_t k,
                int32_t* out, int64_t* taken, int32_t* h) {
  *taken = 0;
  if (k == 0 || n == 0) return FI_OK;
  uint64_t prefix = 0, hi_mask = 0;
  // candidates in total: a histogram of the top digit counts them all
  int64_t remaining = k;  // rank (1-based, from the top) still to locate
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 64 - kDigitBits * (pass + 1);
    hipLaunchKernelGGL(k_zero_i32, dim3(blocks(kBins)), dim3(kBlock), 0, st, (int64_t)kBins,
                       W.hist);
    int g = (int)std::min<int64_t>(blocks(n), 2048);
    hipLaunchKernelGGL(k_hist, dim3(g), dim3(kBlock), 0, st, n, key, W.excl, shift, prefix,
                       hi_mask, W.hist);
    FI_HIP_TRY(hipGetLastError());
    FI_HIP_TRY(hipMemcpyAsync(h, W.hist, sizeof(int32_t) * kBins, hipMemcpyDeviceToHost, st));
    FI_HIP_TRY(hipStreamSynchronize(st));
    if (pass == 0) {
      int64_t total = 0;
      for (int d = 0; d < kBins; ++d) total += h[d];
      if (total == 0) return FI_OK;
      if (total < remaining) remaining = total;
      *taken = remaining;
    }
    int64_t acc = 0;
    int d = kBins - 1;
    for (; d >= 0; --d) {
      if (acc + h[d] >= remaining) break;
      acc += h[d];
    }
    remaining -= acc;
    prefix |= (uint64_t)d << shift;
    hi_mask |= (uint64_t)(kBins - 1) << shift;
  }
  const uint64_t tau = prefix;  // the k-th largest key; `remaining` ties are needed
  hipLaunchKernelGGL(k_flags, dim3(blocks(n + 1)), dim3(kBlock), 0, st, n, key, W.excl, tau, W.gt,
                     W.eq);
  FI_HIP_TRY(hipGetLastError());
  int rc = scan_exclusive(st, W.eq, W.rank, n + 1, W.scan_tmp);
  if (rc) return rc;
  hipLaunchKernelGGL(k_select, dim3(blocks(n + 1)), dim3(kBlock), 0, st, n, W.gt, W.eq, W.rank,
                     (int32_t)remaining, W.sel);
  FI_HIP_TRY(hipGetLastError());
  rc = scan_exclusive(st, W.sel, W.pos, n + 1, W.scan_tmp);
  if (rc) return rc;
  hipLaunchKernelGGL(k_scatter, dim3(blocks(n)), dim3(kBlock), 0, st, n, W.sel, W.pos, out);
  FI_HIP_TRY(hipGetLastError());
  return FI_OK;
}

// The global top-k step on the workspace W (laid out for P keys) with the
// host histogram buffer h.
int topk_in(fi_mesh* M, const double* e, int64_t k, int32_t* out, SelectSpace& W, int32_t* h) {
  hipStream_t st = M->ctx->stream;
  const int64_t P = M->P;
  hipLaunchKernelGGL(k_zero_u8, dim3(blocks(P)), dim3(kBlock), 0, st, P, W.excl);
  hipLaunchKernelGGL(k_mark_mask, dim3(blocks(M->m)), dim3(kBlock), 0, st, (int)M->m,
                     M->d_mask_pix, W.excl);
  FI_HIP_TRY(hipGetLastError());
  int64_t taken = 0;
  int rc = select_topk(st, P, e, W, k, out, &taken, h);
  if (rc) return rc;
  if (taken < k) return fail(FI_E_INVALID, "top-k: fewer candidates than requested");
  FI_HIP_TRY(hipStreamSynchronize(st));
  return FI_OK;
}

}  // namespace

int topk_new_pixels(fi_mesh* M, const double* e, int64_t k, int32_t* out) {
  if (k == 0) return FI_OK;
  SelectSpace W;
  int rc = select_space(M, M->P, W);
  if (rc) return rc;
  std::vector<int32_t> h(kBins);
  return topk_in(M, e, k, out, W, h.data());
}

// Section 3's densification step: triangles in descending order of their
// total squared error, one new mask pixel in each (its empty pixel of
// largest error), k pixels in all.
int paper_densify_step(fi_mesh* M, const double* e, int64_t k, int32_t* out, int64_t* added) {
  *added = 0;
  if (k == 0) return FI_OK;
  hipStream_t st = M->ctx->stream;
  const int64_t T = M->T, P = M->P;
  // per-triangle error and best empty pixel (the pixel mask travels in the
  // selection workspace's byte array, sized for max(P, T))
  const int64_t n = std::max(P, T);
  SelectSpace W;
  int rc = select_space(M, n, W);
  if (rc) return rc;
  if (!M->d_tri_err) {
    if ((rc = device_alloc(M, (void**)&M->d_tri_err, (size_t)T * sizeof(double))) ||
        (rc = device_alloc(M, (void**)&M->d_tri_best, (size_t)T * sizeof(int32_t))) ||
        (rc = device_alloc(M, (void**)&M->d_sel_tri, (size_t)std::max<int64_t>(T, 1) *
                                                         sizeof(int32_t))))
      return rc;
  }
  hipLaunchKernelGGL(k_zero_u8, dim3(blocks(P)), dim3(kBlock), 0, st, P, W.excl);
  hipLaunchKernelGGL(k_mark_mask, dim3(blocks(M->m)), dim3(kBlock), 0, st, (int)M->m,
                     M->d_mask_pix, W.excl);
  FI_HIP_TRY(hipGetLastError());
  if ((rc = launch_tri_best(M, e, W.excl, M->d_tri_err, M->d_tri_best))) return rc;
  // exclusion over triangles: those without an empty pixel
  hipLaunchKernelGGL(k_excl_no_best, dim3(blocks(T)), dim3(kBlock), 0, st, T, M->d_tri_best,
                     W.excl);
  FI_HIP_TRY(hipGetLastError());
  int64_t taken = 0;
  std::vector<int32_t> h(kBins);
  if ((rc = select_topk(st, T, M->d_tri_err, W, k, M->d_sel_tri, &taken, h.data()))) return rc;
  // their pixels, in ascending pixel order: flag, scan, scatter over P
  int32_t* flag = W.gt;  // reuse (n + 1 ints each)
  hipLaunchKernelGGL(k_zero_i32, dim3(blocks(P + 1)), dim3(kBlock), 0, st, P + 1, flag);
  if (taken > 0)
    hipLaunchKernelGGL(k_flag_best, dim3(blocks(taken)), dim3(kBlock), 0, st, taken,
                       M->d_sel_tri, M->d_tri_best, flag);
  FI_HIP_TRY(hipGetLastError());
  if ((rc = scan_exclusive(st, flag, W.pos, P + 1, W.scan_tmp))) return rc;
  hipLaunchKernelGGL(k_scatter, dim3(blocks(P)), dim3(kBlock), 0, st, P, flag, W.pos, out);
  FI_HIP_TRY(hipGetLastError());
  FI_HIP_TRY(hipStreamSynchronize(st));
  *added = taken;
  return FI_OK;
}

}  // namespace fi

// Workspace of the allocation-free top-k entry point: a file-scope device
// array, one copy per GPU the library runs on, held until the process ends.
// In host code `scratch` only names the symbol; its device address comes from
// hipGetSymbolAddress, once per device (fi::scratch_on).
constexpr int64_t kNoAllocMaxPixels = (int64_t)1 << 20;  // a 1024 x 1024 image
constexpr size_t kScratchBytes = (size_t)24 << 20;       // >= select_space_bytes(2^20)
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace fi {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;          // held for a whole call of the entry point
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` on each device
int32_t g_noalloc_hist[kBins];     // host copy of one histogram

// Device address of `scratch` on `dev` (the current device); g_noalloc_mu held.
int scratch_on(int dev, void** ptr) {
  if (dev < 0 || dev >= kMaxDevices) return fail(FI_E_INVALID, "device index out of range");
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(FI_E_HIP, std::string("scratch symbol address: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return FI_OK;
}

}  // namespace
}  // namespace fi

using namespace fi;

extern "C" int fi_topk_new_pixels_noalloc(fi_mesh* M, const double* e_dev, int64_t k,
                                          int32_t* out_dev) {
  if (!M || !M->ctx) return fail(FI_E_INVALID, "mesh is NULL");
  if (!e_dev || (!out_dev && k > 0)) return fail(FI_E_INVALID, "e_dev and out_dev are required");
  if (k < 0 || k > M->P - M->m) return fail(FI_E_INVALID, "k out of range");
  if (M->P > kNoAllocMaxPixels || select_space_bytes(M->P) > kScratchBytes)
    return fail(FI_E_INVALID, "fi_topk_new_pixels_noalloc: more than 2^20 pixels");
  if (k == 0) return FI_OK;
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  void* base = nullptr;
  int rc = scratch_on(M->ctx->device, &base);
  if (rc) return rc;
  SelectSpace W;
  select_space_carve(base, M->P, W);
  return topk_in(M, e_dev, k, out_dev, W, g_noalloc_hist);
}
