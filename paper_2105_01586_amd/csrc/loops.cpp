// Multi-call procedures built on the single-mesh calls: error-driven mask
// growth (Section 3), by the global top-k rule or the paper's per-triangle
// step.
#include <algorithm>
#include <cstring>
#include <iterator>
#include <vector>

#include "internal.h"

namespace fi {
namespace {

struct DevMem {
  void* p = nullptr;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
};

struct Event {
  hipEvent_t e = nullptr;
  ~Event() {
    if (e) (void)hipEventDestroy(e);
  }
};

}  // namespace
}  // namespace fi

using namespace fi;

namespace {

// Shared loop of fi_grow_mask and fi_densify: rule 0 adds the global top-k
// (exactly k_add per round), rule 1 the per-triangle step (up to k_add).
// With `unknowns` (the Delaunay mesh), every round triangulates the current
// mask and the unknown vertices that are not mask pixels yet: a chosen pixel
// that was an unknown vertex becomes a mask vertex.
int densify_loop(fi_ctx* ctx, int side, const uint8_t* f_dev, const int32_t* mask0, int64_t m0,
                 int64_t k_add, int rounds, int rule, const fi_solve_opts* opts, int32_t* mask_out,
                 double* mse_out, double* gpu_ms_out, int64_t* total_out,
                 const std::vector<int32_t>* unknowns = nullptr) {
  if (!ctx || !f_dev || !mask0 || !mask_out || !mse_out)
    return fail(FI_E_INVALID, "densify: NULL argument");
  if (side < 2 || k_add < 0 || rounds < 0) return fail(FI_E_INVALID, "densify: bad sizes");
  if (rule != FI_DENSIFY_TOPK && rule != FI_DENSIFY_TRIANGLES)
    return fail(FI_E_INVALID, "densify: unknown rule");
  const int64_t P = (int64_t)side * side;
  if (m0 + (int64_t)rounds * k_add > P) return fail(FI_E_INVALID, "densify: mask would exceed the image");
  FI_HIP_TRY(hipSetDevice(ctx->device));
  DevMem u, e, sel;
  FI_HIP_TRY(hipMalloc(&u.p, (size_t)P * sizeof(double)));
  FI_HIP_TRY(hipMalloc(&e.p, (size_t)P * sizeof(double)));
  FI_HIP_TRY(hipMalloc(&sel.p, (size_t)std::max<int64_t>(k_add, 1) * sizeof(int32_t)));
  Event t0, t1;
  if (gpu_ms_out) {
    FI_HIP_TRY(hipEventCreate(&t0.e));
    FI_HIP_TRY(hipEventCreate(&t1.e));
  }
  std::vector<int32_t> mask(mask0, mask0 + m0);
  std::memcpy(mask_out, mask0, (size_t)m0 * sizeof(int32_t));
  int64_t written = m0;
  std::vector<int32_t> add((size_t)std::max<int64_t>(k_add, 1));
  std::vector<int32_t> unk;
  for (int r = 0; r <= rounds; ++r) {
    fi_mesh* M = nullptr;
    int rc;
    if (unknowns) {
      unk.clear();
      std::set_difference(unknowns->begin(), unknowns->end(), mask.begin(), mask.end(),
                          std::back_inserter(unk));
      rc = fi_mesh_build_delaunay(ctx, side, mask.data(), (int64_t)mask.size(), unk.data(),
                                  (int64_t)unk.size(), &M);
    } else {
      rc = fi_mesh_build(ctx, side, side, mask.data(), (int64_t)mask.size(), &M);
    }
    if (rc) return rc;
    if (gpu_ms_out) FI_HIP_TRY(hipEventRecord(t0.e, ctx->stream));
    fi_solve_stats st{};
    rc = fi_inpaint(M, f_dev, nullptr, (double*)u.p, opts, &st);
    double mse = 0.0;
    if (rc == FI_OK) rc = fi_error(M, (double*)u.p, f_dev, &mse, (double*)e.p, nullptr);
    if (gpu_ms_out && rc == FI_OK) {
      (void)hipEventRecord(t1.e, ctx->stream);
      (void)hipEventSynchronize(t1.e);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, t0.e, t1.e);
      gpu_ms_out[r] = ms;
    }
    if (rc == FI_OK) mse_out[r] = mse;
    int64_t got = 0;
    if (rc == FI_OK && r < rounds && k_add > 0) {
      if (rule == FI_DENSIFY_TOPK) {
        rc = fi_topk_new_pixels(M, (double*)e.p, k_add, (int32_t*)sel.p);
        got = k_add;
      } else {
        rc = paper_densify_step(M, (double*)e.p, k_add, (int32_t*)sel.p, &got);
      }
      if (rc == FI_OK && got > 0) {
        hipError_t he = hipMemcpy(add.data(), sel.p, (size_t)got * sizeof(int32_t),
                                  hipMemcpyDeviceToHost);
        if (he != hipSuccess) rc = fail(FI_E_HIP, hipGetErrorString(he));
      }
    }
    fi_mesh_destroy(M);
    if (rc) return rc;
    if (got > 0) {
      std::memcpy(mask_out + written, add.data(), (size_t)got * sizeof(int32_t));
      written += got;
      std::vector<int32_t> merged(mask.size() + (size_t)got);
      std::merge(mask.begin(), mask.end(), add.begin(), add.begin() + got, merged.begin());
      mask.swap(merged);
    }
  }
  if (total_out) *total_out = written;
  return FI_OK;
}

}  // namespace

extern "C" int fi_grow_mask(fi_ctx* ctx, int side, const uint8_t* f_dev, const int32_t* mask0,
                            int64_t m0, int64_t k_add, int rounds, const fi_solve_opts* opts,
                            int32_t* mask_out, double* mse_out, double* gpu_ms_out) {
  return densify_loop(ctx, side, f_dev, mask0, m0, k_add, rounds, FI_DENSIFY_TOPK, opts, mask_out,
                      mse_out, gpu_ms_out, nullptr);
}

extern "C" int fi_densify(fi_ctx* ctx, int side, const uint8_t* f_dev, const int32_t* mask0,
                          int64_t m0, int64_t k_add, int rounds, int rule,
                          const fi_solve_opts* opts, int32_t* mask_out, double* mse_out,
                          double* gpu_ms_out, int64_t* mask_size_out) {
  return densify_loop(ctx, side, f_dev, mask0, m0, k_add, rounds, rule, opts, mask_out, mse_out,
                      gpu_ms_out, mask_size_out);
}

extern "C" int fi_densify_delaunay(fi_ctx* ctx, int side, const uint8_t* f_dev,
                                   const int32_t* mask0, int64_t m0, const int32_t* unknowns,
                                   int64_t nu, int64_t k_add, int rounds,
                                   const fi_solve_opts* opts, int32_t* mask_out, double* mse_out,
                                   double* gpu_ms_out, int64_t* mask_size_out) {
  if (nu > 0 && !unknowns) return fail(FI_E_INVALID, "densify: unknown vertices are NULL");
  std::vector<int32_t> unk(unknowns, unknowns + std::max<int64_t>(nu, 0));
  for (size_t i = 1; i < unk.size(); ++i)
    if (unk[i] <= unk[i - 1])
      return fail(FI_E_INVALID, "densify: unknown vertices must be strictly ascending");
  return densify_loop(ctx, side, f_dev, mask0, m0, k_add, rounds, FI_DENSIFY_TRIANGLES, opts,
                      mask_out, mse_out, gpu_ms_out, mask_size_out, &unk);
}

extern "C" int fi_paper_densify_step(fi_mesh* M, const double* e_dev, int64_t k, int32_t* out_dev,
                                     int64_t* added) {
  if (!M || !M->ctx || !e_dev || !added || (k > 0 && !out_dev))
    return fail(FI_E_INVALID, "fi_paper_densify_step: NULL argument");
  if (k < 0) return fail(FI_E_INVALID, "fi_paper_densify_step: k < 0");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  return paper_densify_step(M, e_dev, k, out_dev, added);
}
