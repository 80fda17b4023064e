// Multi-call procedures built on the single-mesh calls: error-driven mask
// growth (Section 3).
#include <algorithm>
#include <cstring>
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

extern "C" int fi_grow_mask(fi_ctx* ctx, int side, const uint8_t* f_dev, const int32_t* mask0,
                            int64_t m0, int64_t k_add, int rounds, const fi_solve_opts* opts,
                            int32_t* mask_out, double* mse_out, double* gpu_ms_out) {
  if (!ctx || !f_dev || !mask0 || !mask_out || !mse_out)
    return fail(FI_E_INVALID, "fi_grow_mask: NULL argument");
  if (side < 2 || k_add < 0 || rounds < 0) return fail(FI_E_INVALID, "fi_grow_mask: bad sizes");
  const int64_t P = (int64_t)side * side;
  if (m0 + (int64_t)rounds * k_add > P) return fail(FI_E_INVALID, "fi_grow_mask: mask would exceed the image");
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
  for (int r = 0; r <= rounds; ++r) {
    fi_mesh* M = nullptr;
    int rc = fi_mesh_build(ctx, side, side, mask.data(), (int64_t)mask.size(), &M);
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
    if (rc == FI_OK && r < rounds && k_add > 0) {
      rc = fi_topk_new_pixels(M, (double*)e.p, k_add, (int32_t*)sel.p);
      if (rc == FI_OK) {
        hipError_t he = hipMemcpy(add.data(), sel.p, (size_t)k_add * sizeof(int32_t),
                                  hipMemcpyDeviceToHost);
        if (he != hipSuccess) rc = fail(FI_E_HIP, hipGetErrorString(he));
      }
    }
    fi_mesh_destroy(M);
    if (rc) return rc;
    if (r < rounds && k_add > 0) {
      std::memcpy(mask_out + written, add.data(), (size_t)k_add * sizeof(int32_t));
      written += k_add;
      std::vector<int32_t> merged(mask.size() + (size_t)k_add);
      std::merge(mask.begin(), mask.end(), add.begin(), add.begin() + k_add, merged.begin());
      mask.swap(merged);
    }
  }
  return FI_OK;
}
