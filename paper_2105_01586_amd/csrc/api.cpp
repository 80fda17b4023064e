// C ABI of the library (declared in include/fi.h): contexts, meshes, and the
// inpainting, error, adjoint and tonal-optimisation calls.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>

#include "internal.h"

namespace fi {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int device_alloc(fi_mesh* M, void** p, size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~(size_t)255;
  if (M->arena) {
    *p = M->arena->alloc(bytes);
    if (!*p) return fail(FI_E_NOMEM, "device arena exhausted");
    M->allocations.push_back(*p);
    M->device_bytes += (int64_t)bytes;
    return FI_OK;
  }
  size_t got = bytes;
  *p = M->cache ? M->cache->take(bytes, &got) : nullptr;
  if (!*p) {
    hipError_t e = hipMalloc(p, bytes);
    if (e == hipErrorOutOfMemory && M->cache) {  // the kept blocks may be what is missing
      (void)hipGetLastError();
      M->cache->release_all();
      e = hipMalloc(p, bytes);
    }
    if (e != hipSuccess) {
      *p = nullptr;
      (void)hipGetLastError();
      return fail(e == hipErrorOutOfMemory ? FI_E_NOMEM : FI_E_HIP,
                  std::string("device allocation failed: ") + hipGetErrorString(e));
    }
  }
  M->allocations.push_back(*p);
  M->alloc_sizes.push_back(got);
  M->device_bytes += (int64_t)bytes;
  return FI_OK;
}

void* DeviceCache::take(size_t bytes, size_t* got) {
  std::lock_guard<std::mutex> lk(mu_);
  auto it = kept_.lower_bound(bytes);
  if (it == kept_.end() || it->first > bytes + bytes / 4 + ((size_t)1 << 20)) return nullptr;
  void* p = it->second;
  *got = it->first;
  kept_bytes_ -= it->first;
  kept_.erase(it);
  return p;
}

void DeviceCache::give(void* p, size_t bytes) {
  {
    std::lock_guard<std::mutex> lk(mu_);
    if (kept_bytes_ + bytes <= kKeepBytes) {
      kept_.emplace(bytes, p);
      kept_bytes_ += bytes;
      return;
    }
  }
  (void)hipSetDevice(device_);
  (void)hipFree(p);
}

bool TmpBlock::take(size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  got = bytes;
  if (M->arena) return (p = M->arena->alloc(bytes)) != nullptr;
  if (M->cache && (p = M->cache->take(bytes, &got))) return true;
  got = bytes;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    return false;
  }
  return true;
}

int TmpBlock::alloc(size_t bytes) {
  return take(bytes) ? FI_OK : fail(FI_E_NOMEM, "device scratch of a build step");
}

TmpBlock::~TmpBlock() {
  if (!p) return;
  (void)hipStreamSynchronize(M->ctx->stream);
  if (M->arena) M->arena->free(p);
  else if (M->cache && got <= kKeepTmp) M->cache->give(p, got);
  else (void)hipFree(p);
}

DeviceCache::~DeviceCache() {
  release_all();
  if (staging_) (void)hipHostFree(staging_);
}

void* DeviceCache::staging(size_t bytes, std::unique_lock<std::mutex>& hold) {
  if (bytes > kStagingMax) return nullptr;
  hold = std::unique_lock<std::mutex>(staging_mu_);
  if (staging_bytes_ < bytes) {
    (void)hipSetDevice(device_);
    if (staging_) (void)hipHostFree(staging_);
    staging_ = nullptr;
    staging_bytes_ = 0;
    const size_t want = std::min(kStagingMax, std::max(bytes, staging_bytes_ * 2));
    if (hipHostMalloc(&staging_, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      staging_ = nullptr;
      hold.unlock();
      return nullptr;
    }
    staging_bytes_ = want;
  }
  return staging_;
}

void DeviceCache::release_all() {
  std::multimap<size_t, void*> blocks;
  {
    std::lock_guard<std::mutex> lk(mu_);
    blocks.swap(kept_);
    kept_bytes_ = 0;
  }
  if (blocks.empty()) return;
  (void)hipSetDevice(device_);
  for (auto& b : blocks) (void)hipFree(b.second);
}

namespace {

template <typename T>
int alloc_n(fi_mesh* M, T** p, int64_t n) {
  return device_alloc(M, (void**)p, (size_t)std::max<int64_t>(n, 1) * sizeof(T));
}

template <typename T, typename A>
int upload(fi_mesh* M, T** p, const std::vector<T, A>& h) {
  int rc = alloc_n(M, p, (int64_t)h.size());
  if (rc) return rc;
  if (!h.empty())
    FI_HIP_TRY(hipMemcpyAsync(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice,
                              M->ctx->stream));
  return FI_OK;
}

}  // namespace

void free_mesh(fi_mesh* M) {
  if (!M) return;
  for (fi_mesh*& c : M->chan) {
    free_mesh(c);
    c = nullptr;
  }
  (void)hipSetDevice(M->device);
  if (M->arena) {
    // arena meshes: the owner has waited for the mesh's last work
    solver_release(M);
    for (void* p : M->allocations) M->arena->free(p);
  } else {
    // The device must be done with the blocks before they are freed or kept
    // for another mesh; the context (and its stream) may already be gone, so
    // only the device id is used here (the cache is shared with the mesh).
    (void)hipDeviceSynchronize();
    solver_release(M);
    for (size_t k = 0; k < M->allocations.size(); ++k) {
      if (M->cache) M->cache->give(M->allocations[k], M->alloc_sizes[k]);
      else (void)hipFree(M->allocations[k]);
    }
  }
  if (M->h_red) (void)hipHostFree(M->h_red);
  if (M->h_ctl) (void)hipHostFree(M->h_ctl);
  delete M;
}

namespace {

#define TRY(x) do { rc = (x); if (rc) return rc; } while (0)

// Vectors of one right-hand side: the solve's b, iterate and residual and
// the per-pixel / per-vertex work vectors (the one-iteration CG vectors are
// allocated by their first solve).
int alloc_rhs_space(fi_mesh* M) {
  int rc = 0;
  const int64_t n = M->n, m = M->m, V = M->V, T = M->T;
  TRY(alloc_n(M, &M->d_b64, n));
  TRY(alloc_n(M, &M->d_x64buf[0], n));
  TRY(alloc_n(M, &M->d_x64buf[1], n));
  M->d_x64 = M->d_x64buf[0];
  TRY(alloc_n(M, &M->d_r64, n));
  // the one-iteration CG vectors come with the first solve that uses them
  M->cg32 = CGState{};
  M->cg64 = CGState{};
  TRY(alloc_n(M, &M->d_red, kMaxGrid));
  TRY(alloc_n(M, &M->d_red_out, 8));
  TRY(alloc_n(M, &M->d_uvert, V));
  TRY(alloc_n(M, &M->d_g, m));
  TRY(alloc_n(M, &M->d_tpart, 3 * T));
  TRY(alloc_n(M, &M->d_tD, m));
  TRY(alloc_n(M, &M->d_rpart, raster_blocks(M)));
  FI_HIP_TRY(hipHostMalloc((void**)&M->h_red, 8 * sizeof(double), hipHostMallocDefault));
  FI_HIP_TRY(hipHostMalloc((void**)&M->h_ctl, 4 * sizeof(int32_t), hipHostMallocDefault));
  return FI_OK;
}

int alloc_workspace(fi_mesh* M) {
  int rc = 0;
  const int64_t n = M->n, m = M->m, T = M->T;
  TRY(alloc_n(M, &M->d_cnt, std::max(2 * (n + 1), m + 1)));
  // scans over free rows, mask rows, triangles and vertices
  TRY(alloc_n(M, &M->d_scan_tmp, scan_tmp_ints(std::max({n, m, T, M->V}) + 1)));
  TRY(alloc_n(M, &M->d_ff_rowptr, n + 1));
  TRY(alloc_n(M, &M->d_fd_rowptr, n + 1));
  TRY(alloc_n(M, &M->d_df_rowptr, m + 1));
  TRY(alloc_n(M, &M->d_diag64, n));
  TRY(alloc_n(M, &M->d_dinv64, n));
  TRY(alloc_n(M, &M->d_dinv32, n));
  TRY(alloc_rhs_space(M));
  TRY(alloc_n(M, &M->d_owner, M->P));
  TRY(alloc_n(M, &M->d_tri_px, M->P));
  TRY(alloc_n(M, &M->d_tri_px_ptr, T + 1));
  return FI_OK;
}

// Channel c of a colour image: shares everything that depends on the mesh
// alone (geometry, matrices, ELL copy, pixel maps) with M and owns what
// depends on the data.
int make_channel(fi_mesh* M, fi_mesh** out) {
  *out = nullptr;
  fi_mesh* S = new fi_mesh();
  S->ctx = M->ctx;
  S->device = M->device;
  S->arena = M->arena;
  S->cache = M->cache;
  S->is_channel = true;
  S->host.N = M->host.N;
  S->host.levels = M->host.levels;
  S->host.delaunay = M->host.delaunay;  // picks the pixel passes and their partial-sum layout
  S->N = M->N;
  S->P = M->P;
  S->V = M->V;
  S->T = M->T;
  S->L = M->L;
  S->n = M->n;
  S->m = M->m;
  S->nnz_off = M->nnz_off;
  S->nnz_fd = M->nnz_fd;
  S->nnz_df = M->nnz_df;
  S->d_vxy = M->d_vxy;
  S->d_tri = M->d_tri;
  S->d_leaves = M->d_leaves;
  S->d_vmap = M->d_vmap;
  S->d_free_vids = M->d_free_vids;
  S->d_mask_vids = M->d_mask_vids;
  S->d_mask_pix = M->d_mask_pix;
  S->d_vt_ptr = M->d_vt_ptr;
  S->d_vt_idx = M->d_vt_idx;
  S->assembled_once = true;
  S->d_ff_rowptr = M->d_ff_rowptr;
  S->d_ff_col = M->d_ff_col;
  S->d_ff_val64 = M->d_ff_val64;
  S->d_ff_val32 = M->d_ff_val32;
  S->d_diag64 = M->d_diag64;
  S->d_dinv64 = M->d_dinv64;
  S->d_dinv32 = M->d_dinv32;
  S->d_fd_rowptr = M->d_fd_rowptr;
  S->d_fd_col = M->d_fd_col;
  S->d_fd_val = M->d_fd_val;
  S->d_df_rowptr = M->d_df_rowptr;
  S->d_df_col = M->d_df_col;
  S->d_df_val = M->d_df_val;
  S->d_owner = M->d_owner;
  S->d_tri_px_ptr = M->d_tri_px_ptr;
  S->d_tri_px = M->d_tri_px;
  int rc = alloc_rhs_space(S);
  if (!rc) rc = solver_channel_setup(S, M);
  if (rc) {
    std::string keep = g_last_error;
    free_mesh(S);
    g_last_error = keep;
    return rc;
  }
  *out = S;
  return FI_OK;
}
#undef TRY

int read_total(fi_mesh* M, const int32_t* dptr, int64_t* out) {
  int32_t v = 0;
  FI_HIP_TRY(hipMemcpyAsync(M->h_ctl + 3, dptr, sizeof(int32_t), hipMemcpyDeviceToHost,
                            M->ctx->stream));
  FI_HIP_TRY(hipStreamSynchronize(M->ctx->stream));
  v = M->h_ctl[3];
  *out = v;
  return FI_OK;
}

int sync_read_scalar(fi_mesh* M, const double* dptr, double* out) {
  FI_HIP_TRY(hipMemcpyAsync(M->h_red, dptr, sizeof(double), hipMemcpyDeviceToHost,
                            M->ctx->stream));
  FI_HIP_TRY(hipStreamSynchronize(M->ctx->stream));
  *out = M->h_red[0];
  return FI_OK;
}

int check_mesh(const fi_mesh* M) {
  if (!M || !M->ctx) return fail(FI_E_INVALID, "mesh is NULL");
  return FI_OK;
}

// u = B g for g on the device (vertex values kept in d_uvert).
int apply_B(fi_mesh* M, const double* g, double* u_out, const fi_solve_opts* o,
            fi_solve_stats* st) {
  int rc = launch_lift(M, g, M->d_b64);
  if (rc) return rc;
  rc = solve_free(M, o, st);
  if (rc) return rc;
  rc = launch_vertex_values(M, M->d_x64, g, M->d_uvert);
  if (rc) return rc;
  return launch_raster(M, M->d_uvert, nullptr, nullptr, u_out, nullptr, nullptr, nullptr,
                       nullptr);
}

// s = B^T r for r on the device.
int apply_BT(fi_mesh* M, const double* r, double* s, const fi_solve_opts* o, fi_solve_stats* st) {
  int rc = launch_raster_transpose(M, r, M->d_tpart);
  if (rc) return rc;
  rc = launch_gather_vertex(M, M->d_tpart, M->d_b64, M->d_tD);  // t_F: the solve's b
  if (rc) return rc;
  rc = solve_free(M, o, st);
  if (rc) return rc;
  return launch_adjoint_tail(M, M->d_tD, M->d_x64, s);
}

int dot_host(fi_mesh* M, const double* a, const double* b, int64_t n, double* out) {
  int rc = launch_dot(M, a, b, n, M->d_red_out);
  if (rc) return rc;
  return sync_read_scalar(M, M->d_red_out, out);
}

// Sum of squared errors of u against f, left on the device in *out_dev.
int sse_dev(fi_mesh* M, const double* u, const uint8_t* f, double* out_dev) {
  int rc = launch_raster(M, nullptr, u, f, nullptr, nullptr, nullptr, nullptr, M->d_rpart);
  if (rc) return rc;
  return launch_reduce(M, M->d_rpart, raster_blocks(M), 1, out_dev);
}


}  // namespace

fi_solve_opts resolve_opts(const fi_solve_opts* o) {
  fi_solve_opts d;
  fi_solve_opts_default(&d);
  if (!o) return d;
  fi_solve_opts r = *o;
  if (r.rtol <= 0) r.rtol = d.rtol;
  if (r.atol == 0) r.atol = d.atol;
  if (r.inner_rtol <= 0 || r.inner_rtol >= 1) r.inner_rtol = d.inner_rtol;
  if (r.max_inner <= 0) r.max_inner = d.max_inner;
  if (r.max_refine <= 0) r.max_refine = d.max_refine;
  if (r.check_every <= 0) r.check_every = d.check_every;
  return r;
}

int channel_views(fi_mesh* M, int nc, fi_mesh** ch) {
  if (M->is_channel) return fail(FI_E_INVALID, "a channel view has no channels");
  if (nc < 1 || nc > kMaxRhs) return fail(FI_E_INVALID, "1 to 3 channels");
  ch[0] = M;
  for (int c = 1; c < nc; ++c) {
    if (!M->chan[c - 1]) {
      int rc = make_channel(M, &M->chan[c - 1]);
      if (rc) return rc;
    }
    ch[c] = M->chan[c - 1];
  }
  return FI_OK;
}

}  // namespace fi

using namespace fi;

extern "C" {

void fi_solve_opts_default(fi_solve_opts* o) {
  if (!o) return;
  o->precision = FI_PREC_FP32_IR;
  o->rtol = 1e-10;
  o->inner_rtol = 1e-5;
  o->max_inner = 20000;
  o->max_refine = 40;
  o->check_every = 32;
  o->atol = kDefaultAtol;
}

void fi_tonal_opts_default(fi_tonal_opts* o) {
  if (!o) return;
  fi_solve_opts_default(&o->inner);
  o->rtol = 1e-8;
  o->max_outer = 500;
  o->start_from_g = 0;
  o->cold_adjoint = 0;
}

const char* fi_last_error(void) { return g_last_error.c_str(); }

const char* fi_version(void) { return "fem-inpaint-mi355x 0.1.0 (gfx950)"; }

int fi_ctx_create(int device, void* stream, fi_ctx** out) {
  if (!out) return fail(FI_E_INVALID, "out is NULL");
  *out = nullptr;
  int count = 0;
  FI_HIP_TRY(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(FI_E_INVALID, "no such device");
  FI_HIP_TRY(hipSetDevice(device));
  fi_ctx* c = new fi_ctx();
  c->device = device;
  c->stream = (hipStream_t)stream;
  c->cache = std::make_shared<DeviceCache>(device);
  *out = c;
  return FI_OK;
}

int fi_ctx_set_stream(fi_ctx* ctx, void* stream) {
  if (!ctx) return fail(FI_E_INVALID, "ctx is NULL");
  ctx->stream = (hipStream_t)stream;
  return FI_OK;
}

int fi_ctx_destroy(fi_ctx* ctx) {
  delete ctx;
  return FI_OK;
}

int fi_host_mesh_build(int width, int height, const int32_t* mask_idx, int64_t m,
                       fi_host_mesh** out) {
  if (!out) return fail(FI_E_INVALID, "out is NULL");
  *out = nullptr;
  if (width != height) return fail(FI_E_INVALID, "image must be square");
  fi_host_mesh* h = new fi_host_mesh();
  int rc = build_host_mesh(width, mask_idx, m, h->mesh);
  if (rc) { delete h; return rc; }
  *out = h;
  return FI_OK;
}

int fi_host_mesh_build_delaunay(int side, const int32_t* mask_idx, int64_t m,
                                const int32_t* unknown_idx, int64_t nu, fi_host_mesh** out) {
  if (!out) return fail(FI_E_INVALID, "out is NULL");
  *out = nullptr;
  if (m < 1) return fail(FI_E_EMPTY_MASK, "the mask is empty");
  fi_host_mesh* h = new fi_host_mesh();
  int rc = build_delaunay_mesh(side, mask_idx, m, unknown_idx, nu, h->mesh);
  if (rc) { delete h; return rc; }
  *out = h;
  return FI_OK;
}

int fi_mesh_build_delaunay(fi_ctx* ctx, int side, const int32_t* mask_idx, int64_t m,
                           const int32_t* unknown_idx, int64_t nu, fi_mesh** out) {
  if (!ctx || !out) return fail(FI_E_INVALID, "ctx or out is NULL");
  *out = nullptr;
  fi_host_mesh* h = nullptr;
  int rc = fi_host_mesh_build_delaunay(side, mask_idx, m, unknown_idx, nu, &h);
  if (rc) return rc;
  rc = fi_mesh_upload(ctx, &h, out);
  if (h) fi_host_mesh_destroy(h);
  return rc;
}

int fi_host_mesh_info(const fi_host_mesh* h, fi_mesh_info* info) {
  if (!h || !info) return fail(FI_E_INVALID, "NULL argument");
  const HostMesh& H = h->mesh;
  std::memset(info, 0, sizeof(*info));
  info->N = H.N;
  info->P = (int64_t)H.N * H.N;
  info->V = H.V();
  info->T = H.T();
  info->L = H.L();
  info->n = (int64_t)H.free_vids.size();
  info->m = (int64_t)H.mask_vids.size();
  return FI_OK;
}

int fi_host_mesh_export(const fi_host_mesh* h, int32_t* vxy, int32_t* tri, int32_t* leaves,
                        int32_t* free_vids, int32_t* mask_vids) {
  if (!h) return fail(FI_E_INVALID, "host mesh is NULL");
  const HostMesh& H = h->mesh;
  if (vxy) std::memcpy(vxy, H.vxy.data(), H.vxy.size() * sizeof(int32_t));
  if (tri) std::memcpy(tri, H.tri.data(), H.tri.size() * sizeof(int32_t));
  if (leaves) {
    for (int64_t i = 0; i < H.L(); ++i) {
      leaves[3 * i] = H.leaves[4 * i];
      leaves[3 * i + 1] = H.leaves[4 * i + 1];
      leaves[3 * i + 2] = H.leaves[4 * i + 2];
    }
  }
  if (free_vids) std::memcpy(free_vids, H.free_vids.data(), H.free_vids.size() * sizeof(int32_t));
  if (mask_vids) std::memcpy(mask_vids, H.mask_vids.data(), H.mask_vids.size() * sizeof(int32_t));
  return FI_OK;
}

int fi_host_mesh_destroy(fi_host_mesh* h) {
  delete h;
  return FI_OK;
}

int fi_mesh_build(fi_ctx* ctx, int width, int height, const int32_t* mask_idx, int64_t m,
                  fi_mesh** out) {
  if (!ctx || !out) return fail(FI_E_INVALID, "ctx or out is NULL");
  *out = nullptr;
  // built on the device; with FI_MESH_HOST=1 on the host and uploaded (the
  // same mesh either way)
  const char* env = std::getenv("FI_MESH_HOST");
  if (!(env && std::atoi(env) == 1)) {
    if (width != height) return fail(FI_E_INVALID, "image must be square");
    return mesh_build_on_device(ctx, width, mask_idx, m, out);
  }
  fi_host_mesh* h = nullptr;
  int rc = fi_host_mesh_build(width, height, mask_idx, m, &h);
  if (rc) return rc;
  rc = fi_mesh_upload(ctx, &h, out);
  if (h) fi_host_mesh_destroy(h);
  return rc;
}

int fi_mesh_upload(fi_ctx* ctx, fi_host_mesh** host, fi_mesh** out) {
  return mesh_upload(ctx, host, nullptr, out);
}

}  // extern "C"

int fi::mesh_build_on_device(fi_ctx* ctx, int N, const int32_t* mask, int64_t m, fi_mesh** out) {
  FI_HIP_TRY(hipSetDevice(ctx->device));
  fi_mesh* M = new fi_mesh();
  M->ctx = ctx;
  M->device = ctx->device;
  M->cache = ctx->cache;
  int rc = FI_OK;
  if ((rc = mesh_geometry_on_device(M, N, mask, m)) || (rc = alloc_workspace(M)) ||
      (rc = build_vertex_triangles(M)) || (rc = build_pixel_maps(M)) || (rc = fi_assemble(M))) {
    std::string keep = g_last_error;
    free_mesh(M);
    g_last_error = keep;
    return rc;
  }
  *out = M;
  return FI_OK;
}

int fi::mesh_host_coords(const fi_mesh* M, std::vector<int32_t>& vxy,
                         std::vector<int32_t>& free_vids) {
  if (!M->host.vxy.empty() || M->V == 0) {
    vxy.assign(M->host.vxy.begin(), M->host.vxy.end());
    free_vids.assign(M->host.free_vids.begin(), M->host.free_vids.end());
    return FI_OK;
  }
  vxy.resize((size_t)(2 * M->V));
  free_vids.resize((size_t)M->n);
  hipStream_t st = M->ctx->stream;
  FI_HIP_TRY(hipMemcpyAsync(vxy.data(), M->d_vxy, vxy.size() * 4, hipMemcpyDeviceToHost, st));
  if (M->n > 0)
    FI_HIP_TRY(hipMemcpyAsync(free_vids.data(), M->d_free_vids, free_vids.size() * 4,
                              hipMemcpyDeviceToHost, st));
  FI_HIP_TRY(hipStreamSynchronize(st));
  return FI_OK;
}

int fi::mesh_upload(fi_ctx* ctx, fi_host_mesh** host, Arena* arena, fi_mesh** out) {
  if (!ctx || !out || !host || !*host) return fail(FI_E_INVALID, "NULL argument");
  *out = nullptr;
  FI_HIP_TRY(hipSetDevice(ctx->device));
  fi_mesh* M = new fi_mesh();
  M->ctx = ctx;
  M->device = ctx->device;
  M->arena = arena;
  if (!arena) M->cache = ctx->cache;
  M->host = std::move((*host)->mesh);
  int rc = FI_OK;
  const HostMesh& H = M->host;
  M->N = H.N;
  M->P = (int64_t)H.N * H.N;
  M->V = H.V();
  M->T = H.T();
  M->L = H.L();
  M->n = (int64_t)H.free_vids.size();
  M->m = (int64_t)H.mask_vids.size();
  if ((rc = upload(M, &M->d_vxy, H.vxy)) || (rc = upload(M, &M->d_tri, H.tri)) ||
      (rc = upload(M, &M->d_leaves, H.leaves)) || (rc = upload(M, &M->d_vmap, H.vmap)) ||
      (rc = upload(M, &M->d_free_vids, H.free_vids)) ||
      (rc = upload(M, &M->d_mask_vids, H.mask_vids)) ||
      (rc = upload(M, &M->d_mask_pix, H.mask_pix)) || (rc = alloc_workspace(M)) ||
      (rc = build_vertex_triangles(M)) ||
      (rc = build_pixel_maps(M)) || (rc = fi_assemble(M))) {
    std::string keep = g_last_error;
    (*host)->mesh = std::move(M->host);
    free_mesh(M);
    g_last_error = keep;
    return rc;
  }
  fi_host_mesh_destroy(*host);
  *host = nullptr;
  *out = M;
  return FI_OK;
}

extern "C" {

int fi_mesh_destroy(fi_mesh* M) {
  free_mesh(M);
  return FI_OK;
}

int fi_mesh_get_info(const fi_mesh* M, fi_mesh_info* info) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!info) return fail(FI_E_INVALID, "info is NULL");
  info->N = M->N;
  info->P = M->P;
  info->V = M->V;
  info->T = M->T;
  info->L = M->L;
  info->n = M->n;
  info->m = M->m;
  info->nnz_ff = M->nnz_off + M->n;
  info->nnz_fd = M->nnz_fd;
  info->device_bytes = M->device_bytes;
  for (const fi_mesh* c : M->chan)
    if (c) info->device_bytes += c->device_bytes;
  info->cg_blocks = M->ss ? M->ss->grid : M->cg_grid;
  info->cg_block_size = M->cg_bs;
  info->large_mode = (M->ss ? M->ss->large : M->large_mode) ? 1 : 0;
  info->cg_iters_per_launch = M->ss ? kSsIters : 1;
  info->cg_max_region = M->ss ? M->ss->max_region : 0;
  info->cg_region_rows = M->ss ? M->ss->region_rows : 0;
  info->cg_lmat_rows = M->ss ? M->ss->lmat_rows : 0;
  return FI_OK;
}

int fi_assemble(fi_mesh* M) {
  int rc = check_mesh(M);
  if (rc) return rc;
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  const int64_t n = M->n, m = M->m;
  // Later assemblies recompute every value (free and mask rows, ELL slots)
  // in one launch.
  if (M->assembled_once) return launch_assemble_refill(M);
  int32_t* cnt_ff = M->d_cnt;
  int32_t* cnt_fd = M->d_cnt + (n + 1);
  // The sparsity pattern depends on the mesh only: counted and scanned on the
  // first assembly, reused after (only the values are recomputed).
  if (!M->assembled_once) {
    if ((rc = launch_assemble_count(M, true))) return rc;
    if ((rc = scan_counts(M, cnt_ff, M->d_ff_rowptr, n + 1))) return rc;
    if ((rc = scan_counts(M, cnt_fd, M->d_fd_rowptr, n + 1))) return rc;
    if ((rc = read_total(M, M->d_ff_rowptr + n, &M->nnz_off))) return rc;
    if ((rc = read_total(M, M->d_fd_rowptr + n, &M->nnz_fd))) return rc;
    if ((rc = alloc_n(M, &M->d_ff_col, M->nnz_off)) || (rc = alloc_n(M, &M->d_ff_val64, M->nnz_off)) ||
        (rc = alloc_n(M, &M->d_ff_val32, M->nnz_off)) || (rc = alloc_n(M, &M->d_fd_col, M->nnz_fd)) ||
        (rc = alloc_n(M, &M->d_fd_val, M->nnz_fd)))
      return rc;
  }
  if ((rc = launch_assemble_fill(M, true))) return rc;
  // mask rows: K_DF (reuses the count scratch after the fill above is queued)
  if (!M->assembled_once) {
    if ((rc = launch_assemble_count(M, false))) return rc;
    if ((rc = scan_counts(M, M->d_cnt, M->d_df_rowptr, m + 1))) return rc;
    if ((rc = read_total(M, M->d_df_rowptr + m, &M->nnz_df))) return rc;
    if ((rc = alloc_n(M, &M->d_df_col, M->nnz_df)) || (rc = alloc_n(M, &M->d_df_val, M->nnz_df)))
      return rc;
  }
  if ((rc = launch_assemble_fill(M, false))) return rc;
  if ((rc = solver_setup(M))) return rc;
  if (!M->assembled_once) FI_HIP_TRY(hipStreamSynchronize(M->ctx->stream));
  M->assembled_once = true;
  return FI_OK;
}

int fi_inpaint(fi_mesh* M, const uint8_t* f_dev, const double* g_dev, double* u_dev,
               const fi_solve_opts* opts, fi_solve_stats* stats) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!u_dev) return fail(FI_E_INVALID, "u_dev is NULL");
  if (!g_dev && !f_dev) return fail(FI_E_INVALID, "need f_dev or g_dev");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  const fi_solve_opts o = resolve_opts(opts);
  fi_solve_stats st{};
  const double* g = g_dev;
  if (!g) {
    if ((rc = launch_gather_mask(M, f_dev, M->d_g))) return rc;
    g = M->d_g;
  }
  rc = apply_B(M, g, u_dev, &o, &st);
  if (stats) *stats = st;
  if (rc) return rc;
  if (st.status != FI_OK)
    return fail(FI_E_NO_CONVERGENCE, "inpainting solve did not reach the tolerance");
  return FI_OK;
}

int fi_inpaint_image(fi_ctx* ctx, int width, int height, const uint8_t* f_dev,
                     const uint8_t* mask_u8_host, const double* g_dev, double* u_dev,
                     const fi_solve_opts* opts, fi_solve_stats* stats) {
  if (!ctx || !mask_u8_host) return fail(FI_E_INVALID, "ctx or mask is NULL");
  if (width < 1 || height < 1) return fail(FI_E_INVALID, "bad image size");
  std::vector<int32_t> idx;
  const int64_t P = (int64_t)width * height;
  for (int64_t p = 0; p < P; ++p)
    if (mask_u8_host[p]) idx.push_back((int32_t)p);
  fi_mesh* M = nullptr;
  int rc = fi_mesh_build(ctx, width, height, idx.data(), (int64_t)idx.size(), &M);
  if (rc) return rc;
  rc = fi_inpaint(M, f_dev, g_dev, u_dev, opts, stats);
  std::string keep = g_last_error;
  if (rc == FI_OK || rc == FI_E_NO_CONVERGENCE) (void)hipStreamSynchronize(ctx->stream);
  free_mesh(M);
  g_last_error = keep;
  return rc;
}

int fi_vertex_values(fi_mesh* M, double* u_vertex_dev) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!u_vertex_dev) return fail(FI_E_INVALID, "output is NULL");
  FI_HIP_TRY(hipMemcpyAsync(u_vertex_dev, M->d_uvert, (size_t)M->V * sizeof(double),
                            hipMemcpyDeviceToDevice, M->ctx->stream));
  FI_HIP_TRY(hipStreamSynchronize(M->ctx->stream));
  return FI_OK;
}

int fi_error(fi_mesh* M, const double* u_dev, const uint8_t* f_dev, double* mse_host,
             double* pix_err_dev, double* tri_err_dev) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!u_dev || !f_dev) return fail(FI_E_INVALID, "u_dev and f_dev are required");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  rc = launch_raster(M, nullptr, u_dev, f_dev, nullptr, pix_err_dev, tri_err_dev, nullptr,
                     M->d_rpart);
  if (rc) return rc;
  rc = launch_reduce(M, M->d_rpart, raster_blocks(M), 1, M->d_red_out);
  if (rc) return rc;
  double s = 0.0;
  rc = sync_read_scalar(M, M->d_red_out, &s);
  if (rc) return rc;
  if (mse_host) *mse_host = s / (double)M->P;
  return FI_OK;
}

int fi_error_dev(fi_mesh* M, const double* u_dev, const uint8_t* f_dev, double* sum_dev) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!u_dev || !f_dev || !sum_dev) return fail(FI_E_INVALID, "u_dev, f_dev and sse_dev are required");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  return fi::sse_dev(M, u_dev, f_dev, sum_dev);
}

int fi_mse_dev(fi_mesh* M, const double* u_dev, const uint8_t* f_dev, double* mse_dev) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!u_dev || !f_dev || !mse_dev) return fail(FI_E_INVALID, "u_dev, f_dev and mse_dev are required");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  rc = launch_raster(M, nullptr, u_dev, f_dev, nullptr, nullptr, nullptr, nullptr, M->d_rpart);
  if (rc) return rc;
  return launch_reduce(M, M->d_rpart, raster_blocks(M), 1, mse_dev, (double)M->P);
}

int fi_mse_backward(fi_mesh* M, const double* u_dev, const uint8_t* f_dev, const double* scale_dev,
                    double* grad_dev, const fi_solve_opts* opts, fi_solve_stats* stats) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!u_dev || !f_dev || !grad_dev) return fail(FI_E_INVALID, "u_dev, f_dev and grad_dev are required");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  if (!M->d_rgrad && (rc = device_alloc(M, (void**)&M->d_rgrad, (size_t)M->P * sizeof(double))))
    return rc;
  const fi_solve_opts o = resolve_opts(opts);
  fi_solve_stats st{};
  if ((rc = launch_mse_residual(M, f_dev, u_dev, scale_dev, M->d_rgrad))) return rc;
  rc = apply_BT(M, M->d_rgrad, grad_dev, &o, &st);
  if (stats) *stats = st;
  if (rc) return rc;
  FI_HIP_TRY(hipStreamSynchronize(M->ctx->stream));
  if (st.status != FI_OK)
    return fail(FI_E_NO_CONVERGENCE, "adjoint solve did not reach the tolerance");
  return FI_OK;
}

int fi_adjoint(fi_mesh* M, const double* r_dev, double* s_dev, const fi_solve_opts* opts,
               fi_solve_stats* stats) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!r_dev || !s_dev) return fail(FI_E_INVALID, "r_dev and s_dev are required");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  const fi_solve_opts o = resolve_opts(opts);
  fi_solve_stats st{};
  rc = apply_BT(M, r_dev, s_dev, &o, &st);
  if (stats) *stats = st;
  if (rc) return rc;
  FI_HIP_TRY(hipStreamSynchronize(M->ctx->stream));
  if (st.status != FI_OK)
    return fail(FI_E_NO_CONVERGENCE, "adjoint solve did not reach the tolerance");
  return FI_OK;
}


int fi_solve(fi_mesh* M, const double* b_dev, const double* x0_dev, double* x_dev,
             const fi_solve_opts* opts, fi_solve_stats* stats) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (M->n > 0 && (!b_dev || !x_dev)) return fail(FI_E_INVALID, "b_dev and x_dev are required");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  const fi_solve_opts o = resolve_opts(opts);
  fi_solve_stats st{};
  const size_t bytes = (size_t)M->n * sizeof(double);
  if (M->n > 0) {
    FI_HIP_TRY(hipMemcpyAsync(M->d_b64, b_dev, bytes, hipMemcpyDeviceToDevice, M->ctx->stream));
    rc = solve_free(M, &o, &st, x0_dev);
    if (stats) *stats = st;
    if (rc) return rc;
    FI_HIP_TRY(hipMemcpyAsync(x_dev, M->d_x64, bytes, hipMemcpyDeviceToDevice, M->ctx->stream));
    FI_HIP_TRY(hipStreamSynchronize(M->ctx->stream));
  } else if (stats) {
    *stats = st;
  }
  if (st.status != FI_OK)
    return fail(FI_E_NO_CONVERGENCE, "solve did not reach the tolerance");
  return FI_OK;
}

int fi_mesh_export_geometry(const fi_mesh* M, int32_t* vxy, int32_t* tri, int32_t* leaves,
                            int32_t* free_vids, int32_t* mask_vids) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (M->host.vxy.empty() && M->V > 0) {  // built on the device: read the arrays back
    FI_HIP_TRY(hipSetDevice(M->ctx->device));
    hipStream_t st = M->ctx->stream;
    FI_HIP_TRY(hipStreamSynchronize(st));
    if (vxy) FI_HIP_TRY(hipMemcpy(vxy, M->d_vxy, (size_t)(2 * M->V) * 4, hipMemcpyDeviceToHost));
    if (tri) FI_HIP_TRY(hipMemcpy(tri, M->d_tri, (size_t)(3 * M->T) * 4, hipMemcpyDeviceToHost));
    if (leaves) {
      std::vector<int32_t> lv((size_t)(4 * (M->L + 1)));
      FI_HIP_TRY(hipMemcpy(lv.data(), M->d_leaves, lv.size() * 4, hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < M->L; ++i)
        for (int k = 0; k < 3; ++k) leaves[3 * i + k] = lv[(size_t)(4 * i + k)];
    }
    if (free_vids && M->n > 0)
      FI_HIP_TRY(hipMemcpy(free_vids, M->d_free_vids, (size_t)M->n * 4, hipMemcpyDeviceToHost));
    if (mask_vids && M->m > 0)
      FI_HIP_TRY(hipMemcpy(mask_vids, M->d_mask_vids, (size_t)M->m * 4, hipMemcpyDeviceToHost));
    return FI_OK;
  }
  fi_host_mesh view;
  view.mesh = M->host;  // copy: exports are for checking, not the hot path
  return fi_host_mesh_export(&view, vxy, tri, leaves, free_vids, mask_vids);
}

int fi_mesh_export_ss_plan(const fi_mesh* M, int32_t* perm, int32_t* blocks, int32_t* region,
                           uint16_t* lmat) {
  int rc = check_mesh(M);
  if (rc) return rc;
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  return ss_export_plan(M, perm, blocks, region, lmat);
}

int fi_mesh_export_csr(const fi_mesh* Mc, int32_t* ff_rowptr, int32_t* ff_col, double* ff_val,
                       int32_t* fd_rowptr, int32_t* fd_col, double* fd_val) {
  int rc = check_mesh(Mc);
  if (rc) return rc;
  fi_mesh* M = const_cast<fi_mesh*>(Mc);
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  FI_HIP_TRY(hipStreamSynchronize(M->ctx->stream));
  const int64_t n = M->n;
  std::vector<int32_t> rp(n + 1), col(M->nnz_off), frp(n + 1), fcol(M->nnz_fd);
  std::vector<double> val(M->nnz_off), diag(n), fval(M->nnz_fd);
  FI_HIP_TRY(hipMemcpy(rp.data(), M->d_ff_rowptr, (n + 1) * 4, hipMemcpyDeviceToHost));
  if (M->nnz_off) {
    FI_HIP_TRY(hipMemcpy(col.data(), M->d_ff_col, M->nnz_off * 4, hipMemcpyDeviceToHost));
    FI_HIP_TRY(hipMemcpy(val.data(), M->d_ff_val64, M->nnz_off * 8, hipMemcpyDeviceToHost));
  }
  FI_HIP_TRY(hipMemcpy(diag.data(), M->d_diag64, n * 8, hipMemcpyDeviceToHost));
  FI_HIP_TRY(hipMemcpy(frp.data(), M->d_fd_rowptr, (n + 1) * 4, hipMemcpyDeviceToHost));
  if (M->nnz_fd) {
    FI_HIP_TRY(hipMemcpy(fcol.data(), M->d_fd_col, M->nnz_fd * 4, hipMemcpyDeviceToHost));
    FI_HIP_TRY(hipMemcpy(fval.data(), M->d_fd_val, M->nnz_fd * 8, hipMemcpyDeviceToHost));
  }
  // K_FF with its diagonal merged in column order
  int64_t pos = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (ff_rowptr) ff_rowptr[i] = (int32_t)pos;
    bool placed = false;
    for (int32_t j = rp[i]; j < rp[i + 1]; ++j) {
      if (!placed && col[j] > i) {
        if (ff_col) ff_col[pos] = (int32_t)i;
        if (ff_val) ff_val[pos] = diag[i];
        ++pos;
        placed = true;
      }
      if (ff_col) ff_col[pos] = col[j];
      if (ff_val) ff_val[pos] = val[j];
      ++pos;
    }
    if (!placed) {
      if (ff_col) ff_col[pos] = (int32_t)i;
      if (ff_val) ff_val[pos] = diag[i];
      ++pos;
    }
  }
  if (ff_rowptr) ff_rowptr[n] = (int32_t)pos;
  if (fd_rowptr) std::memcpy(fd_rowptr, frp.data(), (n + 1) * 4);
  if (fd_col) std::memcpy(fd_col, fcol.data(), fcol.size() * 4);
  if (fd_val) std::memcpy(fd_val, fval.data(), fval.size() * 8);
  return FI_OK;
}

int fi_owner_map(fi_mesh* M, int32_t* owner_dev) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!owner_dev) return fail(FI_E_INVALID, "owner_dev is NULL");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  // the map the interpolation kernels use (built once with the mesh)
  FI_HIP_TRY(hipMemcpyAsync(owner_dev, M->d_owner, (size_t)M->P * sizeof(int32_t),
                            hipMemcpyDeviceToDevice, M->ctx->stream));
  FI_HIP_TRY(hipStreamSynchronize(M->ctx->stream));
  return FI_OK;
}

int fi_topk_new_pixels(fi_mesh* M, const double* e_dev, int64_t k, int32_t* out_dev) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!e_dev || (!out_dev && k > 0)) return fail(FI_E_INVALID, "e_dev and out_dev are required");
  if (k < 0 || k > M->P - M->m) return fail(FI_E_INVALID, "k out of range");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  return topk_new_pixels(M, e_dev, k, out_dev);
}

int fi_time_cg_kernel(fi_mesh* M, int precision, int reps, double* ms_per_launch) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!ms_per_launch) return fail(FI_E_INVALID, "output is NULL");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  return time_cg_kernel(M, precision, reps, ms_per_launch);
}

int fi_inpaint_rgb(fi_mesh* M, const uint8_t* f_dev, const double* g_dev, double* u_dev,
                   const fi_solve_opts* opts, fi_solve_stats* stats) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!u_dev) return fail(FI_E_INVALID, "u_dev is NULL");
  if (!g_dev && !f_dev) return fail(FI_E_INVALID, "need f_dev or g_dev");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  fi_mesh* ch[kMaxRhs];
  if ((rc = channel_views(M, kMaxRhs, ch))) return rc;
  const fi_solve_opts o = resolve_opts(opts);
  const double* g[kMaxRhs];
  for (int c = 0; c < kMaxRhs; ++c) {
    if (g_dev) {
      g[c] = g_dev + (size_t)c * M->m;
    } else {
      if ((rc = launch_gather_mask(ch[c], f_dev + (size_t)c * M->P, ch[c]->d_g))) return rc;
      g[c] = ch[c]->d_g;
    }
    if ((rc = launch_lift(ch[c], g[c], ch[c]->d_b64))) return rc;
  }
  fi_solve_stats st[kMaxRhs] = {};
  rc = solve_multi(ch, kMaxRhs, &o, st);
  if (stats)
    for (int c = 0; c < kMaxRhs; ++c) stats[c] = st[c];
  if (rc) return rc;
  for (int c = 0; c < kMaxRhs; ++c) {
    if ((rc = launch_vertex_values(ch[c], ch[c]->d_x64, g[c], ch[c]->d_uvert)) ||
        (rc = launch_raster(ch[c], ch[c]->d_uvert, nullptr, nullptr, u_dev + (size_t)c * M->P,
                            nullptr, nullptr, nullptr, nullptr)))
      return rc;
  }
  for (int c = 0; c < kMaxRhs; ++c)
    if (st[c].status != FI_OK)
      return fail(FI_E_NO_CONVERGENCE, "inpainting solve of a channel did not reach the tolerance");
  return FI_OK;
}

int fi_error_rgb(fi_mesh* M, const double* u_dev, const uint8_t* f_dev, double* mse_host,
                 double* mse_ch_host) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!u_dev || !f_dev) return fail(FI_E_INVALID, "u_dev and f_dev are required");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  for (int c = 0; c < kMaxRhs; ++c)
    if ((rc = sse_dev(M, u_dev + (size_t)c * M->P, f_dev + (size_t)c * M->P, M->d_red_out + c)))
      return rc;
  FI_HIP_TRY(hipMemcpyAsync(M->h_red, M->d_red_out, kMaxRhs * sizeof(double),
                            hipMemcpyDeviceToHost, M->ctx->stream));
  FI_HIP_TRY(hipStreamSynchronize(M->ctx->stream));
  double total = 0.0;
  for (int c = 0; c < kMaxRhs; ++c) {
    total += M->h_red[c];
    if (mse_ch_host) mse_ch_host[c] = M->h_red[c] / (double)M->P;
  }
  if (mse_host) *mse_host = total / (double)(kMaxRhs * M->P);
  return FI_OK;
}

int fi_time_cg_multi_kernel(fi_mesh* M, int nrhs, int precision, int reps, double* ms) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!ms) return fail(FI_E_INVALID, "output is NULL");
  FI_HIP_TRY(hipSetDevice(M->ctx->device));
  fi_mesh* ch[kMaxRhs];
  if ((rc = channel_views(M, nrhs, ch))) return rc;
  return time_multi_kernel(ch, nrhs, precision, reps, ms);
}

int fi_cg_multi_kernel_bytes(const fi_mesh* M, int nrhs, int precision, int64_t* bytes) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!bytes || nrhs < 1 || nrhs > kMaxRhs) return fail(FI_E_INVALID, "bad argument");
  *bytes = cg_multi_kernel_bytes(M, nrhs, precision);
  return FI_OK;
}

int fi_cg_kernel_bytes(const fi_mesh* M, int precision, int64_t* bytes) {
  int rc = check_mesh(M);
  if (rc) return rc;
  if (!bytes) return fail(FI_E_INVALID, "output is NULL");
  *bytes = cg_kernel_bytes(M, precision);
  return FI_OK;
}

}  // extern "C"
