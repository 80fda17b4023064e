// Internal declarations shared by the host code and the HIP kernels of the
// library. Nothing here is part of the C ABI (see include/fi.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fi.h"
#include "host_pool.h"

namespace fi {

// ---------------------------------------------------------------- errors --
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define FI_HIP_TRY(expr)                                                                 \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::fi::fail(FI_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

// ------------------------------------------------------------- host mesh --
// The quadtree mesh as built on the host (integer data only).
struct HostMesh {
  int N = 0;                       // image side (power of two)
  int levels = 0;                  // log2(N)
  HostVec<int32_t> leaves;     // (L+1) x 4: x0, y0, level, first triangle;
                                   // the extra row holds (0, 0, 0, T)
  HostVec<int32_t> vxy;        // V x 2: x, y
  HostVec<int32_t> tri;        // T x 3 vertex ids, positive orientation
  HostVec<int32_t> vmap;       // V: free row (>= 0) or -(mask slot + 1)
  HostVec<int32_t> free_vids;  // n
  HostVec<int32_t> mask_vids;  // m
  HostVec<int32_t> mask_pix;   // m: linear pixel index of each mask slot
  bool delaunay = false;           // the Delaunay mesh (no quadtree leaves)

  int64_t L() const { return (int64_t)leaves.size() / 4 - 1; }
  int64_t V() const { return (int64_t)vxy.size() / 2; }
  int64_t T() const { return (int64_t)tri.size() / 3; }
};

// Builds the balanced quadtree mesh. Returns FI_OK or an error code (with
// set_error). Checks: N power of two >= 2, mask strictly ascending in range.
int build_host_mesh(int N, const int32_t* mask, int64_t m, HostMesh& out);

// Incident triangles per vertex never exceed this on a 2:1 balanced quadtree
// with centre fans (four leaves meet at a point, each gives at most two).
constexpr int kMaxIncident = 8;
// Cap on incident triangles per vertex of a Delaunay mesh (the assembly's
// per-row neighbour list).
constexpr int kMaxIncidentGeneral = 31;
// Events per mesh for pacing queued step launches (the ring fi_mesh holds).
constexpr int kChunkEvents = 4;
// Launch-count predictions a mesh keeps (FP32 / FP64 x cold / warm start).
constexpr int kPredSlots = 4;
// Right-hand sides one multi-RHS step advances (a mesh and its channel views).
constexpr int kMaxRhs = 3;

// Builds the paper's Delaunay mesh of the mask pixels, the unknown vertices
// and the four corner pixels (delaunay.cpp). Checks: N power of two in
// [2, 8192], both lists strictly ascending in range, no unknown on a mask
// pixel.
int build_delaunay_mesh(int N, const int32_t* mask, int64_t m, const int32_t* unknown, int64_t nu,
                        HostMesh& out);

// ----------------------------------------------------------- device mesh --
template <typename T>
struct DevBuf {
  T* p = nullptr;
  int64_t n = 0;
};

// Device memory carved out of one allocation (the serving path): first fit
// over a sorted free list, 256-byte granules, neighbours merged on free. The
// bookkeeping is on the host; no call here touches the device except
// init/release, so taking and returning memory never synchronises it.
class Arena {
 public:
  int init(int device, size_t bytes);  // one hipMalloc of `bytes`
  void init_view(void* base, size_t bytes);  // over memory another arena owns
  void release();                      // hipFree of the whole block (if owned)
  void* alloc(size_t bytes);           // nullptr when no free range fits
  void free(void* p);
  size_t capacity() const { return cap_; }
  size_t used() const;
  size_t peak() const;

 private:
  mutable std::mutex mu_;
  char* base_ = nullptr;
  bool owned_ = false;
  size_t cap_ = 0, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;   // offset -> bytes
  std::map<size_t, size_t> live_;   // offset -> bytes
};

// Device blocks a context keeps after the meshes that used them are
// destroyed, for the meshes built after them. hipMalloc and hipFree each
// update the device's page tables, and hipFree waits for the device, so a
// loop that builds a mesh per round would pay both for every array of every
// mesh. A request takes the smallest kept block of at least its size and at
// most a quarter (plus 1 MiB) above it; blocks are given back only after
// the device has finished with them. Up to kKeepBytes are kept; the rest is
// freed, and everything is freed when a hipMalloc fails and when the last
// owner (the context or one of its meshes) goes away.
class DeviceCache {
 public:
  static constexpr size_t kKeepBytes = (size_t)2 << 30;
  explicit DeviceCache(int device) : device_(device) {}
  ~DeviceCache();
  void* take(size_t bytes, size_t* got);
  void give(void* p, size_t bytes);
  void release_all();
  // Pinned host memory of at least `bytes` (up to kStagingMax; null past it
  // or on failure) for copies from the device, kept and grown across calls.
  // One user at a time: the buffer is the caller's while `hold` is locked.
  static constexpr size_t kStagingMax = (size_t)256 << 20;
  void* staging(size_t bytes, std::unique_lock<std::mutex>& hold);

 private:
  std::mutex mu_;
  int device_;
  size_t kept_bytes_ = 0;
  std::multimap<size_t, void*> kept_;  // block size -> block
  std::mutex staging_mu_;
  void* staging_ = nullptr;
  size_t staging_bytes_ = 0;
};

// Device scratch of one build step (the device mesh builder, the device
// s-step plan). For a mesh in an arena (a server request) it comes from the
// arena and goes back to it; otherwise it is a block the mesh's context
// keeps, else its own allocation, and once the stream is done with it it is
// handed to the context (up to kKeepTmp, for the next mesh's build) or freed
// (a large mesh's scratch would otherwise stay held beside the mesh).
struct TmpBlock {
  static constexpr size_t kKeepTmp = (size_t)256 << 20;
  fi_mesh* M;
  void* p = nullptr;
  size_t got = 0;
  explicit TmpBlock(fi_mesh* m) : M(m) {}
  TmpBlock(const TmpBlock&) = delete;
  TmpBlock& operator=(const TmpBlock&) = delete;
  int alloc(size_t bytes);  // FI_E_NOMEM (with the error message) on failure
  bool take(size_t bytes);  // false on failure, no error recorded
  ~TmpBlock();
};

// The S-iteration CG launch (sstep.hip): its plan on the device and its
// vectors, all in the plan's Hilbert-order numbering of the free rows.
struct SsState {
  int grid = 0;             // blocks of one launch (a multiple of 8)
  int max_region = 0;       // largest block region (rows)
  bool large = false;       // a separate launch sums the Gram partials
  int64_t region_rows = 0;  // region rows over all blocks (own rows included)
  int64_t lmat_rows = 0;    // local matrix rows over all blocks
  int32_t* perm = nullptr;  // new index -> natural free row
  void* blocks = nullptr;   // BlockPlan per block
  int32_t* region = nullptr;  // region rows of every block, own rows first
  void* lmat = nullptr;     // 8 x uint16 per local matrix row
  float* W[2] = {nullptr, nullptr};  // per row: P_0..P_S, Z_0..Z_{S-1}, D^-1 (8 floats)
  float* x = nullptr;       // FP32 correction of the inner solve
  float* d = nullptr;       // diagonal of K_FF
  double* b = nullptr;      // right-hand side
  double* r64 = nullptr;    // FP64 residual
  double* x64[2] = {nullptr, nullptr};  // FP64 iterate, by buffer parity
  float* part = nullptr;    // Gram partials (FP32): 2 parities x 32 value rows (value-major)
  double* red = nullptr;    // reduced Gram (large systems): 32 doubles
  // the reduction launch's first-level sums (32 per block of 1024 partials)
  // and the coefficients of the next step launch's iterations, which it
  // computes once for all blocks
  double* level1 = nullptr;
  double* ctl = nullptr;
};

struct CGState {  // state of one fused-CG inner solver in precision T
  void* x = nullptr;
  void* p = nullptr;
  void* rq[2] = {nullptr, nullptr};  // per-row (r, s, q, D^-1), by launch parity
};

}  // namespace fi

struct fi_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::shared_ptr<fi::DeviceCache> cache;  // shared with the meshes built on it
};

struct fi_host_mesh {
  fi::HostMesh mesh;
};

struct fi_mesh {
  fi_ctx* ctx = nullptr;  // borrowed: the context outlives the mesh
  int device = 0;         // copy of ctx->device, used on destruction
  fi::HostMesh host;
  int N = 0;
  int64_t P = 0, V = 0, T = 0, L = 0, n = 0, m = 0;
  int64_t nnz_off = 0;  // off-diagonal entries of K_FF
  int64_t nnz_fd = 0;   // entries of K_FD
  int64_t nnz_df = 0;   // entries of K_DF
  int64_t device_bytes = 0;
  std::vector<void*> allocations;
  std::vector<size_t> alloc_sizes;  // block sizes of `allocations` (outside an arena)
  fi::Arena* arena = nullptr;  // set: memory comes from (and returns to) it
  std::shared_ptr<fi::DeviceCache> cache;  // the context's, outside an arena

  // geometry (device)
  int32_t* d_vxy = nullptr;
  int32_t* d_tri = nullptr;
  int32_t* d_leaves = nullptr;
  int32_t* d_vmap = nullptr;
  int32_t* d_free_vids = nullptr;
  int32_t* d_mask_vids = nullptr;
  int32_t* d_mask_pix = nullptr;
  int32_t* d_vt_ptr = nullptr;
  int32_t* d_vt_idx = nullptr;

  // matrices (device)
  bool assembled_once = false;
  int32_t* d_ff_rowptr = nullptr;  // off-diagonal part of K_FF
  int32_t* d_ff_col = nullptr;
  double* d_ff_val64 = nullptr;
  float* d_ff_val32 = nullptr;
  double* d_diag64 = nullptr;
  double* d_dinv64 = nullptr;
  float* d_dinv32 = nullptr;
  int32_t* d_fd_rowptr = nullptr;
  int32_t* d_fd_col = nullptr;
  double* d_fd_val = nullptr;
  int32_t* d_df_rowptr = nullptr;
  int32_t* d_df_col = nullptr;
  double* d_df_val = nullptr;
  int32_t* d_cnt = nullptr;       // counts scratch (max(n, m) + 1)
  int32_t* d_scan_tmp = nullptr;  // scan scratch

  // solver workspace (device)
  double* d_b64 = nullptr;
  double* d_x64 = nullptr;        // the last solve's result (one of d_x64buf)
  double* d_x64buf[2] = {nullptr, nullptr};
  double* d_r64 = nullptr;
  void* d_rec = nullptr;          // solver state records, two by launch parity
  void* h_mirror = nullptr;       // pinned host copy of the solver state (host pointer)
  void* d_mirror = nullptr;       // the same memory as the device addresses it
  int epoch = 0;                  // id of the latest solve started on this mesh
  // step launches the last solve of each kind took (FP32 / FP64 x cold /
  // warm start), which paces the next one; 0: none yet
  int64_t pred_launches[fi::kPredSlots] = {};
  hipEvent_t chunk_ev[fi::kChunkEvents] = {};  // one after each queued chunk of step launches
  fi::CGState cg32, cg64;
  fi::SsState* ss = nullptr;  // the S-iteration launch's plan and state (FP32 solves), or NULL
  double* d_part = nullptr;   // per-block partial sums: 2 parities x cg_grid x 4
  double* d_red = nullptr;    // reduction scratch (kMaxGrid doubles)
  double* d_red_out = nullptr;  // final reduced scalars (8 doubles)
  double* h_red = nullptr;    // pinned host copies of small device results
  int32_t* h_ctl = nullptr;   // pinned host copy of the packing flags
  int cg_grid = 0;            // blocks of the fused CG kernel
  int cg_bs = 512;            // threads per block of the fused CG kernel
  // ELL copy of the off-diagonal part of K_FF, column-major by row: slot k of
  // row i at d_ell[k * n_pad + i]; each entry is the column (bits 0-29), bit
  // 30 for an empty slot (weight 0, column = the row), bit 31 for weight -1
  // (clear: -1/2). ell_w == 0: CSR is used.
  int32_t* d_ell = nullptr;
  int ell_w = 0;
  int64_t n_pad = 0;
  bool large_mode = false;    // n too large for in-kernel partial re-reduction
  double* d_red4 = nullptr;   // reduced partial sums (large mode)
  double* d_lvl1 = nullptr;   // first-level sums of that reduction
  double* d_prm = nullptr;    // inner-solve parameters read by the CG kernels
  int32_t* d_flag = nullptr;  // packing flags

  // pixel / vertex work vectors (device)
  double* d_uvert = nullptr;  // V
  double* d_g = nullptr;      // m (working copy of g)
  double* d_tpart = nullptr;  // 3T adjoint partials
  double* d_tD = nullptr;     // m
  double* d_rpart = nullptr;  // raster partial sums (one per leaf block)
  int32_t* d_owner = nullptr;      // P: owner triangle of every pixel
  int32_t* d_tri_px_ptr = nullptr; // T + 1: pixel list of each triangle (CSR)
  int32_t* d_tri_px = nullptr;     // P: pixels by owner triangle, ascending within one

  // tonal workspace (device, allocated on first use)
  double* d_tg = nullptr;  // m: p
  double* d_ts = nullptr;  // m: s
  double* d_tr = nullptr;  // P: r
  double* d_tq = nullptr;  // P: q
  double* d_tsc = nullptr; // CGLS scalars (see Cgls)
  double* d_ywarm = nullptr; // n: the last adjoint solve's solution (its next start)
  double* d_rgrad = nullptr; // P: pixel factor of the MSE gradient (first use)
  double* d_wsqrt = nullptr; // P: IRLS weights^(1/2) (L1 tonal optimisation, first use)

  // mask-growth workspace (device, allocated on first use)
  void* d_topk = nullptr;
  int64_t topk_bytes = 0;
  double* d_tri_err = nullptr;   // T: per-triangle error
  int32_t* d_tri_best = nullptr; // T: empty pixel of largest error
  int32_t* d_sel_tri = nullptr;  // selected triangles

  // channels 1 and 2 of a colour image (created on first use): views that
  // share this mesh's geometry, matrices and pixel maps and own their solver
  // state and work vectors
  fi_mesh* chan[fi::kMaxRhs - 1] = {};
  bool is_channel = false;
};

namespace fi {

constexpr int kBlock = 256;      // threads per block of the vector kernels
constexpr int kMaxGrid = 1024;   // cap on blocks of the fused CG kernel
// ELL entry of K_FF: bits 0-29 the column, bit 30 padding (weight 0, column =
// the row itself), bit 31 weight -1 (clear: -1/2).
constexpr int32_t kEllColMask = 0x3FFFFFFF;
constexpr int32_t kEllPadBit = 0x40000000;
constexpr int kRedMaxBlocks = 256;  // blocks of the large-system partial-sum reduction

int device_alloc(fi_mesh* M, void** p, size_t bytes);
// Uploads a host mesh and assembles it; memory from `arena` when not NULL.
// On success the host mesh is consumed (*host set to NULL).
int mesh_upload(fi_ctx* ctx, fi_host_mesh** host, Arena* arena, fi_mesh** out);
// The quadtree mesh built on the device from the mask (host array), then the
// same set-up as mesh_upload.
int mesh_build_on_device(fi_ctx* ctx, int N, const int32_t* mask, int64_t m, fi_mesh** out);
// The quadtree mesh's geometry built on the device (mesh_build_dev.hip; the
// host builder's arrays, bit for bit) into M's device arrays and sizes; the
// host copy keeps N and levels only (its arrays stay empty).
int mesh_geometry_on_device(fi_mesh* M, int N, const int32_t* mask, int64_t m);
// Host copies of a mesh's coordinates and free vertex ids: the host mesh's,
// or read back when the mesh was built on the device.
int mesh_host_coords(const fi_mesh* M, std::vector<int32_t>& vxy, std::vector<int32_t>& free_vids);
// Frees a mesh. A mesh without an arena waits for the device first; an arena
// mesh returns its memory at once (its owner has waited for its last work).
void free_mesh(fi_mesh* M);

// Kernel launchers (kernels.hip). All stream-ordered, no host sync.
int launch_assemble_count(fi_mesh* M, bool free_rows);
int launch_assemble_fill(fi_mesh* M, bool free_rows);
// Re-assembly of a mesh whose pattern and ELL width are known: free and mask
// rows in one launch, the free rows' ELL slots written alongside their CSR
// entries (the same encoding as the packing of the first assembly).
int launch_assemble_refill(fi_mesh* M);
int scan_counts(fi_mesh* M, const int32_t* cnt, int32_t* rowptr, int64_t n);
// Exclusive prefix sum of n ints with caller scratch of scan_tmp_ints(n) ints.
int scan_exclusive(hipStream_t st, const int32_t* in, int32_t* out, int64_t n, int32_t* tmp);
int64_t scan_tmp_ints(int64_t n);
// Default absolute residual bound of a solve (fi_solve_opts.atol). A
// pixel's error is the residual amplified by K_FF^-1; measured against FP64
// solves to 1e-13 (512^2 to 8192^2 images, masks of 1 to 10%), the worst
// pixel error over ||b - K_FF x||_2 was 0.06 to 0.21, so stopping at
// ||r|| <= 3e-6 keeps every pixel within about 6e-7.
constexpr double kDefaultAtol = 3e-6;
// Solve options with every unset (0 or out-of-range) field at its default.
fi_solve_opts resolve_opts(const fi_solve_opts* o);
int launch_lift(fi_mesh* M, const double* g, double* b);
int launch_gather_mask(fi_mesh* M, const uint8_t* f, double* g);
int launch_vertex_values(fi_mesh* M, const double* xF, const double* g, double* uvert);
// Leaf-major interpolation / error pass. Pixel values come from u_in when
// given, else from interpolating the vertex values uvert (NULL: zeros).
int launch_raster(fi_mesh* M, const double* uvert, const double* u_in, const uint8_t* f,
                  double* u_out, double* e_out, double* tri_err_out, int32_t* owner_out,
                  double* partial_out);
int raster_blocks(const fi_mesh* M);
// u_out = B u (pixel values from vertex values) and *sq_dev = ||u_out||^2,
// with the bits of launch_raster followed by launch_dot.
int launch_interp_sq(fi_mesh* M, const double* uvert, double* u_out, double* sq_dev);
// Owner map and per-triangle pixel lists (geometry only; once per mesh).
int build_pixel_maps(fi_mesh* M);
// Vertex -> (triangle, corner) lists on the device from the uploaded
// triangles (needs the workspace); checks the incident-triangle bounds.
int build_vertex_triangles(fi_mesh* M);
// t = R^T r, or R^T (w r) when w is given (weighted least squares).
int launch_raster_transpose(fi_mesh* M, const double* r, double* tpart,
                            const double* w = nullptr);
// Per triangle: total error of its pixels, and its empty pixel of largest
// error (-1 if none); in_mask holds one byte per pixel.
int launch_tri_best(fi_mesh* M, const double* e, const uint8_t* in_mask, double* tri_err,
                    int32_t* tri_best);
int launch_gather_vertex(fi_mesh* M, const double* tpart, double* tF, double* tD);
int launch_adjoint_tail(fi_mesh* M, const double* tD, const double* y, double* s);
// out[c] = sum of component c of the partials, divided by div
int launch_reduce(fi_mesh* M, const double* part, int nparts, int ncomp, double* out,
                  double div = 1.0);
int launch_dot(fi_mesh* M, const double* a, const double* b, int64_t n, double* out_dev);
// y += sign * (num / den) x and y = x + (num / den) y, the ratio read from
// device scalars (0 when den <= 0).
// y1 += (num / den) x1 (length n1) and y2 -= (num / den) x2 (length n2), one launch.
int launch_axpy2_ratio(fi_mesh* M, int64_t n1, int64_t n2, const double* num, const double* den,
                       const double* x1, double* y1, const double* x2, double* y2);
int launch_axpy_ratio(fi_mesh* M, int64_t n, const double* num, const double* den, double sign,
                      const double* x, double* y);
int launch_xpby_ratio(fi_mesh* M, int64_t n, const double* x, const double* num, const double* den,
                      double* y);
// r = f - u, or w (f - u) when w is given.
int launch_pixel_residual(fi_mesh* M, const uint8_t* f, const double* u, double* r,
                          const double* w = nullptr);
int launch_scale(fi_mesh* M, int64_t n, const double* w, double* x);  // x *= w
// r = 2 s (u - f) / P with s = *scale (NULL: 1)
int launch_mse_residual(fi_mesh* M, const uint8_t* f, const double* u, const double* scale,
                        double* r);
// IRLS weights w^(1/2) = sqrt(1 / max(|f - u|, eps)) per pixel.
int launch_irls_weights(fi_mesh* M, const uint8_t* f, const double* u, double eps,
                        double* wsqrt);
// sum |u - f| into *out_dev (fixed-order reduction).
int launch_abs_err(fi_mesh* M, const double* u, const uint8_t* f, double* out_dev);

// Solver pieces (solver.hip).
constexpr int kMaxEll = 8;
int solver_setup(fi_mesh* M);      // after assembly: ELL packing, launch shape
void solver_release(fi_mesh* M);   // events and the host mirror
// Solves K_FF x = b64 from x0 (device, n doubles, not a buffer of the mesh's
// solver; NULL: from 0), to the same relative residual ||b - K x|| / ||b||.
int solve_free(fi_mesh* M, const fi_solve_opts* opts, fi_solve_stats* stats,
               const double* x0 = nullptr);
int time_cg_kernel(fi_mesh* M, int precision, int reps, double* ms);
int64_t cg_kernel_bytes(const fi_mesh* M, int precision);
int64_t cg_multi_kernel_bytes(const fi_mesh* M, int nrhs, int precision);
// Solver state of one solve (records, partials, mirror, events); solver_setup
// calls it, and a channel view gets its own with the parent's launch shape.
int alloc_solver_state(fi_mesh* M);
int solver_channel_setup(fi_mesh* S, const fi_mesh* M);

// The S-iteration CG launch (sstep.hip). ss_setup builds its plan after the
// first assembly of a quadtree mesh (nothing for other meshes, or when
// FI_CG_SSTEP=0) and refreshes the matrix values after later ones.
constexpr int kSsIters = 3;  // CG iterations per launch
int ss_setup(fi_mesh* M);
// The plan built on the device (ss_plan_dev.hip) into Z's plan arrays and
// shape; *built stays false when a region would exceed max_region rows or a
// row has more entries than the plan's slots (the mesh keeps the
// one-iteration launch).
int ss_plan_on_device(fi_mesh* M, int S, int max_region, SsState& Z, bool* built);
// Bound of the device scratch ss_plan_on_device takes for n rows (a server
// request's footprint reserves it).
int64_t ss_plan_scratch_bound(int64_t n);
// Copies the plan to host buffers (fi_mesh_export_ss_plan).
int ss_export_plan(const fi_mesh* M, int32_t* perm, int32_t* blocks, int32_t* region,
                   uint16_t* lmat);
void ss_release(fi_mesh* M);
// FP32 solve of K_FF x = b64 from x0 (natural order, may be NULL) with the
// S-iteration launch; the result in d_x64 (natural order).
int ss_solve(fi_mesh* M, const fi_solve_opts* opts, fi_solve_stats* stats, const double* x0);
int ss_time_kernel(fi_mesh* M, int reps, double* ms);
// The same for the channel views ch[0..nc-1] of one mesh in one launch per
// step (each channel the bits of its own ss_solve), and its timing.
int ss_solve_multi(fi_mesh* const* ch, int nc, const fi_solve_opts* opts, fi_solve_stats* stats,
                   const double* const* x0);
int ss_time_multi(fi_mesh* const* ch, int nc, int reps, double* ms);
int ss_channel_setup(fi_mesh* S, const fi_mesh* M);
// Batched steps of meshes that all have the plan (see batch_launch_steps),
// and the start of such a solve.
int ss_batch_launch(hipStream_t st, const std::vector<fi_mesh*>& ms, int count);
int ss_arm(fi_mesh* M, const fi_solve_opts* opts, int epoch, const double* x0);
// Device bytes the S-iteration state of a system with n rows may take.
int64_t ss_footprint(int64_t n);

// Multi-RHS solves (solver.hip): K_FF x_c = b64 of channel view c, for the nc
// views in ch (ch[0] the mesh itself), advanced together by one step launch
// per iteration whose blocks for the same rows share an XCD (and so the
// matrix in its L2); each channel's result and stats are those of its own
// solve_free, bit for bit.
// x0: NULL, or a start for each channel (entries may be NULL).
int solve_multi(fi_mesh* const* ch, int nc, const fi_solve_opts* opts, fi_solve_stats* stats,
                const double* const* x0 = nullptr);
int time_multi_kernel(fi_mesh* const* ch, int nc, int precision, int reps, double* ms);
// The mesh and its channel views 1..nc-1 (created on first use) into ch.
int channel_views(fi_mesh* M, int nc, fi_mesh** ch);

// Batched stepping (solver.hip): the FP32 solves of several meshes advance
// together, one step launch for all of them (for up to 20 meshes; more take
// further launches per step).
constexpr int kMaxSlots = 64;  // meshes a server keeps resident at once
constexpr int kBatchBS = 512;  // the batched step needs this block size
struct BatchSlot {
  fi_mesh* M;
};
// `count` (even) step launches over the meshes in `act`, parity 0 first.
int batch_launch_steps(hipStream_t st, const std::vector<BatchSlot>& act, int count);
// Start of an FP32 solve of K_FF x = b64 that the batch then steps; *epoch
// identifies it in the host mirror.
int solve_arm(fi_mesh* M, const fi_solve_opts* opts, int* epoch, const double* x0 = nullptr);
// Reads the host mirror of the solve `epoch`: *done = 1 once it has ended
// (stats filled, d_x64 set to the result). Never blocks.
int solve_poll(fi_mesh* M, int epoch, fi_solve_stats* stats, int* done);

// CGLS on the normal equations B^T B g = B^T f (Section 4), split into
// segments that each end in one solve with K_FF: the caller runs pre(),
// then the solve of K_FF x = b64, then post(). All scalars of the method stay
// on the device, so the same segments serve the host-driven call and the
// batched server bit for bit.
struct Cgls {
  enum Seg : int { kInpaint = 0, kAdjoint = 1, kApplyP = 2, kFinal = 3, kDone = 4 };
  // device scalar slots in d_tsc
  enum : int { kScRR0 = 0, kScGamma = 1 /* and 2, by iteration parity */, kScQQ = 3, kScSSE = 4,
               kScAbs = 5 /* sum |B g - f| (L1 optimisation) */ };
  fi_mesh* M = nullptr;
  const uint8_t* f = nullptr;  // device image
  double* g = nullptr;         // device, m: in the start (if start_from_g), out g
  const double* wsqrt = nullptr;  // device, P: weights^(1/2) (weighted least squares), or none
  bool start_from_g = false;
  int k = 0;                   // B p products applied
  Seg seg = kInpaint;
  // Start of the segment's solve (set by pre()): the adjoint solve starts
  // from the previous adjoint solution, since r, and with it R^T r, changes
  // less and less from one iteration to the next; other solves start at 0.
  const double* x0 = nullptr;
  bool use_warm = true;        // keep adjoint solutions as starts
  bool warm = false;           // d_ywarm holds an adjoint solution

  int alloc();                 // tonal workspace (first use)
  int pre();                   // right-hand side of the segment's solve into b64
  int post();                  // consumes d_x64; does not advance seg
  const double* scalar(int i) const { return M->d_tsc + i; }
};

// Mask growth (topk.hip).
int topk_new_pixels(fi_mesh* M, const double* e, int64_t k, int32_t* out);
// Section 3's step: up to k new pixels (ascending) into out; *added of them.
int paper_densify_step(fi_mesh* M, const double* e, int64_t k, int32_t* out, int64_t* added);

}  // namespace fi
