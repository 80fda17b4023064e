/*
 * fi.h - C ABI of the MI355X library for FEM harmonic inpainting with
 * optimised data (Chizhov and Weickert, arXiv 2105.01586).
 *
 * The library computes, on one AMD Instinct MI355X (gfx950):
 *   inpaint(f, mask, g) -> u   harmonic inpainting with P1 finite elements
 *                              (Section 2.1 eqs. (1)-(3), Section 2.2);
 *   error(u, f)                squared error map, MSE and per-triangle L2
 *                              error (Section 3);
 *   adjoint(r) -> B^T r        transpose of the inpainting map u = B g
 *                              (Section 4);
 *   tonal_opt(f, mask) -> g    least-squares grey values, CG on the normal
 *                              equations B^T B g = B^T f (Section 4, eqs. (4),
 *                              (5)), with inner solves instead of forming B.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Images are N x N with N a power of two >= 2, stored row-major: pixel
 *   (r, c) has linear index r * N + c and sits at the mesh lattice point
 *   (x = c, y = r). f is uint8, u and every pixel-sized vector are float64.
 * - The mask is a host array of m >= 1 strictly ascending int32 linear pixel
 *   indices. g (the stored values) is float64 of length m in that order.
 * - The mesh is the 2:1 edge-balanced quadtree on [0, N]^2 refined to unit
 *   cells at every mask pixel, each leaf cut into right isosceles triangles
 *   (two per leaf, or a fan from the centre when a neighbour is finer). Every
 *   mask pixel is a vertex (Section 2.2). Vertices are numbered in row-major
 *   (y, x) order; free rows are the non-mask vertices in that order.
 * - Pointers named *_dev are device pointers on the context's device; the
 *   caller owns them and keeps them alive for the duration of the call. All
 *   device work is ordered on the context's HIP stream; a call returns after
 *   the stream work it needs for host-visible results has finished. The
 *   library never frees caller memory.
 * - Every call returns a status code (FI_OK = 0). On failure
 *   fi_last_error() gives a message (per calling thread). Outputs are left
 *   unspecified unless stated, except FI_E_NO_CONVERGENCE, where outputs hold
 *   the last iterate and the stats report the residual reached.
 * - One fi_mesh must not be used by two calls at the same time.
 */
#ifndef FI_H
#define FI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum fi_status {
  FI_OK = 0,
  FI_E_INVALID = 1,        /* bad argument: shape, ordering, range, NaN */
  FI_E_EMPTY_MASK = 2,     /* m == 0: the system is singular (Section 2.2) */
  FI_E_NO_CONVERGENCE = 3, /* iteration cap reached before the tolerance */
  FI_E_NOMEM = 4,          /* device or host allocation failed */
  FI_E_HIP = 5             /* a HIP runtime call failed */
};

enum fi_precision {
  FI_PREC_FP32_IR = 0, /* FP32 Jacobi-PCG inner solves, FP64 residual and
                          iterative refinement (default) */
  FI_PREC_FP64 = 1     /* plain FP64 Jacobi-PCG, FP64 residual check */
};

typedef struct fi_ctx fi_ctx;
typedef struct fi_mesh fi_mesh;

/* Options of one solve of K_FF u_F = b (the harmonic extension). */
typedef struct fi_solve_opts {
  int precision;     /* enum fi_precision */
  double rtol;       /* stop when ||b - K_FF x||_2 <= rtol * ||b||_2 (FP64)
                        and <= atol (below). A pixel's error is the residual
                        amplified by K_FF^-1: measured against FP64 solves to
                        1e-13 on 512^2 to 8192^2 images with 1-10% masks, the
                        worst pixel error was 0.06-0.21 times ||r||_2, so the
                        relative test alone does not hold a fixed pixel bound
                        (1e-10 left 3.9e-6 at 8192^2, 2.4e-6 at 2048^2 with a
                        10% mask). The default atol, 3e-6, keeps every pixel
                        of those images within 1e-6 (at most 3e-7 measured). */
  double inner_rtol; /* each inner solve reduces its residual by this factor
                        (default 1e-5); the final stop above, not this, sets
                        the accuracy */
  int max_inner;     /* iteration cap of one inner solve */
  int max_refine;    /* cap on refinement steps (outer FP64 residual checks) */
  int check_every;   /* unused (the host reads the solver state once per
                        chunk of launches); kept for the layout */
  double atol;       /* absolute bound: the solve also runs until
                        ||b - K_FF x||_2 <= atol (FP64; b in grey levels, as
                        g), i.e. it stops at ||r|| <= min(rtol ||b||, atol).
                        0: the default, 3e-6; negative: no absolute bound. */
} fi_solve_opts;

typedef struct fi_solve_stats {
  int64_t iterations;  /* CG iterations, all inner solves together */
  int32_t refinements; /* inner solves (refinement steps) performed */
  int32_t status;      /* FI_OK or FI_E_NO_CONVERGENCE */
  double rel_residual; /* final ||b - K_FF x||_2 / ||b||_2 in FP64 */
  double residual;     /* final ||b - K_FF x||_2 in FP64 */
  double rhs_norm;     /* ||b||_2 */
  int64_t launches;    /* step launches until the solve ended (the start launch
                          and launches queued past the end not counted; each
                          advances up to fi_mesh_info.cg_iters_per_launch
                          iterations, or applies a refinement) */
} fi_solve_stats;

typedef struct fi_tonal_opts {
  fi_solve_opts inner; /* options of every inner solve */
  double rtol;         /* stop when ||B^T(f - B g)|| <= rtol ||B^T(f - B g0)||;
                          0: run max_outer iterations (then FI_OK);
                          < 0: 1e-8 */
  int max_outer;       /* cap on outer CG iterations */
  int start_from_g;    /* 0: start from g0 = f on the mask; 1: from g_dev */
  int cold_adjoint;    /* 0: each adjoint solve starts from the previous one's
                          solution (same stopping test, fewer iterations);
                          1: from 0 */
} fi_tonal_opts;

typedef struct fi_tonal_stats {
  int32_t outer_iterations;
  int32_t status;         /* FI_OK or FI_E_NO_CONVERGENCE */
  int64_t inner_iterations;
  double rel_normal_residual; /* ||s_k|| / ||s_0|| with s = B^T (f - B g) */
  double mse_initial;     /* MSE of B g0 against f */
  double mse_final;       /* MSE of B g against f */
} fi_tonal_stats;

/* L1 tonal optimisation by iteratively reweighted least squares (see
 * fi_tonal_opt_l1). */
typedef struct fi_l1_opts {
  fi_solve_opts inner; /* every solve with K_FF */
  double eps;          /* floor of |r| in the weights 1 / max(|r|, eps) (grey levels) */
  int irls_iters;      /* K: reweighting steps */
  int cgls_iters;      /* J: CGLS iterations per step (from the current g) */
  int start_from_g;    /* nonzero: g_dev holds the start values */
} fi_l1_opts;

typedef struct fi_l1_stats {
  int32_t irls_iters;
  int32_t status;
  int64_t inner_iterations; /* CG iterations over all solves */
  double mae_initial;       /* mean |B g0 - f| */
  double mae_final;         /* mean |B g - f| */
  double mse_final;         /* MSE of B g */
} fi_l1_stats;

typedef struct fi_mesh_info {
  int64_t N;      /* image side */
  int64_t P;      /* pixels, N * N */
  int64_t V;      /* mesh vertices */
  int64_t T;      /* triangles */
  int64_t L;      /* quadtree leaves */
  int64_t n;      /* free vertices (unknowns) */
  int64_t m;      /* mask pixels */
  int64_t nnz_ff; /* stored entries of K_FF, diagonal included */
  int64_t nnz_fd; /* stored entries of K_FD */
  int64_t device_bytes; /* device memory held by the mesh */
  int64_t cg_blocks;    /* blocks of one FP32 CG step launch (0 before assembly) */
  int64_t cg_block_size; /* threads per block of that launch */
  int64_t large_mode;   /* 1: a separate launch sums the step's partial sums */
  int64_t cg_iters_per_launch; /* CG iterations one FP32 step launch advances:
                                  3 on the quadtree mesh (blocks of rows in
                                  Hilbert order with 3-hop halos), else 1 */
  int64_t cg_max_region;  /* rows of the largest block region (3 per launch), or 0 */
  int64_t cg_region_rows; /* region rows over all blocks (own rows included), or 0 */
  int64_t cg_lmat_rows;   /* local matrix rows over all blocks (rows within S - 1
                             hops), or 0 */
} fi_mesh_info;

/* Default solve options: FP32 inner PCG with FP64 refinement to 1e-10. */
void fi_solve_opts_default(fi_solve_opts* opts);
/* Default tonal options: inner defaults, rtol 1e-8, 500 outer iterations. */
void fi_tonal_opts_default(fi_tonal_opts* opts);

/* Message of the last failure on the calling thread ("" if none). */
const char* fi_last_error(void);

/* Library version string. */
const char* fi_version(void);

/* Context: binds a device and a HIP stream (hipStream_t passed as void*; NULL
 * means the null stream). The stream is borrowed, not owned. A context must
 * outlive every mesh built on it: destroy the meshes first.
 * A context keeps the device blocks of meshes destroyed on it (up to 2 GiB)
 * for the meshes built after them (a request takes a kept block of at least
 * its size and at most a quarter plus 1 MiB above it), and one pinned host
 * staging buffer (up to 256 MiB); fi_ctx_destroy frees them once no mesh
 * built on the context is left. A failed device allocation frees the kept
 * blocks and tries again. */
int fi_ctx_create(int device, void* stream, fi_ctx** out);
int fi_ctx_set_stream(fi_ctx* ctx, void* stream);
int fi_ctx_destroy(fi_ctx* ctx);

/* Builds the quadtree mesh for an N x N image (width == height == N) and the
 * mask (host array, strictly ascending, in range) on the device (the mask is
 * checked on the host and uploaded), and assembles the stiffness matrix
 * (fi_assemble). The mesh rules are those of Section 2.2 with the quadtree
 * reading stated above; the mesh equals fi_host_mesh_build's array for array
 * (with the environment variable FI_MESH_HOST=1 it is built by that host
 * builder and uploaded). Synchronous. Errors: FI_E_INVALID (shape, ordering,
 * range), FI_E_EMPTY_MASK (m == 0). */
int fi_mesh_build(fi_ctx* ctx, int width, int height, const int32_t* mask_idx, int64_t m,
                  fi_mesh** out);
/* Waits for the device, then returns the mesh's device blocks to its
 * context (see fi_ctx_create) or, for a server request, to its arena. */
int fi_mesh_destroy(fi_mesh* mesh);
int fi_mesh_get_info(const fi_mesh* mesh, fi_mesh_info* info);

/* Host-only mesh: the same quadtree mesh built on the CPU with no device
 * work, for building meshes on worker threads (or checking them without a
 * GPU). fi_host_mesh_info fills the geometric counts (nnz fields are 0).
 * fi_mesh_upload moves a host mesh to the device, assembles it, and consumes
 * the host mesh (*host is set to NULL on success). Errors as fi_mesh_build. */
typedef struct fi_host_mesh fi_host_mesh;
int fi_host_mesh_build(int width, int height, const int32_t* mask_idx, int64_t m,
                       fi_host_mesh** out);
int fi_host_mesh_info(const fi_host_mesh* host, fi_mesh_info* info);
int fi_host_mesh_export(const fi_host_mesh* host, int32_t* vxy, int32_t* tri, int32_t* leaves,
                        int32_t* free_vids, int32_t* mask_vids);
int fi_host_mesh_destroy(fi_host_mesh* host);
int fi_mesh_upload(fi_ctx* ctx, fi_host_mesh** host, fi_mesh** out);

/* The paper's own mesh (Section 2.2): every mask pixel is a vertex, the
 * unknown_idx pixels are the "unknown vertices" (Section 3 draws them at
 * random; here they are an input), and the point set, with the four corner
 * pixels always included, is triangulated by Delaunay. Pixel (r, c) is the
 * point (x = c, y = r); vertex ids follow the pixel index. Where four or more
 * vertices are cocircular the triangulation is made unique by symbolic
 * perturbation of the lifted heights (lower vertex ids perturbed more), and
 * triangles are listed counter-clockwise from their lowest vertex id in
 * lexicographic order. A pixel's owner triangle is the lowest-index triangle
 * holding it. Everything else (assembly, solves, interpolation, error,
 * adjoint, tonal, colour, the per-triangle densification step) works on it
 * as on the quadtree mesh; its stiffness entries are general cotangent
 * weights, so the solver uses the CSR layout. The batched server takes
 * quadtree meshes only.
 *   side: power of two in [2, 8192]; mask_idx, unknown_idx: host int32,
 *   each strictly ascending and in range, disjoint.
 * Errors: FI_E_INVALID (shape, ordering, range, overlap, a vertex with more
 * than 31 incident triangles), FI_E_EMPTY_MASK (m == 0). The host variant
 * builds without a device (for checking). */
int fi_mesh_build_delaunay(fi_ctx* ctx, int side, const int32_t* mask_idx, int64_t m,
                           const int32_t* unknown_idx, int64_t nu, fi_mesh** out);
int fi_host_mesh_build_delaunay(int side, const int32_t* mask_idx, int64_t m,
                                const int32_t* unknown_idx, int64_t nu, fi_host_mesh** out);

/* (Re)assembles the P1 stiffness matrix on the device: element matrices
 * K^e_ij = (b_i b_j + c_i c_j) / (4A) summed per vertex row, split into the
 * free block K_FF, the coupling K_FD and its transpose K_DF; exact zeros are
 * dropped (Section 2.2). Stream-ordered; no host sync except the first call,
 * which sizes the matrices. */
int fi_assemble(fi_mesh* mesh);

/* Inpainting u = B g (Section 2.2, Section 4): solves K_FF u_F = -K_FD g
 * (Section 2.2: SPD with at least one mask pixel, solved by CG; here Jacobi
 * PCG) and interpolates linearly inside each triangle to all P pixels.
 *   f_dev:  uint8[P] image; used only when g_dev is NULL (then g = f on the
 *           mask). May be NULL when g_dev is given.
 *   g_dev:  float64[m] mask values, or NULL.
 *   u_dev:  float64[P] output pixels.
 *   opts:   NULL for defaults. stats: may be NULL. */
int fi_inpaint(fi_mesh* mesh, const uint8_t* f_dev, const double* g_dev, double* u_dev,
               const fi_solve_opts* opts, fi_solve_stats* stats);

/* One-shot inpainting of an image given as a mask bitmap: builds the
 * quadtree mesh of the pixels where mask_u8_host is nonzero (host
 * uint8[width * height], row-major), inpaints as fi_inpaint, and frees the
 * mesh. For repeated calls on one mask, build the mesh once instead.
 * Errors as fi_mesh_build and fi_inpaint. */
int fi_inpaint_image(fi_ctx* ctx, int width, int height, const uint8_t* f_dev,
                     const uint8_t* mask_u8_host, const double* g_dev, double* u_dev,
                     const fi_solve_opts* opts, fi_solve_stats* stats);

/* The vertex values of the last fi_inpaint on this mesh, float64[V] in
 * vertex order, copied to a device buffer. */
int fi_vertex_values(fi_mesh* mesh, double* u_vertex_dev);

/* Error measures of Section 3: e_i = (u_i - f_i)^2, MSE = sum(e) / P, and the
 * total e over the pixels each triangle owns (a pixel belongs to the first
 * triangle of its quadtree leaf, in listing order, that contains it).
 *   mse_host:    output scalar (may be NULL);
 *   pix_err_dev: float64[P] output, or NULL;
 *   tri_err_dev: float64[T] output, or NULL.
 * Sums use a fixed order, so results are reproducible run to run. */
int fi_error(fi_mesh* mesh, const double* u_dev, const uint8_t* f_dev, double* mse_host,
             double* pix_err_dev, double* tri_err_dev);

/* The harmonic-extension system itself (Section 2.2: K_FF x = b, SPD, solved
 * by CG; here Jacobi PCG, FP32 iterations with FP64 refinement, or FP64), for
 * a caller's right-hand side, started from x0.
 *   b_dev:  float64[n] right-hand side, free unknowns in ascending free-vertex
 *           order (the order fi_mesh_export_geometry gives free_vids).
 *   x0_dev: float64[n] start, or NULL for 0. The stopping test is
 *           ||b - K_FF x|| <= opts->rtol ||b|| whatever the start, so a good
 *           start only saves iterations; with b = 0 the result is x = 0.
 *   x_dev:  float64[n] output (may be x0_dev or b_dev).
 * Stream-ordered on the context's stream; returns after the solve has ended.
 * Errors: FI_E_INVALID (NULL b_dev or x_dev while n > 0, non-finite values),
 * FI_E_NO_CONVERGENCE (x_dev still written). */
int fi_solve(fi_mesh* mesh, const double* b_dev, const double* x0_dev, double* x_dev,
             const fi_solve_opts* opts, fi_solve_stats* stats);

/* The squared-error sum of fi_error, sum_i (u_i - f_i)^2 (MSE = sum / P),
 * left in device memory: stream-ordered, no host synchronisation, the same
 * bits as fi_error's sum (the same kernels and order).
 *   sse_dev: one float64 output on the device. */
int fi_error_dev(fi_mesh* mesh, const double* u_dev, const uint8_t* f_dev, double* sse_dev);

/* The MSE of Section 3, sum_i (u_i - f_i)^2 / P over all P pixels (mask
 * pixels included), left in device memory: stream-ordered, no host
 * synchronisation. The sum is fi_error_dev's (same kernels, same order)
 * divided by P on the device.
 *   u_dev: float64[P]; f_dev: uint8[P]; mse_dev: one float64 output. */
int fi_mse_dev(fi_mesh* mesh, const double* u_dev, const uint8_t* f_dev, double* mse_dev);

/* Gradient of the MSE with respect to the stored values g (Section 4: for
 * MSE(g) = ||B g - f||^2 / P it is (2 / P) B^T (B g - f)), scaled by a
 * caller's factor: grad = s (2 / P) B^T (u - f), with u = B g the caller's
 * inpainting result (fi_inpaint of the same g). This is the backward pass of
 * the MSE as a function of g: s is d loss / d MSE.
 *   u_dev: float64[P]; f_dev: uint8[P];
 *   scale_dev: one float64 on the device holding s, or NULL for s = 1;
 *   grad_dev: float64[m] output, in mask order.
 * One adjoint solve (as fi_adjoint) with opts (NULL: defaults); returns after
 * it has ended. Errors as fi_adjoint. */
int fi_mse_backward(fi_mesh* mesh, const double* u_dev, const uint8_t* f_dev,
                    const double* scale_dev, double* grad_dev, const fi_solve_opts* opts,
                    fi_solve_stats* stats);

/* Adjoint of the inpainting map, s = B^T r = t_D - K_DF K_FF^{-1} t_F with
 * t = R^T r (R: interpolation to pixels). Section 4's nested CG applies it
 * through one more solve with the same symmetric matrix.
 *   r_dev: float64[P]; s_dev: float64[m] output. */
int fi_adjoint(fi_mesh* mesh, const double* r_dev, double* s_dev, const fi_solve_opts* opts,
               fi_solve_stats* stats);

/* Tonal optimisation (Section 4): g* = argmin ||B g - f||^2 by CG on the
 * normal equations in least-squares form (CGLS): residual r = f - B g,
 * s = B^T r; B is applied through inner solves, never formed.
 *   f_dev: uint8[P]; g_dev: float64[m], start value if opts->start_from_g,
 *   result on return. opts: NULL for defaults. */
int fi_tonal_opt(fi_mesh* mesh, const uint8_t* f_dev, double* g_dev, const fi_tonal_opts* opts,
                 fi_tonal_stats* stats);

/* Defaults: eps = 0.5, irls_iters = 8, cgls_iters = 20, inner as
 * fi_solve_opts_default, start_from_g = 0. */
void fi_l1_opts_default(fi_l1_opts* opts);

/* Tonal optimisation for the L1 error E1(g) = sum_i |(B g)_i - f_i| (the
 * paper optimises its large colour result for it and states no method; this
 * is iteratively reweighted least squares). From g0 = f on the mask (or the
 * given g), each of irls_iters steps computes r = f - B g, the weights
 * w = 1 / max(|r|, eps), and runs cgls_iters iterations of the CGLS of
 * fi_tonal_opt on W^(1/2) B with right side W^(1/2) f, started from g. The
 * Huber function of the residual (|r| above eps, r^2 / (2 eps) + eps / 2
 * below) never increases from step to step.
 *   f_dev: uint8[P]; g_dev: float64[m] (start if start_from_g; result);
 *   mae_hist: host float64[irls_iters + 1] or NULL, the mean |B g - f| at
 *   the start and after each step. Synchronous (one host read per step). */
int fi_tonal_opt_l1(fi_mesh* mesh, const uint8_t* f_dev, double* g_dev, const fi_l1_opts* opts,
                    fi_l1_stats* stats, double* mae_hist);

/* Export of the mesh for checking (host buffers of the stated sizes, each may
 * be NULL): vertex lattice coordinates int32[V][2] (x, y); triangles
 * int32[T][3] (vertex ids, positive orientation); leaves int32[L][3]
 * (x0, y0, level) in Morton order; free vertex ids int32[n]; mask vertex ids
 * int32[m]. Synchronous. */
int fi_mesh_export_geometry(const fi_mesh* mesh, int32_t* vxy, int32_t* tri, int32_t* leaves,
                            int32_t* free_vids, int32_t* mask_vids);

/* Export of the assembled matrices as CSR (host buffers, each may be NULL):
 * K_FF int32 rowptr[n+1], int32 col[nnz_ff], float64 val[nnz_ff] (diagonal
 * included, columns ascending); K_FD int32 rowptr[n+1], col[nnz_fd] (mask
 * slots), float64 val[nnz_fd]. Synchronous. */
int fi_mesh_export_csr(const fi_mesh* mesh, int32_t* ff_rowptr, int32_t* ff_col, double* ff_val,
                       int32_t* fd_rowptr, int32_t* fd_col, double* fd_val);

/* Export of the plan of the S-iteration launch (rows in blocks of 512 with
 * S-hop halos over a Hilbert-order numbering of the free rows; see
 * cg_iters_per_launch), for checking it against a builder of its own (host
 * buffers, each may be NULL): perm int32[n] (new index -> free row);
 * blocks int32[cg_blocks][8] (region offset, local matrix offset, own rows,
 * rows within 1 hop, within S - 1 hops, within S hops, the largest region in
 * block 0's seventh field, 0); region int32[cg_region_rows] (each block's
 * rows: own rows, then the rings at distance 1..S, ascending within a ring);
 * lmat uint16[cg_lmat_rows][6] (per local matrix row: neighbour slot = local
 * index + 1 in bits 0-13, 0 and bit 14 for padding, bit 15 for weight -1).
 * FI_E_INVALID if the mesh has no such plan. Synchronous. */
int fi_mesh_export_ss_plan(const fi_mesh* mesh, int32_t* perm, int32_t* blocks, int32_t* region,
                           uint16_t* lmat);

/* Owner triangle of every pixel, int32[P] device output (the rule of
 * fi_error). */
int fi_owner_map(fi_mesh* mesh, int32_t* owner_dev);

/* Global top-k mask growth: the k non-mask pixels with the largest e
 * (float64[P] device input), ties broken by the lower linear index. Writes
 * the k selected indices in ascending order to out_dev (int32[k], device).
 * Errors: FI_E_INVALID if k exceeds the number of non-mask pixels. */
int fi_topk_new_pixels(fi_mesh* mesh, const double* e_dev, int64_t k, int32_t* out_dev);

/* fi_topk_new_pixels without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). Same arguments, kernels and result (bit
 * for bit) as fi_topk_new_pixels; its workspace (flags, histogram, ranks,
 * scan partials) is a fixed 24 MiB device array inside the library, one copy
 * per GPU, held until the process ends, instead of memory the mesh allocates
 * on first use. It calls no hipMalloc, hipFree or other allocating routine.
 * Limit: P <= 2^20 pixels (images up to 1024 x 1024); larger meshes give
 * FI_E_INVALID. Every call on a GPU reuses that GPU's array (each call
 * clears what it reads before use). Calls in one process are serialised: a
 * call holds a library lock and waits for its stream before it returns, so
 * two calls never use the array at the same time; a caller that bypassed
 * this (e.g. replaying captured work of two calls concurrently) would race. */
int fi_topk_new_pixels_noalloc(fi_mesh* mesh, const double* e_dev, int64_t k, int32_t* out_dev);

/* Error-driven mask growth (Section 3: densification on the inpainting
 * error map, here its global top-k form): starting from mask0, for `rounds`
 * rounds rebuild the mesh on the current mask, inpaint with g = f on the
 * mask, compute e_i = (u_i - f_i)^2 and add the k_add non-mask pixels with
 * the largest e_i (ties to the lower index); finally inpaint once more.
 *   f_dev:     uint8[side * side] device image;
 *   mask0:     host int32[m0], strictly ascending;
 *   mask_out:  host int32[m0 + rounds * k_add]: mask0, then each round's
 *              additions in ascending order, round after round;
 *   mse_out:   host float64[rounds + 1], MSE after each round's inpainting
 *              (index r: the mask of round r; index rounds: the final mask);
 *   gpu_ms_out: host float64[rounds + 1] or NULL: milliseconds of device
 *              time for the solve, interpolation and error of each round
 *              (HIP events on the context stream; mesh building excluded).
 * Errors as fi_mesh_build / fi_inpaint; FI_E_INVALID if a round cannot add
 * k_add pixels. */
int fi_grow_mask(fi_ctx* ctx, int side, const uint8_t* f_dev, const int32_t* mask0, int64_t m0,
                 int64_t k_add, int rounds, const fi_solve_opts* opts, int32_t* mask_out,
                 double* mse_out, double* gpu_ms_out);

/* Section 3's densification step, as the paper states it: the total squared
 * error E_T of every triangle (its pixels' e, added in ascending pixel
 * order); triangles taken in descending E_T (ties: lower triangle index),
 * skipping those that own no pixel outside the mask; from each, its non-mask
 * pixel of largest e (ties: lower index); k pixels in all, or every
 * candidate triangle's if there are fewer.
 *   e_dev:   float64[P] device, the pointwise error (fi_error's pix_err);
 *   out_dev: int32[k] device, the chosen pixels in ascending order;
 *   added:   host, how many were chosen (<= k).
 * Synchronous. */
int fi_paper_densify_step(fi_mesh* mesh, const double* e_dev, int64_t k, int32_t* out_dev,
                          int64_t* added);

/* Mask-growth rules of fi_densify. */
enum fi_densify_rule {
  FI_DENSIFY_TOPK = 0,      /* the k_add non-mask pixels of largest e (fi_grow_mask) */
  FI_DENSIFY_TRIANGLES = 1  /* Section 3's per-triangle step (fi_paper_densify_step) */
};

/* fi_grow_mask with a choice of rule. With FI_DENSIFY_TRIANGLES a round may
 * add fewer than k_add pixels; mask_out is sized for m0 + rounds * k_add and
 * *mask_size_out (host, may be NULL) receives how many were written. */
int fi_densify(fi_ctx* ctx, int side, const uint8_t* f_dev, const int32_t* mask0, int64_t m0,
               int64_t k_add, int rounds, int rule, const fi_solve_opts* opts, int32_t* mask_out,
               double* mse_out, double* gpu_ms_out, int64_t* mask_size_out);

/* Section 3's spatial optimisation on the paper's own mesh: fi_densify with
 * FI_DENSIFY_TRIANGLES, where every round triangulates (Delaunay, as
 * fi_mesh_build_delaunay) the current mask and the unknown vertices. The
 * unknown vertices are drawn once, before the first round (an input here:
 * unknowns, host int32[nu], strictly ascending, none in mask0); a pixel the
 * step adds that was an unknown vertex becomes a mask vertex. Arguments,
 * outputs and errors otherwise as fi_densify. */
int fi_densify_delaunay(fi_ctx* ctx, int side, const uint8_t* f_dev, const int32_t* mask0,
                        int64_t m0, const int32_t* unknowns, int64_t nu, int64_t k_add,
                        int rounds, const fi_solve_opts* opts, int32_t* mask_out,
                        double* mse_out, double* gpu_ms_out, int64_t* mask_size_out);

/* Timing helper: runs `reps` launches of the FP32 (precision =
 * FI_PREC_FP32_IR) or FP64 (FI_PREC_FP64) CG step kernel on this mesh,
 * forced to iterate, between two HIP events recorded on the context stream,
 * and returns the mean milliseconds per launch. An FP32 launch advances
 * fi_mesh_info.cg_iters_per_launch iterations. The solver state is left
 * undefined. */
int fi_time_cg_kernel(fi_mesh* mesh, int precision, int reps, double* ms_per_launch);

/* Algorithmic bytes of one step launch, what it must move at the least:
 * - the one-iteration launch: the matrix (one 4-byte code per stored
 *   off-diagonal entry on the quadtree mesh; column, value and row pointers
 *   otherwise) and each vector of one-pass Jacobi PCG read or written once
 *   (4 nnz_off + 44 n in FP32);
 * - the three-iteration launch (FP32 on the quadtree mesh): per row the
 *   basis record read and the new one written (32 bytes each), the
 *   correction read and written and the diagonal read (4 bytes each), and
 *   the matrix once as 16-bit entries: 76 n + 2 nnz_off. It reads the matrix
 *   and the vectors once for three iterations; the halo rows that
 *   neighbouring blocks read again, the region lists and the local matrix
 *   padding are its layout's overhead, not counted here. */
int fi_cg_kernel_bytes(const fi_mesh* mesh, int precision, int64_t* bytes);

/* ------------------------------------------------------------- colour --
 * Section 5 calls the extension to colour images straightforward; it is
 * read here as the method applied channel by channel. The
 * three channels share the mask, so they share the mesh, K_FF, K_FD and the
 * interpolation; each channel is the grey problem with its own data. Arrays
 * are planar: channel c of a per-pixel array occupies [c * P, (c + 1) * P),
 * of the mask values [c * m, (c + 1) * m).
 *
 * The three solves of every step run in ONE multi-right-hand-side launch
 * whose blocks for the same rows of the three channels run side by side on
 * one XCD, so the rows' matrix entries come from HBM once and from that
 * XCD's L2 for the other channels. Every channel keeps its own solver state
 * and runs the grey step on its own data, so each channel's result is bit
 * for bit what the grey call returns for that channel (also its iteration
 * counts). A channel whose solve has ended leaves the launches.
 * The first colour call on a mesh allocates the data-dependent state of
 * channels 1 and 2 (solver vectors and work vectors, about twice the
 * per-image part of the mesh's memory); fi_mesh_get_info's device_bytes
 * includes it from then on. Colour calls are synchronous like the grey ones. */

/* u_c = B g_c for c = 0, 1, 2 (Section 4's B, Section 5).
 *   f_dev: uint8[3P] device, planar; used only when g_dev is NULL (then
 *          g_c = f_c on the mask). May be NULL when g_dev is given.
 *   g_dev: float64[3m] device, planar, or NULL.
 *   u_dev: float64[3P] device output, planar.
 *   opts:  NULL for defaults. stats: host array of 3 (one per channel) or NULL.
 * Errors: FI_E_INVALID (NULL u_dev, or both f_dev and g_dev NULL);
 * FI_E_NO_CONVERGENCE when a channel's solve missed the tolerance (u_dev is
 * written all the same); FI_E_NOMEM / FI_E_HIP. */
int fi_inpaint_rgb(fi_mesh* mesh, const uint8_t* f_dev, const double* g_dev, double* u_dev,
                   const fi_solve_opts* opts, fi_solve_stats* stats);

/* Colour MSE: the mean over all 3P values of (u - f)^2, i.e. the mean of
 * the three channel MSEs (the paper defines no colour error; this reading
 * weights the channels equally).
 *   u_dev: float64[3P], f_dev: uint8[3P], both device, planar;
 *   mse_host: output scalar (may be NULL); mse_ch_host: host float64[3],
 *   the channel MSEs (may be NULL). Synchronous. */
int fi_error_rgb(fi_mesh* mesh, const double* u_dev, const uint8_t* f_dev, double* mse_host,
                 double* mse_ch_host);

/* Tonal optimisation of a colour image (Section 4 per channel, Section 5):
 * three independent least-squares problems, each solved by the CGLS of
 * fi_tonal_opt, whose solves share the multi-right-hand-side launches.
 * A channel stops at its own relative normal residual opts->rtol (rtol 0:
 * every channel runs opts->max_outer iterations); the others go on.
 *   f_dev: uint8[3P] device, planar; g_dev: float64[3m] device, planar
 *   (start values if opts->start_from_g; the result on return);
 *   stats: host array of 3 or NULL. Channel c's g and stats equal
 *   fi_tonal_opt's on channel c's data, bit for bit.
 * Errors: as fi_tonal_opt; FI_E_NO_CONVERGENCE if any channel missed rtol. */
int fi_tonal_opt_rgb(fi_mesh* mesh, const uint8_t* f_dev, double* g_dev,
                     const fi_tonal_opts* opts, fi_tonal_stats* stats);

/* Timing helper for the multi-right-hand-side step: `reps` launches with
 * nrhs (1..3) channels all in the iteration phase, as fi_time_cg_kernel;
 * returns mean milliseconds per launch (with the large-system reduction
 * launch when the mesh uses one). Channel states are left undefined. */
int fi_time_cg_multi_kernel(fi_mesh* mesh, int nrhs, int precision, int reps,
                            double* ms_per_launch);

/* Algorithmic bytes of one multi-right-hand-side step launch over nrhs
 * channels: the matrix once, and per channel each vector read or written
 * once (as fi_cg_kernel_bytes). */
int fi_cg_multi_kernel_bytes(const fi_mesh* mesh, int nrhs, int precision, int64_t* bytes);

/* ------------------------------------------------------------- serving --
 * Batched serving of requests "inpaint, then run tonal_iters CGLS iterations
 * of tonal optimisation" (Sections 2.2 and 4) for images of any power-of-two
 * side and mask density. Builder threads build each request's mesh on the
 * host and admit it when its device footprint (an upper bound computed from
 * the mesh, see fi_server_footprint) fits in the server's memory budget;
 * the engine keeps up to max_slots requests resident and advances all their
 * FP32 solves together, one step launch per CG step for all of them, while
 * requests arrive and leave (continuous batching). Each request computes the
 * same values as fi_inpaint + fi_tonal_opt with max_outer = tonal_iters,
 * bit for bit, whatever else is in the batch.
 *
 * With precision FI_PREC_FP64, or max_slots == 1, the server runs one
 * request at a time with the single-mesh solver instead (the sequential
 * comparator).
 *
 * Device memory: one allocation of hbm_budget bytes at creation (the arena);
 * requests take and return parts of it without further device allocation.
 * Admission by footprint: a request becomes resident once one contiguous
 * region of its footprint bound is free in the arena; its mesh and buffers
 * are carved out of that region, which returns to the arena when the
 * request finishes (arena_used_bytes counts whole regions).
 * All request data is copied at submission, so the caller's buffers (except
 * g_out) may be reused at once. */
typedef struct fi_server fi_server;

typedef struct fi_server_opts {
  int max_slots;      /* requests resident at once, 1..64 (default 16) */
  int precision;      /* FI_PREC_FP32_IR (batched) or FI_PREC_FP64 (sequential) */
  size_t hbm_budget;  /* bytes of the arena (default 32 GiB) */
  int build_threads;  /* host threads building meshes (default 4) */
  int chunk;          /* step launches per submission, even (default 8) */
} fi_server_opts;

typedef struct fi_job_desc {
  int side;              /* image side, a power of two, 2..16384 */
  const uint8_t* f;      /* host uint8[side * side], row-major (copied) */
  const int32_t* mask;   /* host int32[m], strictly ascending (copied) */
  int64_t m;             /* mask pixels, >= 1 */
  int tonal_iters;       /* CGLS iterations after the inpainting (0: none) */
  double* g_out;         /* host float64[m] or NULL: the optimised g (f on
                            the mask if tonal_iters == 0), written before the
                            request reports done; must stay valid until then */
  fi_solve_opts inner;   /* solve options; precision is the server's */
} fi_job_desc;

typedef struct fi_job_result {
  int32_t done;           /* 0: still running (other fields unset) */
  int32_t status;         /* FI_OK or the request's error code */
  double mse_inpaint;     /* MSE of the inpainting with g = f on the mask */
  double mse_tonal;       /* MSE after the tonal iterations */
  int64_t inner_iterations; /* CG iterations of all the request's solves */
  double t_submit, t_admit, t_start, t_done; /* seconds on the server clock:
                            submitted, mesh uploaded, resident, finished */
  int64_t device_bytes;   /* bytes of its region the request's mesh and
                             buffers took (at most footprint_bound) */
  int64_t footprint_bound; /* its admission bound */
  char error[128];        /* message when status != FI_OK */
} fi_job_result;

typedef struct fi_server_stats {
  int64_t jobs_submitted, jobs_done, jobs_failed;
  int64_t peak_resident;  /* most requests resident at once */
  int64_t step_rounds;    /* batched step rounds launched */
  int64_t slot_steps;     /* sum over rounds of the requests stepped */
  int64_t arena_bytes, arena_used_bytes, arena_peak_bytes;
  double clock;           /* server clock now, seconds */
} fi_server_stats;

void fi_server_opts_default(fi_server_opts* opts);
/* Creates a server on ctx's device (its own streams; ctx is not kept).
 * Errors: FI_E_INVALID (options), FI_E_NOMEM (arena), FI_E_HIP. */
int fi_server_create(fi_ctx* ctx, const fi_server_opts* opts, fi_server** out);
/* Queues a request; returns its ticket. Errors: FI_E_INVALID (side, mask,
 * sizes), FI_E_EMPTY_MASK (m == 0). Thread-safe. */
int fi_server_submit(fi_server* server, const fi_job_desc* job, uint64_t* ticket);
/* Result of a request; wait != 0 blocks until it is done. A done result is
 * returned once: the ticket is then released. A request that could not be
 * admitted (its bound exceeds the budget) ends with FI_E_NOMEM. */
int fi_server_poll(fi_server* server, uint64_t ticket, int wait, fi_job_result* result);
int fi_server_stats_get(fi_server* server, fi_server_stats* stats);
/* Seconds since the server was created (the clock of fi_job_result). */
double fi_server_clock(fi_server* server);
/* Finishes every queued request, then frees the server. */
int fi_server_destroy(fi_server* server);
/* Admission bound (bytes) of a request with this mask, computed on the host
 * from its mesh; no device use. It covers every device allocation of the
 * request, including the scratch of the device build of its s-step plan. */
int fi_server_footprint(int side, const int32_t* mask, int64_t m, int tonal_iters, int64_t* bytes);

#ifdef __cplusplus
}
#endif

#endif /* FI_H */
