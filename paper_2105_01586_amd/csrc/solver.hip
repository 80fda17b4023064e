// Jacobi-preconditioned CG for K_FF x = b with FP64 iterative refinement.
//
// Section 2.2 solves the SPD FEM system with conjugate gradients. Here each
// CG iteration is ONE kernel launch: the Chronopoulos-Gear form of PCG needs
// a single global reduction per iteration (the dots (r, z), (z, A z) and
// (r, r) are taken together), and the next iteration's SpMV input is
// recomputed on the fly from the previous vectors, so one launch covers
//     p = z + beta p,   q = s + beta q,   x += alpha p,   r -= alpha q,
//     z = D^-1 r,       s = A z,          partial dots of the new state.
// r, s and q are double-buffered because neighbours read the old values
// while their owners write the new ones; x and p are only touched by their
// owner. Every block reduces the previous kernel's per-block partial sums
// itself, in a fixed order, so no atomics and no extra reduction launch are
// needed, and results are reproducible bit for bit.
//
// Precision (mixed mode): the inner iterations run in FP32 with FP32
// SpMV accumulation (dots accumulate in FP64); the outer loop forms the true
// residual b - K x in FP64 on the GPU, solves for a correction in FP32 and
// adds it in FP64 until ||b - K x|| <= rtol ||b||. In FP64 mode the same
// kernel runs in double and the FP64 residual check confirms the result.
#include <cmath>
#include <cstdint>

#include "internal.h"
#include "reduce.h"

namespace fi {

namespace {

inline int grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : g);
}

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// New residual of row j from the previous state: r - alpha (s + beta q).
// Owners and neighbours call the same function, so both see the same bits.
template <typename T>
__device__ __forceinline__ T next_r(T r, T s, T q, T a, T b) {
  return fmaT(-a, fmaT(b, q, s), r);
}

// Reads the per-block partial sums of the previous launch and reduces them
// in a fixed order (strided per thread, then the block tree).
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int G,
                                                double (&v)[3], double* lds) {
  v[0] = v[1] = v[2] = 0.0;
  for (int j = threadIdx.x; j < G; j += kBlock) {
    v[0] += part[4 * j];
    v[1] += part[4 * j + 1];
    v[2] += part[4 * j + 2];
  }
  block_sum<3>(v, lds);
}

// State 0 of an inner solve: x = 0, p = 0, q_prev = 0, r = rhs * scale (rhs
// in FP64), s = A D^-1 r, and the partial dots of that state.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_init(
    int n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const T* __restrict__ val, const T* __restrict__ dinv, const double* __restrict__ rhs,
    double scale, T* __restrict__ x, T* __restrict__ p, T* __restrict__ r0,
    T* __restrict__ s0, T* __restrict__ q0, double* __restrict__ part_out,
    int32_t* __restrict__ ctl) {
  __shared__ double lds[12];
  if (blockIdx.x == 0 && threadIdx.x == 0) { ctl[0] = 0; ctl[1] = 0; }
  double v[3] = {0.0, 0.0, 0.0};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const T ri = (T)(rhs[i] * scale);
    const T zi = dinv[i] * ri;
    T acc = ri;  // diagonal term: K_ii z_i = r_i
    for (int j = rowptr[i]; j < rowptr[i + 1]; ++j) {
      const int c = col[j];
      acc = fmaT(val[j], dinv[c] * (T)(rhs[c] * scale), acc);
    }
    x[i] = (T)0;
    p[i] = (T)0;
    q0[i] = (T)0;
    r0[i] = ri;
    s0[i] = acc;
    v[0] += (double)ri * (double)zi;
    v[1] += (double)zi * (double)acc;
    v[2] += (double)ri * (double)ri;
  }
  block_sum<3>(v, lds);
  if (threadIdx.x == 0) {
    part_out[4 * blockIdx.x] = v[0];
    part_out[4 * blockIdx.x + 1] = v[1];
    part_out[4 * blockIdx.x + 2] = v[2];
    part_out[4 * blockIdx.x + 3] = 0.0;
  }
}

// One fused Chronopoulos-Gear PCG iteration (state `iter` -> iter + 1).
// ctl[0]: 0 running, 1 converged, 2 breakdown, 3 iteration cap; ctl[1]:
// iterations done. scal_in/out: gamma_prev, alpha_prev, rho_ref.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_iter(
    int n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const T* __restrict__ val, const T* __restrict__ dinv, T* __restrict__ x, T* __restrict__ p,
    const T* __restrict__ r_in, const T* __restrict__ s_in, const T* __restrict__ q_in,
    T* __restrict__ r_out, T* __restrict__ s_out, T* __restrict__ q_out,
    const double* __restrict__ part_in, double* __restrict__ part_out,
    const double* __restrict__ scal_in, double* __restrict__ scal_out, int32_t* __restrict__ ctl,
    int iter, double tol2, int maxit, int force) {
  __shared__ double lds[12];
  __shared__ int done;
  // One read per block, so the whole block takes the same branch (the flag
  // can change while this launch runs, but only to stop a solve that every
  // block is about to stop anyway).
  if (threadIdx.x == 0) done = force ? 0 : ctl[0];
  __syncthreads();
  if (done) return;
  double red[3];
  reduce_partials(part_in, gridDim.x, red, lds);
  const double gamma = red[0], delta = red[1], rho = red[2];
  const double rho_ref = iter == 0 ? rho : scal_in[2];
  double alpha, beta;
  if (iter == 0) {
    beta = 0.0;
    alpha = gamma / delta;
  } else {
    beta = gamma / scal_in[0];
    alpha = gamma / (delta - beta * gamma / scal_in[1]);
  }
  if (!force) {
    int stop = 0;
    if (!(rho > tol2 * rho_ref)) stop = 1;            // converged (also rho == 0)
    else if (!(alpha > 0.0) || !isfinite(alpha)) stop = 2;  // breakdown / loss of SPD-ness
    else if (iter >= maxit) stop = 3;
    if (stop) {
      if (blockIdx.x == 0 && threadIdx.x == 0) { ctl[0] = stop; ctl[1] = iter; }
      return;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal_out[0] = gamma;
    scal_out[1] = alpha;
    scal_out[2] = rho_ref;
  }
  const T a = (T)alpha, b = (T)beta;
  double v[3] = {0.0, 0.0, 0.0};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const T ri0 = r_in[i], si0 = s_in[i], qi0 = q_in[i], di = dinv[i];
    const T pi = fmaT(b, p[i], di * ri0);
    const T qi = fmaT(b, qi0, si0);
    x[i] = fmaT(a, pi, x[i]);
    p[i] = pi;
    const T ri = next_r(ri0, si0, qi0, a, b);
    const T zi = di * ri;
    T acc = ri;  // diagonal term
    const int j1 = rowptr[i + 1];
    for (int j = rowptr[i]; j < j1; ++j) {
      const int c = col[j];
      const T rc = next_r(r_in[c], s_in[c], q_in[c], a, b);
      acc = fmaT(val[j], dinv[c] * rc, acc);
    }
    r_out[i] = ri;
    q_out[i] = qi;
    s_out[i] = acc;
    v[0] += (double)ri * (double)zi;
    v[1] += (double)zi * (double)acc;
    v[2] += (double)ri * (double)ri;
  }
  block_sum<3>(v, lds);
  if (threadIdx.x == 0) {
    part_out[4 * blockIdx.x] = v[0];
    part_out[4 * blockIdx.x + 1] = v[1];
    part_out[4 * blockIdx.x + 2] = v[2];
    part_out[4 * blockIdx.x + 3] = 0.0;
  }
}

// r = b - K_FF x in FP64 (diagonal separate), with per-block partial ||r||^2.
__global__ __launch_bounds__(kBlock) void k_residual64(
    int n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ diag, const double* __restrict__ b,
    const double* __restrict__ x, double* __restrict__ r, double* __restrict__ part) {
  __shared__ double lds[4];
  double v[1] = {0.0};
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    double acc = diag[i] * x[i];
    for (int j = rowptr[i]; j < rowptr[i + 1]; ++j) acc += val[j] * x[col[j]];
    const double ri = b[i] - acc;
    r[i] = ri;
    v[0] += ri * ri;
  }
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_refine(int n, double scale, const T* __restrict__ d,
                                                   double* __restrict__ x) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] += scale * (double)d[i];
}

__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, double v, double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = v;
}

struct InnerArgs {
  const int32_t* rowptr;
  const int32_t* col;
  const void* val;
  const void* dinv;
  CGState st;
};

template <typename T>
InnerArgs inner_args(fi_mesh* M);

template <>
InnerArgs inner_args<float>(fi_mesh* M) {
  return InnerArgs{M->d_ff_rowptr, M->d_ff_col, M->d_ff_val32, M->d_dinv32, M->cg32};
}
template <>
InnerArgs inner_args<double>(fi_mesh* M) {
  return InnerArgs{M->d_ff_rowptr, M->d_ff_col, M->d_ff_val64, M->d_dinv64, M->cg64};
}

template <typename T>
int launch_init(fi_mesh* M, const double* rhs, double scale) {
  InnerArgs A = inner_args<T>(M);
  hipLaunchKernelGGL(k_cg_init<T>, dim3(M->cg_grid), dim3(kBlock), 0, M->ctx->stream, (int)M->n,
                     A.rowptr, A.col, (const T*)A.val, (const T*)A.dinv, rhs, scale, (T*)A.st.x,
                     (T*)A.st.p, (T*)A.st.r[0], (T*)A.st.s[0], (T*)A.st.q[0], M->d_part, M->d_ctl);
  FI_HIP_TRY(hipGetLastError());
  return FI_OK;
}

template <typename T>
int launch_iter(fi_mesh* M, int iter, double tol2, int maxit, int force) {
  InnerArgs A = inner_args<T>(M);
  const int a = iter & 1, b = a ^ 1;
  double* part_in = M->d_part + (size_t)a * 4 * kMaxGrid;
  double* part_out = M->d_part + (size_t)b * 4 * kMaxGrid;
  double* scal_in = M->d_scal + 4 * a;
  double* scal_out = M->d_scal + 4 * b;
  hipLaunchKernelGGL(k_cg_iter<T>, dim3(M->cg_grid), dim3(kBlock), 0, M->ctx->stream, (int)M->n,
                     A.rowptr, A.col, (const T*)A.val, (const T*)A.dinv, (T*)A.st.x, (T*)A.st.p,
                     (const T*)A.st.r[a], (const T*)A.st.s[a], (const T*)A.st.q[a],
                     (T*)A.st.r[b], (T*)A.st.s[b], (T*)A.st.q[b], part_in, part_out, scal_in,
                     scal_out, M->d_ctl, iter, tol2, maxit, force);
  FI_HIP_TRY(hipGetLastError());
  return FI_OK;
}

// Runs one inner solve of K d = rhs * scale to relative residual `rtol`
// (FP(T) recurrence residual); returns iterations used and the stop code.
template <typename T>
int inner_solve(fi_mesh* M, const double* rhs, double scale, double rtol, int maxit,
                int check_every, int64_t* iters, int* stop_code) {
  int rc = launch_init<T>(M, rhs, scale);
  if (rc) return rc;
  const double tol2 = rtol * rtol;
  int it = 0;
  for (;;) {
    const int chunk = check_every;
    for (int k = 0; k < chunk; ++k) {
      rc = launch_iter<T>(M, it + k, tol2, maxit, 0);
      if (rc) return rc;
    }
    it += chunk;
    FI_HIP_TRY(hipMemcpyAsync(M->h_ctl, M->d_ctl, 2 * sizeof(int32_t), hipMemcpyDeviceToHost,
                              M->ctx->stream));
    FI_HIP_TRY(hipStreamSynchronize(M->ctx->stream));
    if (M->h_ctl[0] != 0) {
      *iters = M->h_ctl[1];
      *stop_code = M->h_ctl[0];
      return FI_OK;
    }
    if (it > maxit + chunk) {  // cannot happen: the kernel stops at maxit
      return fail(FI_E_HIP, "inner solver did not report termination");
    }
  }
}

template <typename T>
int refine_update(fi_mesh* M, double scale) {
  InnerArgs A = inner_args<T>(M);
  hipLaunchKernelGGL(k_refine<T>, dim3(grid_for(M->n)), dim3(kBlock), 0, M->ctx->stream, (int)M->n,
                     scale, (const T*)A.st.x, M->d_x64);
  FI_HIP_TRY(hipGetLastError());
  return FI_OK;
}

int residual64(fi_mesh* M, double* rnorm2_host) {
  hipLaunchKernelGGL(k_residual64, dim3(M->cg_grid), dim3(kBlock), 0, M->ctx->stream, (int)M->n,
                     M->d_ff_rowptr, M->d_ff_col, M->d_ff_val64, M->d_diag64, M->d_b64, M->d_x64,
                     M->d_r64, M->d_red);
  FI_HIP_TRY(hipGetLastError());
  int rc = launch_reduce(M, M->d_red, M->cg_grid, 1, M->d_red_out);
  if (rc) return rc;
  FI_HIP_TRY(hipMemcpyAsync(M->h_red, M->d_red_out, sizeof(double), hipMemcpyDeviceToHost,
                            M->ctx->stream));
  FI_HIP_TRY(hipStreamSynchronize(M->ctx->stream));
  *rnorm2_host = M->h_red[0];
  return FI_OK;
}

template <typename T>
int solve_ir(fi_mesh* M, const fi_solve_opts* o, fi_solve_stats* stats) {
  const int64_t n = M->n;
  stats->iterations = 0;
  stats->refinements = 0;
  stats->status = FI_OK;
  stats->rel_residual = 0.0;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(kBlock), 0, M->ctx->stream, n, 0.0, M->d_x64);
  FI_HIP_TRY(hipGetLastError());
  int rc = launch_dot(M, M->d_b64, M->d_b64, n, M->d_red_out);
  if (rc) return rc;
  FI_HIP_TRY(hipMemcpyAsync(M->h_red, M->d_red_out, sizeof(double), hipMemcpyDeviceToHost,
                            M->ctx->stream));
  FI_HIP_TRY(hipStreamSynchronize(M->ctx->stream));
  const double bnorm = std::sqrt(M->h_red[0]);
  if (!std::isfinite(bnorm)) return fail(FI_E_INVALID, "right-hand side is not finite");
  if (bnorm == 0.0) return FI_OK;  // x = 0 solves it exactly
  double rnorm = bnorm;
  const double* rhs = M->d_b64;  // residual of x = 0
  const bool mixed = sizeof(T) == sizeof(float);
  int stagnant = 0;
  for (int step = 0;; ++step) {
    const double rel = rnorm / bnorm;
    stats->rel_residual = rel;
    if (rel <= o->rtol) return FI_OK;
    if (step >= o->max_refine) break;
    // Inner target: what the outer tolerance still needs, never looser than
    // inner_rtol in mixed mode.
    const double want = 0.5 * o->rtol * bnorm / rnorm;
    const double itol = mixed ? std::max(o->inner_rtol, want) : std::max(want, 1e-15);
    int64_t its = 0;
    int code = 0;
    rc = inner_solve<T>(M, rhs, 1.0 / rnorm, itol, o->max_inner, std::max(1, o->check_every), &its,
                        &code);
    if (rc) return rc;
    stats->iterations += its;
    rc = refine_update<T>(M, rnorm);
    if (rc) return rc;
    double r2 = 0.0;
    rc = residual64(M, &r2);
    if (rc) return rc;
    stats->refinements += 1;
    const double rnew = std::sqrt(r2);
    if (!std::isfinite(rnew)) return fail(FI_E_HIP, "non-finite residual in refinement");
    stagnant = (rnew > 0.5 * rnorm) ? stagnant + 1 : 0;
    rnorm = rnew;
    rhs = M->d_r64;
    if (stagnant >= 3) break;
  }
  stats->rel_residual = rnorm / bnorm;
  stats->status = FI_E_NO_CONVERGENCE;
  return FI_OK;
}

}  // namespace

// Solves K_FF x64 = b64 (both in the mesh workspace).
int solve_free(fi_mesh* M, const fi_solve_opts* opts, fi_solve_stats* stats) {
  if (M->n == 0) {
    stats->iterations = 0;
    stats->refinements = 0;
    stats->status = FI_OK;
    stats->rel_residual = 0.0;
    return FI_OK;
  }
  if (opts->precision == FI_PREC_FP64) return solve_ir<double>(M, opts, stats);
  return solve_ir<float>(M, opts, stats);
}

int time_cg_kernel(fi_mesh* M, int precision, int reps, double* ms) {
  if (M->n == 0 || reps < 1) return fail(FI_E_INVALID, "nothing to time");
  hipStream_t st = M->ctx->stream;
  // a fresh state from the current right-hand side
  int rc = precision == FI_PREC_FP64 ? launch_init<double>(M, M->d_b64, 1.0)
                                     : launch_init<float>(M, M->d_b64, 1.0);
  if (rc) return rc;
  hipEvent_t e0, e1;
  FI_HIP_TRY(hipEventCreate(&e0));
  FI_HIP_TRY(hipEventCreate(&e1));
  for (int k = 0; k < 4; ++k) {
    rc = precision == FI_PREC_FP64 ? launch_iter<double>(M, k, 0.0, 1 << 30, 1)
                                   : launch_iter<float>(M, k, 0.0, 1 << 30, 1);
    if (rc) return rc;
  }
  FI_HIP_TRY(hipEventRecord(e0, st));
  for (int k = 0; k < reps; ++k) {
    rc = precision == FI_PREC_FP64 ? launch_iter<double>(M, 4 + k, 0.0, 1 << 30, 1)
                                   : launch_iter<float>(M, 4 + k, 0.0, 1 << 30, 1);
    if (rc) return rc;
  }
  FI_HIP_TRY(hipEventRecord(e1, st));
  FI_HIP_TRY(hipEventSynchronize(e1));
  float t = 0.f;
  FI_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *ms = (double)t / reps;
  return FI_OK;
}

// Bytes one fused iteration must move: matrix (column index + value per
// off-diagonal entry), row pointers, and per row the reads of r, s, q, D^-1,
// x, p and the writes of x, p, r, s, q.
int64_t cg_kernel_bytes(const fi_mesh* M, int precision) {
  const int64_t w = precision == FI_PREC_FP64 ? 8 : 4;
  return M->nnz_off * (4 + w) + (M->n + 1) * 4 + M->n * w * 11;
}

}  // namespace fi
