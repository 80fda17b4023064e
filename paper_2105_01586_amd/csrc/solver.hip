// Jacobi-preconditioned CG for K_FF x = b with FP64 iterative refinement,
// driven by the device.
//
// Section 2.2 solves the SPD FEM system with conjugate gradients. The whole
// solve is a sequence of launches of ONE "step" kernel; each launch reads a
// small state record, does the work of the current phase, and writes the
// next record:
//   INIT  start an inner solve: r0 = r64 / ||r64||, s0 = A D^-1 r0, or stop
//         the solve when ||r64|| <= rtol ||b|| (or on stagnation / cap);
//   ITER  one Jacobi-PCG iteration in the Chronopoulos-Gear form: a single
//         global reduction per iteration (the dots (r, z), (z, A z), (r, r)
//         together), the next SpMV input recomputed from the previous
//         vectors, so one launch covers
//            p = z + beta p,  q = s + beta q,  x += alpha p,  r -= alpha q,
//            z = D^-1 r,      s = A z,         partial dots of the new state;
//         when the inner solve has converged the same launch instead adds
//         the correction in FP64 and forms the FP64 residual b - K x;
//   DONE  nothing.
// Every per-launch quantity (state record, partial sums, r, s, q) is double
// buffered by launch parity: launch k reads slot k % 2 and writes the other,
// so blocks of one launch never see each other's writes. The host only
// queues step launches, a couple of chunks ahead of the device, until the
// launch that ends the solve reports the outcome in pinned host memory; it
// makes no decision between refinements.
//
// Matrix layout: the off-diagonal part of K_FF in column-major ELL (slot k of
// row i at ell[k * n_pad + i], coalesced across a wavefront); on the
// quadtree mesh every off-diagonal entry is -1/2 or -1, so an entry is the
// column with the sign bit marking -1 and a padding bit for empty slots
// (which point at the row itself with weight 0, so every load is
// unconditional: no divergent branches between the loads). The diagonal
// enters through K_ii z_i = r_i. A CSR path covers other matrices.
//
// All loads of an iteration that do not depend on alpha and beta (the
// previous partial sums, the thread's row, its neighbours' values) are
// issued before the block reduction. Block sums use DPP within each wave and
// one barrier (two per launch), with the two sums of a launch in separate LDS
// regions. When the rows fit in at most kMaxGrid
// blocks, every block re-reduces the previous launch's per-block partial sums
// in a fixed order; larger systems put a one-block reduction launch between
// steps. No atomics: results are reproducible bit for bit. Each row's r, s,
// q and D^-1 sit together (one load per neighbour), and blocks are mapped to
// rows so that every XCD works on one contiguous slab of rows.
//
// Precision: in mixed mode the iterations run in FP32 with FP32 SpMV
// accumulation (dots accumulate in FP64); corrections, residuals and the
// iterate are FP64. FP64 mode runs the same kernel in double.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <string>

#include "internal.h"
#include "cg_common.h"
#include "pacer.h"
#include "reduce.h"

namespace fi {

namespace {

inline int grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : g);
}


// New residual of row j from the previous state: r - alpha (s + beta q).
// Owners and neighbours call the same function, so both see the same bits.
template <typename T>
__device__ __forceinline__ T next_r(T r, T s, T q, T a, T b) {
  return fmaT(-a, fmaT(b, q, s), r);
}

// ELL entry: bits 0-29 column, bit 30 set for padding (weight 0; the column
// is then the row itself, so every gather stays in bounds and unconditional),
// bit 31 set for weight -1, clear for weight -1/2.
constexpr int32_t kColMask = kEllColMask;
constexpr int32_t kPadBit = kEllPadBit;

__device__ __forceinline__ int ell_col(int32_t e) { return e & kColMask; }

template <typename T>
__device__ __forceinline__ T ell_weight(int32_t e) {
  return (e & kPadBit) ? T(0) : (e < 0 ? T(-1) : T(-0.5));
}

// Per-row solver values (r, s, q, D^-1) side by side: a neighbour costs
// one aligned load instead of four.
template <typename T>
struct alignas(4 * sizeof(T)) Quad {
  T r, s, q, d;
};


template <typename T>
struct StepArgs {
  int n;
  int n_pad;
  int W;                  // ELL slots (0: CSR)
  const int32_t* ell;
  const int32_t* rowptr;  // CSR (always present; used when W == 0)
  const int32_t* col;
  const T* val;
  const double* val64;
  const T* dinv;
  const double* diag64;
  T* x;                   // the correction of the current inner solve
  T* p;
  const Quad<T>* rq_in;
  Quad<T>* rq_out;
  const double* part_in;
  int nparts_in;
  double* part_out;
  const Rec* rec_in;
  Rec* rec_out;
  const Params* prm;
  const double* b64;
  double* r64;
  double* x64a;           // x64 buffers; rec.xp selects the current one
  double* x64b;
  Mirror* mirror;         // pinned host memory (device-visible), or NULL
  int force;              // timing only: always iterate, ignore stop tests
};


// Partial sums of block `lb` (the logical block: the index is what fixes the
// order in which the next launch adds them up).
__device__ __forceinline__ void store_partials(double* part_out, int lb, double (&v)[3]) {
  if (threadIdx.x == 0) {
    part_out[4 * lb] = v[0];
    part_out[4 * lb + 1] = v[1];
    part_out[4 * lb + 2] = v[2];
    part_out[4 * lb + 3] = 0.0;
  }
}

// Start of a solve: x64 = x0 (0 when x0 is NULL), r64 = b - K_FF x0 in
// FP64, partial sums ||r64||^2 and ||b||^2, first record. The stopping test
// stays relative to ||b|| whatever the start: a good x0 only saves
// iterations. x0 must not alias x64 buffer a, r64 or b64.
template <typename T, int BS>
__global__ __launch_bounds__(BS) void k_solve_start(StepArgs<T> A, Params prm, Params* prm_out,
                                                    const double* __restrict__ x0) {
  __shared__ double lds[3 * (BS / 64)];
  double v[3] = {0.0, 0.0, 0.0};
  const int lb = logical_block();
  const int i = lb * BS + threadIdx.x;
  if (i < A.n) {
    const double bi = A.b64[i];
    double ri = bi, xi = 0.0;
    if (x0) {
      xi = x0[i];
      double acc = A.diag64[i] * xi;
      if (A.W > 0) {
        for (int k = 0; k < A.W; ++k) {
          const int32_t e = A.ell[(size_t)k * A.n_pad + i];
          acc += ell_weight<double>(e) * x0[ell_col(e)];
        }
      } else {
        for (int j = A.rowptr[i]; j < A.rowptr[i + 1]; ++j) acc += A.val64[j] * x0[A.col[j]];
      }
      ri = bi - acc;
    }
    A.x64a[i] = xi;
    A.r64[i] = ri;
    v[0] = ri * ri;
    v[1] = bi * bi;
  }
  block_sum_w<3, BS / 64>(v, lds);
  store_partials(A.part_out, lb, v);
  if (lb == 0 && threadIdx.x == 0) {
    prm_out->rtol = prm.rtol;  // field by field, as for the record
    prm_out->inner_rtol = prm.inner_rtol;
    prm_out->max_inner = prm.max_inner;
    prm_out->max_refine = prm.max_refine;
    prm_out->mixed = prm.mixed;
    prm_out->epoch = prm.epoch;
    prm_out->atol = prm.atol;
    put_rec(A.rec_out, nullptr, (int)prm.epoch, 0, kInit, 0, 0, 0, 0, 0, 0.0, 0.0, 0.0, 0.0, 0.0,
            0.0);
  }
}

// One step of the solve (see the file comment) for the rows of logical block
// lb. One thread per row, BS threads per block.
// W: ELL width (4, 6 or 8 slots per row), 0 for the CSR path.
// SUMMED: the previous launch's dots arrive already summed by a separate
// launch (large systems): they are uniform loads, alpha and beta are known
// before the neighbour values arrive, and each neighbour is folded into the
// product as its load returns (few registers, more waves in flight). Else
// every block re-reduces the per-block partials, and the neighbour loads
// are issued before that reduction to overlap with it.
// LATE: gather the neighbours after the reduction even when the block
// re-reduces the partials itself (fewer registers: more blocks per CU when
// one launch carries several solves).
// CSR entries per row loaded in one batch by the step (most rows of the
// meshes here have fewer: the Delaunay mesh's free rows hold about 3
// off-diagonal entries, at most 8 to 11).
constexpr int kCsrBatch = 8;

template <typename T, int W, bool SUMMED, int BS, bool LATE = false>
__device__ __forceinline__ void step_body(const StepArgs<T>& A, const int lb, double* lds) {
  constexpr bool PRE = !SUMMED && !LATE;  // neighbour values loaded before the reduction
  // The record slot read here is written only by the next launch, so every
  // thread reads it directly: uniform scalar loads, values kept read-only.
  const Rec Rin = *A.rec_in;
  const Params P = *A.prm;
  // ---- loads that do not depend on the phase or on alpha, beta --------
  double red[3] = {0.0, 0.0, 0.0};
  if constexpr (!SUMMED) {
    constexpr int kPer = (kMaxGrid + BS - 1) / BS;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int j = threadIdx.x + u * BS;
      const bool in = j < A.nparts_in;
      const int jc = in ? j : 0;  // unconditional loads; out-of-range slots add 0
      const double a0 = A.part_in[4 * jc], a1 = A.part_in[4 * jc + 1],
                   a2 = A.part_in[4 * jc + 2];
      red[0] += in ? a0 : 0.0;
      red[1] += in ? a1 : 0.0;
      red[2] += in ? a2 : 0.0;
    }
  }
  const int i = lb * BS + threadIdx.x;
  const bool live = i < A.n;
  const int ic = live ? i : A.n - 1;  // the tail loads a valid row, stores nothing
  const Quad<T> own = A.rq_in[ic];
  const T r0 = own.r, s0 = own.s, q0 = own.q, d0 = own.d;
  const T p0 = A.p[ic], x0 = A.x[ic];
  constexpr int WA = W > 0 ? W : 1;
  T nr[WA], ns[WA], nq[WA], nd[WA], nw[WA];
  int32_t e[WA];
  if constexpr (W > 0) {
    const int32_t* ell = A.ell + ic;
#pragma unroll
    for (int k = 0; k < W; ++k) e[k] = ell[(size_t)k * A.n_pad];
    if constexpr (PRE) {
#pragma unroll
      for (int k = 0; k < W; ++k) {
        const Quad<T> qn = A.rq_in[ell_col(e[k])];
        nr[k] = qn.r;
        ns[k] = qn.s;
        nq[k] = qn.q;
        nd[k] = qn.d;
        nw[k] = ell_weight<T>(e[k]);
      }
    }
  }
  // CSR rows: the first kCsrBatch entries are loaded together (column and
  // value, then the neighbour's record; before the reduction when PRE), so a
  // row costs two dependent rounds of loads whatever its length; longer rows
  // finish in a loop. Every index read stays inside the arrays (they hold at
  // least one entry): slots past the row end read the row's last entry or
  // slot 0 and are masked.
  constexpr int kCB = W == 0 ? kCsrBatch : 1;
  int j0 = 0, j1 = 0;
  int32_t cc[kCB];
  T cv[kCB];
  Quad<T> cq[kCB];
  if constexpr (W == 0) {
    j0 = A.rowptr[ic];
    j1 = A.rowptr[ic + 1];
    const int jl = j1 > 0 ? j1 - 1 : 0;
#pragma unroll
    for (int k = 0; k < kCB; ++k) {
      const bool in = j0 + k < j1;
      const int jc = min(j0 + k, jl);
      const int32_t c = A.col[jc];
      const T v = A.val[jc];
      cc[k] = in ? c : ic;
      cv[k] = in ? v : T(0);
    }
    if constexpr (PRE) {
#pragma unroll
      for (int k = 0; k < kCB; ++k) cq[k] = A.rq_in[cc[k]];
    }
  }
  const bool writer = lb == 0 && threadIdx.x == 0;
  const int phase = A.force ? (int)kIter : Rin.phase;
  if constexpr (SUMMED) {
    red[0] = A.part_in[0];
    red[1] = A.part_in[1];
    red[2] = A.part_in[2];
  } else {
    block_sum_once<3, BS / 64>(red, lds);
  }
  // A launch queued after the solve has ended leaves here (the phase is
  // uniform). Testing it before the reduction above would put the record
  // load on every working launch's critical path.
  if (phase >= kDoneOk) {
    // carry the record forward field by field (a whole-struct copy of the
    // local record would put it in LDS); the host mirror already shows the end
    if (writer)
      put_rec(A.rec_out, nullptr, Rin.epoch, Rin.seq, Rin.phase, Rin.iter, Rin.total, Rin.ninner,
              Rin.stagnant, Rin.xp, Rin.gamma_prev, Rin.alpha_prev, Rin.rho_ref, Rin.tol2,
              Rin.rnorm, Rin.bnorm);
    return;
  }
  double v[3] = {0.0, 0.0, 0.0};

  if (phase == kInit) {
    // red[0] = ||r64||^2 from the start or refinement launch; the start
    // launch also sends red[1] = ||b||^2
    double rnorm = sqrt(red[0]);
    const double bnorm = Rin.ninner == 0 ? sqrt(red[1]) : Rin.bnorm;
    // stop at ||r|| <= rtol ||b||, and (atol > 0) at ||r|| <= atol too
    const double tol = P.atol > 0.0 ? fmin(P.rtol * bnorm, P.atol) : P.rtol * bnorm;
    int stagnant = Rin.stagnant;
    int next = 0;
    if (!isfinite(rnorm)) next = kDoneBad;
    else if (rnorm <= tol) next = kDoneOk;
    else if (bnorm == 0.0 && Rin.ninner == 0) {
      // b = 0 with a non-zero start: the solution is x = 0
      if (live) (Rin.xp ? A.x64b : A.x64a)[i] = 0.0;
      rnorm = 0.0;
      next = kDoneOk;
    }
    else if ((double)Rin.ninner >= P.max_refine) next = kDoneNoConv;
    else if (Rin.ninner > 0) {
      stagnant = rnorm > 0.5 * Rin.rnorm ? stagnant + 1 : 0;
      if (stagnant >= 3) next = kDoneNoConv;
    }
    if (next) {
      if (writer)
        put_rec(A.rec_out, A.mirror, Rin.epoch, Rin.seq + 1, next, Rin.iter, Rin.total,
                Rin.ninner, stagnant, Rin.xp,
                Rin.gamma_prev, Rin.alpha_prev, Rin.rho_ref, Rin.tol2, rnorm, bnorm);
      return;
    }
    // Inner target: what the outer tolerance still needs, never looser than
    // inner_rtol in mixed mode.
    const double want = 0.5 * tol / rnorm;
    const double itol = P.mixed != 0.0 ? fmax(P.inner_rtol, want) : fmax(want, 1e-15);
    const double scale = 1.0 / rnorm;
    if (live) {
      // D^-1 from the matrix (the per-row records may not hold it yet)
      const T di = A.dinv[i];
      const T ri = (T)(A.r64[i] * scale);
      const T zi = di * ri;
      T acc = ri;  // diagonal term: K_ii z_i = r_i
      if constexpr (W > 0) {
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const int c = ell_col(e[k]);
          acc = fmaT(ell_weight<T>(e[k]), A.dinv[c] * (T)(A.r64[c] * scale), acc);
        }
      } else {
        for (int j = A.rowptr[i]; j < A.rowptr[i + 1]; ++j) {
          const int c = A.col[j];
          acc = fmaT(A.val[j], A.dinv[c] * (T)(A.r64[c] * scale), acc);
        }
      }
      A.x[i] = T(0);
      A.p[i] = T(0);
      A.rq_out[i] = Quad<T>{ri, acc, T(0), di};
      v[0] = (double)ri * (double)zi;
      v[1] = (double)zi * (double)acc;
      v[2] = (double)ri * (double)ri;
    }
    block_sum_once<3, BS / 64>(v, lds + 3 * (BS / 64));
    store_partials(A.part_out, lb, v);
    if (writer)
      put_rec(A.rec_out, A.mirror, Rin.epoch, Rin.seq + 1, kIter, 0, Rin.total, Rin.ninner + 1,
              stagnant, Rin.xp, 0.0, 0.0, 0.0,
              itol * itol, rnorm, bnorm);
    return;
  }

  // ---- kIter --------------------------------------------------------------
  const int iter = Rin.iter;
  const double gamma = red[0], delta = red[1], rho = red[2];
  const double rho_ref = iter == 0 ? rho : Rin.rho_ref;
  double alpha, beta;
  if (iter == 0) {
    beta = 0.0;
    alpha = gamma / delta;
  } else {
    beta = gamma / Rin.gamma_prev;
    alpha = gamma / (delta - beta * gamma / Rin.alpha_prev);
  }
  bool stop = false;
  if (!A.force) {
    stop = !(rho > Rin.tol2 * rho_ref)          // converged (also rho == 0)
           || !(alpha > 0.0) || !isfinite(alpha)  // breakdown
           || (double)iter >= P.max_inner;        // iteration cap
  }
  if (stop) {
    // Inner solve over: x64 += rnorm * d (d = the correction in x),
    // r64 = b - K_FF x64, partial ||r64||^2. Neighbours' new x64 values are
    // recomputed from their old value and correction.
    const double* xo = Rin.xp ? A.x64b : A.x64a;
    double* xn = Rin.xp ? A.x64a : A.x64b;
    const double sc = Rin.rnorm;
    if (live) {
      const double xi = xo[i] + sc * (double)x0;
      double acc = A.diag64[i] * xi;
      if constexpr (W > 0) {
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const int c = ell_col(e[k]);
          acc += ell_weight<double>(e[k]) * (xo[c] + sc * (double)A.x[c]);
        }
      } else {
        for (int j = A.rowptr[i]; j < A.rowptr[i + 1]; ++j) {
          const int c = A.col[j];
          acc += A.val64[j] * (xo[c] + sc * (double)A.x[c]);
        }
      }
      const double ri = A.b64[i] - acc;
      xn[i] = xi;
      A.r64[i] = ri;
      v[0] = ri * ri;
    }
    block_sum_once<3, BS / 64>(v, lds + 3 * (BS / 64));
    store_partials(A.part_out, lb, v);
    if (writer)
      put_rec(A.rec_out, A.mirror, Rin.epoch, Rin.seq + 1, kInit, iter, Rin.total + iter,
              Rin.ninner, Rin.stagnant, Rin.xp ^ 1,
              gamma, alpha, rho_ref, Rin.tol2, Rin.rnorm, Rin.bnorm);
    return;
  }
  const T a = (T)alpha, b = (T)beta;
  if (live) {
    const T pi = fmaT(b, p0, d0 * r0);
    const T qi = fmaT(b, q0, s0);
    A.x[i] = fmaT(a, pi, x0);
    A.p[i] = pi;
    const T ri = next_r(r0, s0, q0, a, b);
    const T zi = d0 * ri;
    T acc = ri;  // diagonal term: K_ii z_i = r_i
    if constexpr (W > 0 && !PRE) {
#pragma unroll
      for (int k = 0; k < W; ++k) {
        const Quad<T> qn = A.rq_in[ell_col(e[k])];
        const T rc = next_r(qn.r, qn.s, qn.q, a, b);
        acc = fmaT(ell_weight<T>(e[k]), qn.d * rc, acc);
      }
    } else if constexpr (W > 0) {
#pragma unroll
      for (int k = 0; k < W; ++k) {
        const T rc = next_r(nr[k], ns[k], nq[k], a, b);
        acc = fmaT(nw[k], nd[k] * rc, acc);
      }
    } else {
      if constexpr (!PRE) {
#pragma unroll
        for (int k = 0; k < kCB; ++k) cq[k] = A.rq_in[cc[k]];
      }
#pragma unroll
      for (int k = 0; k < kCB; ++k) {
        if (j0 + k < j1) {
          const T rc = next_r(cq[k].r, cq[k].s, cq[k].q, a, b);
          acc = fmaT(cv[k], cq[k].d * rc, acc);
        }
      }
      for (int j = j0 + kCB; j < j1; ++j) {
        const Quad<T> qc = A.rq_in[A.col[j]];
        const T rc = next_r(qc.r, qc.s, qc.q, a, b);
        acc = fmaT(A.val[j], qc.d * rc, acc);
      }
    }
    A.rq_out[i] = Quad<T>{ri, acc, qi, d0};
    v[0] = (double)ri * (double)zi;
    v[1] = (double)zi * (double)acc;
    v[2] = (double)ri * (double)ri;
  }
  block_sum_once<3, BS / 64>(v, lds + 3 * (BS / 64));
  store_partials(A.part_out, lb, v);
  if (writer)
    put_rec(A.rec_out, A.mirror, Rin.epoch, Rin.seq + 1, kIter, iter + 1, Rin.total, Rin.ninner,
            Rin.stagnant, Rin.xp, gamma, alpha,
            rho_ref, Rin.tol2, Rin.rnorm, Rin.bnorm);
}

template <typename T, int W, bool SUMMED, int BS>
__global__ __launch_bounds__(BS) void k_step(StepArgs<T> A) {
  __shared__ double lds[6 * (BS / 64)];
  step_body<T, W, SUMMED, BS>(A, logical_block(), lds);
}

// Systems handled by one batched launch (bounded by the kernel-argument size).
constexpr int kArgSlots = 20;

// Large systems: a separate launch sums the per-block partials between
// steps, in two levels. Block b of that launch adds partials
// [b * kRedChunk, (b + 1) * kRedChunk) in a fixed order; the block that ends
// last (an integer counter tells) adds the block sums in a fixed order and
// writes the total. Which block ends last does not change any bit. The block
// sums travel through device-scope atomic stores and loads, so they are
// coherent across the XCDs' L2 caches.
constexpr int kRedChunk = 1024;   // partials per block of the reduction launch

struct ReduceArgs {
  int n;                               // systems summed by this launch
  int32_t start[kArgSlots + 1];     // first block of each system; start[n] = grid
  int32_t nparts[kArgSlots];
  const double* part[kArgSlots];    // per-block partials (4 doubles each)
  double* level1[kArgSlots];        // block sums (4 doubles each)
  int32_t* counter[kArgSlots];      // blocks done (0 between launches)
  double* out[kArgSlots];           // total: 3 doubles (+ one 0)
};

__global__ __launch_bounds__(kBlock) void k_reduce_partials(ReduceArgs R) {
  __shared__ double lds[12];
  __shared__ int last;
  const int g = blockIdx.x;
  int j = 0;  // system of this block (uniform)
#pragma unroll
  for (int k = 1; k < kArgSlots; ++k) j += (k < R.n && R.start[k] <= g) ? 1 : 0;
  const int b = g - R.start[j], nb = R.start[j + 1] - R.start[j];
  const double* part = R.part[j];
  const int j0 = b * kRedChunk, j1 = min(R.nparts[j], j0 + kRedChunk);
  double v[3] = {0.0, 0.0, 0.0};
  for (int q = j0 + threadIdx.x; q < j1; q += kBlock) {
    v[0] += part[4 * q];
    v[1] += part[4 * q + 1];
    v[2] += part[4 * q + 2];
  }
  block_sum<3>(v, lds);
  double* out = R.out[j];
  if (nb == 1) {
    if (threadIdx.x == 0) {
      out[0] = v[0];
      out[1] = v[1];
      out[2] = v[2];
      out[3] = 0.0;
    }
    return;
  }
  double* l1 = R.level1[j];
  if (threadIdx.x == 0) {
    for (int c = 0; c < 3; ++c)
      __hip_atomic_store(&l1[4 * b + c], v[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const int t = atomicAdd(R.counter[j], 1);
    last = t == nb - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double w[3] = {0.0, 0.0, 0.0};
  for (int q = threadIdx.x; q < nb; q += kBlock)
    for (int c = 0; c < 3; ++c)
      w[c] += __hip_atomic_load(&l1[4 * q + c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  block_sum<3>(w, lds);
  if (threadIdx.x == 0) {
    out[0] = w[0];
    out[1] = w[1];
    out[2] = w[2];
    out[3] = 0.0;
    __hip_atomic_store(R.counter[j], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------- batched steps --
// Several meshes' FP32 solves advance in one launch. The grid is the
// concatenation of every slot's own grid (each a multiple of 8); a block finds
// its slot from the start offsets, then runs exactly the code of the
// single-mesh step on that slot's arguments with its slot-local logical block,
// so a solve gives the same bits alone or in any batch. The arguments travel
// by value (pointers in by-value kernel arguments are known to be global, so
// the step keeps its SGPR-based addressing), which caps a launch at
// kArgSlots slots.

struct BatchArgs {
  int n;                         // slots in this launch
  int32_t start[kArgSlots + 1];  // first logical block of each slot; start[n] = grid
  StepArgs<float> a[kArgSlots];
};

static_assert(sizeof(BatchArgs) <= 4096, "kernel arguments of a batched step");

template <int W, bool SUMMED, int BS>
__global__ __launch_bounds__(BS) void k_step_batch(BatchArgs B) {
  __shared__ double lds[6 * (BS / 64)];
  const int lb = logical_block();
  int j = 0;  // slot of this block (uniform: scalar registers)
#pragma unroll
  for (int k = 1; k < kArgSlots; ++k) j += (k < B.n && B.start[k] <= lb) ? 1 : 0;
  const StepArgs<float>& A = B.a[j];
  const int lblk = lb - B.start[j];
  if (A.rec_in->phase >= kDoneOk) {  // idle slot: keep its record, skip the work
    if (lblk == 0 && threadIdx.x == 0) *A.rec_out = *A.rec_in;
    return;
  }
  step_body<float, W, SUMMED, BS>(A, lblk, lds);
}

// ------------------------------------------------------ multi-RHS steps --
// The channels of a colour image share the mask, hence K_FF: one launch
// advances up to kMaxRhs solves with the same matrix. Hardware block b runs
// on XCD b % 8; the k-th block of an XCD takes solve k % nrhs and row block
// (b % 8) * (G / 8) + k / nrhs (G row blocks per solve), so the solves'
// blocks for the same rows run side by side on one XCD: the rows' matrix
// entries and D^-1, fetched from HBM by the first of them, are L2 hits for
// the others. Every block runs the single-solve step on its solve's
// arguments and the row block the single-solve launch would give it, so
// each solve gets the bits of its own single solve (records, partial sums
// and vectors are per solve; the solves may be in different phases).
template <typename T>
struct MultiArgs {
  int nrhs;  // solves in this launch, 1..kMaxRhs; the grid is nrhs * G
  StepArgs<T> a[kMaxRhs];
};

template <typename T, int W, bool SUMMED, int BS>
__global__ __launch_bounds__(BS) void k_step_multi(MultiArgs<T> B) {
  __shared__ double lds[6 * (BS / 64)];
  const int nr = B.nrhs;
  const int per = (int)(gridDim.x / nr) >> 3;  // row blocks per XCD slab
  const int k = blockIdx.x >> 3;
  const int c = k % nr;
  step_body<T, W, SUMMED, BS, true>(B.a[c], (blockIdx.x & 7) * per + k / nr, lds);
}

// ELL packing of the CSR off-diagonal part; flags values other than -1/2, -1.
__global__ __launch_bounds__(kBlock) void k_pack_ell(int n, int n_pad, int W,
                                                     const int32_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ val,
                                                     int32_t* __restrict__ ell,
                                                     int32_t* __restrict__ flag) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_pad) return;
  const int j0 = i < n ? rowptr[i] : 0, j1 = i < n ? rowptr[i + 1] : 0;
  for (int k = 0; k < W; ++k) {
    int32_t e = kPadBit | (i < n ? i : 0);
    if (j0 + k < j1) {
      const double w = val[j0 + k];
      e = col[j0 + k];
      if (w == -1.0) e |= (int32_t)0x80000000;
      else if (w != -0.5) atomicOr(flag, 1);
    }
    ell[(int64_t)k * n_pad + i] = e;
  }
  if (i < n && j1 - j0 > W) atomicOr(flag, 2);
}

__global__ __launch_bounds__(kBlock) void k_max_rowlen(int n, const int32_t* __restrict__ rowptr,
                                                       int32_t* __restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) atomicMax(out, rowptr[i + 1] - rowptr[i]);
}

__global__ void k_zero_flag(int32_t* f) { f[0] = 0; f[1] = 0; f[2] = 0; f[3] = 0; }

// ---------------------------------------------------------------- host ----
template <typename T>
struct Prec;
template <>
struct Prec<float> {
  static constexpr int idx = 0;
  static const float* val(fi_mesh* M) { return M->d_ff_val32; }
  static const float* dinv(fi_mesh* M) { return M->d_dinv32; }
  static CGState& st(fi_mesh* M) { return M->cg32; }
};
template <>
struct Prec<double> {
  static constexpr int idx = 1;
  static const double* val(fi_mesh* M) { return M->d_ff_val64; }
  static const double* dinv(fi_mesh* M) { return M->d_dinv64; }
  static CGState& st(fi_mesh* M) { return M->cg64; }
};

Rec* rec_slot(fi_mesh* M, int k) { return (Rec*)M->d_rec + k; }

// Arguments of the launch of parity `par` (reads slot par, writes slot par^1).
template <typename T>
StepArgs<T> make_args(fi_mesh* M, int par, int force) {
  CGState& S = Prec<T>::st(M);
  const int a = par, b = par ^ 1;
  StepArgs<T> A;
  A.n = (int)M->n;
  A.n_pad = (int)M->n_pad;
  A.W = M->ell_w;
  A.ell = M->d_ell;
  A.rowptr = M->d_ff_rowptr;
  A.col = M->d_ff_col;
  A.val = Prec<T>::val(M);
  A.val64 = M->d_ff_val64;
  A.dinv = Prec<T>::dinv(M);
  A.diag64 = M->d_diag64;
  A.x = (T*)S.x;
  A.p = (T*)S.p;
  A.rq_in = (const Quad<T>*)S.rq[a];
  A.rq_out = (Quad<T>*)S.rq[b];
  if (M->large_mode) {
    A.part_in = M->d_red4;
    A.nparts_in = 1;
  } else {
    A.part_in = M->d_part + (size_t)a * 4 * M->cg_grid;
    A.nparts_in = M->cg_grid;
  }
  A.part_out = M->d_part + (size_t)b * 4 * M->cg_grid;
  A.rec_in = rec_slot(M, a);
  A.rec_out = rec_slot(M, b);
  A.prm = (const Params*)M->d_prm;
  A.b64 = M->d_b64;
  A.r64 = M->d_r64;
  A.x64a = M->d_x64buf[0];
  A.x64b = M->d_x64buf[1];
  A.mirror = (Mirror*)M->d_mirror;
  A.force = force;
  return A;
}

template <typename T, int W, bool SUMMED>
void* step_ptr(int bs) {
  switch (bs) {
    case 256: return (void*)k_step<T, W, SUMMED, 256>;
    default: return (void*)k_step<T, W, SUMMED, 512>;
  }
}

template <typename T, bool SUMMED>
void* step_ptr_w(int w, int bs) {
  switch (w) {
    case 4: return step_ptr<T, 4, SUMMED>(bs);
    case 6: return step_ptr<T, 6, SUMMED>(bs);
    case 8: return step_ptr<T, 8, SUMMED>(bs);
    default: return step_ptr<T, 0, SUMMED>(bs);
  }
}

template <typename T>
void* step_kernel(fi_mesh* M) {
  return M->large_mode ? step_ptr_w<T, true>(M->ell_w, M->cg_bs)
                       : step_ptr_w<T, false>(M->ell_w, M->cg_bs);
}

template <bool SUMMED>
void* batch_kernel_w(int w) {
  switch (w) {
    case 4: return (void*)k_step_batch<4, SUMMED, kBatchBS>;
    case 6: return (void*)k_step_batch<6, SUMMED, kBatchBS>;
    default: return (void*)k_step_batch<8, SUMMED, kBatchBS>;
  }
}

void* batch_kernel(int w, bool large) {
  return large ? batch_kernel_w<true>(w) : batch_kernel_w<false>(w);
}

// ELL width used for a widest row of w entries (0: too wide, CSR).
int ell_width_for(int w) { return w <= 4 ? 4 : w <= 6 ? 6 : w <= kMaxEll ? 8 : 0; }

template <typename T>
void* start_kernel(fi_mesh* M) {
  switch (M->cg_bs) {
    case 256: return (void*)k_solve_start<T, 256>;
    default: return (void*)k_solve_start<T, 512>;
  }
}

// Adds a large system's reduction after the step of parity `par` (which
// wrote partial slot par ^ 1) to R, whose grid grows by the system's blocks.
void add_reduce(ReduceArgs& R, fi_mesh* M, int par) {
  const int q = R.n;
  const int nb = (M->cg_grid + kRedChunk - 1) / kRedChunk;
  R.start[q + 1] = R.start[q] + nb;
  R.nparts[q] = M->cg_grid;
  R.part[q] = M->d_part + (size_t)(par ^ 1) * 4 * M->cg_grid;
  R.level1[q] = M->d_lvl1;
  R.counter[q] = M->d_flag + 2;
  R.out[q] = M->d_red4;
  R.n = q + 1;
}

int launch_reduce_after(fi_mesh* M, int par) {
  ReduceArgs R{};
  add_reduce(R, M, par);
  void* args[1] = {&R};
  FI_HIP_TRY(hipLaunchKernel((void*)k_reduce_partials, dim3(R.start[1]), dim3(kBlock), args, 0,
                             M->ctx->stream));
  return FI_OK;
}

template <typename T>
int launch_step(fi_mesh* M, int par, int force) {
  StepArgs<T> A = make_args<T>(M, par, force);
  void* args[1] = {&A};
  FI_HIP_TRY(hipLaunchKernel(step_kernel<T>(M), dim3(M->cg_grid), dim3(M->cg_bs), args, 0,
                             M->ctx->stream));
  if (M->large_mode) return launch_reduce_after(M, par);
  return FI_OK;
}

// The one-iteration launch's vectors in precision T (x, p and the two
// record buffers), allocated by the first solve that uses them: a quadtree
// mesh with the S-iteration plan never does in FP32, and FP64 only when
// asked for.
template <typename T>
int ensure_cg_state(fi_mesh* M) {
  CGState& S = Prec<T>::st(M);
  if (S.x) return FI_OK;
  const size_t n = (size_t)std::max<int64_t>(M->n, 1);
  void* p[4] = {nullptr, nullptr, nullptr, nullptr};
  int rc = 0;
  if ((rc = device_alloc(M, &p[0], n * sizeof(T))) || (rc = device_alloc(M, &p[1], n * sizeof(T))) ||
      (rc = device_alloc(M, &p[2], 4 * n * sizeof(T))) ||
      (rc = device_alloc(M, &p[3], 4 * n * sizeof(T))))
    return rc;
  S = CGState{p[0], p[1], {p[2], p[3]}};
  return FI_OK;
}

// Every solve in the one-iteration launch starts here.
template <typename T>
int launch_start(fi_mesh* M, const fi_solve_opts* o, int epoch, const double* x0 = nullptr) {
  if (const int rc = ensure_cg_state<T>(M)) return rc;
  StepArgs<T> A = make_args<T>(M, 1, 0);  // writes record and partials of slot 0
  Params prm{};
  prm.rtol = o->rtol;
  prm.atol = o->atol;
  prm.inner_rtol = o->inner_rtol;
  prm.max_inner = o->max_inner;
  prm.max_refine = o->max_refine;
  prm.mixed = sizeof(T) == sizeof(float) ? 1.0 : 0.0;
  prm.epoch = epoch;
  Params* pout = (Params*)M->d_prm;
  void* args[4] = {&A, &prm, &pout, &x0};
  FI_HIP_TRY(hipLaunchKernel(start_kernel<T>(M), dim3(M->cg_grid), dim3(M->cg_bs), args, 0,
                             M->ctx->stream));
  if (M->large_mode) return launch_reduce_after(M, 1);
  return FI_OK;
}



// The host queues chunks of kChunk step launches, each followed by an event
// (plain launches: measured faster here than replaying a recorded graph),
// keeps at most kAhead chunks queued, and stops as soon as the mirror shows
// the end of this solve. Chunks still queued then run as idle launches;
// later work on the stream is ordered after them. Pacing and the launch
// prediction: pacer.h.
static_assert(kAhead <= kChunkEvents, "every queued chunk needs its own event");

// Which prediction slot a solve uses: precision and cold or warm start.
template <typename T>
int pred_slot(const double* x0) {
  return (sizeof(T) == sizeof(double) ? 2 : 0) + (x0 ? 1 : 0);
}
static_assert(kPredSlots == 4, "one slot per precision and start");

Pacer pacer_for(const fi_solve_opts* o, int64_t pred) {
  return make_pacer(o->max_inner, o->max_refine, pred);
}

template <typename T>
int solve_dev(fi_mesh* M, const fi_solve_opts* o, fi_solve_stats* stats, const double* x0) {
  hipStream_t st = M->ctx->stream;
  const int epoch = next_epoch(M);
  int rc = launch_start<T>(M, o, epoch, x0);
  if (rc) return rc;
  const int slot = pred_slot<T>(x0);
  Pacer pc = pacer_for(o, M->pred_launches[slot]);
  for (;;) {
    int drc = FI_OK;
    int64_t nl = 0;
    if (read_mirror(M, epoch, stats, &drc, &nl)) {
      M->pred_launches[slot] = nl;
      return drc;
    }
    if (const int n = pc.next()) {
      for (int q = 0; q < n; ++q) {
        rc = launch_step<T>(M, q & 1, 0);
        if (rc) return rc;
      }
      FI_HIP_TRY(hipEventRecord(M->chunk_ev[pc.launched % kChunkEvents], st));
      pc.queued_chunk(n);
      continue;
    }
    if (pc.completed < pc.launched) {
      const hipError_t q = hipEventQuery(M->chunk_ev[pc.completed % kChunkEvents]);
      if (q == hipSuccess) {
        ++pc.completed;
        continue;
      }
      if (q != hipErrorNotReady)
        return fail(FI_E_HIP, std::string("stream failed: ") + hipGetErrorString(q));
    } else {  // everything launched (up to the limit) has run and the solve never ended
      if (read_mirror(M, epoch, stats, &drc, nullptr)) return drc;
      return fail(FI_E_HIP, "solver did not report termination");
    }
    __builtin_ia32_pause();
  }
}

template <typename T, int W, bool SUMMED>
void* multi_ptr(int bs) {
  return bs == 256 ? (void*)k_step_multi<T, W, SUMMED, 256> : (void*)k_step_multi<T, W, SUMMED, 512>;
}

template <typename T, bool SUMMED>
void* multi_kernel_w(int w, int bs) {
  switch (w) {
    case 4: return multi_ptr<T, 4, SUMMED>(bs);
    case 6: return multi_ptr<T, 6, SUMMED>(bs);
    case 8: return multi_ptr<T, 8, SUMMED>(bs);
    default: return multi_ptr<T, 0, SUMMED>(bs);
  }
}

template <typename T>
void* multi_kernel(const fi_mesh* M) {
  return M->large_mode ? multi_kernel_w<T, true>(M->ell_w, M->cg_bs)
                       : multi_kernel_w<T, false>(M->ell_w, M->cg_bs);
}

// Launch arguments of a multi-RHS step for both parities (and, for large
// systems, of the reduction that follows it: one launch sums every solve's
// partials).
template <typename T>
struct MultiLaunch {
  MultiArgs<T> a[2];
  ReduceArgs r[2];
};

template <typename T>
void multi_prepare(fi_mesh* const* ch, int nc, int force, MultiLaunch<T>& L) {
  for (int par = 0; par < 2; ++par) {
    L.a[par] = MultiArgs<T>{};
    L.a[par].nrhs = nc;
    L.r[par] = ReduceArgs{};
    for (int c = 0; c < nc; ++c) {
      L.a[par].a[c] = make_args<T>(ch[c], par, force);
      if (ch[0]->large_mode) add_reduce(L.r[par], ch[c], par);
    }
  }
}

template <typename T>
int multi_launch(fi_mesh* M0, MultiLaunch<T>& L, int par) {
  void* args[1] = {&L.a[par]};
  const unsigned grid = (unsigned)L.a[par].nrhs * (unsigned)M0->cg_grid;
  FI_HIP_TRY(hipLaunchKernel(multi_kernel<T>(M0), dim3(grid), dim3(M0->cg_bs), args, 0,
                             M0->ctx->stream));
  if (!M0->large_mode) return FI_OK;
  void* rargs[1] = {&L.r[par]};
  FI_HIP_TRY(hipLaunchKernel((void*)k_reduce_partials, dim3(L.r[par].start[L.r[par].n]),
                             dim3(kBlock), rargs, 0, M0->ctx->stream));
  return FI_OK;
}

// The solves of all channels advance together, one launch per step, paced
// like solve_dev (events of channel 0), until every channel's mirror shows
// its end.
template <typename T>
int solve_multi_dev(fi_mesh* const* ch, int nc, const fi_solve_opts* o, fi_solve_stats* stats,
                    const double* const* x0) {
  fi_mesh* M0 = ch[0];
  hipStream_t st = M0->ctx->stream;
  int epoch[kMaxRhs];
  bool done[kMaxRhs] = {};
  int rc = FI_OK, first_rc = FI_OK;
  for (int c = 0; c < nc; ++c) {
    epoch[c] = next_epoch(ch[c]);
    if ((rc = launch_start<T>(ch[c], o, epoch[c], x0 ? x0[c] : nullptr))) return rc;
  }
  // Launch arguments for the solves still running; a solve that has ended
  // leaves the launches from the next chunk on (chunks start at parity 0).
  MultiLaunch<T> L;
  fi_mesh* run[kMaxRhs];
  int nrun = nc;
  for (int c = 0; c < nc; ++c) run[c] = ch[c];
  multi_prepare<T>(run, nrun, 0, L);
  // paced to the longest predicted channel (no cap while one has none)
  int64_t pred = 0;
  bool every = true;
  for (int c = 0; c < nc; ++c) {
    const int64_t p = ch[c]->pred_launches[pred_slot<T>(x0 ? x0[c] : nullptr)];
    every = every && p > 0;
    pred = std::max(pred, p);
  }
  if (!every) pred = 0;
  Pacer pc = pacer_for(o, pred);
  auto all_done = [&]() {
    bool all = true;
    for (int c = 0; c < nc; ++c) {
      if (!done[c]) {
        int drc = FI_OK;
        int64_t nl = 0;
        done[c] = read_mirror(ch[c], epoch[c], &stats[c], &drc, &nl) != 0;
        if (done[c]) {
          ch[c]->pred_launches[pred_slot<T>(x0 ? x0[c] : nullptr)] = nl;
          if (drc && !first_rc) first_rc = drc;
        }
      }
      all = all && done[c];
    }
    return all;
  };
  for (;;) {
    if (all_done()) return first_rc;
    int left = 0;
    for (int c = 0; c < nc; ++c)
      if (!done[c]) run[left++] = ch[c];
    if (left < nrun) {
      nrun = left;
      multi_prepare<T>(run, nrun, 0, L);
    }
    if (const int n = pc.next()) {
      for (int q = 0; q < n; ++q)
        if ((rc = multi_launch<T>(M0, L, q & 1))) return rc;
      FI_HIP_TRY(hipEventRecord(M0->chunk_ev[pc.launched % kChunkEvents], st));
      pc.queued_chunk(n);
      continue;
    }
    if (pc.completed < pc.launched) {
      const hipError_t q = hipEventQuery(M0->chunk_ev[pc.completed % kChunkEvents]);
      if (q == hipSuccess) {
        ++pc.completed;
        continue;
      }
      if (q != hipErrorNotReady)
        return fail(FI_E_HIP, std::string("stream failed: ") + hipGetErrorString(q));
    } else {
      if (all_done()) return first_rc;
      return fail(FI_E_HIP, "solver did not report termination");
    }
    __builtin_ia32_pause();
  }
}

}  // namespace

int next_epoch(fi_mesh* M) {
  M->epoch = (M->epoch + 1) & kEpochMask;
  if (M->epoch == 0) M->epoch = 1;  // 0 never names a solve
  return M->epoch;
}

// Reads the host mirror: 1 with stats filled when solve `epoch` has ended,
// 0 while it runs.
int read_mirror(fi_mesh* M, int epoch, fi_solve_stats* stats, int* rc, int64_t* launches) {
  Mirror* m = (Mirror*)M->h_mirror;
  const uint64_t w = __atomic_load_n(&m->word, __ATOMIC_ACQUIRE);
  *rc = FI_OK;
  if ((int)((w & 0x7FFFFFFFu) >> 4) != epoch) return 0;
  const int phase = (int)(w & 15);
  if (phase < kDoneOk) return 0;
  stats->iterations = (int64_t)((w >> 32) & 0xFFFFFFu);
  stats->refinements = (int32_t)((w >> 56) & 0x7Fu);
  double rn, bn;
  int64_t nl;
  __atomic_load(&m->launches, &nl, __ATOMIC_RELAXED);
  if (launches) *launches = nl;
  stats->launches = nl;
  __atomic_load(&m->rnorm, &rn, __ATOMIC_RELAXED);
  __atomic_load(&m->bnorm, &bn, __ATOMIC_RELAXED);
  stats->rel_residual = bn > 0 ? rn / bn : 0.0;
  stats->residual = rn;
  stats->rhs_norm = bn;
  stats->status = phase == kDoneOk ? FI_OK : FI_E_NO_CONVERGENCE;
  M->d_x64 = M->d_x64buf[(w >> 63) & 1];
  if (phase == kDoneBad) *rc = fail(FI_E_INVALID, "right-hand side or residual not finite");
  return 1;
}

int solve_multi(fi_mesh* const* ch, int nc, const fi_solve_opts* opts, fi_solve_stats* stats,
                const double* const* x0) {
  if (nc < 1 || nc > kMaxRhs) return fail(FI_E_INVALID, "1 to 3 right-hand sides per solve");
  for (int c = 0; c < nc; ++c) {
    stats[c].iterations = 0;
    stats[c].refinements = 0;
    stats[c].status = FI_OK;
    stats[c].rel_residual = 0.0;
    stats[c].residual = 0.0;
    stats[c].rhs_norm = 0.0;
    stats[c].launches = 0;
  }
  if (ch[0]->n == 0) return FI_OK;
  if (opts->precision == FI_PREC_FP64) return solve_multi_dev<double>(ch, nc, opts, stats, x0);
  if (ch[0]->ss) return ss_solve_multi(ch, nc, opts, stats, x0);
  return solve_multi_dev<float>(ch, nc, opts, stats, x0);
}

// Times `reps` multi-RHS steps over nc channels forced into the iteration
// phase (every channel iterating), between two HIP events on the stream.
int time_multi_kernel(fi_mesh* const* ch, int nc, int precision, int reps, double* ms) {
  fi_mesh* M0 = ch[0];
  if (M0->n == 0 || reps < 1 || nc < 1 || nc > kMaxRhs)
    return fail(FI_E_INVALID, "nothing to time");
  if (precision != FI_PREC_FP64 && M0->ss) return ss_time_multi(ch, nc, reps, ms);
  hipStream_t st = M0->ctx->stream;
  const bool d = precision == FI_PREC_FP64;
  fi_solve_opts o;
  fi_solve_opts_default(&o);
  int rc = FI_OK;
  for (int c = 0; c < nc; ++c) {
    const int epoch = next_epoch(ch[c]);
    rc = d ? launch_start<double>(ch[c], &o, epoch) : launch_start<float>(ch[c], &o, epoch);
    if (rc) return rc;
  }
  MultiLaunch<float> Lf;
  MultiLaunch<double> Ld;
  if (d) {
    multi_prepare<double>(ch, nc, 0, Ld);
    if ((rc = multi_launch<double>(M0, Ld, 0))) return rc;
    multi_prepare<double>(ch, nc, 1, Ld);
  } else {
    multi_prepare<float>(ch, nc, 0, Lf);
    if ((rc = multi_launch<float>(M0, Lf, 0))) return rc;
    multi_prepare<float>(ch, nc, 1, Lf);
  }
  hipEvent_t e0, e1;
  FI_HIP_TRY(hipEventCreate(&e0));
  FI_HIP_TRY(hipEventCreate(&e1));
  auto step = [&](int k) { return d ? multi_launch<double>(M0, Ld, k & 1) : multi_launch<float>(M0, Lf, k & 1); };
  for (int k = 0; k < 4; ++k)
    if ((rc = step(k + 1))) return rc;
  FI_HIP_TRY(hipEventRecord(e0, st));
  for (int k = 0; k < reps; ++k)
    if ((rc = step(k + 1))) return rc;
  FI_HIP_TRY(hipEventRecord(e1, st));
  FI_HIP_TRY(hipEventSynchronize(e1));
  float t = 0.f;
  FI_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = (double)t / reps;
  return FI_OK;
}

int batch_launch_steps(hipStream_t st, const std::vector<BatchSlot>& all, int count) {
  if (all.empty() || count <= 0) return FI_OK;
  // meshes with the S-iteration plan step in their own launches
  std::vector<fi_mesh*> ssm;
  std::vector<BatchSlot> act;
  for (const BatchSlot& s : all) {
    if (s.M->ss) ssm.push_back(s.M);
    else act.push_back(s);
  }
  if (!ssm.empty()) {
    const int rc = ss_batch_launch(st, ssm, count);
    if (rc) return rc;
  }
  if (act.empty()) return FI_OK;
  for (const BatchSlot& s : act)
    if (s.M->ell_w <= 0 || s.M->cg_bs != kBatchBS || s.M->n <= 0)
      return fail(FI_E_INVALID, "mesh cannot take part in a batched solve");
  // one launch per ELL width and per kArgSlots slots, both parities prepared
  struct Launch {
    BatchArgs b[2];
    ReduceArgs r[2];
    int64_t grid;
    int w;
    bool large;
  };
  std::vector<BatchSlot> order(act);
  auto key = [](const BatchSlot& a) { return a.M->ell_w * 2 + (a.M->large_mode ? 1 : 0); };
  std::stable_sort(order.begin(), order.end(),
                   [&](const BatchSlot& a, const BatchSlot& b) { return key(a) < key(b); });
  std::vector<Launch> L;
  for (size_t j0 = 0; j0 < order.size();) {
    Launch l{};
    size_t j1 = j0;
    while (j1 < order.size() && j1 - j0 < (size_t)kArgSlots && key(order[j1]) == key(order[j0]))
      ++j1;
    l.w = order[j0].M->ell_w;
    l.large = order[j0].M->large_mode;
    int64_t total = 0;
    for (int par = 0; par < 2; ++par) {
      l.b[par].n = (int)(j1 - j0);
      l.r[par].n = 0;
    }
    for (size_t j = j0; j < j1; ++j) {
      fi_mesh* M = order[j].M;
      const int q = (int)(j - j0);
      for (int par = 0; par < 2; ++par) {
        l.b[par].start[q] = (int32_t)total;
        l.b[par].a[q] = make_args<float>(M, par, 0);
        if (M->large_mode) add_reduce(l.r[par], M, par);
      }
      total += M->cg_grid;
    }
    if (total >= (int64_t)1 << 30) return fail(FI_E_INVALID, "batch grid too large");
    for (int par = 0; par < 2; ++par) l.b[par].start[j1 - j0] = (int32_t)total;
    l.grid = total;
    L.push_back(l);
    j0 = j1;
  }
  for (int k = 0; k < count; ++k) {
    const int par = k & 1;
    for (Launch& l : L) {
      void* args[1] = {&l.b[par]};
      FI_HIP_TRY(hipLaunchKernel(batch_kernel(l.w, l.large), dim3((unsigned)l.grid),
                                 dim3(kBatchBS), args, 0, st));
    }
    for (Launch& l : L) {
      if (l.r[par].n == 0) continue;
      void* rargs[1] = {&l.r[par]};
      FI_HIP_TRY(hipLaunchKernel((void*)k_reduce_partials, dim3(l.r[par].start[l.r[par].n]),
                                 dim3(kBlock), rargs, 0, st));
    }
  }
  return FI_OK;
}

int solve_arm(fi_mesh* M, const fi_solve_opts* o, int* epoch, const double* x0) {
  if (M->n <= 0) return fail(FI_E_INVALID, "nothing to solve");
  *epoch = next_epoch(M);
  if (M->ss) return ss_arm(M, o, *epoch, x0);
  return launch_start<float>(M, o, *epoch, x0);
}

int solve_poll(fi_mesh* M, int epoch, fi_solve_stats* stats, int* done) {
  int rc = FI_OK;
  *done = read_mirror(M, epoch, stats, &rc, nullptr);
  return rc;
}

void solver_release(fi_mesh* M) {
  ss_release(M);
  for (int k = 0; k < kChunkEvents; ++k) {
    if (M->chunk_ev[k]) (void)hipEventDestroy(M->chunk_ev[k]);
    M->chunk_ev[k] = nullptr;
  }
  if (M->h_mirror) (void)hipHostFree(M->h_mirror);
  M->h_mirror = nullptr;
  M->d_mirror = nullptr;
}

// The state of one solve: flags and reduction counter, reduced and
// first-level sums, parameters, the two records, the per-block partial sums
// of both parities, the host mirror and the pacing events. Needs cg_grid.
int alloc_solver_state(fi_mesh* M) {
  int rc = 0;
  if ((rc = device_alloc(M, (void**)&M->d_flag, 4 * sizeof(int32_t)))) return rc;
  if ((rc = device_alloc(M, (void**)&M->d_red4, 4 * sizeof(double)))) return rc;
  if ((rc = device_alloc(M, (void**)&M->d_lvl1, 4 * kRedMaxBlocks * sizeof(double)))) return rc;
  if ((rc = device_alloc(M, (void**)&M->d_prm, sizeof(Params)))) return rc;
  if ((rc = device_alloc(M, &M->d_rec, 2 * sizeof(Rec)))) return rc;
  if ((rc = device_alloc(M, (void**)&M->d_part, (size_t)2 * 4 * M->cg_grid * sizeof(double))))
    return rc;
  // the host mirror: fine-grained pinned memory the kernels write through to
  FI_HIP_TRY(hipHostMalloc(&M->h_mirror, sizeof(Mirror),
                           hipHostMallocMapped | hipHostMallocCoherent));
  std::memset(M->h_mirror, 0, sizeof(Mirror));
  FI_HIP_TRY(hipHostGetDevicePointer(&M->d_mirror, M->h_mirror, 0));
  for (int k = 0; k < kChunkEvents; ++k)
    // pacing only: the host reads no device memory on the strength of these
    // events (the outcome arrives through the mirror), so no system fence
    FI_HIP_TRY(hipEventCreateWithFlags(&M->chunk_ev[k],
                                       hipEventDisableTiming | hipEventDisableSystemFence));
  // the reduction counter starts at zero (the flag words are cleared too)
  hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(1), 0, M->ctx->stream, M->d_flag);
  FI_HIP_TRY(hipGetLastError());
  return FI_OK;
}

int solver_channel_setup(fi_mesh* S, const fi_mesh* M) {
  S->cg_bs = M->cg_bs;
  S->cg_grid = M->cg_grid;
  S->large_mode = M->large_mode;
  S->n_pad = M->n_pad;
  S->ell_w = M->ell_w;
  S->d_ell = M->d_ell;
  const int rc = alloc_solver_state(S);
  return rc ? rc : ss_channel_setup(S, M);
}

// Called after every assembly: picks the launch shape and packs the ELL copy.
int solver_setup(fi_mesh* M) {
  hipStream_t st = M->ctx->stream;
  const int64_t n = M->n;
  const bool first = M->d_flag == nullptr;
  if (first) {
    // Block size of the step kernel: fewer, larger blocks cut the partial
    // sums every block re-reads (G^2 traffic); FI_CG_BLOCK overrides.
    int bs = 512;
    if (const char* env = std::getenv("FI_CG_BLOCK")) bs = std::atoi(env);
    if (bs != 256 && bs != 512) bs = 512;  // 1024 would spill the ELL kernel
    M->cg_bs = bs;
  }
  // grid rounded up to a multiple of 8 (the XCD-aware block mapping)
  const int64_t blocks = ((n + M->cg_bs - 1) / M->cg_bs + 7) / 8 * 8;
  if (first) {
    // FI_CG_LARGE=1 forces the separate-reduction launch shape (tests use it
    // to check that path on systems small enough for the oracle).
    const char* force_large = std::getenv("FI_CG_LARGE");
    M->large_mode = blocks > kMaxGrid || (force_large && std::atoi(force_large) == 1);
    M->cg_grid = (int)std::max<int64_t>(1, blocks);
    M->n_pad = (n + 63) / 64 * 64;
    if (M->large_mode && (M->cg_grid + kRedChunk - 1) / kRedChunk > kRedMaxBlocks)
      return fail(FI_E_INVALID, "system too large for the partial-sum reduction");
    int rc = alloc_solver_state(M);
    if (rc) return rc;
    // widest row decides the ELL width
    hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(1), 0, st, M->d_flag);
    if (n > 0)
      hipLaunchKernelGGL(k_max_rowlen, dim3(grid_for(n)), dim3(kBlock), 0, st, (int)n,
                         M->d_ff_rowptr, M->d_flag);
    FI_HIP_TRY(hipGetLastError());
    FI_HIP_TRY(hipMemcpyAsync(M->h_ctl, M->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FI_HIP_TRY(hipStreamSynchronize(st));
    const int32_t w = M->h_ctl[0];
    M->ell_w = ell_width_for(w);
    if (M->ell_w > 0) {
      if ((rc = device_alloc(M, (void**)&M->d_ell, (size_t)M->ell_w * M->n_pad * sizeof(int32_t))))
        return rc;
    }
  }
  if (M->ell_w > 0) {
    hipLaunchKernelGGL(k_zero_flag, dim3(1), dim3(1), 0, st, M->d_flag);
    hipLaunchKernelGGL(k_pack_ell, dim3(grid_for(M->n_pad)), dim3(kBlock), 0, st, (int)n,
                       (int)M->n_pad, M->ell_w, M->d_ff_rowptr, M->d_ff_col, M->d_ff_val64,
                       M->d_ell, M->d_flag);
    FI_HIP_TRY(hipGetLastError());
    if (first) {
      FI_HIP_TRY(hipMemcpyAsync(M->h_ctl, M->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      FI_HIP_TRY(hipStreamSynchronize(st));
      if (M->h_ctl[0] != 0) M->ell_w = 0;  // values other than -1/2, -1: use CSR
    }
  }
  // the S-iteration launch: its plan (first assembly) or its values
  return ss_setup(M);
}

// Solves K_FF x = b64 (both in the mesh workspace) from x0 (device, n; NULL
// for 0); the result is in d_x64.
int solve_free(fi_mesh* M, const fi_solve_opts* opts, fi_solve_stats* stats, const double* x0) {
  stats->iterations = 0;
  stats->refinements = 0;
  stats->status = FI_OK;
  stats->rel_residual = 0.0;
  stats->residual = 0.0;
  stats->rhs_norm = 0.0;
  stats->launches = 0;
  if (M->n == 0) return FI_OK;
  if (opts->precision == FI_PREC_FP64) return solve_dev<double>(M, opts, stats, x0);
  if (M->ss) return ss_solve(M, opts, stats, x0);
  return solve_dev<float>(M, opts, stats, x0);
}

// Times `reps` CG iterations (step launches forced into the iteration
// phase) between two HIP events on the context stream.
int time_cg_kernel(fi_mesh* M, int precision, int reps, double* ms) {
  if (M->n == 0 || reps < 1) return fail(FI_E_INVALID, "nothing to time");
  if (precision != FI_PREC_FP64 && M->ss) return ss_time_kernel(M, reps, ms);
  hipStream_t st = M->ctx->stream;
  const bool d = precision == FI_PREC_FP64;
  fi_solve_opts o;
  fi_solve_opts_default(&o);
  // a start launch plus one init step give a valid state to iterate from
  const int epoch = next_epoch(M);
  int rc = d ? launch_start<double>(M, &o, epoch) : launch_start<float>(M, &o, epoch);
  if (rc) return rc;
  rc = d ? launch_step<double>(M, 0, 0) : launch_step<float>(M, 0, 0);
  if (rc) return rc;
  hipEvent_t e0, e1;
  FI_HIP_TRY(hipEventCreate(&e0));
  FI_HIP_TRY(hipEventCreate(&e1));
  for (int k = 0; k < 4; ++k) {
    rc = d ? launch_step<double>(M, (k + 1) & 1, 1) : launch_step<float>(M, (k + 1) & 1, 1);
    if (rc) return rc;
  }
  FI_HIP_TRY(hipEventRecord(e0, st));
  for (int k = 0; k < reps; ++k) {
    rc = d ? launch_step<double>(M, (k + 1) & 1, 1) : launch_step<float>(M, (k + 1) & 1, 1);
    if (rc) return rc;
  }
  FI_HIP_TRY(hipEventRecord(e1, st));
  FI_HIP_TRY(hipEventSynchronize(e1));
  float t = 0.f;
  FI_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = (double)t / reps;
  return FI_OK;
}

// Algorithmic bytes of one step launch. One iteration per launch: the matrix
// (one int32 per stored off-diagonal entry in the encoded layout, or column +
// value per CSR entry plus row pointers), and per row the reads of r, s, q,
// D^-1, x, p and the writes of x, p, r, s, q. Three iterations per launch (the
// S-iteration plan): per row and solve the basis record read and written
// (32 bytes each), the correction read and written, the diagonal (4 bytes
// each), and the matrix once as 16-bit entries.
int64_t cg_kernel_bytes(const fi_mesh* M, int precision) {
  return cg_multi_kernel_bytes(M, 1, precision);
}

// With nrhs solves per launch the matrix counts once.
int64_t cg_multi_kernel_bytes(const fi_mesh* M, int nrhs, int precision) {
  const int64_t w = precision == FI_PREC_FP64 ? 8 : 4;
  const int64_t mat = M->ell_w > 0 ? M->nnz_off * 4  // encoded entries; padding not counted
                                   : M->nnz_off * (4 + w) + (M->n + 1) * 4;
  if (precision != FI_PREC_FP64 && M->ss)
    return M->nnz_off * 2 + (int64_t)nrhs * M->n * (32 + 32 + 4 + 4 + 4);
  return mat + (int64_t)nrhs * M->n * w * 11;
}

}  // namespace fi
