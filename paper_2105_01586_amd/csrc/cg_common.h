// Solver state shared by the CG launches of the library (the one-iteration
// step in solver.hip and the S-iteration step in sstep.hip): phases, the
// per-launch record, the host mirror, solve parameters and the XCD-aware
// block order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace fi {

enum Phase : int32_t { kInit = 1, kIter = 2, kDoneOk = 3, kDoneNoConv = 4, kDoneBad = 5 };

// Solver state, one record per launch parity.
struct Rec {
  int32_t phase;
  int32_t iter;       // iteration within the current inner solve
  int32_t total;      // iterations over all inner solves
  int32_t ninner;     // inner solves started
  int32_t stagnant;   // consecutive refinements that did not halve ||r||
  int32_t xp;         // x64 buffer holding the iterate
  int32_t epoch;      // solve this record belongs to (set by the start launch)
  int32_t seq;        // launches since the start
  double gamma_prev, alpha_prev, rho_ref;
  double tol2;        // inner tolerance, squared
  double rnorm;       // FP64 residual norm at the start of this inner solve
  double bnorm;
  double pad2, pad3;
};
static_assert(sizeof(Rec) == 96, "record layout");

// What the host sees of a solve: the launch that ends it writes the outcome
// into pinned host memory with system-scope stores (they go through to host
// memory; nobody waits for them). Other launches do not write here: a store
// to host memory costs a working launch several microseconds. `word` holds,
// in one 64-bit store,
//   bits  0-3   phase            bits 4-30  epoch (the solve)
//   bits 32-55  iterations       bits 56-62 inner solves     bit 63 x64 buffer,
// so the host reads phase, epoch and counts consistently; the launch count
// and the residual norms are stored first, to the same cache line.
struct Mirror {
  uint64_t word;
  int64_t launches;  // step launches the solve took (the record's seq)
  double rnorm, bnorm;
};
constexpr int kEpochMask = (1 << 27) - 1;

// Constant parameters of a solve (written by the start launch).
struct Params {
  double rtol, inner_rtol, max_inner, max_refine, mixed, epoch, atol, pad;
};

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Blocks are dispatched round-robin over the 8 XCDs (hardware block b runs on
// XCD b % 8; the grid is a multiple of 8). Logical block (b % 8) * (G / 8) +
// b / 8 gives each XCD one contiguous slab of rows, so the neighbour values a
// block gathers mostly sit in its own XCD's L2.
__device__ __forceinline__ int logical_block() {
  const int b = blockIdx.x, per = gridDim.x >> 3;
  return (b & 7) * per + (b >> 3);
}

// Builds a record from explicit fields (no copy of an input record, whose
// unused bytes the compiler would otherwise carry through the kernel), and
// reports it to the host mirror.
__device__ __forceinline__ void put_rec(Rec* out, Mirror* mirror, int epoch, int seq, int phase,
                                        int iter, int total, int ninner, int stagnant, int xp,
                                        double gamma_prev, double alpha_prev, double rho_ref,
                                        double tol2, double rnorm, double bnorm) {
  Rec r;
  r.phase = phase;
  r.iter = iter;
  r.total = total;
  r.ninner = ninner;
  r.stagnant = stagnant;
  r.xp = xp;
  r.epoch = epoch;
  r.seq = seq;
  r.gamma_prev = gamma_prev;
  r.alpha_prev = alpha_prev;
  r.rho_ref = rho_ref;
  r.tol2 = tol2;
  r.rnorm = rnorm;
  r.bnorm = bnorm;
  r.pad2 = 0.0;
  r.pad3 = 0.0;
  *out = r;
  if (mirror && phase >= kDoneOk) {
    __hip_atomic_store(&mirror->launches, (int64_t)seq, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&mirror->rnorm, rnorm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&mirror->bnorm, bnorm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    const uint64_t w = (uint64_t)(uint32_t)((epoch << 4) | phase) |
                       ((uint64_t)((uint32_t)total & 0xFFFFFFu) << 32) |
                       ((uint64_t)((uint32_t)ninner & 0x7Fu) << 56) | ((uint64_t)(xp & 1) << 63);
    // release: the count and norms above are visible to a host that reads this word
    // with acquire (read_mirror) and sees this solve's epoch
    __hip_atomic_store(&mirror->word, w, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

// Host side (solver.hip): the id of a new solve on M, and the mirror read:
// 1 with stats (and the launches the solve took) filled when solve `epoch`
// has ended, 0 while it runs.
int next_epoch(fi_mesh* M);
int read_mirror(fi_mesh* M, int epoch, fi_solve_stats* stats, int* rc, int64_t* launches);

}  // namespace fi
