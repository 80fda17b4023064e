// Jacobi-preconditioned CG with S = 3 iterations per launch (the s-step, or
// communication-avoiding, form of the same method), for FP32 inner solves
// on the quadtree mesh, with FP64 iterative refinement.
//
// Section 2.2 solves the SPD FEM system with conjugate gradients. One CG
// iteration needs a global reduction, so the one-iteration step kernel
// (solver.hip) pays one kernel boundary per iteration; on systems that fit
// in the caches that boundary, not memory traffic, sets the time. Here one
// launch advances S iterations:
//   - each block owns BS consecutive rows of a Hilbert-order numbering of the
//     free rows and reads the basis of the previous launch on its region (its rows
//     and the rows within S hops, ss_plan.h);
//   - every block reduces the Gram matrix G = W^T D W of the previous basis
//     W = [P_0..P_S, Z_0..Z_{S-1}] (28 values; block sums exact or FP64,
//     stored in FP32, totals in FP64), then runs the S CG
//     iterations on coefficient vectors of length 2S+1 (redundantly, the same
//     in every block): with M = D^-1 K and T the change of basis of M,
//        alpha = (z, r) / (p, K p) = zc'G zc / pc'G T pc,
//        xc += alpha pc,  zc -= alpha T pc,  beta = zc'G zc (new / old),
//        pc = zc + beta pc;
//   - it forms p = W pc and z = W zc on its region, adds W xc to the
//     correction of its rows, and builds the next basis in LDS: the
//     Chebyshev polynomials of M on [0, 2] (its spectrum), rho_0 = v,
//     rho_1 = (M - I) v = D^-1 K_off v, rho_k+1 = 2 (M - I) rho_k - rho_k-1,
//     for p (S + 1 of them) and z (S), on the shrinking rings of its region;
//   - it writes its rows' new basis and its partial Gram sums.
// In exact arithmetic the iterates are those of Jacobi PCG. The inner solve
// stops when (r, z) falls below its tolerance squared times the starting
// (r, z); the launch that finds this adds the correction in FP64 and forms
// the FP64 residual b - K x on its rows (from the rows within one hop), and
// the next launch starts the next inner solve or ends the solve, exactly as
// in the one-iteration kernel.
//
// Every per-launch quantity (basis, partial sums, record, FP64 iterate) is
// double buffered by launch parity, so blocks of one launch never read each
// other's writes. No atomics: every sum has a fixed order, results are
// reproducible bit for bit.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "cg_common.h"
#include "internal.h"
#include "pacer.h"
#include "reduce.h"
#include "ss_plan.h"

namespace fi {

namespace {

constexpr int S = kSsIters;
static_assert(S == 3, "the launch below is written for three iterations");
constexpr int NB = 2 * S + 1;           // basis vectors: P_0..P_S, Z_0..Z_{S-1}
constexpr int NG = NB * (NB + 1) / 2;   // Gram entries (upper triangle)
constexpr int NGP = 32;                 // Gram slots per block (NG used)
constexpr int BS = 512;                 // threads and own rows per block
// Blocks up to which a single solve's blocks re-reduce the partials
// themselves (one block per compute unit at most: those launches run in
// one round even at the occupancy the in-block iterations allow); larger
// grids, and multi-solve or batched launches past it, sum them in a
// reduction launch. Up to 256 blocks both ways give the same bits.
constexpr int kSmallGrid = 256;
constexpr int kMaxRegion = 2048;        // region rows per block (LDS: 5 floats per row)
constexpr int kZ0 = S + 1;              // index of Z_0 in the basis
// A value's partial sums (one per block) are a row of the partials buffer
// whose length, the grid rounded up to this, is a whole number of chunks of
// 256 zero-padded entries: every reduction loads whole chunks, unmasked.
constexpr int kPartPad = 256;

__host__ __device__ constexpr int part_stride(int grid) {
  return (grid + kPartPad - 1) / kPartPad * kPartPad;
}

// Index of G[a][b] (a <= b) in the upper triangle, row by row.
__host__ __device__ constexpr int gi(int a, int b) {
  return a <= b ? a * NB - a * (a - 1) / 2 + (b - a) : b * NB - b * (b - 1) / 2 + (a - b);
}

// One local matrix row: kPlanSlots 16-bit entries in three dwords (one
// 12-byte load).
struct LmRow {
  uint32_t w[3];
};
static_assert(kPlanSlots == 6 && sizeof(LmRow) == 2 * kPlanSlots, "local matrix row layout");

struct SsArgs {
  int n;
  int grid;
  int gstride;         // length of a value's row of partial sums (part_stride)
  const int32_t* perm;
  const BlockPlan* blocks;
  const int32_t* region;  // region rows of every block (own rows first)
  const LmRow* lmat;
  const float4* Win;   // 2 float4 per row: P_0..P_3 | Z_0..Z_2, D^-1
  float4* Wout;
  float* x;
  const float* d;
  double* b;
  double* r64;
  double* x64a;
  double* x64b;
  double* xout;        // natural-order result (written when the solve ends)
  const float* part_in;   // partial sums of the previous launch (FP32)
  float* part_out;
  const double* tot_in;   // their totals, summed by the reduction launch
  const Rec* rec_in;
  Rec* rec_out;
  const Params* prm;
  Mirror* mirror;
  const double* ctl;   // large systems: the coefficients of this launch's iterations
  int force;           // timing only: always iterate
};

// -1 or -1/2 from bit 15 (the bit pattern of -1/2 with its exponent raised
// by one); a padding entry points at the zero slot, so its weight is moot.
__device__ __forceinline__ float lm_weight(uint32_t e) {
  return __uint_as_float(0xBF000000u | ((e & kPlanMinusOne) << 8));
}

__device__ __forceinline__ uint32_t lm_entry(const LmRow& m, int k) {
  const uint32_t w = k < 2 ? m.w[0] : k < 4 ? m.w[1] : m.w[2];
  return (k & 1) ? (w >> 16) : (w & 0xFFFFu);
}

// Region row l of a block -> row (new numbering).
__device__ __forceinline__ int region_row(const SsArgs& A, const BlockPlan& B, int base, int l) {
  (void)base;
  return A.region[B.reg_off + l];
}

// sum_k w_k vs[idx_k] over one local matrix row, for p and z at once
// (FP32, slot order; vs holds (p, z) per LDS slot: 0 the zero slot, l + 1
// region row l).
__device__ __forceinline__ float2 lm_apply(const LmRow& m, const float2* vs) {
  float2 acc = make_float2(0.0f, 0.0f);
#pragma unroll
  for (int k = 0; k < kPlanSlots; ++k) {
    const uint32_t e = lm_entry(m, k);
    const float w = lm_weight(e);
    const float2 x = vs[e & (kPlanLocalMax - 1)];
    acc.x = __builtin_fmaf(w, x.x, acc.x);
    acc.y = __builtin_fmaf(w, x.y, acc.y);
  }
  return acc;
}

// Coefficients of M v for v = sum c_a rho_a (P block 0..S, Z block S+1..2S;
// the top coefficient of each block is zero wherever this is used):
// M rho_0 = rho_1 + rho_0, M rho_k = rho_k+1 / 2 + rho_k + rho_k-1 / 2.
__device__ __forceinline__ void tcoef(const double (&c)[NB], double (&o)[NB]) {
#pragma unroll
  for (int a = 0; a < NB; ++a) o[a] = 0.0;
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    const int base = blk == 0 ? 0 : kZ0, m = blk == 0 ? S + 1 : S;
#pragma unroll
    for (int k = 0; k < m - 1; ++k) {
      const double ck = c[base + k];
      if (k == 0) {
        o[base + 1] += ck;
        o[base] += ck;
      } else {
        o[base + k + 1] += 0.5 * ck;
        o[base + k] += ck;
        o[base + k - 1] += 0.5 * ck;
      }
    }
  }
}

// G v for G symmetric, stored as its upper triangle (seven independent
// FMA chains).
__device__ __forceinline__ void gmul(const double (&G)[NG], const double (&v)[NB],
                                     double (&o)[NB]) {
#pragma unroll
  for (int a = 0; a < NB; ++a) {
    double t = G[gi(a, 0)] * v[0];
#pragma unroll
    for (int b = 1; b < NB; ++b) t = __builtin_fma(G[gi(a, b)], v[b], t);
    o[a] = t;
  }
}

__device__ __forceinline__ double dotv(const double (&x)[NB], const double (&y)[NB]) {
  double t = x[0] * y[0];
#pragma unroll
  for (int a = 1; a < NB; ++a) t = __builtin_fma(x[a], y[a], t);
  return t;
}

// a / b from the hardware reciprocal and two Newton steps (within an ulp
// or so; the iteration's scalars are a chain of these divisions).
__device__ __forceinline__ double qdiv(double a, double b) {
  double y = __builtin_amdgcn_rcp(b);
  y = __builtin_fma(y, __builtin_fma(-b, y, 1.0), y);
  y = __builtin_fma(y, __builtin_fma(-b, y, 1.0), y);
  return a * y;
}

// sum_a w_a c_a in FP64 over the 7 basis values of one row.
__device__ __forceinline__ double combine(const float4& a0, const float4& a1,
                                          const double (&c)[NB]) {
  double s = (double)a0.x * c[0];
  s = __builtin_fma((double)a0.y, c[1], s);
  s = __builtin_fma((double)a0.z, c[2], s);
  s = __builtin_fma((double)a0.w, c[3], s);
  s = __builtin_fma((double)a1.x, c[4], s);
  s = __builtin_fma((double)a1.y, c[5], s);
  s = __builtin_fma((double)a1.z, c[6], s);
  return s;
}

// Writes the block's partial sums: slot v at part_out[v * gstride + lb],
// from thread 16 v (which holds it), rounded to FP32. Each block's sums are
// exact or FP64 up to here; what the rounding leaves (a relative 6e-8 per
// block) is far below what the FP32 basis vectors carry, and the totals are
// summed in FP64. Halving the bytes every block of the next launch reads
// took 5% off a 512^2 launch, with the same iteration counts.
__device__ __forceinline__ void store_slot(const SsArgs& A, int lb, double v) {
  if ((threadIdx.x & 15) == 0 && (threadIdx.x >> 4) < NGP)
    A.part_out[(size_t)(threadIdx.x >> 4) * A.gstride + lb] = (float)v;
}

typedef double d4v __attribute__((ext_vector_type(4)));

// Sum over the 16 lanes of each DPP row, every lane of the row receiving it
// (neighbours, pairs, half-row and row mirrors; each step adds two equal
// partial sums, in either order).
__device__ __forceinline__ double row_sum(double v) {
  v += dpp_move<0xB1>(v);
  v += dpp_move<0x4E>(v);
  v += dpp_move<0x141>(v);
  v += dpp_move<0x140>(v);
  return v;
}

// The block's partial Gram sums G_ab = sum over its rows of d w_a w_b, on
// the FP64 matrix cores: each wave stages its 64 rows' values (and d) in LDS
// and adds W' (D W) over them with 8 products of 16 x 4 by 4 x 16. Each
// product takes two groups of four rows: lane l supplies element (row
// 8 m + 4 h + l / 16, value c) with h = (l % 16) / 8, c = l % 8, so the
// first group's sums land in the 8 x 8 block at (0, 0) of the product and
// the second group's in the block at (8, 8) (the other blocks mix the two
// groups and are not used); values 7 and 15 are 0. The products of FP32
// values and the small half-integer d are exact in FP64. The waves' sums
// are then added in wave order. Returns value v's total in thread 16 v
// (v < NG), 0 elsewhere. wst: BS x 8 floats; wg: 8 x NGP.
__device__ __forceinline__ double block_gram(const float (&w)[NB], float dd, float* wst,
                                             double* wg) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  __syncthreads();  // wst shares LDS with the basis levels read last
  float4* st = (float4*)(wst + 8 * t);
  st[0] = make_float4(w[0], w[1], w[2], w[3]);
  st[1] = make_float4(w[4], w[5], w[6], dd);
  __builtin_amdgcn_wave_barrier();  // each wave reads only its own rows
  const int col = lane & 15, kq = lane >> 4, h = col >> 3, c = col & 7;
  // all operands first (unconditional reads, masked after), then the products
  float xv[8], dv[8];
  const int cc = c < NB ? c : 0;
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const float* row = wst + 8 * (64 * wave + 8 * m + 4 * h + kq);
    xv[m] = row[cc];
    dv[m] = row[7];
  }
  d4v acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const double a = c < NB ? (double)xv[m] : 0.0;
    const double b = (double)dv[m] * a;
    if (m & 1) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc1, 0, 0, 0);
    else acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc0, 0, 0, 0);
  }
  // lane l holds D[4 v + l / 16][l % 16] in element v: G[i][j] = D[i][j] +
  // D[8 + i][8 + j], the second term from lane l + 8 (row rotation by 8)
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    const double g = (acc0[v] + acc1[v]) + dpp_move<0x128>(acc0[v + 2] + acc1[v + 2]);
    const int i = 4 * v + kq, j = col;
    if (i <= j && j < NB) wg[wave * NGP + gi(i, j)] = g;
  }
  __syncthreads();
  const int v = t >> 4;
  double s = 0.0;
  if ((t & 15) == 0 && v < NG) {
    s = wg[v];
#pragma unroll
    for (int q = 1; q < BS / 64; ++q) s += wg[q * NGP + v];
  }
  return s;
}

// The launch's Gram matrix of the previous basis: the totals of the
// previous launch's partial sums, summed by every block in a fixed order
// (value v by the 16 lanes of one DPP row, partials j, j + 16, ... each, in
// chunks of 16 loads issued together), or read as totals summed by a
// separate launch (large systems). gram_issue starts the first chunk's
// loads, so that other loads can follow before the sum waits for them.
struct GramLoads {
  float a[16];
};

template <bool LARGE>
__device__ __forceinline__ void gram_issue(const SsArgs& A, GramLoads& L) {
  if constexpr (!LARGE) {
    const int v = threadIdx.x >> 4, j = threadIdx.x & 15;
    const float* pv = A.part_in + (size_t)(v < NG ? v : 0) * A.gstride + j;
#pragma unroll
    for (int k = 0; k < 16; ++k) L.a[k] = pv[16 * k];  // padding entries are 0
  }
}

template <bool LARGE>
__device__ __forceinline__ void gram_finish(const SsArgs& A, const GramLoads& L, double* red) {
  if constexpr (!LARGE) {
    const int v = threadIdx.x >> 4, j = threadIdx.x & 15;
    const float* pv = A.part_in + (size_t)(v < NG ? v : 0) * A.gstride + j;
    double h[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) h[k] = (double)L.a[k];
#pragma unroll
    for (int w = 8; w >= 1; w >>= 1)
#pragma unroll
      for (int k = 0; k < w; ++k) h[k] += h[k + w];  // pairwise, fixed order
    double acc = h[0];
    for (int c0 = 256; c0 < A.grid; c0 += 256) {
      float a[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) a[k] = pv[c0 + 16 * k];
#pragma unroll
      for (int k = 0; k < 16; ++k) acc += (double)a[k];
    }
    if (v >= NG) acc = 0.0;
    acc += dpp_move<0xB1>(acc);
    acc += dpp_move<0x4E>(acc);
    acc += dpp_move<0x141>(acc);
    acc += dpp_move<0x140>(acc);
    if (j == 0 && v < NG) red[v] = acc;
    __syncthreads();
  }
}

// A thread's first two region rows (l = t and l = t + BS), loaded before the
// Gram reduction: row, basis record, local matrix row. Most regions have at
// most 2 BS rows; later rows are loaded where they are used.
struct Pre {
  int i[2];        // rows (new numbering), 0 past the region
  float4 a[2], b[2];
  LmRow m[2];      // local matrix rows (zeros past the inner rows)
};

// Rows and local matrix rows (loads that need only the block table). The
// own rows are the block's consecutive rows (the region list starts with
// them): large systems, which are bound by HBM traffic, read only the halo
// rows from the list (4 bytes per row and launch less); at small sizes, bound
// by latency, the unconditional load of every row measured faster. Loads are
// at clamped positions that stay inside the lists (an empty block points at
// their start); entries past the region or past the inner rows are never
// used.
template <bool LARGE>
__device__ __forceinline__ void prefetch_rows(const SsArgs& A, const BlockPlan& B, int base,
                                              Pre& R) {
  const int t = threadIdx.x;
  if constexpr (LARGE)
    R.i[0] = t < B.nown ? base + t : A.region[B.reg_off + max(0, min(t, B.nreg - 1))];
  else
    R.i[0] = A.region[B.reg_off + max(0, min(t, B.nreg - 1))];
  R.i[1] = A.region[B.reg_off + max(0, min(t + BS, B.nreg - 1))];
#pragma unroll
  for (int k = 0; k < 2; ++k) R.m[k] = A.lmat[B.lmat_off + max(0, min(t + k * BS, B.ninner - 1))];
}

// The rows' basis records (loads that need the rows; every row is valid).
__device__ __forceinline__ void prefetch_recs(const SsArgs& A, Pre& R) {
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    R.a[k] = A.Win[2 * (size_t)R.i[k]];
    R.b[k] = A.Win[2 * (size_t)R.i[k] + 1];
  }
}

// Region row l = t + k BS: its row, record and local matrix row.
__device__ __forceinline__ int row_at(const SsArgs& A, const BlockPlan& B, int base, const Pre& R,
                                      int l, int k) {
  return k < 2 ? R.i[k] : region_row(A, B, base, l);
}
__device__ __forceinline__ void rec_at(const SsArgs& A, const Pre& R, int i, int k, float4& a,
                                       float4& b) {
  if (k < 2) {
    a = R.a[k];
    b = R.b[k];
  } else {
    a = A.Win[2 * (size_t)i];
    b = A.Win[2 * (size_t)i + 1];
  }
}
__device__ __forceinline__ LmRow lm_at(const SsArgs& A, const BlockPlan& B, const Pre& R, int l,
                                       int k) {
  return k < 2 ? R.m[k] : A.lmat[B.lmat_off + l];
}

// The next basis from level 0 (pz0 = (p, z) on the whole region, ld =
// D^-1), in LDS: round k computes level k on the rows within S - k hops.
// pz0 and pz1 point at region row 0 of their slot arrays, whose slot 0 (at
// index -1) holds zeros. Returns the own row's seven values (thread t: row
// t, zeros past nown).
__device__ __forceinline__ void build_basis(const SsArgs& A, const BlockPlan& B, const Pre& R,
                                            float2* pz0, float2* pz1, const float* ld,
                                            float (&w)[NB]) {
  const int t = threadIdx.x;
  const bool own = t < B.nown;
  const float2* s0 = pz0 - 1;
  const float2* s1 = pz1 - 1;
  if (t == 0) {
    pz0[-1] = make_float2(0.f, 0.f);
    pz1[-1] = make_float2(0.f, 0.f);
  }
  float2 l0 = make_float2(0.f, 0.f), l1 = l0, l2 = l0;
  float p3 = 0.0f;
  __syncthreads();
  // level 1: rows within S - 1 hops
  for (int l = t, k = 0; l < B.ninner; l += BS, ++k) {
    const LmRow m = lm_at(A, B, R, l, k);
    const float dv = ld[l];
    const float2 acc = lm_apply(m, s0);
    pz1[l] = make_float2(dv * acc.x, dv * acc.y);
  }
  __syncthreads();
  if (own) {
    l0 = pz0[t];
    l1 = pz1[t];
  }
  // level 2 over level 0 (each row reads its own level 0 before writing it;
  // the neighbours' values come from level 1)
  for (int l = t, k = 0; l < B.n1; l += BS, ++k) {
    const LmRow m = lm_at(A, B, R, l, k);
    const float dv2 = 2.0f * ld[l];
    const float2 acc = lm_apply(m, s1);
    const float2 old = pz0[l];
    pz0[l] = make_float2(__builtin_fmaf(dv2, acc.x, -old.x), __builtin_fmaf(dv2, acc.y, -old.y));
  }
  __syncthreads();
  // level 3 of p on the own rows
  if (own) {
    l2 = pz0[t];
    p3 = __builtin_fmaf(2.0f * ld[t], lm_apply(R.m[0], s0).x, -l1.x);
  }
  w[0] = l0.x;
  w[1] = l1.x;
  w[2] = l2.x;
  w[3] = p3;
  w[kZ0] = l0.y;
  w[kZ0 + 1] = l1.y;
  w[kZ0 + 2] = l2.y;
}

// Stores the own row's new basis and the block's partial Gram sums.
__device__ __forceinline__ void finish_basis(const SsArgs& A, const BlockPlan& B, int lb, int base,
                                             const float (&w)[NB], float dinv, float dd,
                                             float* wst, double* wred) {
  const int t = threadIdx.x;
  if (t < B.nown) {
    A.Wout[2 * (size_t)(base + t)] = make_float4(w[0], w[1], w[2], w[3]);
    A.Wout[2 * (size_t)(base + t) + 1] = make_float4(w[4], w[5], w[6], dinv);
  }
  store_slot(A, lb, block_gram(w, t < B.nown ? dd : 0.0f, wst, wred));
}

// The S CG iterations of one launch on the coefficient vectors (one wave,
// every lane alike; lane 0 writes out = pc, zc, xc, (r, z), iteration count,
// stop flag: 3 NB + 3 doubles). G is the Gram matrix of the launch's basis,
// Rin the record the launch reads. G z is kept up to date (z -= alpha T p
// gives G z -= alpha G T p, which the step has formed anyway), so each step
// needs one product with G.
__device__ __forceinline__ void ss_recur(const double* Gsrc, const Rec& Rin, const Params& P,
                                         int force, double* out) {
  int iter = Rin.iter;
  double rz = iter == 0 ? Gsrc[gi(kZ0, kZ0)] : Rin.gamma_prev;
  const double rho_ref = iter == 0 ? rz : Rin.rho_ref;
  double pc[NB], zc[NB], xc[NB];
  bool stop = false;
  double Gw[NG];
#pragma unroll
  for (int q = 0; q < NG; ++q) Gw[q] = Gsrc[q];
  double gz[NB];
#pragma unroll
  for (int a = 0; a < NB; ++a) {
    pc[a] = a == 0 ? 1.0 : 0.0;
    zc[a] = a == kZ0 ? 1.0 : 0.0;
    xc[a] = 0.0;
    gz[a] = Gw[gi(a, kZ0)];
  }
#pragma unroll
  for (int j = 0; j < S; ++j) {
    if (!stop) {
      double tp[NB], gtp[NB];
      tcoef(pc, tp);
      gmul(Gw, tp, gtp);
      const double alpha = qdiv(rz, dotv(pc, gtp));
      if (!force && (!(alpha > 0.0) || !isfinite(alpha))) {
        stop = true;  // breakdown: refine with what has been reached
      } else {
#pragma unroll
        for (int a = 0; a < NB; ++a) {
          xc[a] = __builtin_fma(alpha, pc[a], xc[a]);
          zc[a] = __builtin_fma(-alpha, tp[a], zc[a]);
          gz[a] = __builtin_fma(-alpha, gtp[a], gz[a]);
        }
        ++iter;
        const double rzn = dotv(zc, gz);
        if (!force && (!(rzn > Rin.tol2 * rho_ref) || (double)iter >= P.max_inner)) {
          stop = true;
        } else {
          const double beta = qdiv(rzn, rz);
          rz = rzn;
#pragma unroll
          for (int a = 0; a < NB; ++a) pc[a] = __builtin_fma(beta, pc[a], zc[a]);
        }
      }
    }
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      out[a] = pc[a];
      out[NB + a] = zc[a];
      out[2 * NB + a] = xc[a];
    }
    out[3 * NB] = rz;
    out[3 * NB + 1] = (double)iter;
    out[3 * NB + 2] = stop ? 1.0 : 0.0;
  }
}

template <bool LARGE>
__device__ __forceinline__ void ss_body(const SsArgs& A, const int lb, float* dyn, double* red,
                                        double* wred, double* coef, float* wst) {
  const int t = threadIdx.x;
  const Rec Rin = *A.rec_in;
  const Params P = *A.prm;
  const BlockPlan B = A.blocks[lb];
  const int base = lb * BS;
  const bool own = t < B.nown;
  const int ro = own ? base + t : 0;
  // loads that depend neither on the phase nor on the Gram matrix: the first
  // region rows' records, the own row's correction and diagonal (unconditional
  // at row 0 past the own rows; those values are never used)
  Pre R;
  prefetch_rows<LARGE>(A, B, base, R);
  GramLoads L;
  gram_issue<LARGE>(A, L);
  prefetch_recs(A, R);
  const float xo = A.x[ro];
  const float dd = A.d[ro];
  gram_finish<LARGE>(A, L, red);
  // the reduced Gram matrix: in LDS, or summed by the previous reduction launch
  const double* Gsrc = LARGE ? A.tot_in : red;
  const int phase = A.force ? (int)kIter : Rin.phase;
  const bool writer = lb == 0 && t == 0;
  // LDS: two slot arrays of (p, z) (zero slot, then the region rows), D^-1
  const int RM = A.blocks[0].pad0;  // region rows the LDS is laid out for
  float2* pz0 = (float2*)dyn + 1;
  float2* pz1 = (float2*)dyn + RM + 2;
  float* ld = dyn + 4 * (RM + 1);
  const float dinv_own = R.b[0].w;

  if (phase >= kDoneOk) {  // a launch queued after the end: carry the record
    if (writer)
      put_rec(A.rec_out, nullptr, Rin.epoch, Rin.seq, Rin.phase, Rin.iter, Rin.total, Rin.ninner,
              Rin.stagnant, Rin.xp, Rin.gamma_prev, Rin.alpha_prev, Rin.rho_ref, Rin.tol2,
              Rin.rnorm, Rin.bnorm);
    return;
  }

  if (phase == kInit) {
    // G[0] = ||r64||^2 from the start or refinement launch; the start launch
    // also sends G[1] = ||b||^2
    double rnorm = sqrt(Gsrc[0]);
    const double bnorm = Rin.ninner == 0 ? sqrt(Gsrc[1]) : Rin.bnorm;
    const double tol = P.atol > 0.0 ? fmin(P.rtol * bnorm, P.atol) : P.rtol * bnorm;
    int stagnant = Rin.stagnant;
    int next = 0;
    bool zero = false;
    if (!isfinite(rnorm)) next = kDoneBad;
    else if (rnorm <= tol) next = kDoneOk;
    else if (bnorm == 0.0 && Rin.ninner == 0) {  // b = 0 with a non-zero start: x = 0
      zero = true;
      rnorm = 0.0;
      next = kDoneOk;
    }
    else if ((double)Rin.ninner >= P.max_refine) next = kDoneNoConv;
    else if (Rin.ninner > 0) {
      stagnant = rnorm > 0.5 * Rin.rnorm ? stagnant + 1 : 0;
      if (stagnant >= 3) next = kDoneNoConv;
    }
    if (next) {
      // the result, in the natural order of the free rows
      if (own) A.xout[A.perm[ro]] = zero ? 0.0 : (Rin.xp ? A.x64b : A.x64a)[ro];
      if (writer)
        put_rec(A.rec_out, A.mirror, Rin.epoch, Rin.seq + 1, next, Rin.iter, Rin.total,
                Rin.ninner, stagnant, 0, Rin.gamma_prev, Rin.alpha_prev, Rin.rho_ref, Rin.tol2,
                rnorm, bnorm);
      return;
    }
    const double want = 0.5 * tol / rnorm;
    const double itol = fmax(P.inner_rtol, want);
    const double scale = 1.0 / rnorm;
    for (int l = t, k = 0; l < B.nreg; l += BS, ++k) {
      const int i = row_at(A, B, base, R, l, k);
      float4 a, b;
      rec_at(A, R, i, k, a, b);
      const float r = (float)(A.r64[i] * scale);
      const float z = b.w * r;
      pz0[l] = make_float2(z, z);
      ld[l] = b.w;
    }
    if (own) A.x[ro] = 0.0f;
    float w[NB];
    build_basis(A, B, R, pz0, pz1, ld, w);
    finish_basis(A, B, lb, base, w, dinv_own, dd, wst, wred);
    if (writer)
      put_rec(A.rec_out, A.mirror, Rin.epoch, Rin.seq + 1, kIter, 0, Rin.total, Rin.ninner + 1,
              stagnant, Rin.xp, 0.0, 0.0, 0.0, itol * itol, rnorm, bnorm);
    return;
  }

  // ---- kIter: S iterations on the coefficients -----------------------------
  // One wave runs them (every other wave would repeat the same FP64 chain on
  // the same SIMDs) and hands the coefficients over through LDS; for large
  // systems the reduction launch has run them once for every block.
  const int iter0 = Rin.iter;
  const double rho_ref = iter0 == 0 ? Gsrc[gi(kZ0, kZ0)] : Rin.rho_ref;
  const double* cf = coef;
  if constexpr (LARGE) {
    cf = A.ctl;
  } else {
    if (t < 64) ss_recur(Gsrc, Rin, P, A.force, coef);
    __syncthreads();
  }
  double pc[NB], zc[NB], xc[NB];
#pragma unroll
  for (int a = 0; a < NB; ++a) {
    pc[a] = cf[a];
    zc[a] = cf[NB + a];
    xc[a] = cf[2 * NB + a];
  }
  const double rz = cf[3 * NB];
  const int iter = (int)cf[3 * NB + 1];
  const bool stop = cf[3 * NB + 2] != 0.0;

  if (stop) {
    // Inner solve over: x64 += rnorm * (x + W xc) on the rows within one hop,
    // then r64 = b - K x64 on the own rows (FP64), and ||r64||^2.
    const double* xo64 = Rin.xp ? A.x64b : A.x64a;
    double* xn64 = Rin.xp ? A.x64a : A.x64b;
    double* lx = (double*)dyn + 1;  // slot array, zero slot at -1
    if (t == 0) lx[-1] = 0.0;
    const double sc = Rin.rnorm;
    for (int l = t, k = 0; l < B.n1; l += BS, ++k) {
      const int i = row_at(A, B, base, R, l, k);
      float4 a, b;
      rec_at(A, R, i, k, a, b);
      const float xv = k == 0 ? (own ? xo : A.x[i]) : A.x[i];
      lx[l] = __builtin_fma(sc, (double)xv + combine(a, b, xc), xo64[i]);
    }
    __syncthreads();
    double v0 = 0.0;
    if (own) {
      const double xi = lx[t];
      double acc = (double)dd * xi;
#pragma unroll
      for (int k = 0; k < kPlanSlots; ++k) {
        const uint32_t e = lm_entry(R.m[0], k);
        acc = __builtin_fma((double)lm_weight(e), lx[(int)(e & (kPlanLocalMax - 1)) - 1], acc);
      }
      const double ri = A.b[ro] - acc;
      xn64[ro] = xi;
      A.r64[ro] = ri;
      v0 = ri * ri;
    }
    double v[1] = {v0};
    block_sum_once<1, BS / 64>(v, wred);
    store_slot(A, lb, threadIdx.x == 0 ? v[0] : 0.0);  // slot 0; other slots 0
    if (writer)
      put_rec(A.rec_out, A.mirror, Rin.epoch, Rin.seq + 1, kInit, iter, Rin.total + iter,
              Rin.ninner, Rin.stagnant, Rin.xp ^ 1, rz, 0.0, rho_ref, Rin.tol2, Rin.rnorm,
              Rin.bnorm);
    return;
  }

  // p = W pc, z = W zc on the region; x += W xc on the own rows
  for (int l = t, k = 0; l < B.nreg; l += BS, ++k) {
    float4 a, b;
    rec_at(A, R, k < 2 ? 0 : region_row(A, B, base, l), k, a, b);
    pz0[l] = make_float2((float)combine(a, b, pc), (float)combine(a, b, zc));
    ld[l] = b.w;
  }
  if (own) A.x[ro] = (float)((double)xo + combine(R.a[0], R.b[0], xc));
  float w[NB];
  build_basis(A, B, R, pz0, pz1, ld, w);
  finish_basis(A, B, lb, base, w, dinv_own, dd, wst, wred);
  if (writer)
    put_rec(A.rec_out, A.mirror, Rin.epoch, Rin.seq + 1, kIter, iter, Rin.total, Rin.ninner,
            Rin.stagnant, Rin.xp, rz, 0.0, rho_ref, Rin.tol2, Rin.rnorm, Rin.bnorm);
}

template <bool LARGE>
__global__ __launch_bounds__(BS) void k_ss_step(SsArgs A) {
  extern __shared__ float dyn[];
  __shared__ double red[NGP];
  __shared__ double wred[(BS / 64) * NGP];  // per-wave Gram sums
  __shared__ double coef[3 * NB + 3];       // the iteration's coefficients
  ss_body<LARGE>(A, logical_block(), dyn, red, wred, coef, dyn);
}

// Several right-hand sides with one matrix (the channels of a colour image):
// the k-th block of XCD x takes solve k % nrhs and row block
// x (G / 8) + k / nrhs, so the solves' blocks for the same rows run side by
// side on one XCD and share the rows' plan and matrix in its L2. Each block
// runs the single-solve body on its solve's arguments and the row block the
// single-solve launch would give it: every solve gets the bits of its own
// single solve.
struct SsMultiArgs {
  int nrhs;
  SsArgs a[kMaxRhs];
};

template <bool LARGE>
__device__ __forceinline__ void multi_body(const SsMultiArgs& M) {
  extern __shared__ float dyn[];
  __shared__ double red[NGP];
  __shared__ double wred[(BS / 64) * NGP];
  __shared__ double coef[3 * NB + 3];
  const int nr = M.nrhs;
  const int per = (int)(gridDim.x / nr) >> 3;
  const int k = blockIdx.x >> 3;
  ss_body<LARGE>(M.a[k % nr], (blockIdx.x & 7) * per + k / nr, dyn, red, wred, coef, dyn);
}

// The launch that re-reduces in every block fits its solves' blocks in one
// round; the other runs three blocks per compute unit (at most 80 VGPRs).
__global__ __launch_bounds__(BS) void k_ss_multi_small(SsMultiArgs M) { multi_body<false>(M); }
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(6))) void k_ss_multi_large(
    SsMultiArgs M) {
  multi_body<true>(M);
}

// Several meshes' solves in one launch (the server): the grid is the
// concatenation of every slot's own grid (each a multiple of 8); a block
// finds its slot from the start offsets and runs the single-mesh body with
// its slot-local block index, so a solve gives the same bits alone or in any
// batch. A slot whose solve has ended only carries its record forward.
constexpr int kSsArgSlots = 20;

struct SsBatchArgs {
  int n;
  int32_t start[kSsArgSlots + 1];
  SsArgs a[kSsArgSlots];
};
static_assert(sizeof(SsBatchArgs) <= 4096, "kernel arguments of a batched launch");

// Batched solves always take the reduction launch (ss_arm, ss_batch_launch).
__global__ __launch_bounds__(BS) void k_ss_batch(SsBatchArgs Bt) {
  extern __shared__ float dyn[];
  __shared__ double red[NGP];
  __shared__ double wred[(BS / 64) * NGP];
  __shared__ double coef[3 * NB + 3];
  const int lb = logical_block();
  int j = 0;  // slot of this block (uniform)
#pragma unroll
  for (int k = 1; k < kSsArgSlots; ++k) j += (k < Bt.n && Bt.start[k] <= lb) ? 1 : 0;
  const SsArgs& A = Bt.a[j];
  const int lblk = lb - Bt.start[j];
  if (A.rec_in->phase >= kDoneOk) {
    if (lblk == 0 && threadIdx.x == 0) *A.rec_out = *A.rec_in;
    return;
  }
  ss_body<true>(A, lblk, dyn, red, wred, coef, dyn);
}

// Start of a solve: b and x0 in the launch's numbering, x64 = x0 (0 when
// x0 is NULL), r64 = b - K_FF x0 in FP64, ||r64||^2 and ||b||^2, the first
// record. b_nat and x0 are in the natural order of the free rows.
__global__ __launch_bounds__(BS) void k_ss_start(SsArgs A, Params prm, Params* prm_out,
                                                 const double* __restrict__ b_nat,
                                                 const double* __restrict__ x0) {
  extern __shared__ float dyn[];
  __shared__ double wred[(BS / 64) * 2];
  const int t = threadIdx.x, lb = logical_block();
  const BlockPlan B = A.blocks[lb];
  const int base = lb * BS;
  const bool own = t < B.nown;
  const int ro = own ? base + t : 0;
  double* lx = (double*)dyn + 1;  // slot array, zero slot at -1
  if (x0) {
    if (t == 0) lx[-1] = 0.0;
    for (int l = t; l < B.n1; l += BS) lx[l] = x0[A.perm[region_row(A, B, base, l)]];
    __syncthreads();
  }
  double v[2] = {0.0, 0.0};
  if (own) {
    const double bi = b_nat[A.perm[ro]];
    double ri = bi, xi = 0.0;
    if (x0) {
      const LmRow m = A.lmat[B.lmat_off + t];
      xi = lx[t];
      double acc = (double)A.d[ro] * xi;
#pragma unroll
      for (int k = 0; k < kPlanSlots; ++k) {
        const uint32_t e = lm_entry(m, k);
        acc = __builtin_fma((double)lm_weight(e), lx[(int)(e & (kPlanLocalMax - 1)) - 1], acc);
      }
      ri = bi - acc;
    }
    A.b[ro] = bi;
    A.x64a[ro] = xi;
    A.r64[ro] = ri;
    v[0] = ri * ri;
    v[1] = bi * bi;
  }
  block_sum_once<2, BS / 64>(v, wred);
  store_slot(A, lb, threadIdx.x == 0 ? v[0] : threadIdx.x == 16 ? v[1] : 0.0);
  if (lb == 0 && t == 0) {
    prm_out->rtol = prm.rtol;
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

// Large systems: a separate launch sums the Gram partials of the step launch
// before it and runs the next launch's iterations on the coefficients once,
// for every block of that launch. First level: block b sums partials
// [256 b, 256 b + 256) of every value (value v by the 16 lanes of one DPP
// row, partials j, j + 16, ... each: a tree over each lane's sixteen, as in
// the step's own re-reduction, so a system of up to 256 blocks gets the
// step's own bits); a system of one such block is done there (totals, and
// the coefficients when the next launch iterates), larger ones in a second
// launch of one block per system that sums the first-level sums in block
// order. Several systems (channels, batched meshes) share the launches, each
// with its own blocks. Chunks of 256 give a 8192^2 system (47k step blocks)
// 185 first-level blocks, enough to spread the partials' loads over the chip.
constexpr int kGramChunk = 256;

struct SsRedSys {
  const float* part;  // NGP rows of partials (value-major, rows of part_stride(grid))
  double* level1;      // first-level sums, NGP per block
  double* out;         // NGP totals
  const Rec* rec;      // the record the next step launch reads
  const Params* prm;
  double* ctl;         // that launch's coefficients (3 NB + 3 doubles)
  int grid;
  int force;
};

struct SsRedArgs {
  int n;
  int32_t start[kSsArgSlots + 1];  // first block of each system
  SsRedSys s[kSsArgSlots];
};
static_assert(sizeof(SsRedArgs) <= 4096, "kernel arguments of a reduction launch");

__host__ __device__ constexpr int gram_blocks(int grid) {
  return (part_stride(grid) + kGramChunk - 1) / kGramChunk;
}
static_assert(kGramChunk % kPartPad == 0, "a first-level block covers whole padded chunks");

__global__ __launch_bounds__(BS) void k_ss_gram(SsRedArgs R) {
  __shared__ double tot[NGP];
  int j = 0;  // system of this block (uniform)
#pragma unroll
  for (int k = 1; k < kSsArgSlots; ++k) j += (k < R.n && R.start[k] <= (int)blockIdx.x) ? 1 : 0;
  const SsRedSys& Y = R.s[j];
  const int b = (int)blockIdx.x - R.start[j], nb = R.start[j + 1] - R.start[j];
  const int t = threadIdx.x, v = t >> 4, l = t & 15;
  const int vv = v < NG ? v : 0;
  const int gs = part_stride(Y.grid), c0 = b * kGramChunk;
  const float* pv = Y.part + (size_t)vv * gs + c0 + l;
  // every chunk's loads first (a chunk past the row is skipped as a whole)
  constexpr int kSub = kGramChunk / kPartPad;
  double h[kSub][16];
#pragma unroll
  for (int c = 0; c < kSub; ++c) {
    const bool in = c == 0 || c0 + c * kPartPad < gs;  // uniform
#pragma unroll
    for (int k = 0; k < 16; ++k) h[c][k] = in ? (double)pv[c * kPartPad + 16 * k] : 0.0;
  }
#pragma unroll
  for (int w = 8; w >= 1; w >>= 1)
#pragma unroll
    for (int k = 0; k < w; ++k) h[0][k] += h[0][k + w];
  double acc = h[0][0];
#pragma unroll
  for (int c = 1; c < kSub; ++c)
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += h[c][k];  // zeros past the row
  const double sum = row_sum(acc);
  if (nb == 1) {  // one block: its sums are the totals
    if (l == 0 && v < NG) {
      tot[v] = sum;
      Y.out[v] = sum;
    }
    __syncthreads();
    if (t < 64 && (Y.force || Y.rec->phase == kIter)) ss_recur(tot, *Y.rec, *Y.prm, Y.force, Y.ctl);
    return;
  }
  if (l == 0 && v < NG) Y.level1[(size_t)b * NGP + v] = sum;
}

// Second level, for systems of more than one first-level block (one block
// per system): the first-level sums in block order, the totals, and the
// coefficients of the next launch.
__global__ __launch_bounds__(BS) void k_ss_gram_final(SsRedArgs R) {
  __shared__ double tot[NGP];
  const int j = blockIdx.x;
  const SsRedSys& Y = R.s[j];
  const int nb = R.start[j + 1] - R.start[j];
  if (nb <= 1) return;  // summed by the first level
  const int t = threadIdx.x, v = t >> 4, l = t & 15;
  const int vv = v < NG ? v : 0;
  const double* l1 = Y.level1 + vv;
  double acc = 0.0;
  for (int q0 = 0; q0 < nb; q0 += 256) {
    double h[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int q = q0 + l + 16 * k;
      h[k] = l1[(size_t)(q < nb ? q : 0) * NGP];  // clamped in range, masked after
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) h[k] = (q0 + l + 16 * k < nb) ? h[k] : 0.0;
#pragma unroll
    for (int w = 8; w >= 1; w >>= 1)
#pragma unroll
      for (int k = 0; k < w; ++k) h[k] += h[k + w];
    acc += h[0];
  }
  acc = row_sum(acc);
  if (l == 0 && v < NG) {
    tot[v] = acc;
    Y.out[v] = acc;
  }
  __syncthreads();
  if (t < 64 && (Y.force || Y.rec->phase == kIter)) ss_recur(tot, *Y.rec, *Y.prm, Y.force, Y.ctl);
}

// Values of the plan's rows after an assembly: the FP32 diagonal and D^-1
// (slot 7 of both basis buffers), in the plan's numbering.
__global__ __launch_bounds__(kBlock) void k_ss_values(int n, const int32_t* __restrict__ perm,
                                                      const double* __restrict__ diag64,
                                                      const float* __restrict__ dinv32,
                                                      float* __restrict__ d, float* __restrict__ W0,
                                                      float* __restrict__ W1) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int r = perm[i];
  if (d) d[i] = (float)diag64[r];
  W0[8 * (size_t)i + 7] = dinv32[r];
  W1[8 * (size_t)i + 7] = dinv32[r];
}

// ---------------------------------------------------------------- host ----
// Launch arguments; `large`: the partials are summed by a reduction launch
// (the step reads the totals and the coefficients it computed).
SsArgs ss_args(fi_mesh* M, int par, int force, bool large) {
  (void)large;  // the kernel instantiation decides which inputs it reads
  SsState& Z = *M->ss;
  SsArgs A;
  A.n = (int)M->n;
  A.grid = Z.grid;
  A.gstride = part_stride(Z.grid);
  A.perm = Z.perm;
  A.blocks = (const BlockPlan*)Z.blocks;
  A.region = Z.region;
  A.lmat = (const LmRow*)Z.lmat;
  A.Win = (const float4*)Z.W[par];
  A.Wout = (float4*)Z.W[par ^ 1];
  A.x = Z.x;
  A.d = Z.d;
  A.b = Z.b;
  A.r64 = Z.r64;
  A.x64a = Z.x64[0];
  A.x64b = Z.x64[1];
  A.xout = M->d_x64buf[0];
  A.part_in = Z.part + (size_t)par * NGP * A.gstride;
  A.tot_in = Z.red;
  A.part_out = Z.part + (size_t)(par ^ 1) * NGP * A.gstride;
  A.rec_in = (const Rec*)M->d_rec + par;
  A.rec_out = (Rec*)M->d_rec + (par ^ 1);
  A.prm = (const Params*)M->d_prm;
  A.mirror = (Mirror*)M->d_mirror;
  A.ctl = Z.ctl;
  A.force = force;
  return A;
}

// The reduction after a step launch of parity par: its partials, and the
// record and coefficients of the next launch.
SsRedSys red_sys(fi_mesh* M, int par, int force) {
  SsState& Z = *M->ss;
  SsRedSys y;
  y.part = Z.part + (size_t)(par ^ 1) * NGP * part_stride(Z.grid);
  y.level1 = Z.level1;
  y.out = Z.red;
  y.rec = (const Rec*)M->d_rec + (par ^ 1);
  y.prm = (const Params*)M->d_prm;
  y.ctl = Z.ctl;
  y.grid = Z.grid;
  y.force = force;
  return y;
}

// Appends system y to a reduction launch (false when the launch is full).
bool red_add(SsRedArgs& R, const SsRedSys& y) {
  if (R.n >= kSsArgSlots) return false;
  if (R.n == 0) R.start[0] = 0;
  R.s[R.n] = y;
  R.start[R.n + 1] = R.start[R.n] + gram_blocks(y.grid);
  ++R.n;
  return true;
}

int red_launch(const SsRedArgs& R, hipStream_t st) {
  if (R.n == 0) return FI_OK;
  void* args[1] = {(void*)&R};
  FI_HIP_TRY(hipLaunchKernel((void*)k_ss_gram, dim3((unsigned)R.start[R.n]), dim3(BS), args, 0, st));
  bool two = false;
  for (int k = 0; k < R.n; ++k) two = two || R.start[k + 1] - R.start[k] > 1;
  if (two)
    FI_HIP_TRY(hipLaunchKernel((void*)k_ss_gram_final, dim3((unsigned)R.n), dim3(BS), args, 0, st));
  return FI_OK;
}

// Dynamic LDS of a launch: the basis levels (5 floats per region row, and
// the two zero slots), and at least room for the rows' values staged for
// the matrix cores.
size_t ss_lds_bytes(const SsState& Z) {
  return std::max((size_t)(5 * Z.max_region + 4) * sizeof(float), (size_t)BS * 8 * sizeof(float));
}

int ss_reduce_after(fi_mesh* M, int par, int force) {
  SsRedArgs R{};
  red_add(R, red_sys(M, par, force));
  return red_launch(R, M->ctx->stream);
}

int ss_launch_step(fi_mesh* M, int par, int force) {
  SsState& Z = *M->ss;
  SsArgs A = ss_args(M, par, force, Z.large);
  void* args[1] = {&A};
  void* fn = Z.large ? (void*)k_ss_step<true> : (void*)k_ss_step<false>;
  FI_HIP_TRY(hipLaunchKernel(fn, dim3(Z.grid), dim3(BS), args, ss_lds_bytes(Z), M->ctx->stream));
  return Z.large ? ss_reduce_after(M, par, force) : FI_OK;
}

int ss_launch_start(fi_mesh* M, const fi_solve_opts* o, int epoch, const double* x0, bool large) {
  SsState& Z = *M->ss;
  SsArgs A = ss_args(M, 1, 0, large);  // writes record and partials of slot 0
  Params prm{};
  prm.rtol = o->rtol;
  prm.atol = o->atol;
  prm.inner_rtol = o->inner_rtol;
  prm.max_inner = o->max_inner;
  prm.max_refine = o->max_refine;
  prm.mixed = 1.0;
  prm.epoch = epoch;
  Params* pout = (Params*)M->d_prm;
  const double* bnat = M->d_b64;
  void* args[5] = {&A, &prm, &pout, &bnat, &x0};
  FI_HIP_TRY(hipLaunchKernel((void*)k_ss_start, dim3(Z.grid), dim3(BS), args, ss_lds_bytes(Z),
                             M->ctx->stream));
  return large ? ss_reduce_after(M, 1, 0) : FI_OK;
}

// Both parities of the partial sums.
size_t part_bytes(int grid) { return (size_t)2 * NGP * part_stride(grid) * sizeof(float); }

// The reduction launch's first-level sums and the coefficient block (every mesh: multi-solve and batched launches may sum
// a small system's partials that way too).
int large_alloc(fi_mesh* M, SsState& Z) {
  Z.level1 = nullptr;
  Z.ctl = nullptr;
  int rc = 0;
  if ((rc = device_alloc(M, (void**)&Z.level1, (size_t)gram_blocks(Z.grid) * NGP * 8)) ||
      (rc = device_alloc(M, (void**)&Z.ctl, NGP * 8)))
    return rc;
  FI_HIP_TRY(hipMemsetAsync(Z.ctl, 0, NGP * 8, M->ctx->stream));
  return FI_OK;
}

int slot_of(const double* x0) { return 0 + (x0 ? 1 : 0); }  // FP32 cold / warm prediction slots

// The host builder's plan (ss_plan.h), from the ELL copied back from the
// device: what the device builder is checked against, and its stand-in with
// FI_SS_PLAN=host.
int plan_on_host(fi_mesh* M, SsState& Z, bool* built) {
  *built = false;
  hipStream_t st = M->ctx->stream;
  const int64_t n = M->n;
  // the ELL comes back through the context's pinned staging buffer when it
  // fits there (several times faster than a copy to pageable memory)
  const size_t ell_words = (size_t)M->ell_w * M->n_pad;
  std::unique_lock<std::mutex> staging_hold;
  int32_t* ell = M->cache ? (int32_t*)M->cache->staging(ell_words * 4, staging_hold) : nullptr;
  std::vector<int32_t> ell_pageable;
  if (!ell) {
    ell_pageable.resize(ell_words);
    ell = ell_pageable.data();
  }
  FI_HIP_TRY(hipMemcpyAsync(ell, M->d_ell, ell_words * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  FI_HIP_TRY(hipStreamSynchronize(st));
  std::vector<int32_t> hv, hf;
  int rc = mesh_host_coords(M, hv, hf);
  if (rc) return rc;
  HostVec<int32_t> xy((size_t)2 * n);
  pool_run(16, [&](int64_t t, int64_t nt) {
    const auto [i0, i1] = split_range(n, nt, t);
    for (int64_t i = i0; i < i1; ++i) {
      const int32_t v = hf[i];
      xy[2 * i] = hv[2 * (size_t)v];
      xy[2 * i + 1] = hv[2 * (size_t)v + 1];
    }
  });
  SsPlan plan;
  if (!build_ss_plan(S, BS, n, xy.data(), ell, M->n_pad, M->ell_w, 16, kMaxRegion, plan))
    return FI_OK;  // keep the one-iteration launch
  if (staging_hold.owns_lock()) staging_hold.unlock();
  plan.blocks[0].pad0 = plan.max_region;  // the LDS layout size, in the first block's spare field
  if ((rc = device_alloc(M, (void**)&Z.perm, (size_t)n * 4)) ||
      (rc = device_alloc(M, &Z.blocks, plan.blocks.size() * sizeof(BlockPlan))) ||
      (rc = device_alloc(M, (void**)&Z.region, std::max<size_t>(plan.region.size(), 1) * 4)) ||
      (rc = device_alloc(M, &Z.lmat, std::max<size_t>(plan.lmat.size(), kPlanSlots) * 2)))
    return rc;
  FI_HIP_TRY(hipMemcpyAsync(Z.perm, plan.perm.data(), (size_t)n * 4, hipMemcpyHostToDevice, st));
  FI_HIP_TRY(hipMemcpyAsync(Z.blocks, plan.blocks.data(), plan.blocks.size() * sizeof(BlockPlan),
                            hipMemcpyHostToDevice, st));
  FI_HIP_TRY(hipMemcpyAsync(Z.region, plan.region.data(), plan.region.size() * 4,
                            hipMemcpyHostToDevice, st));
  if (!plan.lmat.empty())
    FI_HIP_TRY(hipMemcpyAsync(Z.lmat, plan.lmat.data(), plan.lmat.size() * 2,
                              hipMemcpyHostToDevice, st));
  // the host copies come from vectors that end with this call
  FI_HIP_TRY(hipStreamSynchronize(st));
  Z.grid = plan.grid;
  Z.max_region = plan.max_region;
  Z.region_rows = (int64_t)plan.region.size();
  Z.lmat_rows = (int64_t)plan.lmat.size() / kPlanSlots;
  *built = true;
  return FI_OK;
}

}  // namespace

// Builds the plan after the first assembly of a quadtree mesh (on the device,
// or on the host with FI_SS_PLAN=host; both give the same plan); later calls
// refresh the values that come from the matrix.
int ss_setup(fi_mesh* M) {
  hipStream_t st = M->ctx->stream;
  if (!M->ss) {
    if (M->ell_w <= 0 || M->n <= 0 || M->is_channel) return FI_OK;
    if (const char* env = std::getenv("FI_CG_SSTEP"))
      if (std::atoi(env) == 0) return FI_OK;
    const int64_t n = M->n;
    std::unique_ptr<SsState> plan(new SsState());
    bool built = false;
    // server requests (meshes carved out of an arena) take the device
    // build's scratch from their arena region; one whose scratch would not
    // fit the region's reserve falls back to the host builder
    const char* where = std::getenv("FI_SS_PLAN");
    const bool on_host = where && std::strcmp(where, "host") == 0;
    int rc = on_host ? plan_on_host(M, *plan, &built)
                     : ss_plan_on_device(M, S, kMaxRegion, *plan, &built);
    if (!rc && !built && !on_host && M->arena) rc = plan_on_host(M, *plan, &built);
    if (rc || !built) return rc;  // not built: keep the one-iteration launch
    SsState* Z = plan.release();
    bool large = Z->grid > kSmallGrid;
    if (const char* env = std::getenv("FI_CG_LARGE"))
      if (std::atoi(env) == 1) large = true;
    Z->large = large;
    M->ss = Z;
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    if ((rc = device_alloc(M, (void**)&Z->W[0], nn * 32)) ||
        (rc = device_alloc(M, (void**)&Z->W[1], nn * 32)) ||
        (rc = device_alloc(M, (void**)&Z->x, nn * 4)) ||
        (rc = device_alloc(M, (void**)&Z->d, nn * 4)) ||
        (rc = device_alloc(M, (void**)&Z->b, nn * 8)) ||
        (rc = device_alloc(M, (void**)&Z->r64, nn * 8)) ||
        (rc = device_alloc(M, (void**)&Z->x64[0], nn * 8)) ||
        (rc = device_alloc(M, (void**)&Z->x64[1], nn * 8)) ||
        (rc = device_alloc(M, (void**)&Z->part, part_bytes(Z->grid))) ||
        (rc = device_alloc(M, (void**)&Z->red, NGP * 8)) ||
        (rc = large_alloc(M, *Z)))
      return rc;
    // every basis slot starts finite (the first launch reads only D^-1)
    FI_HIP_TRY(hipMemsetAsync(Z->W[0], 0, nn * 32, st));
    FI_HIP_TRY(hipMemsetAsync(Z->part, 0, part_bytes(Z->grid), st));  // the padding stays 0
    FI_HIP_TRY(hipMemsetAsync(Z->W[1], 0, nn * 32, st));
  }
  SsState& Z = *M->ss;
  hipLaunchKernelGGL(k_ss_values, dim3((unsigned)((M->n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     st, (int)M->n, Z.perm, M->d_diag64, M->d_dinv32, Z.d, Z.W[0], Z.W[1]);
  FI_HIP_TRY(hipGetLastError());
  return FI_OK;
}

int ss_export_plan(const fi_mesh* M, int32_t* perm, int32_t* blocks, int32_t* region,
                   uint16_t* lmat) {
  if (!M || !M->ss) return fail(FI_E_INVALID, "the mesh has no S-iteration plan");
  const SsState& Z = *M->ss;
  hipStream_t st = M->ctx->stream;
  if (perm)
    FI_HIP_TRY(hipMemcpyAsync(perm, Z.perm, (size_t)M->n * 4, hipMemcpyDeviceToHost, st));
  if (blocks)
    FI_HIP_TRY(hipMemcpyAsync(blocks, Z.blocks, (size_t)Z.grid * sizeof(BlockPlan),
                              hipMemcpyDeviceToHost, st));
  if (region)
    FI_HIP_TRY(hipMemcpyAsync(region, Z.region, (size_t)Z.region_rows * 4, hipMemcpyDeviceToHost,
                              st));
  if (lmat && Z.lmat_rows > 0)
    FI_HIP_TRY(hipMemcpyAsync(lmat, Z.lmat, (size_t)Z.lmat_rows * kPlanSlots * 2,
                              hipMemcpyDeviceToHost, st));
  FI_HIP_TRY(hipStreamSynchronize(st));
  return FI_OK;
}

void ss_release(fi_mesh* M) {
  delete M->ss;  // its device memory is in the mesh's allocations
  M->ss = nullptr;
}

int ss_solve(fi_mesh* M, const fi_solve_opts* o, fi_solve_stats* stats, const double* x0) {
  hipStream_t st = M->ctx->stream;
  const int epoch = next_epoch(M);
  int rc = ss_launch_start(M, o, epoch, x0, M->ss->large);
  if (rc) return rc;
  const int slot = slot_of(x0);
  Pacer pc = make_pacer(o->max_inner, o->max_refine, M->pred_launches[slot],
                        M->ss->large ? kChunk : kChunkShort);
  for (;;) {
    int drc = FI_OK;
    int64_t nl = 0;
    if (read_mirror(M, epoch, stats, &drc, &nl)) {
      M->pred_launches[slot] = nl;
      return drc;
    }
    if (const int nq = pc.next()) {
      for (int q = 0; q < nq; ++q)
        if ((rc = ss_launch_step(M, q & 1, 0))) return rc;
      FI_HIP_TRY(hipEventRecord(M->chunk_ev[pc.launched % kChunkEvents], st));
      pc.queued_chunk(nq);
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
    } else {
      if (read_mirror(M, epoch, stats, &drc, nullptr)) return drc;
      return fail(FI_E_HIP, "solver did not report termination");
    }
    __builtin_ia32_pause();
  }
}

namespace {

void* multi_fn(bool large) { return large ? (void*)k_ss_multi_large : (void*)k_ss_multi_small; }

// Launch arguments of a multi-RHS step for both parities.
struct SsMultiLaunch {
  SsMultiArgs a[2];
  SsRedArgs r[2];
  bool large;
};

// Multi-solve launches sum the partials in a reduction launch when their
// blocks would not fit in one round otherwise.
bool multi_large(fi_mesh* const* ch, int nc) {
  return ch[0]->ss->large || (int64_t)nc * ch[0]->ss->grid > kSmallGrid;
}

void ss_multi_prepare(fi_mesh* const* ch, int nc, int force, bool large, SsMultiLaunch& L) {
  L.large = large;
  for (int par = 0; par < 2; ++par) {
    L.a[par] = SsMultiArgs{};
    L.a[par].nrhs = nc;
    L.r[par] = SsRedArgs{};
    for (int c = 0; c < nc; ++c) {
      L.a[par].a[c] = ss_args(ch[c], par, force, large);
      if (large) red_add(L.r[par], red_sys(ch[c], par, force));
    }
  }
}

int ss_multi_launch(fi_mesh* M0, SsMultiLaunch& L, int par) {
  SsState& Z = *M0->ss;
  void* args[1] = {&L.a[par]};
  const unsigned grid = (unsigned)L.a[par].nrhs * (unsigned)Z.grid;
  FI_HIP_TRY(hipLaunchKernel(multi_fn(L.large), dim3(grid), dim3(BS), args, ss_lds_bytes(Z),
                             M0->ctx->stream));
  return L.large ? red_launch(L.r[par], M0->ctx->stream) : FI_OK;
}

}  // namespace

// The channels' solves advance together, one launch per step, paced like
// ss_solve (events of channel 0), until every channel's mirror shows its end;
// a channel whose solve has ended leaves the launches from the next chunk on.
int ss_solve_multi(fi_mesh* const* ch, int nc, const fi_solve_opts* o, fi_solve_stats* stats,
                   const double* const* x0) {
  fi_mesh* M0 = ch[0];
  hipStream_t st = M0->ctx->stream;
  int epoch[kMaxRhs];
  bool done[kMaxRhs] = {};
  int rc = FI_OK, first_rc = FI_OK;
  // the mode stays for the whole solve, also once fewer channels are left
  const bool large = multi_large(ch, nc);
  for (int c = 0; c < nc; ++c) {
    epoch[c] = next_epoch(ch[c]);
    if ((rc = ss_launch_start(ch[c], o, epoch[c], x0 ? x0[c] : nullptr, large))) return rc;
  }
  SsMultiLaunch L;
  fi_mesh* run[kMaxRhs];
  int nrun = nc;
  for (int c = 0; c < nc; ++c) run[c] = ch[c];
  ss_multi_prepare(run, nrun, 0, large, L);
  int64_t pred = 0;
  bool every = true;
  for (int c = 0; c < nc; ++c) {
    const int64_t p = ch[c]->pred_launches[slot_of(x0 ? x0[c] : nullptr)];
    every = every && p > 0;
    pred = std::max(pred, p);
  }
  if (!every) pred = 0;
  Pacer pc = make_pacer(o->max_inner, o->max_refine, pred);
  auto all_done = [&]() {
    bool all = true;
    for (int c = 0; c < nc; ++c) {
      if (!done[c]) {
        int drc = FI_OK;
        int64_t nl = 0;
        done[c] = read_mirror(ch[c], epoch[c], &stats[c], &drc, &nl) != 0;
        if (done[c]) {
          ch[c]->pred_launches[slot_of(x0 ? x0[c] : nullptr)] = nl;
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
      ss_multi_prepare(run, nrun, 0, large, L);
    }
    if (const int nq = pc.next()) {
      for (int q = 0; q < nq; ++q)
        if ((rc = ss_multi_launch(M0, L, q & 1))) return rc;
      FI_HIP_TRY(hipEventRecord(M0->chunk_ev[pc.launched % kChunkEvents], st));
      pc.queued_chunk(nq);
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

// Times `reps` multi-RHS launches forced to iterate.
int ss_time_multi(fi_mesh* const* ch, int nc, int reps, double* ms) {
  fi_mesh* M0 = ch[0];
  hipStream_t st = M0->ctx->stream;
  fi_solve_opts o;
  fi_solve_opts_default(&o);
  int rc = FI_OK;
  const bool large = multi_large(ch, nc);
  for (int c = 0; c < nc; ++c)
    if ((rc = ss_launch_start(ch[c], &o, next_epoch(ch[c]), nullptr, large))) return rc;
  SsMultiLaunch L;
  ss_multi_prepare(ch, nc, 0, large, L);
  if ((rc = ss_multi_launch(M0, L, 0))) return rc;  // the initial bases
  ss_multi_prepare(ch, nc, 1, large, L);
  hipEvent_t e0, e1;
  FI_HIP_TRY(hipEventCreate(&e0));
  FI_HIP_TRY(hipEventCreate(&e1));
  for (int k = 0; k < 4; ++k)
    if ((rc = ss_multi_launch(M0, L, (k + 1) & 1))) return rc;
  FI_HIP_TRY(hipEventRecord(e0, st));
  for (int k = 0; k < reps; ++k)
    if ((rc = ss_multi_launch(M0, L, (k + 1) & 1))) return rc;
  FI_HIP_TRY(hipEventRecord(e1, st));
  FI_HIP_TRY(hipEventSynchronize(e1));
  float t = 0.f;
  FI_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = (double)t / reps;
  return FI_OK;
}

// `count` (even) launches over the meshes in `ms` (all with the S-iteration
// plan), parity 0 first: one launch per kSsArgSlots meshes, each followed by
// its reduction launch. Batched solves always sum their partials in the
// reduction launch (armed so by ss_arm), whatever the batch holds, so a
// solve's mode never depends on its neighbours; for systems of up to
// kSmallGrid blocks that gives the bits of the single-solve launch.
int ss_batch_launch(hipStream_t st, const std::vector<fi_mesh*>& ms, int count) {
  struct Launch {
    SsBatchArgs b[2];
    SsRedArgs r[2];
    int64_t grid;
    size_t lds;
  };
  const std::vector<fi_mesh*>& order = ms;
  std::vector<Launch> L;
  for (size_t j0 = 0; j0 < order.size();) {
    Launch l{};
    const size_t j1 = std::min(order.size(), j0 + (size_t)kSsArgSlots);
    int64_t total = 0;
    for (int par = 0; par < 2; ++par) l.b[par].n = (int)(j1 - j0);
    for (size_t j = j0; j < j1; ++j) {
      fi_mesh* M = order[j];
      const int q = (int)(j - j0);
      for (int par = 0; par < 2; ++par) {
        l.b[par].start[q] = (int32_t)total;
        l.b[par].a[q] = ss_args(M, par, 0, true);
        red_add(l.r[par], red_sys(M, par, 0));
      }
      total += M->ss->grid;
      l.lds = std::max(l.lds, ss_lds_bytes(*M->ss));
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
      FI_HIP_TRY(hipLaunchKernel((void*)k_ss_batch, dim3((unsigned)l.grid), dim3(BS), args,
                                 l.lds, st));
    }
    for (Launch& l : L) {
      const int rc = red_launch(l.r[par], st);
      if (rc) return rc;
    }
  }
  return FI_OK;
}

int ss_arm(fi_mesh* M, const fi_solve_opts* o, int epoch, const double* x0) {
  return ss_launch_start(M, o, epoch, x0, true);  // batched solves: ss_batch_launch
}

// A channel view's own vectors, with the parent's plan and diagonal.
int ss_channel_setup(fi_mesh* S, const fi_mesh* M) {
  if (!M->ss) return FI_OK;
  const SsState& P = *M->ss;
  SsState* Z = new SsState();
  *Z = P;  // plan, shape and the shared diagonal
  S->ss = Z;
  const size_t nn = (size_t)std::max<int64_t>(M->n, 1);
  int rc = 0;
  if ((rc = device_alloc(S, (void**)&Z->W[0], nn * 32)) ||
      (rc = device_alloc(S, (void**)&Z->W[1], nn * 32)) ||
      (rc = device_alloc(S, (void**)&Z->x, nn * 4)) ||
      (rc = device_alloc(S, (void**)&Z->b, nn * 8)) ||
      (rc = device_alloc(S, (void**)&Z->r64, nn * 8)) ||
      (rc = device_alloc(S, (void**)&Z->x64[0], nn * 8)) ||
      (rc = device_alloc(S, (void**)&Z->x64[1], nn * 8)) ||
      (rc = device_alloc(S, (void**)&Z->part, part_bytes(Z->grid))) ||
      (rc = device_alloc(S, (void**)&Z->red, NGP * 8)) || (rc = large_alloc(S, *Z)))
    return rc;
  hipStream_t st = M->ctx->stream;
  FI_HIP_TRY(hipMemsetAsync(Z->W[0], 0, nn * 32, st));
  FI_HIP_TRY(hipMemsetAsync(Z->W[1], 0, nn * 32, st));
  FI_HIP_TRY(hipMemsetAsync(Z->part, 0, part_bytes(Z->grid), st));  // the padding stays 0
  hipLaunchKernelGGL(k_ss_values, dim3((unsigned)((M->n + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     st, (int)M->n, Z->perm, M->d_diag64, M->d_dinv32, (float*)nullptr, Z->W[0],
                     Z->W[1]);
  FI_HIP_TRY(hipGetLastError());
  return FI_OK;
}

// Device bytes the S-iteration state of a system of n rows may take (each
// allocation rounded to 256 bytes): the plan (at most three region and
// local matrix rows per free row), the two basis buffers, the FP32 and FP64
// vectors, the partial sums, the reduction launch's state.
int64_t ss_footprint(int64_t n) {
  const int64_t grid = ((n + BS - 1) / BS + 7) / 8 * 8;
  int64_t total = 0;
  auto add = [&](int64_t bytes) {
    total += std::max<int64_t>(256, (std::max<int64_t>(bytes, 1) + 255) & ~(int64_t)255);
  };
  add(4 * n); add(32 * grid); add(4 * 3 * n); add(16 * 3 * n);
  add(32 * n); add(32 * n); add(4 * n); add(4 * n);
  add(8 * n); add(8 * n); add(8 * n); add(8 * n);
  add(8 * 2 * NGP * part_stride((int)grid)); add(8 * NGP);
  add(8 * NGP * gram_blocks((int)grid)); add(8 * NGP);  // the reduction launch
  return total;
}

// Times `reps` launches forced to iterate, between two HIP events on the
// context stream (large systems: with their reduction launch).
int ss_time_kernel(fi_mesh* M, int reps, double* ms) {
  hipStream_t st = M->ctx->stream;
  fi_solve_opts o;
  fi_solve_opts_default(&o);
  int rc = ss_launch_start(M, &o, next_epoch(M), nullptr, M->ss->large);
  if (rc) return rc;
  if ((rc = ss_launch_step(M, 0, 0))) return rc;  // the initial basis
  hipEvent_t e0, e1;
  FI_HIP_TRY(hipEventCreate(&e0));
  FI_HIP_TRY(hipEventCreate(&e1));
  for (int k = 0; k < 4; ++k)
    if ((rc = ss_launch_step(M, (k + 1) & 1, 1))) return rc;
  FI_HIP_TRY(hipEventRecord(e0, st));
  for (int k = 0; k < reps; ++k)
    if ((rc = ss_launch_step(M, (k + 1) & 1, 1))) return rc;
  FI_HIP_TRY(hipEventRecord(e1, st));
  FI_HIP_TRY(hipEventSynchronize(e1));
  float t = 0.f;
  FI_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = (double)t / reps;
  return FI_OK;
}

}  // namespace fi
