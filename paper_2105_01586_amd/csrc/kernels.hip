// HIP kernels for gfx950: stiffness assembly, Dirichlet lift, interpolation
// to pixels with error measures, its transpose, and vector reductions.
//
// Assembly is vertex-centric: one thread owns one matrix row and visits the
// triangles incident to its vertex, so rows are written without atomics and
// the result is bitwise reproducible. Rasterisation is leaf-centric: one
// thread owns one quadtree leaf, whose half-open box holds exactly its own
// pixels, so per-triangle sums are private to the thread.
#include <algorithm>
#include <cstdint>

#include "internal.h"
#include "reduce.h"

namespace fi {

namespace {

inline int grid_for(int64_t n, int per_block = kBlock) {
  int64_t g = (n + per_block - 1) / per_block;
  return (int)(g < 1 ? 1 : g);
}

// ------------------------------------------------------------ assembly ----
// Row of the stiffness matrix at vertex v: K_vw = sum over triangles holding
// v and w of (b_v b_w + c_v c_w) / (4A), with b_i = y_j - y_k, c_i = x_k - x_j
// for (i, j, k) cyclic (Section 2.2, P1 elements). Returns the distinct
// neighbours with non-zero weight, sorted by vertex id, and the diagonal.
// NB: capacity of the neighbour list, at least the distinct neighbours of
// any vertex. Quadtree meshes use NB = kMaxIncident: an interior vertex has a
// closed fan (as many neighbours as triangles) and the builder keeps border
// vertices to kMaxIncident - 1 triangles (open fan: one neighbour more).
template <int NB>
__device__ __forceinline__ int stiffness_row(int v, const int32_t* __restrict__ vxy,
                                             const int32_t* __restrict__ tri,
                                             const int32_t* __restrict__ vt_ptr,
                                             const int32_t* __restrict__ vt_idx,
                                             int32_t (&nb)[NB], double (&w)[NB], double& diag) {
  int cnt = 0;
  double d = 0.0;
  const int64_t xa = vxy[2 * v], ya = vxy[2 * v + 1];
  const int e0 = vt_ptr[v], e1 = vt_ptr[v + 1];
  // Quadtree rows (at most kMaxIncident triangles): every index and
  // coordinate is loaded before the arithmetic, three dependent rounds in
  // all instead of three per triangle. Other meshes walk the list.
  constexpr bool PRE = NB == kMaxIncident;
  constexpr int MT = PRE ? kMaxIncident : 1;
  int pb[MT], pc[MT];
  int64_t pxb[MT], pyb[MT], pxc[MT], pyc[MT];
  if constexpr (PRE) {
    const int last = e1 - 1;  // every vertex has a triangle: clamped loads stay in the list
    int code[MT];
#pragma unroll
    for (int q = 0; q < MT; ++q) code[q] = vt_idx[min(e0 + q, last)];
#pragma unroll
    for (int q = 0; q < MT; ++q) {
      const int t = code[q] / 3;
      const int k = code[q] - 3 * t;
      pb[q] = tri[3 * t + (k + 1) % 3];
      pc[q] = tri[3 * t + (k + 2) % 3];
    }
#pragma unroll
    for (int q = 0; q < MT; ++q) {
      pxb[q] = vxy[2 * pb[q]];
      pyb[q] = vxy[2 * pb[q] + 1];
      pxc[q] = vxy[2 * pc[q]];
      pyc[q] = vxy[2 * pc[q] + 1];
    }
  }
  // One incident triangle (b, c its other two corners), in list order: the
  // weights of b and c join their slots, or open new ones.
  if constexpr (PRE) {
    // Slots addressed only by compile-time indices (predicated updates), so
    // no lane-dependent register indexing; then a sorting network.
    int32_t id[NB];
    double wv[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      id[q] = 0x7fffffff;
      wv[q] = 0.0;
    }
    auto put = [&](int32_t u, double wu) {
      bool found = false;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        if (id[q] == u) {
          wv[q] += wu;
          found = true;
        }
      }
      if (!found) {
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          if (q == cnt) {
            id[q] = u;
            wv[q] = wu;
          }
        }
        ++cnt;
      }
    };
    const int ne = e1 - e0;
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      if (t < ne) {
        const int64_t xb = pxb[t], yb = pyb[t], xc = pxc[t], yc = pyc[t];
        const int64_t ba = yb - yc, ca = xc - xb;
        const int64_t bb = yc - ya, cb = xa - xc;
        const int64_t bc = ya - yb, cc = xb - xa;
        const int64_t twoA = (xb - xa) * (yc - ya) - (yb - ya) * (xc - xa);
        const double inv = 1.0 / (2.0 * (double)twoA);
        d += (double)(ba * ba + ca * ca) * inv;
        put(pb[t], (double)(ba * bb + ca * cb) * inv);
        put(pc[t], (double)(ba * bc + ca * cc) * inv);
      }
    }
    // drop exact zeros (hypotenuse couplings), sort by id (odd-even
    // transposition network; ids are distinct)
#pragma unroll
    for (int q = 0; q < NB; ++q)
      if (wv[q] == 0.0) id[q] = 0x7fffffff;
#pragma unroll
    for (int r = 0; r < NB; ++r) {
#pragma unroll
      for (int q = r & 1; q + 1 < NB; q += 2) {
        const bool sw = id[q] > id[q + 1];
        const int32_t i0 = sw ? id[q + 1] : id[q], i1 = sw ? id[q] : id[q + 1];
        const double w0 = sw ? wv[q + 1] : wv[q], w1 = sw ? wv[q] : wv[q + 1];
        id[q] = i0;
        id[q + 1] = i1;
        wv[q] = w0;
        wv[q + 1] = w1;
      }
    }
    int k2 = 0;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      nb[q] = id[q];
      w[q] = wv[q];
      k2 += id[q] != 0x7fffffff;
    }
    diag = d;
    return k2;
  } else {
    auto add = [&](int b, int c, int64_t xb, int64_t yb, int64_t xc, int64_t yc) {
      const int64_t ba = yb - yc, ca = xc - xb;
      const int64_t bb = yc - ya, cb = xa - xc;
      const int64_t bc = ya - yb, cc = xb - xa;
      const int64_t twoA = (xb - xa) * (yc - ya) - (yb - ya) * (xc - xa);
      const double inv = 1.0 / (2.0 * (double)twoA);
      d += (double)(ba * ba + ca * ca) * inv;
      const double wb = (double)(ba * bb + ca * cb) * inv;
      const double wc = (double)(ba * bc + ca * cc) * inv;
      int fb = -1, fc = -1;
      for (int q = 0; q < cnt; ++q) {
        if (nb[q] == b) fb = q;
        if (nb[q] == c) fc = q;
      }
      if (fb >= 0) w[fb] += wb; else { nb[cnt] = b; w[cnt] = wb; ++cnt; }
      if (fc >= 0) w[fc] += wc; else { nb[cnt] = c; w[cnt] = wc; ++cnt; }
    };
    for (int e = e0; e < e1; ++e) {
      const int code = vt_idx[e];
      const int t = code / 3;
      const int k = code - 3 * t;
      const int b = tri[3 * t + (k + 1) % 3];
      const int c = tri[3 * t + (k + 2) % 3];
      add(b, c, vxy[2 * b], vxy[2 * b + 1], vxy[2 * c], vxy[2 * c + 1]);
    }
    // drop exact zeros (hypotenuse couplings), then insertion sort by id
    int k2 = 0;
    for (int q = 0; q < cnt; ++q) {
      if (w[q] != 0.0) { nb[k2] = nb[q]; w[k2] = w[q]; ++k2; }
    }
    for (int q = 1; q < k2; ++q) {
      const int32_t kn = nb[q];
      const double kw = w[q];
      int r = q - 1;
      while (r >= 0 && nb[r] > kn) { nb[r + 1] = nb[r]; w[r + 1] = w[r]; --r; }
      nb[r + 1] = kn;
      w[r + 1] = kw;
    }
    diag = d;
    return k2;
  }
}

// Rows of the free vertices: count entries of K_FF (off-diagonal) and K_FD.
template <int NB>
__global__ __launch_bounds__(kBlock) void k_asm_free_count(
    int n, const int32_t* __restrict__ free_vids, const int32_t* __restrict__ vxy,
    const int32_t* __restrict__ tri, const int32_t* __restrict__ vt_ptr,
    const int32_t* __restrict__ vt_idx, const int32_t* __restrict__ vmap,
    int32_t* __restrict__ cnt_ff, int32_t* __restrict__ cnt_fd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == n) { cnt_ff[n] = 0; cnt_fd[n] = 0; }
  if (i >= n) return;
  int32_t nb[NB];
  double w[NB];
  double d;
  const int k = stiffness_row<NB>(free_vids[i], vxy, tri, vt_ptr, vt_idx, nb, w, d);
  int cf = 0, cd = 0;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if (q < k) {
      if (vmap[nb[q]] >= 0) ++cf; else ++cd;
    }
  }
  cnt_ff[i] = cf;
  cnt_fd[i] = cd;
}

// Free row i: its K_FF and K_FD entries, diagonal and D^-1; with ell, also
// its ELL slots (W of them, column-major with stride n_pad).
template <int NB>
__device__ __forceinline__ void free_row_fill(
    int i, const int32_t* __restrict__ free_vids, const int32_t* __restrict__ vxy,
    const int32_t* __restrict__ tri, const int32_t* __restrict__ vt_ptr,
    const int32_t* __restrict__ vt_idx, const int32_t* __restrict__ vmap,
    const int32_t* __restrict__ ff_ptr, int32_t* __restrict__ ff_col,
    double* __restrict__ ff_val64, float* __restrict__ ff_val32,
    const int32_t* __restrict__ fd_ptr, int32_t* __restrict__ fd_col,
    double* __restrict__ fd_val, double* __restrict__ diag64, double* __restrict__ dinv64,
    float* __restrict__ dinv32, int32_t* __restrict__ ell, int n_pad, int W) {
  int32_t nb[NB];
  double w[NB];
  double d;
  const int k = stiffness_row<NB>(free_vids[i], vxy, tri, vt_ptr, vt_idx, nb, w, d);
  const int p0 = ff_ptr[i];
  int pf = p0, pd = fd_ptr[i];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if (q < k) {
      const int32_t mv = vmap[nb[q]];
      if (mv >= 0) {
        ff_col[pf] = mv;
        ff_val64[pf] = w[q];
        ff_val32[pf] = (float)w[q];
        if (ell && pf - p0 < W)
          ell[(int64_t)(pf - p0) * n_pad + i] = mv | (w[q] == -1.0 ? (int32_t)0x80000000 : 0);
        ++pf;
      } else {
        fd_col[pd] = -mv - 1;
        fd_val[pd] = w[q];
        ++pd;
      }
    }
  }
  if (ell)
    for (int s = pf - p0; s < W; ++s) ell[(int64_t)s * n_pad + i] = kEllPadBit | i;
  diag64[i] = d;
  dinv64[i] = 1.0 / d;
  dinv32[i] = (float)(1.0 / d);
}

template <int NB>
__global__ __launch_bounds__(kBlock) void k_asm_free_fill(
    int n, const int32_t* __restrict__ free_vids, const int32_t* __restrict__ vxy,
    const int32_t* __restrict__ tri, const int32_t* __restrict__ vt_ptr,
    const int32_t* __restrict__ vt_idx, const int32_t* __restrict__ vmap,
    const int32_t* __restrict__ ff_ptr, int32_t* __restrict__ ff_col,
    double* __restrict__ ff_val64, float* __restrict__ ff_val32,
    const int32_t* __restrict__ fd_ptr, int32_t* __restrict__ fd_col,
    double* __restrict__ fd_val, double* __restrict__ diag64, double* __restrict__ dinv64,
    float* __restrict__ dinv32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  free_row_fill<NB>(i, free_vids, vxy, tri, vt_ptr, vt_idx, vmap, ff_ptr, ff_col, ff_val64,
                    ff_val32, fd_ptr, fd_col, fd_val, diag64, dinv64, dinv32, nullptr, 0, 0);
}

// Rows of the mask vertices: K_DF (free columns only).
template <int NB>
__global__ __launch_bounds__(kBlock) void k_asm_mask_count(
    int m, const int32_t* __restrict__ mask_vids, const int32_t* __restrict__ vxy,
    const int32_t* __restrict__ tri, const int32_t* __restrict__ vt_ptr,
    const int32_t* __restrict__ vt_idx, const int32_t* __restrict__ vmap,
    int32_t* __restrict__ cnt_df) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == m) cnt_df[m] = 0;
  if (j >= m) return;
  int32_t nb[NB];
  double w[NB];
  double d;
  const int k = stiffness_row<NB>(mask_vids[j], vxy, tri, vt_ptr, vt_idx, nb, w, d);
  int cf = 0;
#pragma unroll
  for (int q = 0; q < NB; ++q)
    if (q < k) cf += vmap[nb[q]] >= 0;
  cnt_df[j] = cf;
}

// Mask row j: its K_DF entries.
template <int NB>
__device__ __forceinline__ void mask_row_fill(
    int j, const int32_t* __restrict__ mask_vids, const int32_t* __restrict__ vxy,
    const int32_t* __restrict__ tri, const int32_t* __restrict__ vt_ptr,
    const int32_t* __restrict__ vt_idx, const int32_t* __restrict__ vmap,
    const int32_t* __restrict__ df_ptr, int32_t* __restrict__ df_col,
    double* __restrict__ df_val) {
  int32_t nb[NB];
  double w[NB];
  double d;
  const int k = stiffness_row<NB>(mask_vids[j], vxy, tri, vt_ptr, vt_idx, nb, w, d);
  int p = df_ptr[j];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if (q < k) {
      const int32_t mv = vmap[nb[q]];
      if (mv >= 0) { df_col[p] = mv; df_val[p] = w[q]; ++p; }
    }
  }
}

template <int NB>
__global__ __launch_bounds__(kBlock) void k_asm_mask_fill(
    int m, const int32_t* __restrict__ mask_vids, const int32_t* __restrict__ vxy,
    const int32_t* __restrict__ tri, const int32_t* __restrict__ vt_ptr,
    const int32_t* __restrict__ vt_idx, const int32_t* __restrict__ vmap,
    const int32_t* __restrict__ df_ptr, int32_t* __restrict__ df_col,
    double* __restrict__ df_val) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  mask_row_fill<NB>(j, mask_vids, vxy, tri, vt_ptr, vt_idx, vmap, df_ptr, df_col, df_val);
}

// Re-assembly in one launch: blocks [0, free_blocks) fill free rows (and
// their ELL slots when ell is given), the rest fill mask rows.
struct RefillArgs {
  int n, m, free_blocks, n_pad, W;
  const int32_t *free_vids, *mask_vids, *vxy, *tri, *vt_ptr, *vt_idx, *vmap;
  const int32_t* ff_ptr;
  int32_t* ff_col;
  double* ff_val64;
  float* ff_val32;
  const int32_t* fd_ptr;
  int32_t* fd_col;
  double* fd_val;
  double *diag64, *dinv64;
  float* dinv32;
  const int32_t* df_ptr;
  int32_t* df_col;
  double* df_val;
  int32_t* ell;
};

template <int NB>
__global__ __launch_bounds__(kBlock) void k_asm_refill(RefillArgs A) {
  if ((int)blockIdx.x < A.free_blocks) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= A.n) return;
    free_row_fill<NB>(i, A.free_vids, A.vxy, A.tri, A.vt_ptr, A.vt_idx, A.vmap, A.ff_ptr,
                      A.ff_col, A.ff_val64, A.ff_val32, A.fd_ptr, A.fd_col, A.fd_val, A.diag64,
                      A.dinv64, A.dinv32, A.ell, A.n_pad, A.W);
  } else {
    const int j = (blockIdx.x - A.free_blocks) * blockDim.x + threadIdx.x;
    if (j >= A.m) return;
    mask_row_fill<NB>(j, A.mask_vids, A.vxy, A.tri, A.vt_ptr, A.vt_idx, A.vmap, A.df_ptr,
                      A.df_col, A.df_val);
  }
}

// ---------------------------------------------------------------- scan ----
// Exclusive prefix sum, 2048 items per block (256 threads x 8).
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__global__ __launch_bounds__(kBlock) void k_scan_tile(const int32_t* __restrict__ in,
                                                      int32_t* __restrict__ out, int64_t n,
                                                      int32_t* __restrict__ tile_sums) {
  __shared__ int32_t sh[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int32_t tsum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    tsum += v[k];
  }
  sh[threadIdx.x] = tsum;
  __syncthreads();
  for (int off = 1; off < kBlock; off <<= 1) {
    const int32_t add = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  int32_t run = sh[threadIdx.x] - tsum;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kBlock - 1) tile_sums[blockIdx.x] = sh[kBlock - 1];
}

__global__ __launch_bounds__(kBlock) void k_scan_add(int32_t* __restrict__ out, int64_t n,
                                                     const int32_t* __restrict__ offs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += offs[i / kScanTile];
}

int scan_rec(hipStream_t st, const int32_t* in, int32_t* out, int64_t n, int32_t* tmp) {
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  int32_t* sums = tmp;
  int32_t* sums_scanned = tmp + tiles;
  hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)tiles), dim3(kBlock), 0, st, in, out, n, sums);
  if (tiles > 1) {
    int rc = scan_rec(st, sums, sums_scanned, tiles, tmp + 2 * tiles);
    if (rc) return rc;
    hipLaunchKernelGGL(k_scan_add, dim3(grid_for(n)), dim3(kBlock), 0, st, out, n, sums_scanned);
  }
  FI_HIP_TRY(hipGetLastError());
  return FI_OK;
}

// ------------------------------------------------------ lift and gathers --
// b = -K_FD g (Section 2.2: mask values prescribed, moved to the right side).
__global__ __launch_bounds__(kBlock) void k_lift(int n, const int32_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ col,
                                                 const double* __restrict__ val,
                                                 const double* __restrict__ g,
                                                 double* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int j = ptr[i]; j < ptr[i + 1]; ++j) acc += val[j] * g[col[j]];
  b[i] = -acc;
}

__global__ __launch_bounds__(kBlock) void k_gather_mask(int m, const int32_t* __restrict__ pix,
                                                        const uint8_t* __restrict__ f,
                                                        double* __restrict__ g) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) g[j] = (double)f[pix[j]];
}

__global__ __launch_bounds__(kBlock) void k_vertex_values(int V, const int32_t* __restrict__ vmap,
                                                          const double* __restrict__ xF,
                                                          const double* __restrict__ g,
                                                          double* __restrict__ uv) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const int32_t mv = vmap[v];
  uv[v] = mv >= 0 ? xF[mv] : g[-mv - 1];
}

// ------------------------------------------------------- rasterisation ----
// Linear interpolation inside the owner triangle (Section 2.2). A pixel at
// point (x, y) belongs to the leaf whose half-open box holds it, and to the
// first triangle of that leaf (listing order) that contains it, boundary
// included. Weights are orient(p, b, c) / orient(a, b, c) and cyclic; the
// denominators are powers of two, so the weights are exact.
constexpr int kMaxLeafTri = 8;

struct LeafTris {
  int nt;
  int t0;
  int ax[kMaxLeafTri], ay[kMaxLeafTri], bx[kMaxLeafTri], by[kMaxLeafTri], cx[kMaxLeafTri],
      cy[kMaxLeafTri];
  int va[kMaxLeafTri], vb[kMaxLeafTri], vc[kMaxLeafTri];
  double inv[kMaxLeafTri];
};

__device__ __forceinline__ void load_leaf(const int32_t* __restrict__ leaves, int64_t i,
                                          const int32_t* __restrict__ tri,
                                          const int32_t* __restrict__ vxy, LeafTris& L) {
  L.t0 = leaves[4 * i + 3];
  L.nt = leaves[4 * i + 7] - L.t0;
#pragma unroll
  for (int k = 0; k < kMaxLeafTri; ++k) {
    if (k < L.nt) {
      const int t = L.t0 + k;
      L.va[k] = tri[3 * t];
      L.vb[k] = tri[3 * t + 1];
      L.vc[k] = tri[3 * t + 2];
      L.ax[k] = vxy[2 * L.va[k]]; L.ay[k] = vxy[2 * L.va[k] + 1];
      L.bx[k] = vxy[2 * L.vb[k]]; L.by[k] = vxy[2 * L.vb[k] + 1];
      L.cx[k] = vxy[2 * L.vc[k]]; L.cy[k] = vxy[2 * L.vc[k] + 1];
      const int den = (L.bx[k] - L.ax[k]) * (L.cy[k] - L.ay[k]) - (L.by[k] - L.ay[k]) * (L.cx[k] - L.ax[k]);
      L.inv[k] = 1.0 / (double)den;
    }
  }
}

// orientation numerators of point (x, y) against triangle k; owner is the
// first k with all three >= 0
__device__ __forceinline__ int locate(const LeafTris& L, int x, int y, int& oa, int& ob, int& oc) {
  int own = -1;
#pragma unroll
  for (int k = 0; k < kMaxLeafTri; ++k) {
    if (own < 0 && k < L.nt) {
      const int a = (L.bx[k] - x) * (L.cy[k] - y) - (L.by[k] - y) * (L.cx[k] - x);
      const int b = (L.cx[k] - x) * (L.ay[k] - y) - (L.cy[k] - y) * (L.ax[k] - x);
      const int c = (L.ax[k] - x) * (L.by[k] - y) - (L.ay[k] - y) * (L.bx[k] - x);
      if (a >= 0 && b >= 0 && c >= 0) { own = k; oa = a; ob = b; oc = c; }
    }
  }
  return own;
}

__global__ __launch_bounds__(kBlock) void k_raster(
    int64_t nleaves, int N, const int32_t* __restrict__ leaves, const int32_t* __restrict__ tri,
    const int32_t* __restrict__ vxy, const double* __restrict__ uv, const double* __restrict__ u_in,
    const uint8_t* __restrict__ f, double* __restrict__ u_out, double* __restrict__ e_out, double* __restrict__ tri_err,
    int32_t* __restrict__ owner_out, double* __restrict__ partial) {
  __shared__ double lds[4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc[1] = {0.0};
  if (i < nleaves) {
    LeafTris L;
    load_leaf(leaves, i, tri, vxy, L);
    double ua[kMaxLeafTri], ub[kMaxLeafTri], uc[kMaxLeafTri], E[kMaxLeafTri];
#pragma unroll
    for (int k = 0; k < kMaxLeafTri; ++k) {
      E[k] = 0.0;
      if (k < L.nt && uv) { ua[k] = uv[L.va[k]]; ub[k] = uv[L.vb[k]]; uc[k] = uv[L.vc[k]]; }
      else { ua[k] = ub[k] = uc[k] = 0.0; }
    }
    const int x0 = leaves[4 * i], y0 = leaves[4 * i + 1];
    const int s = 1 << leaves[4 * i + 2];
    for (int dy = 0; dy < s; ++dy) {
      for (int dx = 0; dx < s; ++dx) {
        const int x = x0 + dx, y = y0 + dy;
        int oa = 0, ob = 0, oc = 0;
        const int own = locate(L, x, y, oa, ob, oc);
        double u = 0.0, ia = 0.0;
        int tk = 0;
#pragma unroll
        for (int k = 0; k < kMaxLeafTri; ++k) {
          if (k == own) {
            ia = L.inv[k];
            u = ((double)oa * ia) * ua[k] + ((double)ob * ia) * ub[k] + ((double)oc * ia) * uc[k];
            tk = k;
          }
        }
        const int64_t pix = (int64_t)y * N + x;
        if (u_in) u = u_in[pix];
        if (u_out) u_out[pix] = u;
        if (owner_out) owner_out[pix] = L.t0 + tk;
        if (f) {
          const double dlt = u - (double)f[pix];
          const double e = dlt * dlt;
          if (e_out) e_out[pix] = e;
          acc[0] += e;
#pragma unroll
          for (int k = 0; k < kMaxLeafTri; ++k)
            if (k == tk) E[k] += e;
        }
      }
    }
    if (f && tri_err) {
#pragma unroll
      for (int k = 0; k < kMaxLeafTri; ++k)
        if (k < L.nt) tri_err[L.t0 + k] = E[k];
    }
  }
  block_sum<1>(acc, lds);
  if (partial && threadIdx.x == 0) partial[blockIdx.x] = acc[0];
}

// ------------------------------------------------- pixel-major passes ----
// The leaf-major kernels above give one thread a whole leaf; the passes below
// give one thread a pixel (interpolation, error) or a triangle's pixel list
// (the transposed interpolation), with the owner of every pixel found once
// per mesh by the leaf-major rule.

// Per leaf: how many pixels each of its triangles owns.
__global__ __launch_bounds__(kBlock) void k_tri_count(int64_t nleaves,
                                                      const int32_t* __restrict__ leaves,
                                                      const int32_t* __restrict__ tri,
                                                      const int32_t* __restrict__ vxy,
                                                      int32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nleaves) return;
  LeafTris L;
  load_leaf(leaves, i, tri, vxy, L);
  int c[kMaxLeafTri];
#pragma unroll
  for (int k = 0; k < kMaxLeafTri; ++k) c[k] = 0;
  const int x0 = leaves[4 * i], y0 = leaves[4 * i + 1];
  const int s = 1 << leaves[4 * i + 2];
  for (int dy = 0; dy < s; ++dy) {
    for (int dx = 0; dx < s; ++dx) {
      int oa, ob, oc;
      const int own = max(0, locate(L, x0 + dx, y0 + dy, oa, ob, oc));  // (always >= 0)
#pragma unroll
      for (int k = 0; k < kMaxLeafTri; ++k) c[k] += k == own;
    }
  }
#pragma unroll
  for (int k = 0; k < kMaxLeafTri; ++k)
    if (k < L.nt) cnt[L.t0 + k] = c[k];
}

// Per leaf: its pixels into their owners' lists, ascending, and the owner map.
__global__ __launch_bounds__(kBlock) void k_tri_fill(int64_t nleaves, int N,
                                                     const int32_t* __restrict__ leaves,
                                                     const int32_t* __restrict__ tri,
                                                     const int32_t* __restrict__ vxy,
                                                     const int32_t* __restrict__ ptr,
                                                     int32_t* __restrict__ px,
                                                     int32_t* __restrict__ owner) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nleaves) return;
  LeafTris L;
  load_leaf(leaves, i, tri, vxy, L);
  int cur[kMaxLeafTri];
#pragma unroll
  for (int k = 0; k < kMaxLeafTri; ++k) cur[k] = k < L.nt ? ptr[L.t0 + k] : 0;
  const int x0 = leaves[4 * i], y0 = leaves[4 * i + 1];
  const int s = 1 << leaves[4 * i + 2];
  for (int dy = 0; dy < s; ++dy) {
    for (int dx = 0; dx < s; ++dx) {
      int oa, ob, oc;
      const int own = max(0, locate(L, x0 + dx, y0 + dy, oa, ob, oc));  // (always >= 0)
      const int32_t pix = (y0 + dy) * N + (x0 + dx);
      owner[pix] = L.t0 + own;
#pragma unroll
      for (int k = 0; k < kMaxLeafTri; ++k) {
        if (k == own) {
          px[cur[k]] = pix;
          ++cur[k];
        }
      }
    }
  }
}

// ------------------------------------------- Delaunay-mesh pixel maps ----
// Without leaves, a pixel's owner is the lowest-index triangle that holds it
// (boundary included). Work is split into (triangle, bounding-box row)
// items, so a large triangle does not serialise one thread: item g belongs
// to the triangle t with rowstart[t] <= g < rowstart[t + 1] and covers row
// y0(t) + g - rowstart[t] of its box.

struct TriBox {
  int ax, ay, bx, by, cx, cy, x0, x1;
};

__device__ __forceinline__ int item_triangle(const int32_t* __restrict__ rowstart, int T,
                                             int64_t g) {
  int lo = 0, hi = T - 1;  // last t with rowstart[t] <= g
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rowstart[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ TriBox tri_box(const int32_t* __restrict__ tri,
                                          const int32_t* __restrict__ vxy, int t) {
  TriBox B;
  const int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
  B.ax = vxy[2 * a]; B.ay = vxy[2 * a + 1];
  B.bx = vxy[2 * b]; B.by = vxy[2 * b + 1];
  B.cx = vxy[2 * c]; B.cy = vxy[2 * c + 1];
  B.x0 = min(B.ax, min(B.bx, B.cx));
  B.x1 = max(B.ax, max(B.bx, B.cx));
  return B;
}

__device__ __forceinline__ bool tri_holds(const TriBox& B, int x, int y) {
  const int64_t o1 = (int64_t)(B.bx - B.ax) * (y - B.ay) - (int64_t)(B.by - B.ay) * (x - B.ax);
  const int64_t o2 = (int64_t)(B.cx - B.bx) * (y - B.by) - (int64_t)(B.cy - B.by) * (x - B.bx);
  const int64_t o3 = (int64_t)(B.ax - B.cx) * (y - B.cy) - (int64_t)(B.ay - B.cy) * (x - B.cx);
  return o1 >= 0 && o2 >= 0 && o3 >= 0;
}

// Rows of each triangle's bounding box (the item counts).
__global__ __launch_bounds__(kBlock) void k_dt_rows(int T, const int32_t* __restrict__ tri,
                                                    const int32_t* __restrict__ vxy,
                                                    int32_t* __restrict__ rows) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t > T) return;
  if (t == T) { rows[T] = 0; return; }
  const int a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
  const int ya = vxy[2 * a + 1], yb = vxy[2 * b + 1], yc = vxy[2 * c + 1];
  rows[t] = max(ya, max(yb, yc)) - min(ya, min(yb, yc)) + 1;
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int64_t n, int32_t v, int32_t* __restrict__ a) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) a[i] = v;
}

// owner[p] = min over triangles holding p (integer minimum: any order).
__global__ __launch_bounds__(kBlock) void k_dt_owner(int64_t items, int T, int N,
                                                     const int32_t* __restrict__ rowstart,
                                                     const int32_t* __restrict__ tri,
                                                     const int32_t* __restrict__ vxy,
                                                     int32_t* __restrict__ owner) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= items) return;
  const int t = item_triangle(rowstart, T, g);
  const TriBox B = tri_box(tri, vxy, t);
  const int y = min(B.ay, min(B.by, B.cy)) + (int)(g - rowstart[t]);
  for (int x = B.x0; x <= B.x1; ++x)
    if (tri_holds(B, x, y)) atomicMin(&owner[(int64_t)y * N + x], t);
}

// Pixels of row item g that its triangle owns.
__global__ __launch_bounds__(kBlock) void k_dt_count(int64_t items, int T, int N,
                                                     const int32_t* __restrict__ rowstart,
                                                     const int32_t* __restrict__ tri,
                                                     const int32_t* __restrict__ vxy,
                                                     const int32_t* __restrict__ owner,
                                                     int32_t* __restrict__ cnt) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g > items) return;
  if (g == items) { cnt[items] = 0; return; }
  const int t = item_triangle(rowstart, T, g);
  const TriBox B = tri_box(tri, vxy, t);
  const int y = min(B.ay, min(B.by, B.cy)) + (int)(g - rowstart[t]);
  int c = 0;
  for (int x = B.x0; x <= B.x1; ++x) c += owner[(int64_t)y * N + x] == t;
  cnt[g] = c;
}

// The owned pixels of row item g at their offset: rows ascend within a
// triangle and x within a row, so every list is in ascending pixel order.
__global__ __launch_bounds__(kBlock) void k_dt_fill(int64_t items, int T, int N,
                                                    const int32_t* __restrict__ rowstart,
                                                    const int32_t* __restrict__ tri,
                                                    const int32_t* __restrict__ vxy,
                                                    const int32_t* __restrict__ owner,
                                                    const int32_t* __restrict__ off,
                                                    int32_t* __restrict__ px) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= items) return;
  const int t = item_triangle(rowstart, T, g);
  const TriBox B = tri_box(tri, vxy, t);
  const int y = min(B.ay, min(B.by, B.cy)) + (int)(g - rowstart[t]);
  int pos = off[g];
  for (int x = B.x0; x <= B.x1; ++x) {
    const int64_t p = (int64_t)y * N + x;
    if (owner[p] == t) px[pos++] = (int32_t)p;
  }
}

// Start of each triangle's list: the offset of its first row item.
__global__ __launch_bounds__(kBlock) void k_dt_ptr(int T, int64_t items,
                                                   const int32_t* __restrict__ rowstart,
                                                   const int32_t* __restrict__ off,
                                                   int32_t* __restrict__ ptr) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t > T) return;
  ptr[t] = off[t < T ? rowstart[t] : items];
}

// Per triangle over its pixel list (ascending): the total squared error
// (from e, or from u and f), and, when in_mask is given, its pixel of
// largest e outside the mask (ties: lower index; -1 if none).
__global__ __launch_bounds__(kBlock) void k_tri_err_list(int64_t T,
                                                         const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ px,
                                                         const double* __restrict__ e,
                                                         const double* __restrict__ u,
                                                         const uint8_t* __restrict__ f,
                                                         const uint8_t* __restrict__ in_mask,
                                                         double* __restrict__ tri_err,
                                                         int32_t* __restrict__ tri_best) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= T) return;
  double E = 0.0, bv = -1.0;
  int32_t best = -1;
  const int j1 = ptr[t + 1];
  for (int j = ptr[t]; j < j1; ++j) {
    const int p = px[j];
    double ep;
    if (e) {
      ep = e[p];
    } else {
      const double d = u[p] - (double)f[p];
      ep = d * d;
    }
    E += ep;
    if (in_mask && !in_mask[p] && ep > bv) {
      bv = ep;
      best = p;
    }
  }
  tri_err[t] = E;
  if (tri_best) tri_best[t] = best;
}

// u at every pixel from the vertex values (one thread per pixel; the weights
// are formed exactly as in the leaf-major pass).
__device__ __forceinline__ double interp_at(int64_t p, int logN, const int32_t* __restrict__ owner,
                                            const int32_t* __restrict__ tri,
                                            const int32_t* __restrict__ vxy,
                                            const double* __restrict__ uv) {
  const int t = owner[p];
  const int x = (int)(p & ((1 << logN) - 1)), y = (int)(p >> logN);
  const int va = tri[3 * t], vb = tri[3 * t + 1], vc = tri[3 * t + 2];
  const int ax = vxy[2 * va], ay = vxy[2 * va + 1];
  const int bx = vxy[2 * vb], by = vxy[2 * vb + 1];
  const int cx = vxy[2 * vc], cy = vxy[2 * vc + 1];
  const int den = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
  const double ia = 1.0 / (double)den;
  const int oa = (bx - x) * (cy - y) - (by - y) * (cx - x);
  const int ob = (cx - x) * (ay - y) - (cy - y) * (ax - x);
  const int oc = (ax - x) * (by - y) - (ay - y) * (bx - x);
  return ((double)oa * ia) * uv[va] + ((double)ob * ia) * uv[vb] + ((double)oc * ia) * uv[vc];
}

__global__ __launch_bounds__(kBlock) void k_interp_px(int64_t P, int logN,
                                                      const int32_t* __restrict__ owner,
                                                      const int32_t* __restrict__ tri,
                                                      const int32_t* __restrict__ vxy,
                                                      const double* __restrict__ uv,
                                                      double* __restrict__ u_out) {
  const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (p >= P) return;
  u_out[p] = interp_at(p, logN, owner, tri, vxy, uv);
}

// k_interp_px with the per-block partial sums of u_out^2 that k_dot_part
// would take of it (the same grid-stride loop over the same grid), so
// their sum has the bits of the separate dot product.
__global__ __launch_bounds__(kBlock) void k_interp_px_sq(int64_t P, int logN,
                                                         const int32_t* __restrict__ owner,
                                                         const int32_t* __restrict__ tri,
                                                         const int32_t* __restrict__ vxy,
                                                         const double* __restrict__ uv,
                                                         double* __restrict__ u_out,
                                                         double* __restrict__ part) {
  __shared__ double lds[4];
  double v[1] = {0.0};
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * kBlock) {
    const double u = interp_at(p, logN, owner, tri, vxy, uv);
    u_out[p] = u;
    v[0] += u * u;
  }
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// e = (u - f)^2 per pixel and per-block partial sums; `nblocks` blocks cover
// the pixels grid-stride, so the number of partial sums is fixed by the mesh.
__global__ __launch_bounds__(kBlock) void k_err_px(int64_t P, const double* __restrict__ u,
                                                   const uint8_t* __restrict__ f,
                                                   double* __restrict__ e_out,
                                                   double* __restrict__ partial) {
  __shared__ double lds[4];
  double acc[1] = {0.0};
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * kBlock) {
    const double d = u[p] - (double)f[p];
    const double e = d * d;
    if (e_out) e_out[p] = e;
    acc[0] += e;
  }
  block_sum<1>(acc, lds);
  if (partial && threadIdx.x == 0) partial[blockIdx.x] = acc[0];
}

// Transposed interpolation, one thread per triangle over its pixel list (in
// ascending pixel order, as the leaf-major pass adds them).
// WEIGHTED: the residual is scaled by w per pixel first (R^T (w r)).
template <bool WEIGHTED>
__global__ __launch_bounds__(kBlock) void k_interp_T_tri(int64_t T, int logN,
                                                         const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ px,
                                                         const int32_t* __restrict__ tri,
                                                         const int32_t* __restrict__ vxy,
                                                         const double* __restrict__ r,
                                                         const double* __restrict__ w,
                                                         double* __restrict__ tpart) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= T) return;
  const int va = tri[3 * t], vb = tri[3 * t + 1], vc = tri[3 * t + 2];
  const int ax = vxy[2 * va], ay = vxy[2 * va + 1];
  const int bx = vxy[2 * vb], by = vxy[2 * vb + 1];
  const int cx = vxy[2 * vc], cy = vxy[2 * vc + 1];
  const int den = (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
  const double ia = 1.0 / (double)den;
  double Sa = 0.0, Sb = 0.0, Sc = 0.0;
  const int j1 = ptr[t + 1];
  for (int j = ptr[t]; j < j1; ++j) {
    const int p = px[j];
    const int x = p & ((1 << logN) - 1), y = p >> logN;
    const int oa = (bx - x) * (cy - y) - (by - y) * (cx - x);
    const int ob = (cx - x) * (ay - y) - (cy - y) * (ax - x);
    const int oc = (ax - x) * (by - y) - (ay - y) * (bx - x);
    const double rv = WEIGHTED ? r[p] * w[p] : r[p];
    Sa += ((double)oa * ia) * rv;
    Sb += ((double)ob * ia) * rv;
    Sc += ((double)oc * ia) * rv;
  }
  tpart[3 * t] = Sa;
  tpart[3 * t + 1] = Sb;
  tpart[3 * t + 2] = Sc;
}

// Per triangle: the total squared error of the pixels it owns (added in
// ascending pixel order), and its pixel of largest error that is not in the
// mask (ties: the lower index; -1 if it owns none). Section 3's inputs to the
// densification step.
__global__ __launch_bounds__(kBlock) void k_tri_best(int64_t nleaves, int N,
                                                     const int32_t* __restrict__ leaves,
                                                     const int32_t* __restrict__ tri,
                                                     const int32_t* __restrict__ vxy,
                                                     const double* __restrict__ e,
                                                     const uint8_t* __restrict__ in_mask,
                                                     double* __restrict__ tri_err,
                                                     int32_t* __restrict__ tri_best) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nleaves) return;
  LeafTris L;
  load_leaf(leaves, i, tri, vxy, L);
  double E[kMaxLeafTri], bestv[kMaxLeafTri];
  int32_t best[kMaxLeafTri];
#pragma unroll
  for (int k = 0; k < kMaxLeafTri; ++k) {
    E[k] = 0.0;
    bestv[k] = 0.0;
    best[k] = -1;
  }
  const int x0 = leaves[4 * i], y0 = leaves[4 * i + 1];
  const int s = 1 << leaves[4 * i + 2];
  for (int dy = 0; dy < s; ++dy) {
    for (int dx = 0; dx < s; ++dx) {
      const int x = x0 + dx, y = y0 + dy;
      int oa = 0, ob = 0, oc = 0;
      const int own = locate(L, x, y, oa, ob, oc);
      const int64_t pix = (int64_t)y * N + x;
      const double ev = e[pix];
      const bool empty = !in_mask[pix];
#pragma unroll
      for (int k = 0; k < kMaxLeafTri; ++k) {
        if (k == own) {
          E[k] += ev;
          // pixels come in ascending order, so a strictly larger error wins
          if (empty && (best[k] < 0 || ev > bestv[k])) {
            best[k] = (int32_t)pix;
            bestv[k] = ev;
          }
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kMaxLeafTri; ++k) {
    if (k < L.nt) {
      tri_err[L.t0 + k] = E[k];
      tri_best[L.t0 + k] = best[k];
    }
  }
}

// t_v = sum over (triangle, corner) pairs at v of the partial sums, in the
// fixed ascending order of the adjacency list; split into free and mask parts.
__global__ __launch_bounds__(kBlock) void k_gather_vertex(int V, const int32_t* __restrict__ vt_ptr,
                                                          const int32_t* __restrict__ vt_idx,
                                                          const int32_t* __restrict__ vmap,
                                                          const double* __restrict__ tpart,
                                                          double* __restrict__ tF,
                                                          double* __restrict__ tD) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  double acc = 0.0;
  const int e0 = vt_ptr[v], e1 = vt_ptr[v + 1];
  if (e1 - e0 <= kMaxIncident) {
    // all loads first (quadtree lists are this short), then the sum in order
    double t[kMaxIncident];
#pragma unroll
    for (int q = 0; q < kMaxIncident; ++q) t[q] = tpart[vt_idx[min(e0 + q, e1 - 1)]];
#pragma unroll
    for (int q = 0; q < kMaxIncident; ++q)
      if (e0 + q < e1) acc += t[q];
  } else {
    for (int e = e0; e < e1; ++e) acc += tpart[vt_idx[e]];
  }
  const int32_t mv = vmap[v];
  if (mv >= 0) tF[mv] = acc; else tD[-mv - 1] = acc;
}

// s = t_D - K_DF y
__global__ __launch_bounds__(kBlock) void k_adjoint_tail(int m, const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ val,
                                                         const double* __restrict__ tD,
                                                         const double* __restrict__ y,
                                                         double* __restrict__ s) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double acc = 0.0;
  for (int q = ptr[j]; q < ptr[j + 1]; ++q) acc += val[q] * y[col[q]];
  s[j] = tD[j] - acc;
}

// ------------------------------------------------------ vector kernels ----
// out[c] = (sum of component c over the partials) / div.
__global__ __launch_bounds__(kBlock) void k_reduce(const double* __restrict__ part, int nparts,
                                                   int ncomp, double div, double* __restrict__ out) {
  __shared__ double lds[4];
  for (int c = 0; c < ncomp; ++c) {
    double v[1] = {0.0};
    for (int j = threadIdx.x; j < nparts; j += kBlock) v[0] += part[(int64_t)j * ncomp + c];
    block_sum<1>(v, lds);
    if (threadIdx.x == 0) out[c] = v[0] / div;
  }
}

__global__ __launch_bounds__(kBlock) void k_dot_part(const double* __restrict__ a,
                                                     const double* __restrict__ b, int64_t n,
                                                     double* __restrict__ part) {
  __shared__ double lds[4];
  double v[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    v[0] += a[i] * b[i];
  block_sum<1>(v, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = v[0];
}

// Ratio of two device scalars, or 0 when the denominator is not positive
// (a step of length zero where CG would divide by zero).
__device__ __forceinline__ double ratio(const double* num, const double* den) {
  const double d = *den;
  return d > 0.0 ? *num / d : 0.0;
}

// y += sign * (num / den) x
__global__ __launch_bounds__(kBlock) void k_axpy_ratio(int64_t n, const double* __restrict__ num,
                                                       const double* __restrict__ den, double sign,
                                                       const double* __restrict__ x,
                                                       double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] += sign * ratio(num, den) * x[i];
}

// y1 += (num / den) x1 on [0, n1) and y2 -= (num / den) x2 on [0, n2), the
// two updates of k_axpy_ratio (signs 1 and -1) in one launch.
__global__ __launch_bounds__(kBlock) void k_axpy2_ratio(int64_t n1, int64_t n2,
                                                        const double* __restrict__ num,
                                                        const double* __restrict__ den,
                                                        const double* __restrict__ x1,
                                                        double* __restrict__ y1,
                                                        const double* __restrict__ x2,
                                                        double* __restrict__ y2) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n1) y1[i] += 1.0 * ratio(num, den) * x1[i];
  if (i < n2) y2[i] += -1.0 * ratio(num, den) * x2[i];
}

// y = x + (num / den) y
__global__ __launch_bounds__(kBlock) void k_xpby_ratio(int64_t n, const double* __restrict__ x,
                                                       const double* __restrict__ num,
                                                       const double* __restrict__ den,
                                                       double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = x[i] + ratio(num, den) * y[i];
}

__global__ __launch_bounds__(kBlock) void k_pixel_residual(int64_t P, const uint8_t* __restrict__ f,
                                                           const double* __restrict__ u,
                                                           double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < P) r[i] = (double)f[i] - u[i];
}

// Pixel-space factor of the MSE gradient: r = c (u - f) with c = 2 s / P,
// s = *scale (the caller's d loss / d MSE) or 1. Section 4: the gradient of
// MSE(g) = ||B g - f||^2 / P is (2 / P) B^T (B g - f), so B^T r is s times it.
__global__ __launch_bounds__(kBlock) void k_mse_residual(int64_t P, const uint8_t* __restrict__ f,
                                                         const double* __restrict__ u,
                                                         const double* __restrict__ scale,
                                                         double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < P) {
    const double c = 2.0 * (scale ? *scale : 1.0) / (double)P;
    r[i] = c * (u[i] - (double)f[i]);
  }
}

// Weighted residual r = w (f - u).
__global__ __launch_bounds__(kBlock) void k_pixel_residual_w(int64_t P,
                                                             const uint8_t* __restrict__ f,
                                                             const double* __restrict__ u,
                                                             const double* __restrict__ w,
                                                             double* __restrict__ r) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < P) r[i] = w[i] * ((double)f[i] - u[i]);
}

// x *= w elementwise.
__global__ __launch_bounds__(kBlock) void k_scale(int64_t n, const double* __restrict__ w,
                                                  double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) x[i] = w[i] * x[i];
}

// IRLS weights: w^(1/2) = sqrt(1 / max(|f - u|, eps)).
__global__ __launch_bounds__(kBlock) void k_irls_weights(int64_t P, const uint8_t* __restrict__ f,
                                                         const double* __restrict__ u,
                                                         double eps,
                                                         double* __restrict__ wsqrt) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < P) wsqrt[i] = sqrt(1.0 / fmax(fabs((double)f[i] - u[i]), eps));
}

// Per-block partial sums of |u - f| (grid-stride, like k_err_px).
__global__ __launch_bounds__(kBlock) void k_abs_err(int64_t P, const double* __restrict__ u,
                                                    const uint8_t* __restrict__ f,
                                                    double* __restrict__ partial) {
  __shared__ double lds[4];
  double acc[1] = {0.0};
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < P;
       p += (int64_t)gridDim.x * kBlock)
    acc[0] += fabs(u[p] - (double)f[p]);
  block_sum<1>(acc, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc[0];
}

}  // namespace

// ------------------------------------------------------------ launchers ----
#define FI_LAUNCH_CHECK() FI_HIP_TRY(hipGetLastError())

template <int NB>
int assemble_count(fi_mesh* M, bool free_rows) {
  hipStream_t st = M->ctx->stream;
  if (free_rows) {
    hipLaunchKernelGGL(k_asm_free_count<NB>, dim3(grid_for(M->n + 1)), dim3(kBlock), 0, st,
                       (int)M->n, M->d_free_vids, M->d_vxy, M->d_tri, M->d_vt_ptr, M->d_vt_idx,
                       M->d_vmap, M->d_cnt, M->d_cnt + (M->n + 1));
  } else {
    hipLaunchKernelGGL(k_asm_mask_count<NB>, dim3(grid_for(M->m + 1)), dim3(kBlock), 0, st,
                       (int)M->m, M->d_mask_vids, M->d_vxy, M->d_tri, M->d_vt_ptr, M->d_vt_idx,
                       M->d_vmap, M->d_cnt);
  }
  FI_LAUNCH_CHECK();
  return FI_OK;
}

template <int NB>
int assemble_fill(fi_mesh* M, bool free_rows) {
  hipStream_t st = M->ctx->stream;
  if (free_rows) {
    hipLaunchKernelGGL(k_asm_free_fill<NB>, dim3(grid_for(M->n)), dim3(kBlock), 0, st, (int)M->n,
                       M->d_free_vids, M->d_vxy, M->d_tri, M->d_vt_ptr, M->d_vt_idx, M->d_vmap,
                       M->d_ff_rowptr, M->d_ff_col, M->d_ff_val64, M->d_ff_val32, M->d_fd_rowptr,
                       M->d_fd_col, M->d_fd_val, M->d_diag64, M->d_dinv64, M->d_dinv32);
  } else {
    hipLaunchKernelGGL(k_asm_mask_fill<NB>, dim3(grid_for(M->m)), dim3(kBlock), 0, st, (int)M->m,
                       M->d_mask_vids, M->d_vxy, M->d_tri, M->d_vt_ptr, M->d_vt_idx, M->d_vmap,
                       M->d_df_rowptr, M->d_df_col, M->d_df_val);
  }
  FI_LAUNCH_CHECK();
  return FI_OK;
}

template <int NB>
int assemble_refill(fi_mesh* M) {
  RefillArgs A;
  A.n = (int)M->n;
  A.m = (int)M->m;
  A.free_blocks = grid_for(M->n);
  A.n_pad = (int)M->n_pad;
  A.W = M->ell_w;
  A.free_vids = M->d_free_vids;
  A.mask_vids = M->d_mask_vids;
  A.vxy = M->d_vxy;
  A.tri = M->d_tri;
  A.vt_ptr = M->d_vt_ptr;
  A.vt_idx = M->d_vt_idx;
  A.vmap = M->d_vmap;
  A.ff_ptr = M->d_ff_rowptr;
  A.ff_col = M->d_ff_col;
  A.ff_val64 = M->d_ff_val64;
  A.ff_val32 = M->d_ff_val32;
  A.fd_ptr = M->d_fd_rowptr;
  A.fd_col = M->d_fd_col;
  A.fd_val = M->d_fd_val;
  A.diag64 = M->d_diag64;
  A.dinv64 = M->d_dinv64;
  A.dinv32 = M->d_dinv32;
  A.df_ptr = M->d_df_rowptr;
  A.df_col = M->d_df_col;
  A.df_val = M->d_df_val;
  A.ell = M->ell_w > 0 ? M->d_ell : nullptr;
  const int grid = A.free_blocks + grid_for(M->m);
  hipLaunchKernelGGL(k_asm_refill<NB>, dim3(grid), dim3(kBlock), 0, M->ctx->stream, A);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

// A row has at most (incident triangles + 1) neighbours.
int launch_assemble_count(fi_mesh* M, bool free_rows) {
  return M->host.delaunay ? assemble_count<kMaxIncidentGeneral + 1>(M, free_rows)
                          : assemble_count<kMaxIncident>(M, free_rows);
}

int launch_assemble_fill(fi_mesh* M, bool free_rows) {
  return M->host.delaunay ? assemble_fill<kMaxIncidentGeneral + 1>(M, free_rows)
                          : assemble_fill<kMaxIncident>(M, free_rows);
}

int launch_assemble_refill(fi_mesh* M) {
  return M->host.delaunay ? assemble_refill<kMaxIncidentGeneral + 1>(M)
                          : assemble_refill<kMaxIncident>(M);
}

int scan_counts(fi_mesh* M, const int32_t* cnt, int32_t* rowptr, int64_t n_plus_1) {
  return scan_rec(M->ctx->stream, cnt, rowptr, n_plus_1, M->d_scan_tmp);
}

int scan_exclusive(hipStream_t st, const int32_t* in, int32_t* out, int64_t n, int32_t* tmp) {
  return scan_rec(st, in, out, n, tmp);
}

int64_t scan_tmp_ints(int64_t n) {
  int64_t total = 0, t = n;
  for (;;) {
    t = (t + kScanTile - 1) / kScanTile;
    total += 2 * t + 2;
    if (t <= 1) break;
  }
  return total + 16;
}

int launch_lift(fi_mesh* M, const double* g, double* b) {
  if (M->n == 0) return FI_OK;
  hipLaunchKernelGGL(k_lift, dim3(grid_for(M->n)), dim3(kBlock), 0, M->ctx->stream, (int)M->n,
                     M->d_fd_rowptr, M->d_fd_col, M->d_fd_val, g, b);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

int launch_gather_mask(fi_mesh* M, const uint8_t* f, double* g) {
  hipLaunchKernelGGL(k_gather_mask, dim3(grid_for(M->m)), dim3(kBlock), 0, M->ctx->stream,
                     (int)M->m, M->d_mask_pix, f, g);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

int launch_vertex_values(fi_mesh* M, const double* xF, const double* g, double* uvert) {
  hipLaunchKernelGGL(k_vertex_values, dim3(grid_for(M->V)), dim3(kBlock), 0, M->ctx->stream,
                     (int)M->V, M->d_vmap, xF, g, uvert);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

// Interpolation and error passes on a mesh without leaves: pixel-major,
// then the per-triangle sums over the pixel lists and a copy of the owner map.
int raster_general(fi_mesh* M, const double* uvert, const double* u_in, const uint8_t* f,
                   double* u_out, double* e_out, double* tri_err_out, int32_t* owner_out,
                   double* partial_out) {
  hipStream_t st = M->ctx->stream;
  const double* u = u_in;
  if (!u_in && (u_out || f)) {
    if (!uvert) return fail(FI_E_INVALID, "interpolation without vertex values");
    if (!u_out) return fail(FI_E_INVALID, "error of interpolated values needs an output");
    hipLaunchKernelGGL(k_interp_px, dim3(grid_for(M->P)), dim3(kBlock), 0, st, M->P,
                       M->host.levels, M->d_owner, M->d_tri, M->d_vxy, uvert, u_out);
    FI_LAUNCH_CHECK();
    u = u_out;
  } else if (u_in && u_out && u_out != u_in) {
    FI_HIP_TRY(hipMemcpyAsync(u_out, u_in, (size_t)M->P * sizeof(double),
                              hipMemcpyDeviceToDevice, st));
  }
  if (f) {
    hipLaunchKernelGGL(k_err_px, dim3(raster_blocks(M)), dim3(kBlock), 0, st, M->P, u, f, e_out,
                       partial_out);
    FI_LAUNCH_CHECK();
    if (tri_err_out) {
      hipLaunchKernelGGL(k_tri_err_list, dim3(grid_for(M->T)), dim3(kBlock), 0, st, M->T,
                         M->d_tri_px_ptr, M->d_tri_px, (const double*)nullptr, u, f,
                         (const uint8_t*)nullptr, tri_err_out, (int32_t*)nullptr);
      FI_LAUNCH_CHECK();
    }
  }
  if (owner_out)
    FI_HIP_TRY(hipMemcpyAsync(owner_out, M->d_owner, (size_t)M->P * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, st));
  return FI_OK;
}

int launch_raster(fi_mesh* M, const double* uvert, const double* u_in, const uint8_t* f,
                  double* u_out, double* e_out, double* tri_err_out, int32_t* owner_out,
                  double* partial_out) {
  hipStream_t st = M->ctx->stream;
  if (M->host.delaunay) return raster_general(M, uvert, u_in, f, u_out, e_out, tri_err_out,
                                              owner_out, partial_out);
  if (tri_err_out || owner_out || !M->d_owner || (u_in && u_out)) {
    // per-triangle sums and the owner map need the leaf-major pass
    hipLaunchKernelGGL(k_raster, dim3(grid_for(M->L)), dim3(kBlock), 0, st, M->L, M->N,
                       M->d_leaves, M->d_tri, M->d_vxy, uvert, u_in, f, u_out, e_out,
                       tri_err_out, owner_out, partial_out);
    FI_LAUNCH_CHECK();
    return FI_OK;
  }
  const double* u = u_in;
  if (!u_in && u_out) {
    if (!uvert) return fail(FI_E_INVALID, "interpolation without vertex values");
    hipLaunchKernelGGL(k_interp_px, dim3(grid_for(M->P)), dim3(kBlock), 0, st, M->P,
                       M->host.levels, M->d_owner, M->d_tri, M->d_vxy, uvert, u_out);
    FI_LAUNCH_CHECK();
    u = u_out;
  }
  if (f) {
    if (!u) return fail(FI_E_INVALID, "error without pixel values");
    hipLaunchKernelGGL(k_err_px, dim3(raster_blocks(M)), dim3(kBlock), 0, st, M->P, u, f, e_out,
                       partial_out);
    FI_LAUNCH_CHECK();
  }
  return FI_OK;
}

// Temporary device memory of one call (freed on every return path).
struct DevTmp {
  int32_t* p = nullptr;
  ~DevTmp() {
    if (p) (void)hipFree(p);
  }
};

// Owner map and pixel lists of a mesh without leaves (see k_dt_owner).
int build_pixel_maps_general(fi_mesh* M) {
  hipStream_t st = M->ctx->stream;
  const int T = (int)M->T;
  DevTmp rows, tmp, off;
  // item counts and their starts (kept in the list-start array until the end)
  FI_HIP_TRY(hipMalloc(&rows.p, (size_t)(T + 1) * sizeof(int32_t)));
  FI_HIP_TRY(hipMalloc(&tmp.p, (size_t)scan_tmp_ints(T + 1) * sizeof(int32_t)));
  int32_t* rowstart = M->d_tri_px_ptr;
  hipLaunchKernelGGL(k_dt_rows, dim3(grid_for(T + 1)), dim3(kBlock), 0, st, T, M->d_tri,
                     M->d_vxy, rows.p);
  FI_LAUNCH_CHECK();
  int rc = scan_exclusive(st, rows.p, rowstart, T + 1, tmp.p);
  if (rc) return rc;
  int32_t items32 = 0;
  FI_HIP_TRY(hipMemcpyAsync(&items32, rowstart + T, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  FI_HIP_TRY(hipStreamSynchronize(st));
  const int64_t items = items32;
  FI_HIP_TRY(hipFree(tmp.p));
  tmp.p = nullptr;
  FI_HIP_TRY(hipMalloc(&off.p, (size_t)(items + 1) * sizeof(int32_t) * 2));
  FI_HIP_TRY(hipMalloc(&tmp.p, (size_t)scan_tmp_ints(items + 1) * sizeof(int32_t)));
  int32_t* cnt = off.p + (items + 1);
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(M->P)), dim3(kBlock), 0, st, M->P,
                     (int32_t)0x7fffffff, M->d_owner);
  hipLaunchKernelGGL(k_dt_owner, dim3(grid_for(items)), dim3(kBlock), 0, st, items, T, M->N,
                     rowstart, M->d_tri, M->d_vxy, M->d_owner);
  hipLaunchKernelGGL(k_dt_count, dim3(grid_for(items + 1)), dim3(kBlock), 0, st, items, T, M->N,
                     rowstart, M->d_tri, M->d_vxy, M->d_owner, cnt);
  FI_LAUNCH_CHECK();
  if ((rc = scan_exclusive(st, cnt, off.p, items + 1, tmp.p))) return rc;
  // every pixel must have an owner (the triangles tile the square)
  int32_t owned = 0;
  FI_HIP_TRY(hipMemcpyAsync(&owned, off.p + items, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  FI_HIP_TRY(hipStreamSynchronize(st));
  if (owned != M->P) return fail(FI_E_INVALID, "the triangles do not cover every pixel");
  hipLaunchKernelGGL(k_dt_fill, dim3(grid_for(items)), dim3(kBlock), 0, st, items, T, M->N,
                     rowstart, M->d_tri, M->d_vxy, M->d_owner, off.p, M->d_tri_px);
  // the list starts replace the item starts (same array): staged through rows
  hipLaunchKernelGGL(k_dt_ptr, dim3(grid_for(T + 1)), dim3(kBlock), 0, st, T, items, rowstart,
                     off.p, rows.p);
  FI_LAUNCH_CHECK();
  FI_HIP_TRY(hipMemcpyAsync(M->d_tri_px_ptr, rows.p, (size_t)(T + 1) * sizeof(int32_t),
                            hipMemcpyDeviceToDevice, st));
  FI_HIP_TRY(hipStreamSynchronize(st));
  return FI_OK;
}

// Vertex -> (triangle, corner) lists, built on the device from the
// triangles: counts, their exclusive sum, a fill in any order, then each list
// put in ascending order (e = 3 * triangle + corner), so the lists do not
// depend on the order of the atomic additions. The vertex work vector holds
// the counts and fill positions while they are built.
__global__ __launch_bounds__(kBlock) void k_vt_count(int64_t E, const int32_t* __restrict__ tri,
                                                     int32_t* __restrict__ cnt) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < E) atomicAdd(&cnt[tri[e]], 1);
}

__global__ __launch_bounds__(kBlock) void k_vt_fill(int64_t E, const int32_t* __restrict__ tri,
                                                    int32_t* __restrict__ pos,
                                                    int32_t* __restrict__ vt_idx) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < E) vt_idx[atomicAdd(&pos[tri[e]], 1)] = (int32_t)e;
}

// Sorts each list (at most `limit` entries; longer lists set bit 0 of flag);
// with border_limit > 0, a vertex on the square's border with more than that
// many triangles sets bit 1 (its open fan has one neighbour more than
// triangles, and a row holds kMaxIncident neighbours).
__global__ __launch_bounds__(kBlock) void k_vt_sort(int V, int N, const int32_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ vxy,
                                                    int32_t* __restrict__ vt_idx, int limit,
                                                    int border_limit, int32_t* __restrict__ flag) {
  const int v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= V) return;
  const int a = ptr[v], deg = ptr[v + 1] - a;
  if (deg > limit) {
    atomicOr(flag, 1);
    return;
  }
  if (border_limit > 0 && deg > border_limit) {
    const int x = vxy[2 * v], y = vxy[2 * v + 1];
    if (x == 0 || y == 0 || x == N || y == N) atomicOr(flag, 2);
  }
  int32_t l[kMaxIncidentGeneral];
  for (int i = 0; i < deg; ++i) l[i] = vt_idx[a + i];
  for (int i = 1; i < deg; ++i) {
    const int32_t x = l[i];
    int j = i - 1;
    while (j >= 0 && l[j] > x) {
      l[j + 1] = l[j];
      --j;
    }
    l[j + 1] = x;
  }
  for (int i = 0; i < deg; ++i) vt_idx[a + i] = l[i];
}

int build_vertex_triangles(fi_mesh* M) {
  hipStream_t st = M->ctx->stream;
  const int64_t V = M->V, E = 3 * M->T;
  int rc = 0;
  if ((rc = device_alloc(M, (void**)&M->d_vt_ptr, (size_t)(V + 1) * sizeof(int32_t))) ||
      (rc = device_alloc(M, (void**)&M->d_vt_idx, (size_t)std::max<int64_t>(E, 1) * sizeof(int32_t))))
    return rc;
  int32_t* cnt = (int32_t*)M->d_uvert;  // scratch: V doubles hold V + 1 counts
  int32_t* flag = M->d_cnt;             // scratch until the assembly counts rows
  FI_HIP_TRY(hipMemsetAsync(cnt, 0, (size_t)(V + 1) * sizeof(int32_t), st));
  FI_HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
  if (E > 0) {
    hipLaunchKernelGGL(k_vt_count, dim3(grid_for(E)), dim3(kBlock), 0, st, E, M->d_tri, cnt);
    FI_LAUNCH_CHECK();
  }
  int rc2 = scan_exclusive(st, cnt, M->d_vt_ptr, V + 1, M->d_scan_tmp);
  if (rc2) return rc2;
  FI_HIP_TRY(hipMemcpyAsync(cnt, M->d_vt_ptr, (size_t)V * sizeof(int32_t), hipMemcpyDeviceToDevice,
                            st));
  if (E > 0) {
    hipLaunchKernelGGL(k_vt_fill, dim3(grid_for(E)), dim3(kBlock), 0, st, E, M->d_tri, cnt,
                       M->d_vt_idx);
    FI_LAUNCH_CHECK();
  }
  const bool general = M->host.delaunay;
  hipLaunchKernelGGL(k_vt_sort, dim3(grid_for(V)), dim3(kBlock), 0, st, (int)V, M->N,
                     M->d_vt_ptr, M->d_vxy, M->d_vt_idx,
                     general ? kMaxIncidentGeneral : kMaxIncident,
                     general ? 0 : kMaxIncident - 1, flag);
  FI_LAUNCH_CHECK();
  int32_t bad = 0;
  FI_HIP_TRY(hipMemcpyAsync(&bad, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  FI_HIP_TRY(hipStreamSynchronize(st));
  if (bad & 1)
    return fail(FI_E_INVALID, general ? "Delaunay mesh: a vertex has more than 31 incident triangles"
                                      : "internal: vertex with more incident triangles than expected");
  if (bad & 2)
    return fail(FI_E_INVALID, "internal: border vertex with more incident triangles than expected");
  return FI_OK;
}

int build_pixel_maps(fi_mesh* M) {
  if (M->host.delaunay) return build_pixel_maps_general(M);
  hipStream_t st = M->ctx->stream;
  int32_t* cnt = (int32_t*)M->d_tpart;  // scratch: 3T doubles hold T + 1 counts
  hipLaunchKernelGGL(k_tri_count, dim3(grid_for(M->L)), dim3(kBlock), 0, st, M->L, M->d_leaves,
                     M->d_tri, M->d_vxy, cnt);
  FI_LAUNCH_CHECK();
  FI_HIP_TRY(hipMemsetAsync(cnt + M->T, 0, sizeof(int32_t), st));
  int rc = scan_exclusive(st, cnt, M->d_tri_px_ptr, M->T + 1, M->d_scan_tmp);
  if (rc) return rc;
  hipLaunchKernelGGL(k_tri_fill, dim3(grid_for(M->L)), dim3(kBlock), 0, st, M->L, M->N,
                     M->d_leaves, M->d_tri, M->d_vxy, M->d_tri_px_ptr, M->d_tri_px, M->d_owner);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

int launch_tri_best(fi_mesh* M, const double* e, const uint8_t* in_mask, double* tri_err,
                    int32_t* tri_best) {
  if (M->host.delaunay) {
    hipLaunchKernelGGL(k_tri_err_list, dim3(grid_for(M->T)), dim3(kBlock), 0, M->ctx->stream,
                       M->T, M->d_tri_px_ptr, M->d_tri_px, e, (const double*)nullptr,
                       (const uint8_t*)nullptr, in_mask, tri_err, tri_best);
    FI_LAUNCH_CHECK();
    return FI_OK;
  }
  hipLaunchKernelGGL(k_tri_best, dim3(grid_for(M->L)), dim3(kBlock), 0, M->ctx->stream, M->L,
                     M->N, M->d_leaves, M->d_tri, M->d_vxy, e, in_mask, tri_err, tri_best);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

int launch_raster_transpose(fi_mesh* M, const double* r, double* tpart, const double* w) {
  if (w)
    hipLaunchKernelGGL(k_interp_T_tri<true>, dim3(grid_for(M->T)), dim3(kBlock), 0,
                       M->ctx->stream, M->T, M->host.levels, M->d_tri_px_ptr, M->d_tri_px,
                       M->d_tri, M->d_vxy, r, w, tpart);
  else
    hipLaunchKernelGGL(k_interp_T_tri<false>, dim3(grid_for(M->T)), dim3(kBlock), 0,
                       M->ctx->stream, M->T, M->host.levels, M->d_tri_px_ptr, M->d_tri_px,
                       M->d_tri, M->d_vxy, r, (const double*)nullptr, tpart);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

int launch_gather_vertex(fi_mesh* M, const double* tpart, double* tF, double* tD) {
  hipLaunchKernelGGL(k_gather_vertex, dim3(grid_for(M->V)), dim3(kBlock), 0, M->ctx->stream,
                     (int)M->V, M->d_vt_ptr, M->d_vt_idx, M->d_vmap, tpart, tF, tD);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

int launch_adjoint_tail(fi_mesh* M, const double* tD, const double* y, double* s) {
  hipLaunchKernelGGL(k_adjoint_tail, dim3(grid_for(M->m)), dim3(kBlock), 0, M->ctx->stream,
                     (int)M->m, M->d_df_rowptr, M->d_df_col, M->d_df_val, tD, y, s);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

int launch_reduce(fi_mesh* M, const double* part, int nparts, int ncomp, double* out, double div) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, M->ctx->stream, part, nparts, ncomp, div,
                     out);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

int launch_dot(fi_mesh* M, const double* a, const double* b, int64_t n, double* out_dev) {
  int g = grid_for(n);
  if (g > kMaxGrid) g = kMaxGrid;
  hipLaunchKernelGGL(k_dot_part, dim3(g), dim3(kBlock), 0, M->ctx->stream, a, b, n, M->d_red);
  FI_LAUNCH_CHECK();
  return launch_reduce(M, M->d_red, g, 1, out_dev);
}

int launch_interp_sq(fi_mesh* M, const double* uvert, double* u_out, double* sq_dev) {
  if (M->host.delaunay || !M->d_owner) {  // no per-pixel owner map: two passes
    const int rc =
        launch_raster(M, uvert, nullptr, nullptr, u_out, nullptr, nullptr, nullptr, nullptr);
    return rc ? rc : launch_dot(M, u_out, u_out, M->P, sq_dev);
  }
  int g = grid_for(M->P);
  if (g > kMaxGrid) g = kMaxGrid;
  hipLaunchKernelGGL(k_interp_px_sq, dim3(g), dim3(kBlock), 0, M->ctx->stream, M->P,
                     M->host.levels, M->d_owner, M->d_tri, M->d_vxy, uvert, u_out, M->d_red);
  FI_LAUNCH_CHECK();
  return launch_reduce(M, M->d_red, g, 1, sq_dev);
}

int launch_axpy2_ratio(fi_mesh* M, int64_t n1, int64_t n2, const double* num, const double* den,
                       const double* x1, double* y1, const double* x2, double* y2) {
  const int64_t n = std::max(n1, n2);
  if (n == 0) return FI_OK;
  hipLaunchKernelGGL(k_axpy2_ratio, dim3(grid_for(n)), dim3(kBlock), 0, M->ctx->stream, n1, n2,
                     num, den, x1, y1, x2, y2);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

int launch_axpy_ratio(fi_mesh* M, int64_t n, const double* num, const double* den, double sign,
                      const double* x, double* y) {
  if (n == 0) return FI_OK;
  hipLaunchKernelGGL(k_axpy_ratio, dim3(grid_for(n)), dim3(kBlock), 0, M->ctx->stream, n, num, den,
                     sign, x, y);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

int launch_xpby_ratio(fi_mesh* M, int64_t n, const double* x, const double* num, const double* den,
                      double* y) {
  if (n == 0) return FI_OK;
  hipLaunchKernelGGL(k_xpby_ratio, dim3(grid_for(n)), dim3(kBlock), 0, M->ctx->stream, n, x, num,
                     den, y);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

int launch_pixel_residual(fi_mesh* M, const uint8_t* f, const double* u, double* r,
                          const double* w) {
  if (w)
    hipLaunchKernelGGL(k_pixel_residual_w, dim3(grid_for(M->P)), dim3(kBlock), 0,
                       M->ctx->stream, M->P, f, u, w, r);
  else
    hipLaunchKernelGGL(k_pixel_residual, dim3(grid_for(M->P)), dim3(kBlock), 0, M->ctx->stream,
                       M->P, f, u, r);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

int launch_mse_residual(fi_mesh* M, const uint8_t* f, const double* u, const double* scale,
                        double* r) {
  hipLaunchKernelGGL(k_mse_residual, dim3(grid_for(M->P)), dim3(kBlock), 0, M->ctx->stream, M->P,
                     f, u, scale, r);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

int launch_scale(fi_mesh* M, int64_t n, const double* w, double* x) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(kBlock), 0, M->ctx->stream, n, w, x);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

int launch_irls_weights(fi_mesh* M, const uint8_t* f, const double* u, double eps,
                        double* wsqrt) {
  hipLaunchKernelGGL(k_irls_weights, dim3(grid_for(M->P)), dim3(kBlock), 0, M->ctx->stream, M->P,
                     f, u, eps, wsqrt);
  FI_LAUNCH_CHECK();
  return FI_OK;
}

int launch_abs_err(fi_mesh* M, const double* u, const uint8_t* f, double* out_dev) {
  hipLaunchKernelGGL(k_abs_err, dim3(raster_blocks(M)), dim3(kBlock), 0, M->ctx->stream, M->P, u,
                     f, M->d_rpart);
  FI_LAUNCH_CHECK();
  return launch_reduce(M, M->d_rpart, raster_blocks(M), 1, out_dev);
}

}  // namespace fi

namespace fi {
int raster_blocks(const fi_mesh* M) {
  // one partial sum per leaf block; a mesh without leaves: per 2048 pixels
  const int64_t g = M->host.delaunay ? std::min<int64_t>((M->P + 2047) / 2048, 1024)
                                     : (M->L + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : g);
}
}  // namespace fi
