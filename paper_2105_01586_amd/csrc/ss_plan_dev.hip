// The s-step plan (row blocks with S-hop halos, ss_plan.h) built on the
// device: the same plan as the host builder, bit for bit, without copying the
// matrix back.
//   1. Hilbert keys of the free rows' clamped lattice coordinates, paired
//      with the row (key in the high 32 bits), sorted by a stable radix sort
//      on the key bits: ties keep the natural row order.
//   2. perm (new -> natural), its inverse, and every row's neighbour list in
//      the new numbering (ELL slot order, padding dropped; weight -1 in bit
//      30).
//   3. One workgroup per block grows the region ring by ring in LDS: an open
//      addressing table (4096 slots, at most ~2600 used) marks the rows
//      already in, each ring's new rows are gathered, sorted ascending
//      (bitonic) and numbered after the previous rings. The first pass
//      counts the rings; after the host has laid out the block table from
//      the counts, a second pass writes the region lists and the local matrix
//      rows.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "internal.h"
#include "ss_plan.h"

namespace fi {
namespace {

constexpr int kRingThreads = 512;   // the plan's block size: one thread per own row
constexpr int kTabBits = 12;
constexpr int kTab = 1 << kTabBits;   // hash slots
constexpr int kRegionCap = 2048;      // region rows a block may hold (the largest max_region)
constexpr int kNone = -1;

// Position of (x, y) along the Hilbert curve over [0, 2^order)^2 (the host
// builder's hilbert_key).
__device__ __forceinline__ uint32_t hilbert_pos(uint32_t x, uint32_t y, int order) {
  const uint32_t side = 1u << order;
  uint32_t d = 0;
  for (uint32_t s = side >> 1; s > 0; s >>= 1) {
    const uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
    d += s * s * ((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = side - 1 - x;
        y = side - 1 - y;
      }
      const uint32_t t = x;
      x = y;
      y = t;
    }
  }
  return d;
}

// Largest lattice coordinate of a free row.
__global__ void k_plan_maxc(int n, const int32_t* __restrict__ free_vids,
                            const int32_t* __restrict__ vxy, int32_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int32_t v = 0;
  if (i < n) {
    const int r = free_vids[i];
    v = max(vxy[2 * (size_t)r], vxy[2 * (size_t)r + 1]);
  }
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0 && v > 0) atomicMax(out, v);
}

__global__ void k_plan_keys(int n, const int32_t* __restrict__ free_vids,
                            const int32_t* __restrict__ vxy, uint32_t clampc, int order,
                            uint64_t* __restrict__ keys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int v = free_vids[i];
  const uint32_t x = min((uint32_t)vxy[2 * (size_t)v], clampc);
  const uint32_t y = min((uint32_t)vxy[2 * (size_t)v + 1], clampc);
  keys[i] = ((uint64_t)hilbert_pos(x, y, order) << 32) | (uint32_t)i;
}

__global__ void k_plan_perm(int n, const uint64_t* __restrict__ sorted, int32_t* __restrict__ perm,
                            int32_t* __restrict__ inv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int r = (int)(uint32_t)(sorted[i] & 0xFFFFFFFFu);
  perm[i] = r;
  inv[r] = i;
}

// Neighbours of new row q: kPlanSlots entries, the new column (bits 0-29) and
// bit 30 for weight -1, in ELL slot order; kNone past the row's entries.
__global__ void k_plan_nb(int n, int n_pad, int W, const int32_t* __restrict__ perm,
                          const int32_t* __restrict__ inv, const int32_t* __restrict__ ell,
                          int32_t* __restrict__ nb) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int r = perm[q];
  int32_t out[kPlanSlots];
  int c = 0;
#pragma unroll
  for (int k = 0; k < kPlanSlots; ++k) out[k] = kNone;
  for (int k = 0; k < W; ++k) {
    const int32_t e = ell[(size_t)k * n_pad + r];
    if (e & 0x40000000) continue;
    out[c++] = inv[e & 0x3FFFFFFF] | (e < 0 ? 0x40000000 : 0);
  }
#pragma unroll
  for (int k = 0; k < kPlanSlots; ++k) nb[(size_t)q * kPlanSlots + k] = out[k];
}

struct RingArgs {
  int n, S, max_region;
  const int32_t* nb;
  int4* counts;           // pass 1: (nown, n1, ninner, nreg) per block
  int* overflow;          // pass 1: set when a region outgrows max_region
  const BlockPlan* blocks;  // pass 2
  int32_t* region;
  uint32_t* lmat;         // kPlanSlots / 2 words per row
};

__device__ __forceinline__ uint32_t tab_hash(int32_t row) {
  return ((uint32_t)row * 2654435761u) >> (32 - kTabBits);
}

// Slot of a row that is in the table (every lookup below is of such a row).
__device__ __forceinline__ int tab_find(const int32_t* key, int32_t row) {
  uint32_t h = tab_hash(row);
  for (int p = 0; p < kTab && key[h] != row; ++p) h = (h + 1) & (kTab - 1);
  return (int)h;
}

template <bool WRITE>
__global__ __launch_bounds__(kRingThreads) void k_plan_rings(RingArgs A) {
  __shared__ int32_t key[kTab];
  __shared__ int16_t val[kTab];
  __shared__ int32_t reg[kRegionCap];
  __shared__ int32_t nxt[kRegionCap];
  __shared__ int cnt, bad;
  const int b = blockIdx.x, t = threadIdx.x;
  const int r0 = b * kRingThreads;
  const int nown = min(A.n - r0, kRingThreads);
  for (int i = t; i < kTab; i += kRingThreads) key[i] = kNone;
  if (t == 0) bad = 0;
  __syncthreads();
  if (t < nown) {  // own rows: distinct, so each claims a slot of its own
    const int32_t row = r0 + t;
    uint32_t h = tab_hash(row);
    while (atomicCAS(&key[h], kNone, row) != kNone) h = (h + 1) & (kTab - 1);
    val[h] = (int16_t)t;
    reg[t] = row;
  }
  __syncthreads();
  int nreg = nown, lo = 0, n1 = nown, ninner = nown;
  bool over = false;
  for (int d = 1; d <= A.S; ++d) {
    if (t == 0) cnt = 0;
    __syncthreads();
    // candidates past this many cannot fit: stop adding (the table then holds
    // at most max_region + 1 + one insertion in flight per thread)
    const int room = A.max_region - nreg;
    for (int q = lo + t; q < nreg; q += kRingThreads) {
      const int32_t row = reg[q];
      for (int k = 0; k < kPlanSlots; ++k) {
        const int32_t e = A.nb[(size_t)row * kPlanSlots + k];
        if (e == kNone) continue;
        if (*(volatile int*)&cnt > room) break;
        const int32_t c = e & 0x3FFFFFFF;
        uint32_t h = tab_hash(c);
        int p = 0;
        for (; p < kTab; ++p) {
          const int32_t old = atomicCAS(&key[h], kNone, c);
          if (old == kNone) {
            const int at = atomicAdd(&cnt, 1);
            if (at < kRegionCap) nxt[at] = c;
            break;
          }
          if (old == c) break;
          h = (h + 1) & (kTab - 1);
        }
        if (p == kTab) bad = 1;  // never with the bound above; kept as a guard
      }
    }
    __syncthreads();
    const int m = cnt;
    if (bad || nreg + m > A.max_region) {
      over = true;
      break;
    }
    // the ring in ascending order (bitonic sort over a power of two, padded)
    int p2 = 1;
    while (p2 < m) p2 <<= 1;
    for (int i = m + t; i < p2; i += kRingThreads) nxt[i] = 0x7FFFFFFF;
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int i = t; i < p2; i += kRingThreads) {
          const int ixj = i ^ j;
          if (ixj > i) {
            const int32_t a = nxt[i], c = nxt[ixj];
            if ((a > c) == ((i & k) == 0)) {
              nxt[i] = c;
              nxt[ixj] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    for (int i = t; i < m; i += kRingThreads) {
      const int32_t c = nxt[i];
      reg[nreg + i] = c;
      val[tab_find(key, c)] = (int16_t)(nreg + i);
    }
    __syncthreads();
    lo = nreg;
    nreg += m;
    if (d == 1) n1 = nreg;
    if (d == A.S - 1) ninner = nreg;
  }
  if (A.S == 1) ninner = nown;
  if constexpr (!WRITE) {
    if (t == 0) {
      A.counts[b] = make_int4(nown, n1, ninner, nreg);
      if (over) atomicOr(A.overflow, 1);
    }
  } else {
    if (over) return;  // the first pass has refused the plan already
    const BlockPlan B = A.blocks[b];
    for (int l = t; l < nreg; l += kRingThreads) A.region[(size_t)B.reg_off + l] = reg[l];
    for (int l = t; l < ninner; l += kRingThreads) {
      const int32_t row = reg[l];
      uint32_t w[kPlanSlots / 2] = {};
#pragma unroll
      for (int k = 0; k < kPlanSlots; ++k) {
        const int32_t e = A.nb[(size_t)row * kPlanSlots + k];
        uint32_t ent = kPlanPad;  // the zero slot
        if (e != kNone)
          ent = (uint32_t)(val[tab_find(key, e & 0x3FFFFFFF)] + 1) |
                ((e & 0x40000000) ? kPlanMinusOne : 0u);
        w[k >> 1] |= ent << (16 * (k & 1));
      }
      uint32_t* dst = A.lmat + ((size_t)B.lmat_off + l) * (kPlanSlots / 2);
#pragma unroll
      for (int j = 0; j < kPlanSlots / 2; ++j) dst[j] = w[j];
    }
  }
}

unsigned grid_of(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// Device scratch of ss_plan_on_device for n rows, as a bound: the keys in and
// out, the inverse permutation and neighbour lists (52 bytes per row), the
// ring counts, and for the radix sort's storage 12 bytes per row plus 4 MiB
// (a pass over 8-bit digits keeps a second copy of the keys and per-block
// digit counts); with 256-byte rounding of every piece.
int64_t ss_plan_scratch_bound(int64_t n) {
  const int64_t nblk = (n + kRingThreads - 1) / kRingThreads;
  return 256 + 52 * n + (12 * n + ((int64_t)4 << 20)) + 16 * nblk + 8 * 256;
}

int ss_plan_on_device(fi_mesh* M, int S, int max_region, SsState& Z, bool* built) {
  *built = false;
  hipStream_t st = M->ctx->stream;
  const int64_t n = M->n;
  const int W = M->ell_w;
  if (n <= 0 || W > kPlanSlots || S < 1 || max_region > kRegionCap || max_region < kRingThreads)
    return FI_OK;
  // lattice clamp of the host builder: coordinates up to the largest power of
  // two not above the largest coordinate of a free row, minus one
  int32_t maxc = 0;
  {
    TmpBlock mx(M);
    if (!mx.take(256)) return M->arena ? FI_OK : fail(FI_E_NOMEM, "s-step plan: scratch");
    FI_HIP_TRY(hipMemsetAsync(mx.p, 0, sizeof(int32_t), st));
    hipLaunchKernelGGL(k_plan_maxc, dim3(grid_of(n, 256)), dim3(256), 0, st, (int)n,
                       M->d_free_vids, M->d_vxy, (int32_t*)mx.p);
    FI_HIP_TRY(hipGetLastError());
    FI_HIP_TRY(hipMemcpyAsync(&maxc, mx.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    FI_HIP_TRY(hipStreamSynchronize(st));
  }
  uint32_t top = 1;
  while (maxc > 1 && top * 2 <= (uint32_t)maxc) top *= 2;
  const uint32_t clampc = maxc > 1 ? top - 1 : (uint32_t)maxc;
  int order = 0;
  while (order < 31 && (1u << order) <= clampc) ++order;

  const int64_t nblk = (n + kRingThreads - 1) / kRingThreads;
  size_t sort_bytes = 0;
  FI_HIP_TRY(hipcub::DeviceRadixSort::SortKeys(nullptr, sort_bytes, (uint64_t*)nullptr,
                                               (uint64_t*)nullptr, (int)n, 32,
                                               32 + std::max(1, 2 * order), st));
  // one temporary block: keys in and out, the sort's storage, the inverse
  // permutation, the neighbour lists, the ring counts and the overflow flag
  const size_t o_keys2 = (size_t)n * 8, o_sort = 2 * o_keys2;
  const size_t o_inv = (o_sort + sort_bytes + 255) & ~(size_t)255;
  const size_t o_nb = (o_inv + (size_t)n * 4 + 255) & ~(size_t)255;
  const size_t o_cnt = (o_nb + (size_t)n * kPlanSlots * 4 + 255) & ~(size_t)255;
  const size_t o_flag = o_cnt + (size_t)nblk * sizeof(int4);
  if (M->arena && (int64_t)(o_flag + 256) > ss_plan_scratch_bound(n) - 256) return FI_OK;
  // a server request's scratch comes from its arena region, whose bound
  // reserves ss_plan_scratch_bound(n); should the sort need more, the
  // request keeps the host builder
  TmpBlock tmp(M);
  if (!tmp.take(o_flag + 256)) return M->arena ? FI_OK : fail(FI_E_NOMEM, "s-step plan: scratch");
  int rc = 0;
  char* base = (char*)tmp.p;
  uint64_t* keys = (uint64_t*)base;
  uint64_t* sorted = (uint64_t*)(base + o_keys2);
  int32_t* inv = (int32_t*)(base + o_inv);
  int32_t* nb = (int32_t*)(base + o_nb);
  int4* counts = (int4*)(base + o_cnt);
  int* flag = (int*)(base + o_flag);
  if ((rc = device_alloc(M, (void**)&Z.perm, (size_t)n * 4))) return rc;

  hipLaunchKernelGGL(k_plan_keys, dim3(grid_of(n, 256)), dim3(256), 0, st, (int)n,
                     M->d_free_vids, M->d_vxy, clampc, order, keys);
  FI_HIP_TRY(hipGetLastError());
  FI_HIP_TRY(hipcub::DeviceRadixSort::SortKeys(base + o_sort, sort_bytes, keys, sorted, (int)n, 32,
                                               32 + std::max(1, 2 * order), st));
  hipLaunchKernelGGL(k_plan_perm, dim3(grid_of(n, 256)), dim3(256), 0, st, (int)n, sorted, Z.perm,
                     inv);
  hipLaunchKernelGGL(k_plan_nb, dim3(grid_of(n, 256)), dim3(256), 0, st, (int)n, (int)M->n_pad, W,
                     Z.perm, inv, M->d_ell, nb);
  FI_HIP_TRY(hipGetLastError());
  FI_HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), st));
  RingArgs A{};
  A.n = (int)n;
  A.S = S;
  A.max_region = max_region;
  A.nb = nb;
  A.counts = counts;
  A.overflow = flag;
  hipLaunchKernelGGL(k_plan_rings<false>, dim3((unsigned)nblk), dim3(kRingThreads), 0, st, A);
  FI_HIP_TRY(hipGetLastError());
  std::vector<int4> cnt((size_t)nblk);
  int over = 0;
  FI_HIP_TRY(hipMemcpyAsync(cnt.data(), counts, cnt.size() * sizeof(int4), hipMemcpyDeviceToHost, st));
  FI_HIP_TRY(hipMemcpyAsync(&over, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  FI_HIP_TRY(hipStreamSynchronize(st));
  if (over) return FI_OK;  // keep the one-iteration launch

  // the block table, as the host builder lays it out
  const int32_t grid = (int32_t)((nblk + 7) / 8 * 8);
  std::vector<BlockPlan> blocks((size_t)grid, BlockPlan{});
  int64_t roff = 0, loff = 0;
  int32_t maxr = 0;
  for (int64_t b = 0; b < nblk; ++b) {
    BlockPlan& B = blocks[(size_t)b];
    B.nown = cnt[(size_t)b].x;
    B.n1 = cnt[(size_t)b].y;
    B.ninner = cnt[(size_t)b].z;
    B.nreg = cnt[(size_t)b].w;
    B.reg_off = B.nreg > 0 ? (int32_t)roff : 0;
    B.lmat_off = B.ninner > 0 ? (int32_t)loff : 0;
    roff += B.nreg;
    loff += B.ninner;
    maxr = std::max(maxr, B.nreg);
  }
  // the footprint bound reserves at most three region and local matrix rows
  // per free row
  if (roff > 3 * n || loff > 3 * n) return FI_OK;
  blocks[0].pad0 = maxr;  // the LDS layout size travels in the first block's spare field
  if ((rc = device_alloc(M, &Z.blocks, blocks.size() * sizeof(BlockPlan))) ||
      (rc = device_alloc(M, (void**)&Z.region, (size_t)std::max<int64_t>(roff, 1) * 4)) ||
      (rc = device_alloc(M, &Z.lmat, (size_t)std::max<int64_t>(loff, 1) * 2 * kPlanSlots)))
    return rc;
  FI_HIP_TRY(hipMemcpyAsync(Z.blocks, blocks.data(), blocks.size() * sizeof(BlockPlan),
                            hipMemcpyHostToDevice, st));
  A.blocks = (const BlockPlan*)Z.blocks;
  A.region = Z.region;
  A.lmat = (uint32_t*)Z.lmat;
  hipLaunchKernelGGL(k_plan_rings<true>, dim3((unsigned)nblk), dim3(kRingThreads), 0, st, A);
  FI_HIP_TRY(hipGetLastError());
  // the block table's host copy ends with this call
  FI_HIP_TRY(hipStreamSynchronize(st));
  Z.grid = grid;
  Z.max_region = maxr;
  Z.region_rows = roff;
  Z.lmat_rows = loff;
  *built = true;
  return FI_OK;
}

}  // namespace fi
