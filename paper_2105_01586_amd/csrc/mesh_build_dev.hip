// The quadtree mesh built on the device: the host builder's mesh
// (mesh_build.cpp), array for array and bit for bit, from the mask alone.
//   - split flags per level: level 1 from the mask pixels, level l from level
//     l - 1 (a child split, or an edge neighbour's child next to the cell),
//     one launch per level;
//   - leaves: every cell that is not split and whose parent is, emitted with
//     its Morton key (x in the even bits) and level, then sorted by a radix
//     sort: the order of the host builder's depth-first walk (children LL,
//     LR, UL, UR);
//   - vertices: a bitset over the (N+1)^2 lattice (leaf corners, and centres
//     of leaves with a split edge neighbour), ids = ranks in row-major order
//     from per-word popcounts and their prefix sum;
//   - triangles: per leaf two (diagonal cut) or one per ring vertex (fan), at
//     offsets from a prefix sum over the leaves;
//   - mask and free vertex ids, and the vertex map, by a prefix sum over the
//     vertices.
#include <hipcub/hipcub.hpp>

#include <vector>

#include "internal.h"

namespace fi {
namespace {

constexpr int kB = 256;
unsigned gridn(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kB - 1) / kB); }

struct Levels {
  int N, levels;
  int64_t off[16];  // byte offset of level l's flags (row-major, (N >> l)^2 cells)
  const uint8_t* split;
};

__device__ __forceinline__ bool is_split(const Levels& Lv, int l, int cx, int cy) {
  if (l < 1) return false;
  const int nl = Lv.N >> l;
  if (cx < 0 || cy < 0 || cx >= nl || cy >= nl) return false;
  return Lv.split[Lv.off[l] + (int64_t)cy * nl + cx] != 0;
}

__global__ void k_qt_mark(int64_t m, const int32_t* __restrict__ mask, int N,
                          uint8_t* __restrict__ s1) {
  const int64_t j = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (j >= m) return;
  const int r = mask[j] / N, c = mask[j] % N;
  s1[(int64_t)(r >> 1) * (N >> 1) + (c >> 1)] = 1;  // every writer stores 1
}

__global__ void k_qt_level(int nl, const uint8_t* __restrict__ ch, uint8_t* __restrict__ cur) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= (int64_t)nl * nl) return;
  const int cx = (int)(i % nl), cy = (int)(i / nl), nc = 2 * nl;
  const int X = 2 * cx, Y = 2 * cy;
  auto C = [&](int x, int y) -> int { return ch[(int64_t)y * nc + x]; };
  int s = C(X, Y) | C(X + 1, Y) | C(X, Y + 1) | C(X + 1, Y + 1);
  if (!s && cx > 0) s = C(X - 1, Y) | C(X - 1, Y + 1);
  if (!s && cx + 1 < nl) s = C(X + 2, Y) | C(X + 2, Y + 1);
  if (!s && cy > 0) s = C(X, Y - 1) | C(X + 1, Y - 1);
  if (!s && cy + 1 < nl) s = C(X, Y + 2) | C(X + 1, Y + 2);
  cur[i] = (uint8_t)s;
}

__device__ __forceinline__ uint32_t spread_bits(uint32_t v) {  // bit k -> bit 2k (v < 2^16)
  v = (v | (v << 8)) & 0x00FF00FFu;
  v = (v | (v << 4)) & 0x0F0F0F0Fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}
__device__ __forceinline__ uint32_t gather_bits(uint32_t v) {  // bit 2k -> bit k
  v &= 0x55555555u;
  v = (v | (v >> 1)) & 0x33333333u;
  v = (v | (v >> 2)) & 0x0F0F0F0Fu;
  v = (v | (v >> 4)) & 0x00FF00FFu;
  v = (v | (v >> 8)) & 0x0000FFFFu;
  return v;
}

// Leaves of level l: count them (keys == nullptr) or emit (Morton key << 4) |
// l. One atomic per wave.
__global__ void k_qt_leaves(Levels Lv, int l, int* __restrict__ count,
                            uint32_t* __restrict__ keys) {
  const int nl = Lv.N >> l;
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  bool leaf = false;
  int cx = 0, cy = 0;
  if (i < (int64_t)nl * nl) {
    cx = (int)(i % nl);
    cy = (int)(i / nl);
    leaf = !is_split(Lv, l, cx, cy) && (l == Lv.levels || is_split(Lv, l + 1, cx >> 1, cy >> 1));
  }
  const uint64_t bal = __ballot(leaf);
  if (bal == 0) return;
  const int lane = __lane_id();
  const int leader = __ffsll((unsigned long long)bal) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(count, __popcll(bal));
  base = __shfl(base, leader);
  if (keys && leaf) {
    const int at = base + __popcll(bal & ((1ull << lane) - 1));
    const uint32_t x0 = (uint32_t)cx << l, y0 = (uint32_t)cy << l;
    keys[at] = ((spread_bits(x0) | (spread_bits(y0) << 1)) << 4) | (uint32_t)l;
  }
}

struct LeafOut {
  int64_t L;
  const uint32_t* keys;  // sorted
  int32_t* xyl;          // x0, y0, level per leaf
  uint8_t* hang;         // bit 0 bottom, 1 right, 2 top, 3 left
  int32_t* ntri;         // triangles per leaf (L + 1 entries, the last 0)
  uint32_t* vbits;       // lattice bitset
  int N1;
};

__global__ void k_qt_leaf_decode(Levels Lv, LeafOut O) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i == O.L) O.ntri[O.L] = 0;
  if (i >= O.L) return;
  const uint32_t k = O.keys[i];
  const int l = (int)(k & 15u);
  const uint32_t mk = k >> 4;
  const int x0 = (int)gather_bits(mk), y0 = (int)gather_bits(mk >> 1);
  uint8_t hb = 0;
  if (l >= 1) {
    const int cx = x0 >> l, cy = y0 >> l;
    if (is_split(Lv, l, cx, cy - 1)) hb |= 1;
    if (is_split(Lv, l, cx + 1, cy)) hb |= 2;
    if (is_split(Lv, l, cx, cy + 1)) hb |= 4;
    if (is_split(Lv, l, cx - 1, cy)) hb |= 8;
  }
  O.xyl[3 * i] = x0;
  O.xyl[3 * i + 1] = y0;
  O.xyl[3 * i + 2] = l;
  O.hang[i] = hb;
  O.ntri[i] = hb ? 4 + __popc((uint32_t)hb) : 2;
  const int64_t s = (int64_t)1 << l, N1 = O.N1;
  auto mark = [&](int64_t x, int64_t y) {
    const int64_t b = y * N1 + x;
    atomicOr(&O.vbits[b >> 5], 1u << (b & 31));
  };
  mark(x0, y0);
  mark(x0 + s, y0);
  mark(x0, y0 + s);
  mark(x0 + s, y0 + s);
  if (hb) mark(x0 + s / 2, y0 + s / 2);
}

__global__ void k_qt_popc(int64_t nw, const uint32_t* __restrict__ w, int32_t* __restrict__ c) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < nw) c[i] = __popc(w[i]);
  if (i == nw) c[nw] = 0;
}

__device__ __forceinline__ int32_t lattice_rank(const uint32_t* __restrict__ w,
                                                const int32_t* __restrict__ before, int64_t b) {
  const uint32_t word = w[b >> 5];
  const uint32_t low = word & ((1u << (b & 31)) - 1u);
  return before[b >> 5] + __popc(low);
}

__global__ void k_qt_vxy(int64_t nw, int N1, const uint32_t* __restrict__ w,
                         const int32_t* __restrict__ before, int32_t* __restrict__ vxy) {
  const int64_t k = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (k >= nw) return;
  uint32_t word = w[k];
  int32_t v = before[k];
  while (word) {
    const int b = __ffs(word) - 1;
    word &= word - 1;
    const int64_t idx = k * 32 + b;
    vxy[2 * (int64_t)v] = (int32_t)(idx % N1);
    vxy[2 * (int64_t)v + 1] = (int32_t)(idx / N1);
    ++v;
  }
}

struct TriArgs {
  int64_t L;
  int N1;
  const int32_t* xyl;
  const uint8_t* hang;
  const int32_t* off;  // first triangle per leaf (L + 1)
  const uint32_t* vbits;
  const int32_t* before;
  int32_t* tri;
  int32_t* leaves;     // (L + 1) x 4
};

__global__ void k_qt_tris(TriArgs A) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i == A.L) {
    A.leaves[4 * i] = 0;
    A.leaves[4 * i + 1] = 0;
    A.leaves[4 * i + 2] = 0;
    A.leaves[4 * i + 3] = A.off[A.L];
  }
  if (i >= A.L) return;
  const int64_t x0 = A.xyl[3 * i], y0 = A.xyl[3 * i + 1];
  const int l = A.xyl[3 * i + 2];
  const int64_t s = (int64_t)1 << l, h = s / 2, N1 = A.N1;
  auto vid = [&](int64_t x, int64_t y) { return lattice_rank(A.vbits, A.before, y * N1 + x); };
  const int32_t first = A.off[i];
  A.leaves[4 * i] = (int32_t)x0;
  A.leaves[4 * i + 1] = (int32_t)y0;
  A.leaves[4 * i + 2] = l;
  A.leaves[4 * i + 3] = first;
  int32_t* out = A.tri + 3 * (int64_t)first;
  const uint8_t hb = A.hang[i];
  if (!hb) {
    const int32_t a = vid(x0, y0), b = vid(x0 + s, y0), c = vid(x0 + s, y0 + s), d = vid(x0, y0 + s);
    out[0] = a; out[1] = b; out[2] = c;
    out[3] = a; out[4] = c; out[5] = d;
  } else {
    int32_t ring[8];
    int nr = 0;
    ring[nr++] = vid(x0, y0);
    if (hb & 1) ring[nr++] = vid(x0 + h, y0);
    ring[nr++] = vid(x0 + s, y0);
    if (hb & 2) ring[nr++] = vid(x0 + s, y0 + h);
    ring[nr++] = vid(x0 + s, y0 + s);
    if (hb & 4) ring[nr++] = vid(x0 + h, y0 + s);
    ring[nr++] = vid(x0, y0 + s);
    if (hb & 8) ring[nr++] = vid(x0, y0 + h);
    const int32_t cen = vid(x0 + h, y0 + h);
    for (int k = 0; k < nr; ++k) {
      out[3 * k] = cen;
      out[3 * k + 1] = ring[k];
      out[3 * k + 2] = ring[k + 1 < nr ? k + 1 : 0];
    }
  }
}

__global__ void k_qt_mask(int64_t m, int N, int N1, const int32_t* __restrict__ mask,
                          const uint32_t* __restrict__ vbits, const int32_t* __restrict__ before,
                          int32_t* __restrict__ mask_vids, int32_t* __restrict__ vmap,
                          int32_t* __restrict__ flag) {
  const int64_t j = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (j >= m) return;
  const int64_t r = mask[j] / N, c = mask[j] % N;
  const int64_t b = r * N1 + c;
  if (!((vbits[b >> 5] >> (b & 31)) & 1u)) {
    atomicOr(flag, 1);
    return;
  }
  const int32_t v = lattice_rank(vbits, before, b);
  mask_vids[j] = v;
  vmap[v] = -(int32_t)(j + 1);
}

__global__ void k_qt_freeflag(int64_t V, const int32_t* __restrict__ vmap, int32_t* __restrict__ f) {
  const int64_t v = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (v < V) f[v] = vmap[v] == 0;
  if (v == V) f[V] = 0;
}

__global__ void k_qt_free(int64_t V, const int32_t* __restrict__ pos, int32_t* __restrict__ vmap,
                          int32_t* __restrict__ free_vids) {
  const int64_t v = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (v >= V || vmap[v] != 0) return;
  const int32_t p = pos[v];
  free_vids[p] = (int32_t)v;
  vmap[v] = p;
}

int read_i32(hipStream_t st, const int32_t* dev, int32_t* host) {
  FI_HIP_TRY(hipMemcpyAsync(host, dev, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  FI_HIP_TRY(hipStreamSynchronize(st));
  return FI_OK;
}

}  // namespace

int mesh_geometry_on_device(fi_mesh* M, int N, const int32_t* mask, int64_t m) {
  if (N < 2 || (N & (N - 1)) != 0 || N > (1 << 14))
    return fail(FI_E_INVALID, "image side must be a power of two in [2, 16384]");
  if (m < 0) return fail(FI_E_INVALID, "negative mask size");
  if (m == 0) return fail(FI_E_EMPTY_MASK, "empty mask: the FEM system is singular");
  if (mask == nullptr) return fail(FI_E_INVALID, "mask pointer is NULL");
  const int64_t P = (int64_t)N * N;
  for (int64_t j = 0; j < m; ++j) {
    if (mask[j] < 0 || mask[j] >= P) return fail(FI_E_INVALID, "mask index out of range");
    if (j > 0 && mask[j] <= mask[j - 1])
      return fail(FI_E_INVALID, "mask indices must be strictly ascending");
  }
  hipStream_t st = M->ctx->stream;
  int levels = 0;
  while ((1 << levels) < N) ++levels;
  M->host.N = N;
  M->host.levels = levels;
  M->N = N;
  M->P = P;
  M->m = m;
  int rc = 0;
  if ((rc = device_alloc(M, (void**)&M->d_mask_pix, (size_t)m * 4))) return rc;
  FI_HIP_TRY(hipMemcpyAsync(M->d_mask_pix, mask, (size_t)m * 4, hipMemcpyHostToDevice, st));

  // split flags
  Levels Lv{};
  Lv.N = N;
  Lv.levels = levels;
  int64_t sbytes = 0;
  for (int l = 1; l <= levels; ++l) {
    Lv.off[l] = sbytes;
    sbytes += (int64_t)(N >> l) * (N >> l);
  }
  TmpBlock splitb(M), cntb(M);
  if ((rc = splitb.alloc((size_t)sbytes + 256)) || (rc = cntb.alloc(256))) return rc;
  uint8_t* split = (uint8_t*)splitb.p;
  int32_t* counter = (int32_t*)cntb.p;
  Lv.split = split;
  FI_HIP_TRY(hipMemsetAsync(split, 0, (size_t)sbytes, st));
  hipLaunchKernelGGL(k_qt_mark, dim3(gridn(m)), dim3(kB), 0, st, m, M->d_mask_pix, N,
                     split + Lv.off[1]);
  for (int l = 2; l <= levels; ++l) {
    const int nl = N >> l;
    hipLaunchKernelGGL(k_qt_level, dim3(gridn((int64_t)nl * nl)), dim3(kB), 0, st, nl,
                       split + Lv.off[l - 1], split + Lv.off[l]);
  }
  FI_HIP_TRY(hipGetLastError());

  // leaves: count, emit, sort by key
  FI_HIP_TRY(hipMemsetAsync(counter, 0, 2 * sizeof(int32_t), st));
  for (int l = 0; l <= levels; ++l) {
    const int64_t cells = (int64_t)(N >> l) * (N >> l);
    hipLaunchKernelGGL(k_qt_leaves, dim3(gridn(cells)), dim3(kB), 0, st, Lv, l, counter,
                       (uint32_t*)nullptr);
  }
  FI_HIP_TRY(hipGetLastError());
  int32_t L32 = 0;
  if ((rc = read_i32(st, counter, &L32))) return rc;
  const int64_t L = L32;
  size_t sort_bytes = 0;
  FI_HIP_TRY(hipcub::DeviceRadixSort::SortKeys(nullptr, sort_bytes, (uint32_t*)nullptr,
                                               (uint32_t*)nullptr, (int)L, 0, 32, st));
  const int N1 = N + 1;
  const int64_t nw = ((int64_t)N1 * N1 + 31) / 32;
  // leaf scratch: keys in and out, the sort's storage, (x0, y0, level),
  // hanging bits, triangle counts and offsets
  const size_t o_keys2 = ((size_t)L * 4 + 255) & ~(size_t)255;
  const size_t o_sort = 2 * o_keys2;
  const size_t o_xyl = (o_sort + sort_bytes + 255) & ~(size_t)255;
  const size_t o_hang = (o_xyl + (size_t)L * 12 + 255) & ~(size_t)255;
  const size_t o_ntri = (o_hang + (size_t)L + 255) & ~(size_t)255;
  const size_t o_toff = (o_ntri + (size_t)(L + 1) * 4 + 255) & ~(size_t)255;
  const size_t o_end = o_toff + (size_t)(L + 1) * 4;
  TmpBlock leafb(M), latb(M), scanb(M);
  // lattice scratch: the bitset and its word prefix sums
  const size_t o_before = ((size_t)nw * 4 + 255) & ~(size_t)255;
  const size_t lat_end = o_before + (size_t)(nw + 1) * 4 + 256;
  if ((rc = leafb.alloc(o_end + 256)) || (rc = latb.alloc(lat_end))) return rc;
  char* lb = (char*)leafb.p;
  uint32_t* keys = (uint32_t*)lb;
  uint32_t* sorted = (uint32_t*)(lb + o_keys2);
  int32_t* xyl = (int32_t*)(lb + o_xyl);
  uint8_t* hang = (uint8_t*)(lb + o_hang);
  int32_t* ntri = (int32_t*)(lb + o_ntri);
  int32_t* toff = (int32_t*)(lb + o_toff);
  uint32_t* vbits = (uint32_t*)latb.p;
  int32_t* before = (int32_t*)((char*)latb.p + o_before);

  FI_HIP_TRY(hipMemsetAsync(counter, 0, sizeof(int32_t), st));
  for (int l = 0; l <= levels; ++l) {
    const int64_t cells = (int64_t)(N >> l) * (N >> l);
    hipLaunchKernelGGL(k_qt_leaves, dim3(gridn(cells)), dim3(kB), 0, st, Lv, l, counter, keys);
  }
  FI_HIP_TRY(hipGetLastError());
  FI_HIP_TRY(hipcub::DeviceRadixSort::SortKeys(lb + o_sort, sort_bytes, keys, sorted, (int)L, 0,
                                               32, st));
  FI_HIP_TRY(hipMemsetAsync(vbits, 0, (size_t)nw * 4, st));
  LeafOut O{L, sorted, xyl, hang, ntri, vbits, N1};
  hipLaunchKernelGGL(k_qt_leaf_decode, dim3(gridn(L + 1)), dim3(kB), 0, st, Lv, O);
  FI_HIP_TRY(hipGetLastError());

  // vertex ids: popcounts of the bitset words and their prefix sum
  const int64_t V_upper = std::max<int64_t>(nw, L) + 2;
  if ((rc = scanb.alloc((size_t)scan_tmp_ints(V_upper + (int64_t)N1 * N1) * 4))) return rc;
  int32_t* scan_tmp = (int32_t*)scanb.p;
  TmpBlock wcb(M);
  if ((rc = wcb.alloc((size_t)(nw + 1) * 4))) return rc;
  hipLaunchKernelGGL(k_qt_popc, dim3(gridn(nw + 1)), dim3(kB), 0, st, nw, vbits,
                     (int32_t*)wcb.p);
  FI_HIP_TRY(hipGetLastError());
  if ((rc = scan_exclusive(st, (const int32_t*)wcb.p, before, nw + 1, scan_tmp))) return rc;
  int32_t V32 = 0;
  if ((rc = read_i32(st, before + nw, &V32))) return rc;
  const int64_t V = V32;
  if (V >= INT32_MAX / 4) return fail(FI_E_INVALID, "mesh too large for int32 indexing");
  if ((rc = scan_exclusive(st, ntri, toff, L + 1, scan_tmp))) return rc;
  int32_t T32 = 0;
  if ((rc = read_i32(st, toff + L, &T32))) return rc;
  const int64_t T = T32;
  M->V = V;
  M->T = T;
  M->L = L;

  // the mesh's arrays
  if ((rc = device_alloc(M, (void**)&M->d_vxy, (size_t)std::max<int64_t>(2 * V, 1) * 4)) ||
      (rc = device_alloc(M, (void**)&M->d_tri, (size_t)std::max<int64_t>(3 * T, 1) * 4)) ||
      (rc = device_alloc(M, (void**)&M->d_leaves, (size_t)(4 * (L + 1)) * 4)) ||
      (rc = device_alloc(M, (void**)&M->d_vmap, (size_t)std::max<int64_t>(V, 1) * 4)) ||
      (rc = device_alloc(M, (void**)&M->d_mask_vids, (size_t)m * 4)))
    return rc;
  hipLaunchKernelGGL(k_qt_vxy, dim3(gridn(nw)), dim3(kB), 0, st, nw, N1, vbits, before, M->d_vxy);
  TriArgs A{L, N1, xyl, hang, toff, vbits, before, M->d_tri, M->d_leaves};
  hipLaunchKernelGGL(k_qt_tris, dim3(gridn(L + 1)), dim3(kB), 0, st, A);
  FI_HIP_TRY(hipMemsetAsync(M->d_vmap, 0, (size_t)V * 4, st));
  FI_HIP_TRY(hipMemsetAsync(counter, 0, sizeof(int32_t), st));
  hipLaunchKernelGGL(k_qt_mask, dim3(gridn(m)), dim3(kB), 0, st, m, N, N1, M->d_mask_pix, vbits,
                     before, M->d_mask_vids, M->d_vmap, counter);
  FI_HIP_TRY(hipGetLastError());
  // free vertices in ascending order
  TmpBlock fb(M);
  if ((rc = fb.alloc((size_t)(2 * (V + 1)) * 4))) return rc;
  int32_t* flags = (int32_t*)fb.p;
  int32_t* pos = flags + (V + 1);
  hipLaunchKernelGGL(k_qt_freeflag, dim3(gridn(V + 1)), dim3(kB), 0, st, V, M->d_vmap, flags);
  FI_HIP_TRY(hipGetLastError());
  if ((rc = scan_exclusive(st, flags, pos, V + 1, scan_tmp))) return rc;
  int32_t n32 = 0, bad = 0;
  if ((rc = read_i32(st, pos + V, &n32)) || (rc = read_i32(st, counter, &bad))) return rc;
  if (bad) return fail(FI_E_INVALID, "internal: a mask pixel is not a vertex");
  M->n = n32;
  if ((rc = device_alloc(M, (void**)&M->d_free_vids, (size_t)std::max<int64_t>(M->n, 1) * 4)))
    return rc;
  hipLaunchKernelGGL(k_qt_free, dim3(gridn(V)), dim3(kB), 0, st, V, pos, M->d_vmap,
                     M->d_free_vids);
  FI_HIP_TRY(hipGetLastError());
  FI_HIP_TRY(hipStreamSynchronize(st));
  return FI_OK;
}

}  // namespace fi
