// Host construction of the balanced quadtree triangle mesh (integer work).
//
// Section 2.2 asks for a triangle mesh in which every mask pixel is a
// vertex. The mesh here is the 2:1 edge-balanced quadtree on [0, N]^2 refined
// to unit cells at the mask pixels (pixel (r, c) at lattice point (c, r); its
// unit cell [c, c+1] x [r, r+1]). Leaves without a finer edge neighbour are
// cut along the diagonal (x0, y0)-(x0+s, y0+s); leaves with one are fanned
// from their centre through the hanging edge midpoints. All triangles are
// right isosceles, hence non-obtuse, hence Delaunay for their vertex set.
//
// Construction, bottom-up over levels (level l cells have side 2^l):
//   split[1](c)  = c holds a mask pixel;
//   split[l](c)  = some child of c is split, or an edge neighbour of c at
//                  level l has a split child touching c (that child's
//                  children would be leaves < half of c's side).
// One pass from fine to coarse gives the smallest balanced tree: each flag
// only depends on level l-1 flags, and every flag raised is forced.
// Leaves come out of a depth-first walk in Morton order. Vertices are leaf
// corners plus centres of leaves with a split edge neighbour; vertex ids are
// ranks in row-major (y, x) order, found with a bitset and popcounts.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace fi {

namespace {

struct Bitset {
  std::vector<uint64_t> w;
  std::vector<int64_t> before;  // set bits in words before this one
  void init(int64_t nbits) { w.assign((size_t)((nbits + 63) / 64), 0); }
  void set(int64_t i) { w[(size_t)(i >> 6)] |= (uint64_t)1 << (i & 63); }
  bool get(int64_t i) const { return (w[(size_t)(i >> 6)] >> (i & 63)) & 1; }
  void finish() {
    before.resize(w.size() + 1);
    int64_t acc = 0;
    for (size_t k = 0; k < w.size(); ++k) {
      before[k] = acc;
      acc += __builtin_popcountll(w[k]);
    }
    before[w.size()] = acc;
  }
  int64_t count() const { return before.back(); }
  int64_t rank(int64_t i) const {  // number of set bits strictly below i
    const uint64_t word = w[(size_t)(i >> 6)];
    const int b = (int)(i & 63);
    const uint64_t low = b ? (word & ((~(uint64_t)0) >> (64 - b))) : 0;
    return before[(size_t)(i >> 6)] + __builtin_popcountll(low);
  }
};

}  // namespace

int build_host_mesh(int N, const int32_t* mask, int64_t m, HostMesh& H) {
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
  int levels = 0;
  while ((1 << levels) < N) ++levels;

  H = HostMesh();
  H.N = N;
  H.levels = levels;

  // ---- split flags per level ------------------------------------------
  std::vector<std::vector<uint8_t>> split(levels + 1);
  for (int l = 1; l <= levels; ++l) split[l].assign((size_t)(N >> l) * (N >> l), 0);
  {
    const int n1 = N >> 1;
    for (int64_t j = 0; j < m; ++j) {
      const int r = mask[j] / N, c = mask[j] % N;
      split[1][(size_t)(r >> 1) * n1 + (c >> 1)] = 1;
    }
  }
  for (int l = 2; l <= levels; ++l) {
    const int nl = N >> l, nc = N >> (l - 1);
    const std::vector<uint8_t>& ch = split[l - 1];
    std::vector<uint8_t>& cur = split[l];
    for (int cy = 0; cy < nl; ++cy) {
      for (int cx = 0; cx < nl; ++cx) {
        const int X = 2 * cx, Y = 2 * cy;  // lower-left child
        auto C = [&](int x, int y) -> int { return ch[(size_t)y * nc + x]; };
        int s = C(X, Y) | C(X + 1, Y) | C(X, Y + 1) | C(X + 1, Y + 1);
        if (!s && cx > 0) s = C(X - 1, Y) | C(X - 1, Y + 1);
        if (!s && cx + 1 < nl) s = C(X + 2, Y) | C(X + 2, Y + 1);
        if (!s && cy > 0) s = C(X, Y - 1) | C(X + 1, Y - 1);
        if (!s && cy + 1 < nl) s = C(X, Y + 2) | C(X + 1, Y + 2);
        cur[(size_t)cy * nl + cx] = (uint8_t)s;
      }
    }
  }
  auto is_split = [&](int l, int cx, int cy) -> bool {
    if (l < 1) return false;
    const int nl = N >> l;
    if (cx < 0 || cy < 0 || cx >= nl || cy >= nl) return false;
    return split[l][(size_t)cy * nl + cx] != 0;
  };

  // ---- leaves in Morton order (depth-first, children LL, LR, UL, UR) ----
  std::vector<int32_t> leaf_xyl;  // x0, y0, level
  std::vector<uint8_t> hang;      // bit 0 bottom, 1 right, 2 top, 3 left
  {
    std::vector<int32_t> st;
    st.reserve(4 * (size_t)(levels + 1) * 3);
    st.push_back(0); st.push_back(0); st.push_back(levels);
    while (!st.empty()) {
      const int l = st.back(); st.pop_back();
      const int y0 = st.back(); st.pop_back();
      const int x0 = st.back(); st.pop_back();
      if (is_split(l, x0 >> l, y0 >> l)) {
        const int h = 1 << (l - 1);
        const int cx[4] = {x0 + h, x0, x0 + h, x0};  // pushed in reverse: UR UL LR LL
        const int cy[4] = {y0 + h, y0 + h, y0, y0};
        for (int k = 0; k < 4; ++k) { st.push_back(cx[k]); st.push_back(cy[k]); st.push_back(l - 1); }
      } else {
        leaf_xyl.push_back(x0); leaf_xyl.push_back(y0); leaf_xyl.push_back(l);
        uint8_t hb = 0;
        if (l >= 1) {
          const int cx = x0 >> l, cy = y0 >> l;
          if (is_split(l, cx, cy - 1)) hb |= 1;
          if (is_split(l, cx + 1, cy)) hb |= 2;
          if (is_split(l, cx, cy + 1)) hb |= 4;
          if (is_split(l, cx - 1, cy)) hb |= 8;
        }
        hang.push_back(hb);
      }
    }
  }
  split.clear();
  split.shrink_to_fit();
  const int64_t L = (int64_t)hang.size();

  // ---- vertices: bitset over the (N+1)^2 lattice, ranks give ids --------
  const int64_t N1 = (int64_t)N + 1;
  Bitset vb;
  vb.init(N1 * N1);
  for (int64_t i = 0; i < L; ++i) {
    const int64_t x0 = leaf_xyl[3 * i], y0 = leaf_xyl[3 * i + 1];
    const int64_t s = (int64_t)1 << leaf_xyl[3 * i + 2];
    vb.set(y0 * N1 + x0);
    vb.set(y0 * N1 + x0 + s);
    vb.set((y0 + s) * N1 + x0);
    vb.set((y0 + s) * N1 + x0 + s);
    if (hang[(size_t)i]) vb.set((y0 + s / 2) * N1 + x0 + s / 2);
  }
  vb.finish();
  const int64_t V = vb.count();
  if (V >= INT32_MAX / 4) return fail(FI_E_INVALID, "mesh too large for int32 indexing");
  H.vxy.resize((size_t)(2 * V));
  {
    int64_t v = 0;
    for (size_t k = 0; k < vb.w.size(); ++k) {
      uint64_t word = vb.w[k];
      while (word) {
        const int b = __builtin_ctzll(word);
        word &= word - 1;
        const int64_t idx = (int64_t)k * 64 + b;
        H.vxy[(size_t)(2 * v)] = (int32_t)(idx % N1);
        H.vxy[(size_t)(2 * v + 1)] = (int32_t)(idx / N1);
        ++v;
      }
    }
  }
  auto vid = [&](int64_t x, int64_t y) -> int32_t { return (int32_t)vb.rank(y * N1 + x); };

  // ---- triangles ------------------------------------------------------
  H.leaves.resize((size_t)(4 * (L + 1)));
  H.tri.reserve((size_t)(3 * 2 * L + 64));
  int32_t ntri = 0;
  for (int64_t i = 0; i < L; ++i) {
    const int64_t x0 = leaf_xyl[3 * i], y0 = leaf_xyl[3 * i + 1];
    const int l = leaf_xyl[3 * i + 2];
    const int64_t s = (int64_t)1 << l, h = s / 2;
    H.leaves[(size_t)(4 * i)] = (int32_t)x0;
    H.leaves[(size_t)(4 * i + 1)] = (int32_t)y0;
    H.leaves[(size_t)(4 * i + 2)] = l;
    H.leaves[(size_t)(4 * i + 3)] = ntri;
    const uint8_t hb = hang[(size_t)i];
    if (!hb) {
      const int32_t a = vid(x0, y0), b = vid(x0 + s, y0), c = vid(x0 + s, y0 + s), d = vid(x0, y0 + s);
      const int32_t t[6] = {a, b, c, a, c, d};
      H.tri.insert(H.tri.end(), t, t + 6);
      ntri += 2;
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
        H.tri.push_back(cen);
        H.tri.push_back(ring[k]);
        H.tri.push_back(ring[(k + 1) % nr]);
      }
      ntri += nr;
    }
  }
  H.leaves[(size_t)(4 * L)] = 0;
  H.leaves[(size_t)(4 * L + 1)] = 0;
  H.leaves[(size_t)(4 * L + 2)] = 0;
  H.leaves[(size_t)(4 * L + 3)] = ntri;
  const int64_t T = ntri;

  // ---- Dirichlet / free split -----------------------------------------
  H.vmap.assign((size_t)V, 0);
  H.mask_vids.resize((size_t)m);
  H.mask_pix.assign(mask, mask + m);
  for (int64_t j = 0; j < m; ++j) {
    const int64_t r = mask[j] / N, c = mask[j] % N;
    const int64_t idx = r * N1 + c;
    if (!vb.get(idx)) return fail(FI_E_INVALID, "internal: a mask pixel is not a vertex");
    const int32_t v = vid(c, r);
    H.mask_vids[(size_t)j] = v;
    H.vmap[(size_t)v] = -(int32_t)(j + 1);
  }
  H.free_vids.reserve((size_t)(V - m));
  for (int64_t v = 0; v < V; ++v) {
    if (H.vmap[(size_t)v] == 0) {
      H.vmap[(size_t)v] = (int32_t)H.free_vids.size();
      H.free_vids.push_back((int32_t)v);
    }
  }

  // ---- vertex -> (triangle, corner) adjacency ----------------------------
  H.vt_ptr.assign((size_t)(V + 1), 0);
  for (int64_t e = 0; e < 3 * T; ++e) H.vt_ptr[(size_t)H.tri[(size_t)e] + 1]++;
  // A vertex on the square's border has an open fan, one neighbour more than
  // triangles; the assembly's neighbour slots hold kMaxIncident.
  bool border_ok = true;
  for (int64_t v = 0; v < V; ++v) {
    const int32_t inc = H.vt_ptr[(size_t)v + 1];
    const int32_t x = H.vxy[(size_t)(2 * v)], y = H.vxy[(size_t)(2 * v + 1)];
    border_ok &= !(x == 0 || y == 0 || x == N || y == N) || inc <= kMaxIncident - 1;
    H.max_incident = std::max(H.max_incident, inc);
    H.vt_ptr[(size_t)v + 1] += H.vt_ptr[(size_t)v];
  }
  if (H.max_incident > kMaxIncident)
    return fail(FI_E_INVALID, "internal: vertex with more incident triangles than expected");
  if (!border_ok)
    return fail(FI_E_INVALID, "internal: border vertex with more incident triangles than expected");
  H.vt_idx.resize((size_t)(3 * T));
  {
    std::vector<int32_t> fill(H.vt_ptr.begin(), H.vt_ptr.end() - 1);
    for (int64_t e = 0; e < 3 * T; ++e) {
      const int32_t v = H.tri[(size_t)e];
      H.vt_idx[(size_t)fill[(size_t)v]++] = (int32_t)e;  // e = 3 * t + corner
    }
  }
  return FI_OK;
}

}  // namespace fi
