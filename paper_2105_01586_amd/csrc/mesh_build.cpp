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
//
// Every step runs on the host pool in tasks fixed by the data (rows of a
// level, subtrees, chunks of leaves or vertices), so the mesh is the same
// whatever the number of threads: per-task pieces are concatenated in order.
// The vertex -> triangle lists are built on the device from the triangles
// (build_vertex_triangles), which also checks the incident-triangle bounds.

#include <algorithm>
#include <atomic>
#include <cstring>

#include "host_pool.h"
#include "internal.h"

namespace fi {

namespace {

// Chunks for a pass over n items: about 64, none below 4096 items.
int64_t chunks_for(int64_t n) { return std::max<int64_t>(1, std::min<int64_t>(64, n / 4096)); }

// Exclusive prefix sum of per-chunk counts, in place; returns the total.
int64_t exclusive_scan(std::vector<int64_t>& v) {
  int64_t acc = 0;
  for (auto& x : v) {
    const int64_t c = x;
    x = acc;
    acc += c;
  }
  return acc;
}

struct Bitset {
  std::vector<uint64_t> w;
  std::vector<int64_t> before;  // set bits in words before this one
  void init(int64_t nbits) { w.assign((size_t)((nbits + 63) / 64), 0); }
  void set_shared(int64_t i) {  // several tasks set bits of one word
    __atomic_fetch_or(&w[(size_t)(i >> 6)], (uint64_t)1 << (i & 63), __ATOMIC_RELAXED);
  }
  bool get(int64_t i) const { return (w[(size_t)(i >> 6)] >> (i & 63)) & 1; }
  void finish() {
    const int64_t nw = (int64_t)w.size();
    before.resize((size_t)nw + 1);
    const int64_t nc = chunks_for(nw);
    std::vector<int64_t> cs((size_t)nc);
    pool_run(nc, [&](int64_t t, int64_t nt) {
      const auto [k0, k1] = split_range(nw, nt, t);
      int64_t acc = 0;
      for (int64_t k = k0; k < k1; ++k) acc += __builtin_popcountll(w[(size_t)k]);
      cs[(size_t)t] = acc;
    });
    before[(size_t)nw] = exclusive_scan(cs);
    pool_run(nc, [&](int64_t t, int64_t nt) {
      const auto [k0, k1] = split_range(nw, nt, t);
      int64_t acc = cs[(size_t)t];
      for (int64_t k = k0; k < k1; ++k) {
        before[(size_t)k] = acc;
        acc += __builtin_popcountll(w[(size_t)k]);
      }
    });
  }
  int64_t count() const { return before.back(); }
  int64_t rank(int64_t i) const {  // number of set bits strictly below i
    const uint64_t word = w[(size_t)(i >> 6)];
    const int b = (int)(i & 63);
    const uint64_t low = b ? (word & ((~(uint64_t)0) >> (64 - b))) : 0;
    return before[(size_t)(i >> 6)] + __builtin_popcountll(low);
  }
};

// Leaves of one walk: (x0, y0, level) triples and hanging-edge bits.
struct LeafList {
  std::vector<int32_t> xyl;
  std::vector<uint8_t> hang;  // bit 0 bottom, 1 right, 2 top, 3 left
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
    pool_run(chunks_for((int64_t)nl * nl), [&](int64_t t, int64_t nt) {
      const auto [y0, y1] = split_range(nl, nt, t);
      for (int cy = (int)y0; cy < (int)y1; ++cy) {
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
    });
  }
  auto is_split = [&](int l, int cx, int cy) -> bool {
    if (l < 1) return false;
    const int nl = N >> l;
    if (cx < 0 || cy < 0 || cx >= nl || cy >= nl) return false;
    return split[l][(size_t)cy * nl + cx] != 0;
  };

  // ---- leaves in Morton order (depth-first, children LL, LR, UL, UR) ----
  // A walk from (x0, y0, l): leaves go to leaf(x0, y0, l, hanging bits);
  // nodes at level `stop` go to at_stop(x0, y0) instead of being opened.
  auto walk = [&](int x0_, int y0_, int l_, int stop, auto&& leaf, auto&& at_stop) {
    std::vector<int32_t> st;
    st.reserve(4 * (size_t)(levels + 1) * 3);
    st.push_back(x0_); st.push_back(y0_); st.push_back(l_);
    while (!st.empty()) {
      const int l = st.back(); st.pop_back();
      const int y0 = st.back(); st.pop_back();
      const int x0 = st.back(); st.pop_back();
      if (l == stop) {
        at_stop(x0, y0);
      } else if (is_split(l, x0 >> l, y0 >> l)) {
        const int h = 1 << (l - 1);
        const int cx[4] = {x0 + h, x0, x0 + h, x0};  // pushed in reverse: UR UL LR LL
        const int cy[4] = {y0 + h, y0 + h, y0, y0};
        for (int k = 0; k < 4; ++k) { st.push_back(cx[k]); st.push_back(cy[k]); st.push_back(l - 1); }
      } else {
        uint8_t hb = 0;
        if (l >= 1) {
          const int cx = x0 >> l, cy = y0 >> l;
          if (is_split(l, cx, cy - 1)) hb |= 1;
          if (is_split(l, cx + 1, cy)) hb |= 2;
          if (is_split(l, cx, cy + 1)) hb |= 4;
          if (is_split(l, cx - 1, cy)) hb |= 8;
        }
        leaf(x0, y0, l, hb);
      }
    }
  };
  auto append = [](LeafList& p, int x0, int y0, int l, uint8_t hb) {
    p.xyl.push_back(x0); p.xyl.push_back(y0); p.xyl.push_back(l);
    p.hang.push_back(hb);
  };
  // The walk down to level `ls` lists, in Morton order, the coarser leaves
  // and the subtree roots at level ls (up to 64): pieces alternate between
  // the coarse leaves found before a root and the root's subtree, which is
  // walked in parallel afterwards; the pieces are then joined in order.
  const int ls = std::max(0, levels - 3);
  std::vector<LeafList> pieces(1);
  std::vector<int32_t> roots;  // x0, y0, piece index
  walk(0, 0, levels, ls,
       [&](int x0, int y0, int l, uint8_t hb) { append(pieces.back(), x0, y0, l, hb); },
       [&](int x0, int y0) {
         roots.push_back(x0); roots.push_back(y0); roots.push_back((int32_t)pieces.size());
         pieces.emplace_back();  // the subtree
         pieces.emplace_back();  // coarse leaves after it
       });
  const int64_t nroots = (int64_t)roots.size() / 3;
  pool_run(nroots, [&](int64_t t, int64_t) {
    LeafList& p = pieces[(size_t)roots[3 * t + 2]];
    walk(roots[3 * t], roots[3 * t + 1], ls, -1,
         [&](int x0, int y0, int l, uint8_t hb) { append(p, x0, y0, l, hb); }, [](int, int) {});
  });
  std::vector<int64_t> loff(pieces.size());
  for (size_t k = 0; k < pieces.size(); ++k) loff[k] = (int64_t)pieces[k].hang.size();
  const int64_t L = exclusive_scan(loff);
  HostVec<int32_t> leaf_xyl((size_t)(3 * L));
  HostVec<uint8_t> hang((size_t)L);
  pool_run((int64_t)pieces.size(), [&](int64_t k, int64_t) {
    const LeafList& p = pieces[(size_t)k];
    std::copy(p.xyl.begin(), p.xyl.end(), leaf_xyl.begin() + 3 * loff[(size_t)k]);
    std::copy(p.hang.begin(), p.hang.end(), hang.begin() + loff[(size_t)k]);
  });
  pieces.clear();
  split.clear();
  split.shrink_to_fit();

  // ---- vertices: bitset over the (N+1)^2 lattice, ranks give ids --------
  const int64_t N1 = (int64_t)N + 1;
  Bitset vb;
  vb.init(N1 * N1);
  const int64_t lch = chunks_for(L);
  pool_run(lch, [&](int64_t t, int64_t nt) {
    const auto [i0, i1] = split_range(L, nt, t);
    for (int64_t i = i0; i < i1; ++i) {
      const int64_t x0 = leaf_xyl[3 * i], y0 = leaf_xyl[3 * i + 1];
      const int64_t s = (int64_t)1 << leaf_xyl[3 * i + 2];
      vb.set_shared(y0 * N1 + x0);
      vb.set_shared(y0 * N1 + x0 + s);
      vb.set_shared((y0 + s) * N1 + x0);
      vb.set_shared((y0 + s) * N1 + x0 + s);
      if (hang[(size_t)i]) vb.set_shared((y0 + s / 2) * N1 + x0 + s / 2);
    }
  });
  vb.finish();
  const int64_t V = vb.count();
  if (V >= INT32_MAX / 4) return fail(FI_E_INVALID, "mesh too large for int32 indexing");
  H.vxy.resize((size_t)(2 * V));
  {
    const int64_t nw = (int64_t)vb.w.size();
    pool_run(chunks_for(nw), [&](int64_t t, int64_t nt) {
      const auto [k0, k1] = split_range(nw, nt, t);
      int64_t v = vb.before[(size_t)k0];
      for (int64_t k = k0; k < k1; ++k) {
        uint64_t word = vb.w[(size_t)k];
        while (word) {
          const int b = __builtin_ctzll(word);
          word &= word - 1;
          const int64_t idx = k * 64 + b;
          H.vxy[(size_t)(2 * v)] = (int32_t)(idx % N1);
          H.vxy[(size_t)(2 * v + 1)] = (int32_t)(idx / N1);
          ++v;
        }
      }
    });
  }
  auto vid = [&](int64_t x, int64_t y) -> int32_t { return (int32_t)vb.rank(y * N1 + x); };

  // ---- triangles ------------------------------------------------------
  // two per plain leaf; a fan has one per ring vertex (4 corners + midpoints)
  std::vector<int64_t> toff((size_t)lch);
  pool_run(lch, [&](int64_t t, int64_t nt) {
    const auto [i0, i1] = split_range(L, nt, t);
    int64_t c = 0;
    for (int64_t i = i0; i < i1; ++i) {
      const uint8_t hb = hang[(size_t)i];
      c += hb ? 4 + __builtin_popcount(hb) : 2;
    }
    toff[(size_t)t] = c;
  });
  const int64_t T = exclusive_scan(toff);
  if (T >= INT32_MAX / 3) return fail(FI_E_INVALID, "mesh too large for int32 indexing");
  H.leaves.resize((size_t)(4 * (L + 1)));
  H.tri.resize((size_t)(3 * T));
  pool_run(lch, [&](int64_t t, int64_t nt) {
    const auto [i0, i1] = split_range(L, nt, t);
    int32_t ntri = (int32_t)toff[(size_t)t];
    int32_t* out = H.tri.data() + 3 * (size_t)ntri;
    for (int64_t i = i0; i < i1; ++i) {
      const int64_t x0 = leaf_xyl[3 * i], y0 = leaf_xyl[3 * i + 1];
      const int l = leaf_xyl[3 * i + 2];
      const int64_t s = (int64_t)1 << l, h = s / 2;
      H.leaves[(size_t)(4 * i)] = (int32_t)x0;
      H.leaves[(size_t)(4 * i + 1)] = (int32_t)y0;
      H.leaves[(size_t)(4 * i + 2)] = l;
      H.leaves[(size_t)(4 * i + 3)] = ntri;
      const uint8_t hb = hang[(size_t)i];
      if (!hb) {
        const int32_t a = vid(x0, y0), b = vid(x0 + s, y0), c = vid(x0 + s, y0 + s),
                      d = vid(x0, y0 + s);
        const int32_t tt[6] = {a, b, c, a, c, d};
        std::memcpy(out, tt, sizeof(tt));
        out += 6;
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
          *out++ = cen;
          *out++ = ring[k];
          *out++ = ring[(k + 1) % nr];
        }
        ntri += nr;
      }
    }
  });
  H.leaves[(size_t)(4 * L)] = 0;
  H.leaves[(size_t)(4 * L + 1)] = 0;
  H.leaves[(size_t)(4 * L + 2)] = 0;
  H.leaves[(size_t)(4 * L + 3)] = (int32_t)T;

  // ---- Dirichlet / free split -----------------------------------------
  const int64_t vch = chunks_for(V);
  H.vmap.resize((size_t)V);
  pool_run(vch, [&](int64_t t, int64_t nt) {
    const auto [v0, v1] = split_range(V, nt, t);
    std::fill(H.vmap.begin() + v0, H.vmap.begin() + v1, 0);
  });
  H.mask_vids.resize((size_t)m);
  H.mask_pix.assign(mask, mask + m);
  std::atomic<bool> not_vertex{false};
  pool_run(chunks_for(m), [&](int64_t t, int64_t nt) {
    const auto [j0, j1] = split_range(m, nt, t);
    for (int64_t j = j0; j < j1; ++j) {
      const int64_t r = mask[j] / N, c = mask[j] % N;
      if (!vb.get(r * N1 + c)) {
        not_vertex.store(true, std::memory_order_relaxed);
        continue;
      }
      const int32_t v = vid(c, r);
      H.mask_vids[(size_t)j] = v;
      H.vmap[(size_t)v] = -(int32_t)(j + 1);
    }
  });
  if (not_vertex.load()) return fail(FI_E_INVALID, "internal: a mask pixel is not a vertex");
  std::vector<int64_t> foff((size_t)vch);
  pool_run(vch, [&](int64_t t, int64_t nt) {
    const auto [v0, v1] = split_range(V, nt, t);
    int64_t c = 0;
    for (int64_t v = v0; v < v1; ++v) c += H.vmap[(size_t)v] == 0;
    foff[(size_t)t] = c;
  });
  H.free_vids.resize((size_t)exclusive_scan(foff));
  pool_run(vch, [&](int64_t t, int64_t nt) {
    const auto [v0, v1] = split_range(V, nt, t);
    int64_t f = foff[(size_t)t];
    for (int64_t v = v0; v < v1; ++v) {
      if (H.vmap[(size_t)v] == 0) {
        H.vmap[(size_t)v] = (int32_t)f;
        H.free_vids[(size_t)f++] = (int32_t)v;
      }
    }
  });

  return FI_OK;
}

}  // namespace fi
