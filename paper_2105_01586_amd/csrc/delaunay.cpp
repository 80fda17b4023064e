// The paper's own mesh (Section 2.2): every mask pixel is a vertex, some of
// the other pixels are "unknown vertices", and the point set is triangulated
// by Delaunay. Host C++, exact integer predicates.
//
// Pixel (r, c) is the point (x = c, y = r). The four corner pixels are always
// vertices, so the triangulation covers the square [0, N-1]^2 and every pixel
// lies in a triangle. Vertex ids follow the linear pixel index.
//
// Lattice points are often cocircular, and there the Delaunay triangulation
// is not unique. The one built here is the regular triangulation of the
// lifted points (x, y, x^2 + y^2 + e_v) for infinitesimal e_0 >> e_1 >> ...:
// the in-circle determinant is linear in the lifted heights, so when it is
// zero the sign is that of the height cofactor of the lowest vertex id whose
// cofactor is non-zero. This triangulation is Delaunay and unique, so it is
// the same whatever the construction order.
//
// Construction: incremental insertion with edge flips, points taken along a
// Hilbert curve and located by walking from the last new triangle.
// Triangles are then listed counter-clockwise from their lowest vertex id,
// in lexicographic order.
#include <algorithm>
#include <cstdint>
#include <numeric>
#include <vector>

#include "internal.h"

namespace fi {
namespace {

struct Pt {
  int64_t x, y;
};

inline int64_t orient(const Pt& a, const Pt& b, const Pt& c) {
  return (b.x - a.x) * (c.y - a.y) - (b.y - a.y) * (c.x - a.x);
}

// |x y x^2+y^2 1| over rows a, b, c, d (positive: d inside the circle of the
// counter-clockwise a, b, c). Coordinates below 2^14 keep every term below
// 2^58.
inline int64_t incircle(const Pt& a, const Pt& b, const Pt& c, const Pt& d) {
  const int64_t a0 = a.x - d.x, a1 = a.y - d.y, a2 = a0 * a0 + a1 * a1;
  const int64_t b0 = b.x - d.x, b1 = b.y - d.y, b2 = b0 * b0 + b1 * b1;
  const int64_t c0 = c.x - d.x, c1 = c.y - d.y, c2 = c0 * c0 + c1 * c1;
  return a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0);
}

// d strictly inside the perturbed circumcircle of counter-clockwise (a, b, c).
bool inside(const std::vector<Pt>& P, int a, int b, int c, int d) {
  const int64_t D = incircle(P[a], P[b], P[c], P[d]);
  if (D != 0) return D > 0;
  // height cofactors: +orient(b,c,d), -orient(a,c,d), +orient(a,b,d), -orient(a,b,c)
  int id[4] = {a, b, c, d};
  int64_t co[4] = {orient(P[b], P[c], P[d]), -orient(P[a], P[c], P[d]),
                   orient(P[a], P[b], P[d]), -orient(P[a], P[b], P[c])};
  int ord[4] = {0, 1, 2, 3};
  std::sort(ord, ord + 4, [&](int i, int j) { return id[i] < id[j]; });
  for (int k : ord)
    if (co[k] != 0) return co[k] > 0;
  return false;  // unreachable for a non-degenerate (a, b, c)
}

uint64_t hilbert(uint32_t x, uint32_t y, int order) {
  uint64_t d = 0;
  for (uint32_t s = 1u << (order - 1); s > 0; s >>= 1) {
    const uint32_t rx = (x & s) ? 1 : 0, ry = (y & s) ? 1 : 0;
    d += (uint64_t)s * s * ((3 * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = s - 1 - (x & (s - 1));
        y = s - 1 - (y & (s - 1));
      }
      std::swap(x, y);
    }
  }
  return d;
}

// Triangles t: vertices V[3t..3t+2] counter-clockwise; Nb[3t + i] is the
// triangle across the edge opposite vertex i (-1 on the square's border).
class Triangulation {
 public:
  explicit Triangulation(const std::vector<Pt>& P) : P_(P) {}
  std::vector<int32_t> V, Nb;

  int count() const { return (int)(V.size() / 3); }

  int add(int a, int b, int c, int na, int nb, int nc) {
    V.insert(V.end(), {a, b, c});
    Nb.insert(Nb.end(), {na, nb, nc});
    return count() - 1;
  }
  void set(int t, int a, int b, int c, int na, int nb, int nc) {
    V[3 * t] = a; V[3 * t + 1] = b; V[3 * t + 2] = c;
    Nb[3 * t] = na; Nb[3 * t + 1] = nb; Nb[3 * t + 2] = nc;
  }
  void repoint(int t, int from, int to) {
    if (t < 0) return;
    for (int i = 0; i < 3; ++i)
      if (Nb[3 * t + i] == from) { Nb[3 * t + i] = to; return; }
  }
  void rotate_to(int t, int v) {
    int k = V[3 * t] == v ? 0 : V[3 * t + 1] == v ? 1 : 2;
    int a[3], n[3];
    for (int i = 0; i < 3; ++i) {
      a[i] = V[3 * t + (k + i) % 3];
      n[i] = Nb[3 * t + (k + i) % 3];
    }
    set(t, a[0], a[1], a[2], n[0], n[1], n[2]);
  }
  int64_t o(int p, int q, int r) const { return orient(P_[p], P_[q], P_[r]); }

  // Triangle holding p (boundary included), walking from `start`.
  int locate(int p, int start) const {
    int t = start;
    const int64_t cap = 4 * (int64_t)count() + 8;
    for (int64_t step = 0; step < cap; ++step) {
      const int a = V[3 * t], b = V[3 * t + 1], c = V[3 * t + 2];
      int next = -2;
      if (o(b, c, p) < 0) next = Nb[3 * t];
      else if (o(c, a, p) < 0) next = Nb[3 * t + 1];
      else if (o(a, b, p) < 0) next = Nb[3 * t + 2];
      if (next == -2) return t;
      if (next < 0) return -1;  // outside the square (cannot happen for pixels)
      t = next;
    }
    return -1;
  }

  // Flips until every edge opposite the new point in the stacked triangles
  // is locally regular (each stacked triangle has the new point first).
  void legalise(std::vector<int>& stack) {
    while (!stack.empty()) {
      const int t = stack.back();
      stack.pop_back();
      const int u = Nb[3 * t];
      if (u < 0) continue;
      const int p = V[3 * t], b = V[3 * t + 1], c = V[3 * t + 2];
      int k = Nb[3 * u] == t ? 0 : Nb[3 * u + 1] == t ? 1 : 2;
      const int d = V[3 * u + k];
      if (!inside(P_, p, b, c, d)) continue;
      rotate_to(u, d);  // u = (d, c, b)
      const int nu_c = Nb[3 * u + 1], nu_b = Nb[3 * u + 2];
      const int nt_b = Nb[3 * t + 1], nt_c = Nb[3 * t + 2];
      set(t, p, b, d, nu_c, u, nt_c);
      set(u, p, d, c, nu_b, nt_b, t);
      repoint(nu_c, u, t);
      repoint(nt_b, t, u);
      stack.push_back(t);
      stack.push_back(u);
    }
  }

  // Inserts vertex p; returns a triangle holding it (a walk start), or -1.
  int insert(int p, int start, std::vector<int>& stack) {
    int t = locate(p, start);
    if (t < 0) return -1;
    const int a = V[3 * t], b = V[3 * t + 1], c = V[3 * t + 2];
    const int64_t oa = o(b, c, p), ob = o(c, a, p), oc = o(a, b, p);
    const int zeros = (oa == 0) + (ob == 0) + (oc == 0);
    stack.clear();
    if (zeros == 0) {
      const int na = Nb[3 * t], nb = Nb[3 * t + 1], nc = Nb[3 * t + 2];
      const int t1 = add(p, c, a, nb, -1, -1);
      const int t2 = add(p, a, b, nc, -1, -1);
      set(t, p, b, c, na, t1, t2);
      Nb[3 * t1 + 1] = t2; Nb[3 * t1 + 2] = t;
      Nb[3 * t2 + 1] = t;  Nb[3 * t2 + 2] = t1;
      repoint(nb, t, t1);
      repoint(nc, t, t2);
      stack.insert(stack.end(), {t, t1, t2});
      legalise(stack);
      return t;
    }
    if (zeros > 1) return -1;  // on a vertex: duplicate point
    rotate_to(t, oa == 0 ? a : ob == 0 ? b : c);
    const int A = V[3 * t], B = V[3 * t + 1], C = V[3 * t + 2];  // p on edge (B, C)
    const int na = Nb[3 * t], nb = Nb[3 * t + 1], nc = Nb[3 * t + 2];
    if (na < 0) {
      const int t1 = add(p, C, A, nb, t, -1);
      set(t, p, A, B, nc, -1, t1);
      repoint(nb, t, t1);
      stack.insert(stack.end(), {t, t1});
      legalise(stack);
      return t;
    }
    const int u = na;
    int du = -1;
    for (int i = 0; i < 3; ++i)
      if (V[3 * u + i] != B && V[3 * u + i] != C) du = V[3 * u + i];
    rotate_to(u, du);  // u = (d, C, B)
    const int d = du;
    const int uc = Nb[3 * u + 1], ub = Nb[3 * u + 2];
    const int t1 = add(p, C, A, nb, -1, -1);
    const int u1 = add(p, d, C, ub, -1, -1);
    set(t, p, A, B, nc, u, t1);
    set(u, p, B, d, uc, u1, t);
    Nb[3 * u1 + 1] = t1; Nb[3 * u1 + 2] = u;
    Nb[3 * t1 + 1] = t;  Nb[3 * t1 + 2] = u1;
    repoint(nb, t, t1);
    repoint(ub, u, u1);
    stack.insert(stack.end(), {t, u, u1, t1});
    legalise(stack);
    return t;
  }

 private:
  const std::vector<Pt>& P_;
};

int check_sorted(const int32_t* a, int64_t n, int64_t P, const char* what) {
  for (int64_t i = 0; i < n; ++i) {
    if (a[i] < 0 || a[i] >= P) return fail(FI_E_INVALID, std::string(what) + ": index out of range");
    if (i && a[i] <= a[i - 1])
      return fail(FI_E_INVALID, std::string(what) + ": must be strictly ascending");
  }
  return FI_OK;
}

}  // namespace

int build_delaunay_mesh(int N, const int32_t* mask, int64_t m, const int32_t* unknown, int64_t nu,
                        HostMesh& H) {
  if (N < 2 || (N & (N - 1)) != 0) return fail(FI_E_INVALID, "side must be a power of two >= 2");
  if (N > 8192) return fail(FI_E_INVALID, "side above 8192");
  const int64_t P = (int64_t)N * N;
  if (m > 0 && !mask) return fail(FI_E_INVALID, "mask is NULL");
  if (nu > 0 && !unknown) return fail(FI_E_INVALID, "unknown vertices are NULL");
  int rc = check_sorted(mask, m, P, "mask");
  if (!rc) rc = check_sorted(unknown, nu, P, "unknown vertices");
  if (rc) return rc;
  // vertices: mask, unknowns and the four corners, by pixel index
  for (int64_t i = 0; i < nu; ++i)
    if (std::binary_search(mask, mask + m, unknown[i]))
      return fail(FI_E_INVALID, "an unknown vertex lies on a mask pixel");
  std::vector<int32_t> pix;
  pix.reserve((size_t)(m + nu + 4));
  pix.insert(pix.end(), mask, mask + m);
  pix.insert(pix.end(), unknown, unknown + nu);
  for (int32_t c : {(int32_t)0, (int32_t)(N - 1), (int32_t)((int64_t)(N - 1) * N), (int32_t)(P - 1)})
    pix.push_back(c);
  std::sort(pix.begin(), pix.end());
  pix.erase(std::unique(pix.begin(), pix.end()), pix.end());
  std::vector<uint8_t> is_mask(pix.size());
  for (size_t v = 0; v < pix.size(); ++v) is_mask[v] = std::binary_search(mask, mask + m, pix[v]);
  const int V = (int)pix.size();
  std::vector<Pt> Pp(V);
  for (int v = 0; v < V; ++v) Pp[v] = Pt{pix[v] % N, pix[v] / N};
  auto vid = [&](int32_t q) {
    return (int)(std::lower_bound(pix.begin(), pix.end(), q) - pix.begin());
  };
  const int c00 = vid(0), c10 = vid(N - 1), c01 = vid((int32_t)((int64_t)(N - 1) * N)),
            c11 = vid((int32_t)(P - 1));
  Triangulation T(Pp);
  const int t0 = T.add(c00, c10, c11, -1, -1, -1);
  const int t1 = T.add(c00, c11, c01, -1, -1, -1);
  T.Nb[3 * t0 + 1] = t1;
  T.Nb[3 * t1 + 2] = t0;
  std::vector<int> stack;
  T.rotate_to(t0, c10);  // the diagonal by the same rule as every other edge
  stack.push_back(t0);
  T.legalise(stack);
  int order = 1;
  while ((1 << order) < N) ++order;
  std::vector<int> rest;
  rest.reserve(V);
  for (int v = 0; v < V; ++v)
    if (v != c00 && v != c10 && v != c01 && v != c11) rest.push_back(v);
  std::vector<uint64_t> key(V);
  for (int v : rest) key[v] = hilbert((uint32_t)Pp[v].x, (uint32_t)Pp[v].y, order);
  std::stable_sort(rest.begin(), rest.end(), [&](int a, int b) { return key[a] < key[b]; });
  int last = 0;
  for (int v : rest) {
    last = T.insert(v, last, stack);
    if (last < 0) return fail(FI_E_INVALID, "Delaunay insertion failed");
  }
  // canonical listing
  const int nt = T.count();
  std::vector<int32_t> tri(3 * (size_t)nt);
  for (int t = 0; t < nt; ++t) {
    int a = T.V[3 * t], b = T.V[3 * t + 1], c = T.V[3 * t + 2];
    while (a > b || a > c) {
      const int x = a;
      a = b; b = c; c = x;
    }
    tri[3 * t] = a; tri[3 * t + 1] = b; tri[3 * t + 2] = c;
  }
  std::vector<int32_t> idx(nt);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int32_t i, int32_t j) {
    for (int k = 0; k < 3; ++k)
      if (tri[3 * i + k] != tri[3 * j + k]) return tri[3 * i + k] < tri[3 * j + k];
    return false;
  });
  H = HostMesh{};
  H.N = N;
  H.levels = order;
  H.delaunay = true;
  H.tri.resize(3 * (size_t)nt);
  for (int t = 0; t < nt; ++t)
    for (int k = 0; k < 3; ++k) H.tri[3 * t + k] = tri[3 * idx[t] + k];
  H.leaves = {0, 0, 0, nt};  // no quadtree: the sentinel row only
  H.vxy.resize(2 * (size_t)V);
  for (int v = 0; v < V; ++v) {
    H.vxy[2 * v] = (int32_t)Pp[v].x;
    H.vxy[2 * v + 1] = (int32_t)Pp[v].y;
  }
  H.vmap.resize(V);
  for (int v = 0; v < V; ++v) {
    if (is_mask[v]) {
      H.vmap[v] = -(int32_t)H.mask_vids.size() - 1;
      H.mask_vids.push_back(v);
      H.mask_pix.push_back(pix[v]);
    } else {
      H.vmap[v] = (int32_t)H.free_vids.size();
      H.free_vids.push_back(v);
    }
  }
  // incident triangles per vertex (the lists themselves are built on the
  // device): the assembly holds at most kMaxIncidentGeneral
  std::vector<int32_t> inc((size_t)V, 0);
  for (int32_t x : H.tri) ++inc[(size_t)x];
  if (V > 0 && *std::max_element(inc.begin(), inc.end()) > kMaxIncidentGeneral)
    return fail(FI_E_INVALID, "a vertex has more incident triangles than the assembly supports");
  return FI_OK;
}

}  // namespace fi
