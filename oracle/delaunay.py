"""The paper's own mesh: a Delaunay triangulation of the mask pixels and a set
of unknown vertices (Section 2.2).

TEST INFRASTRUCTURE ONLY (see the package header).

Section 2.2 makes every mask pixel a vertex, adds some of the other pixels as
"unknown vertices" (about as many as there are mask pixels; Section 3 places
them uniformly at random in its first iteration) and triangulates the point
set by Delaunay. Readings, where the paper is silent:

* pixel (r, c) is the point (x = c, y = r). The four corner pixels are always
  vertices (unknowns unless they are mask pixels), so the triangulation covers
  the square [0, N-1]^2 and every pixel lies in a triangle.
* The unknown vertices are an input: the random draw happens outside.
* Vertex ids follow the linear pixel index.
* On a pixel lattice, four or more cocircular vertices are common, and there
  the Delaunay triangulation is not unique. The canonical one is the regular
  triangulation of the lifted points (x, y, x^2 + y^2 + e_v) with
  infinitesimal e_0 >> e_1 >> ... (simulation of simplicity). The in-circle
  determinant is linear in the lifted heights, so a zero determinant is
  decided by the height cofactor of the lowest vertex id whose cofactor is
  non-zero. The result is a Delaunay triangulation, and it is unique.
* Triangles are listed counter-clockwise starting at their lowest vertex id,
  in lexicographic order.
* The owner of a pixel is the lowest-index triangle that contains it,
  boundary included. Values do not depend on this rule; exported indices do.

Construction: incremental insertion with edge flips (Lawson), in Hilbert
order, with exact integer predicates. Pure Python, for the modest sizes the
tests use.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


def orient(ax, ay, bx, by, cx, cy):
    """Twice the signed area of (a, b, c); positive when counter-clockwise."""
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)


def incircle_det(P, a, b, c, d) -> int:
    """The 4x4 determinant |x y x^2+y^2 1| over rows a, b, c, d: positive when
    d lies inside the circle through a, b, c (counter-clockwise)."""
    dx, dy = P[d]
    rows = []
    for v in (a, b, c):
        x = P[v][0] - dx
        y = P[v][1] - dy
        rows.append((x, y, x * x + y * y))
    (a0, a1, a2), (b0, b1, b2), (c0, c1, c2) = rows
    return (a0 * (b1 * c2 - b2 * c1) - a1 * (b0 * c2 - b2 * c0) + a2 * (b0 * c1 - b1 * c0))


def inside(P, a, b, c, d) -> bool:
    """d strictly inside the circumcircle of the counter-clockwise triangle
    (a, b, c) for the perturbed lifted heights (never a tie)."""
    D = incircle_det(P, a, b, c, d)
    if D != 0:
        return D > 0
    # D' = D + e_a orient(b,c,d) - e_b orient(a,c,d) + e_c orient(a,b,d)
    #        - e_d orient(a,b,c): the cofactors of the height column
    def o(p, q, r):
        return orient(P[p][0], P[p][1], P[q][0], P[q][1], P[r][0], P[r][1])
    terms = {a: o(b, c, d), b: -o(a, c, d), c: o(a, b, d), d: -o(a, b, c)}
    for v in sorted(terms):
        if terms[v] != 0:
            return terms[v] > 0
    raise AssertionError("all height cofactors vanish: (a, b, c) is degenerate")


def hilbert_key(x: np.ndarray, y: np.ndarray, order: int) -> np.ndarray:
    """Index along the Hilbert curve of side 2^order (vectorised)."""
    x = x.astype(np.int64).copy()
    y = y.astype(np.int64).copy()
    d = np.zeros_like(x)
    s = 1 << (order - 1)
    while s > 0:
        rx = (x & s) > 0
        ry = (y & s) > 0
        d += s * s * ((3 * rx) ^ ry)
        # rotate the quadrant
        flip = ~ry
        x1 = np.where(flip & rx, s - 1 - x, x)
        y1 = np.where(flip & rx, s - 1 - y, y)
        x, y = np.where(flip, y1, x1), np.where(flip, x1, y1)
        s >>= 1
    return d


class _Triangulation:
    """Triangles V[t] = [a, b, c] counter-clockwise; Nb[t][i] = the triangle
    across the edge opposite V[t][i], or -1 on the hull."""

    def __init__(self, P):
        self.P = P
        self.V: list[list[int]] = []
        self.Nb: list[list[int]] = []

    def o(self, p, q, r):
        P = self.P
        return orient(P[p][0], P[p][1], P[q][0], P[q][1], P[r][0], P[r][1])

    def new(self, verts, nbrs) -> int:
        self.V.append(list(verts))
        self.Nb.append(list(nbrs))
        return len(self.V) - 1

    def set(self, t, verts, nbrs):
        self.V[t] = list(verts)
        self.Nb[t] = list(nbrs)

    def repoint(self, t, old, new):
        """Neighbour t (if any) now sees `new` where it saw `old`."""
        if t < 0:
            return
        nb = self.Nb[t]
        nb[nb.index(old)] = new

    def locate(self, p, start):
        t = start
        for _ in range(4 * len(self.V) + 8):
            a, b, c = self.V[t]
            moved = False
            for i, (q, r) in enumerate(((b, c), (c, a), (a, b))):
                if self.o(q, r, p) < 0:
                    t = self.Nb[t][i]
                    if t < 0:
                        raise AssertionError("point outside the triangulated square")
                    moved = True
                    break
            if not moved:
                return t
        raise AssertionError("walk did not terminate")

    def rotate_to(self, t, v):
        """Rotate triangle t so that vertex v is first."""
        k = self.V[t].index(v)
        self.V[t] = self.V[t][k:] + self.V[t][:k]
        self.Nb[t] = self.Nb[t][k:] + self.Nb[t][:k]

    def legalise(self, stack):
        """stack: triangles whose vertex 0 is the new point; check the edge
        opposite it against the neighbour across."""
        while stack:
            t = stack.pop()
            u = self.Nb[t][0]
            if u < 0:
                continue
            p, b, c = self.V[t]
            # u holds (c, b) and its vertex d opposite that edge
            k = self.Nb[u].index(t)
            d = self.V[u][k]
            if not inside(self.P, p, b, c, d):
                continue
            self.rotate_to(u, d)          # u = (d, c, b)
            nu_c = self.Nb[u][1]          # across (b, d)
            nu_b = self.Nb[u][2]          # across (d, c)
            nt_b = self.Nb[t][1]          # across (c, p)
            nt_c = self.Nb[t][2]          # across (p, b)
            # t' = (p, b, d), u' = (p, d, c)
            self.set(t, (p, b, d), (nu_c, u, nt_c))
            self.set(u, (p, d, c), (nu_b, nt_b, t))
            self.repoint(nu_c, u, t)
            self.repoint(nt_b, t, u)
            stack.append(t)
            stack.append(u)

    def insert(self, p, start) -> int:
        t = self.locate(p, start)
        a, b, c = self.V[t]
        oa, ob, oc = self.o(b, c, p), self.o(c, a, p), self.o(a, b, p)
        zero = [i for i, x in enumerate((oa, ob, oc)) if x == 0]
        if not zero:
            na, nb, nc = self.Nb[t]
            t1 = self.new((p, c, a), (nb, -1, -1))
            t2 = self.new((p, a, b), (nc, -1, -1))
            self.set(t, (p, b, c), (na, t1, t2))
            self.Nb[t1][1], self.Nb[t1][2] = t2, t
            self.Nb[t2][1], self.Nb[t2][2] = t, t1
            self.repoint(nb, t, t1)
            self.repoint(nc, t, t2)
            self.legalise([t, t1, t2])
            return t
        if len(zero) > 1:
            raise AssertionError("point coincides with a vertex")
        # p on the edge opposite vertex zero[0] of t
        self.rotate_to(t, self.V[t][zero[0]])
        a, b, c = self.V[t]               # p on edge (b, c)
        na, nb, nc = self.Nb[t]
        u = na
        if u < 0:
            # hull edge: split t into (p, c, a) and (p, a, b)
            t1 = self.new((p, c, a), (nb, t, -1))
            self.set(t, (p, a, b), (nc, -1, t1))
            self.repoint(nb, t, t1)
            self.legalise([t, t1])
            return t
        self.rotate_to(u, [v for v in self.V[u] if v not in (b, c)][0])
        d, _, _ = self.V[u]               # u = (d, c, b)
        ud, uc, ub = self.Nb[u]           # ud = t; uc across (b, d); ub across (d, c)
        # four triangles around p: (p, a, b), (p, b, d), (p, d, c), (p, c, a)
        t1 = self.new((p, c, a), (nb, -1, -1))
        u1 = self.new((p, d, c), (ub, -1, -1))
        self.set(t, (p, a, b), (nc, -1, -1))
        self.set(u, (p, b, d), (uc, -1, -1))
        # neighbours around p, counter-clockwise: t(a,b) -> u(b,d) -> u1(d,c) -> t1(c,a)
        self.Nb[t][1], self.Nb[t][2] = u, t1      # across (b, p) -> u; across (p, a) -> t1
        self.Nb[u][1], self.Nb[u][2] = u1, t      # across (d, p) -> u1; across (p, b) -> t
        self.Nb[u1][1], self.Nb[u1][2] = t1, u    # across (c, p) -> t1; across (p, d) -> u
        self.Nb[t1][1], self.Nb[t1][2] = t, u1    # across (a, p) -> t; across (p, c) -> u1
        self.repoint(nb, t, t1)
        self.repoint(ub, u, u1)
        self.legalise([t, u, u1, t1])
        return t


def vertex_set(N: int, mask_idx, unknown_idx):
    """Sorted linear pixel indices of all vertices and a mask flag per vertex."""
    mask = np.asarray(mask_idx, dtype=np.int64)
    unk = np.asarray(unknown_idx, dtype=np.int64)
    if np.intersect1d(mask, unk).size:
        raise ValueError("unknown vertices must not be mask pixels")
    corners = np.array([0, N - 1, (N - 1) * N, N * N - 1], dtype=np.int64)
    pix = np.unique(np.concatenate([mask, unk, corners]))
    is_mask = np.isin(pix, mask)
    return pix, is_mask


def triangulate(N: int, pix: np.ndarray) -> np.ndarray:
    """(T, 3) canonical triangles (vertex ids = positions in pix)."""
    if N < 2:
        raise ValueError("the image needs at least 2 x 2 pixels")
    xs = (pix % N).astype(np.int64)
    ys = (pix // N).astype(np.int64)
    P = [(int(x), int(y)) for x, y in zip(xs, ys)]
    vid = {int(p): i for i, p in enumerate(pix)}
    c00, c10 = vid[0], vid[N - 1]
    c01, c11 = vid[(N - 1) * N], vid[N * N - 1]
    tr = _Triangulation(P)
    t0 = tr.new((c00, c10, c11), (-1, -1, -1))
    t1 = tr.new((c00, c11, c01), (-1, -1, -1))
    tr.Nb[t0][1] = t1   # across (c11, c00)
    tr.Nb[t1][2] = t0   # across (c00, c11)
    # the square's diagonal by the same rule as every other edge
    tr.rotate_to(t0, c10)
    tr.legalise([t0])
    order = int(max(1, (N - 1).bit_length()))
    rest = np.array([i for i in range(len(P)) if i not in (c00, c10, c01, c11)], dtype=np.int64)
    if rest.size:
        key = hilbert_key(xs[rest], ys[rest], order)
        rest = rest[np.argsort(key, kind="stable")]
    last = 0
    for v in rest.tolist():
        last = tr.insert(v, last)
    tris = np.array(tr.V, dtype=np.int64)
    # canonical listing: rotate to the lowest id (orientation kept), sort
    k = np.argmin(tris, axis=1)
    idx = (k[:, None] + np.arange(3)[None, :]) % 3
    tris = np.take_along_axis(tris, idx, axis=1)
    order_t = np.lexsort((tris[:, 2], tris[:, 1], tris[:, 0]))
    return tris[order_t]


def is_regular(N: int, pix: np.ndarray, tris: np.ndarray) -> bool:
    """Every interior edge is locally regular (the vertex across it is not
    inside the perturbed circumcircle): for a triangulation this makes it THE
    canonical one."""
    P = [(int(p % N), int(p // N)) for p in pix]
    opp = {}
    for a, b, c in tris.tolist():
        for (u, v, w) in ((a, b, c), (b, c, a), (c, a, b)):
            opp[(u, v)] = w
    for (u, v), w in opp.items():
        x = opp.get((v, u))
        if x is not None and inside(P, u, v, w, x):
            return False
    return True


@dataclass
class DelaunayMesh:
    """Same fields as the quadtree mesh where the FEM and tonal code read them."""
    N: int
    mask_idx: np.ndarray
    pix: np.ndarray          # (V,) linear pixel index of each vertex
    vxy: np.ndarray          # (V, 2) (x, y)
    tri: np.ndarray          # (T, 3)
    dirichlet: np.ndarray    # (V,) bool
    slot: np.ndarray         # (V,) mask slot or -1
    free: np.ndarray         # (V,) free row or -1
    free_vids: np.ndarray    # (n,)
    mask_vids: np.ndarray    # (m,)

    @property
    def V(self) -> int:
        return int(self.vxy.shape[0])

    @property
    def T(self) -> int:
        return int(self.tri.shape[0])

    @property
    def n(self) -> int:
        return int(self.free_vids.shape[0])

    @property
    def m(self) -> int:
        return int(self.mask_vids.shape[0])


def build_mesh(N: int, mask_idx, unknown_idx) -> DelaunayMesh:
    mask = np.asarray(mask_idx, dtype=np.int64)
    if mask.size and (np.any(np.diff(mask) <= 0) or mask[0] < 0 or mask[-1] >= N * N):
        raise ValueError("mask must be strictly ascending pixel indices")
    pix, is_mask = vertex_set(N, mask, unknown_idx)
    tri = triangulate(N, pix)
    V = pix.size
    vxy = np.stack([pix % N, pix // N], axis=1).astype(np.int64)
    slot = np.full(V, -1, dtype=np.int64)
    mask_vids = np.nonzero(is_mask)[0]
    slot[mask_vids] = np.arange(mask_vids.size)   # mask slots in ascending pixel order
    free_vids = np.nonzero(~is_mask)[0]
    free = np.full(V, -1, dtype=np.int64)
    free[free_vids] = np.arange(free_vids.size)
    return DelaunayMesh(N=N, mask_idx=mask, pix=pix, vxy=vxy, tri=tri, dirichlet=is_mask,
                        slot=slot, free=free, free_vids=free_vids, mask_vids=mask_vids)


@dataclass
class Raster:
    owner: np.ndarray   # (P,) owner triangle per pixel
    lam: np.ndarray     # (P, 3) barycentric weights w.r.t. tri[owner]
    R: sp.csr_matrix    # (P, V)


def rasteriser(mesh: DelaunayMesh) -> Raster:
    """Owner = lowest-index triangle containing the pixel; linear weights."""
    N = mesh.N
    P = N * N
    owner = np.full(P, -1, dtype=np.int64)
    xy = mesh.vxy
    for t in range(mesh.T - 1, -1, -1):       # lower indices overwrite
        a, b, c = (xy[v] for v in mesh.tri[t])
        x0, x1 = min(a[0], b[0], c[0]), max(a[0], b[0], c[0])
        y0, y1 = min(a[1], b[1], c[1]), max(a[1], b[1], c[1])
        gy, gx = np.mgrid[y0:y1 + 1, x0:x1 + 1]
        ins = ((orient(a[0], a[1], b[0], b[1], gx, gy) >= 0)
               & (orient(b[0], b[1], c[0], c[1], gx, gy) >= 0)
               & (orient(c[0], c[1], a[0], a[1], gx, gy) >= 0))
        owner[(gy[ins] * N + gx[ins])] = t
    if np.any(owner < 0):
        raise AssertionError("a pixel lies in no triangle")
    pixels = np.arange(P, dtype=np.int64)
    px, py = pixels % N, pixels // N
    tv = mesh.tri[owner]
    a, b, c = (xy[tv[:, i]] for i in range(3))
    den = orient(a[:, 0], a[:, 1], b[:, 0], b[:, 1], c[:, 0], c[:, 1]).astype(np.float64)
    la = orient(px, py, b[:, 0], b[:, 1], c[:, 0], c[:, 1]) / den
    lb = orient(px, py, c[:, 0], c[:, 1], a[:, 0], a[:, 1]) / den
    lc = orient(px, py, a[:, 0], a[:, 1], b[:, 0], b[:, 1]) / den
    lam = np.stack([la, lb, lc], axis=1)
    R = sp.csr_matrix((lam.ravel(), (np.repeat(pixels, 3), tv.ravel())), shape=(P, mesh.V))
    R.sum_duplicates()
    return Raster(owner=owner, lam=lam, R=R)
