"""Linear interpolation of the vertex solution to every pixel (Section 2.2).

The FEM solution is linear inside each triangle; pixels that are not vertices
get the value of that linear function. For pixel (r, c) at point p = (c, r):

* its leaf is the one whose half-open box [x0, x0+s) x [y0, y0+s) holds p
  (the leaves tile the pixel lattice exactly);
* its owner triangle is the first triangle of that leaf, in the leaf's
  listing order, that contains p, boundary included;
* its weights are barycentric: lambda_a = orient(p, b, c) / orient(a, b, c)
  and cyclically. Both terms are integers and the denominator is a power of
  two, so the weights are exact in float64.

The value at a pixel does not depend on which of several triangles sharing
an edge is chosen (the interpolant is continuous); only the exported owner
index does, which is why the rule above is fixed.

The result is the sparse P x V interpolation matrix R with u_pixels = R u_vertices.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .mesh import Mesh, orient


def leaf_of_pixel(mesh: Mesh) -> np.ndarray:
    """(N, N) int64 leaf index of the leaf covering each pixel, indexed [r, c]."""
    N = mesh.N
    out = np.full((N, N), -1, dtype=np.int64)
    lv = mesh.leaves
    for l in np.unique(lv[:, 2]):
        l = int(l)
        sel = np.nonzero(lv[:, 2] == l)[0]
        n = N >> l
        blk = np.full((n, n), -1, dtype=np.int64)
        blk[lv[sel, 1] >> l, lv[sel, 0] >> l] = sel
        full = np.repeat(np.repeat(blk, 1 << l, axis=0), 1 << l, axis=1)
        out = np.where(full >= 0, full, out)
    if np.any(out < 0):
        raise AssertionError("leaves do not tile the pixel lattice")
    return out


@dataclass
class Raster:
    owner: np.ndarray   # (P,) owner triangle id per pixel
    lam: np.ndarray     # (P, 3) float64 barycentric weights w.r.t. tri[owner]
    R: sp.csr_matrix    # (P, V)


def rasteriser(mesh: Mesh) -> Raster:
    N = mesh.N
    P = N * N
    leaf = leaf_of_pixel(mesh).ravel()
    pix = np.arange(P, dtype=np.int64)
    px = pix % N
    py = pix // N
    t0 = mesh.leaf_tri_start[leaf]
    nt = mesh.leaf_tri_start[leaf + 1] - t0
    owner = np.full(P, -1, dtype=np.int64)
    for k in range(int(nt.max())):
        cand = (owner < 0) & (nt > k)
        idx = np.nonzero(cand)[0]
        t = t0[idx] + k
        a, b, c = (mesh.vxy[mesh.tri[t, i]] for i in range(3))
        x, y = px[idx], py[idx]
        inside = ((orient(a[:, 0], a[:, 1], b[:, 0], b[:, 1], x, y) >= 0)
                  & (orient(b[:, 0], b[:, 1], c[:, 0], c[:, 1], x, y) >= 0)
                  & (orient(c[:, 0], c[:, 1], a[:, 0], a[:, 1], x, y) >= 0))
        owner[idx[inside]] = t[inside]
    if np.any(owner < 0):
        raise AssertionError("pixel not covered by its leaf's triangles")
    tv = mesh.tri[owner]
    a, b, c = (mesh.vxy[tv[:, i]] for i in range(3))
    den = orient(a[:, 0], a[:, 1], b[:, 0], b[:, 1], c[:, 0], c[:, 1]).astype(np.float64)
    la = orient(px, py, b[:, 0], b[:, 1], c[:, 0], c[:, 1]) / den
    lb = orient(px, py, c[:, 0], c[:, 1], a[:, 0], a[:, 1]) / den
    lc = orient(px, py, a[:, 0], a[:, 1], b[:, 0], b[:, 1]) / den
    lam = np.stack([la, lb, lc], axis=1)
    R = sp.csr_matrix((lam.ravel(), (np.repeat(pix, 3), tv.ravel())), shape=(P, mesh.V))
    R.sum_duplicates()
    return Raster(owner=owner, lam=lam, R=R)


def rasterise(rast: Raster, u_vertex: np.ndarray) -> np.ndarray:
    return rast.R @ np.asarray(u_vertex, dtype=np.float64)
