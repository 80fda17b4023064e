"""Triangle mesh on the balanced quadtree (Section 2.2).

Vertices are all leaf corners plus the centre of every leaf that has a hanging
node, where a hanging node is the midpoint of a leaf edge that is a corner of
some (finer) leaf. Every mask pixel is a vertex, as Section 2.2 requires,
because it is the corner of its unit leaf. Vertex ids are ranks in row-major
(y, x) order, so mask vertices come in ascending linear pixel index.

Triangles, each listed with positive orientation in (x, y):

* a leaf without hanging nodes is cut along the diagonal (x0, y0)-(x0+s, y0+s)
  into {(x0,y0), (x0+s,y0), (x0+s,y0+s)} and {(x0,y0), (x0+s,y0+s), (x0,y0+s)};
* a leaf with hanging nodes is fanned from its centre: walk the boundary
  (x0,y0) -> (x0+s,y0) -> (x0+s,y0+s) -> (x0,y0+s), inserting the midpoints that
  are hanging nodes, and emit (centre, b_i, b_{i+1}) for consecutive boundary
  points, starting at (x0, y0).

All triangles are right isosceles, so none is obtuse: the mesh is a Delaunay
triangulation of its own vertex set, the property Section 2.2 asks of its
mesh.

Dirichlet set D: vertices at mask pixels (Section 2.2: mask values are
prescribed). Free set F: all other vertices, including the apron row/column at
N and the fan centres.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import quadtree


@dataclass
class Mesh:
    N: int
    mask_idx: np.ndarray      # (m,) int64 ascending linear pixel indices
    leaves: np.ndarray        # (L, 3) int64 (x0, y0, level), Morton order
    vxy: np.ndarray           # (V, 2) int64 lattice coordinates, (y, x) order
    tri: np.ndarray           # (T, 3) int64 vertex ids
    tri_leaf: np.ndarray      # (T,) leaf index of each triangle
    leaf_tri_start: np.ndarray  # (L+1,) first triangle of each leaf
    vid_lattice: np.ndarray   # ((N+1)^2,) vertex id at lattice point y*(N+1)+x, or -1
    dirichlet: np.ndarray     # (V,) bool
    slot: np.ndarray          # (V,) mask slot of a Dirichlet vertex, else -1
    free: np.ndarray          # (V,) free row of a free vertex, else -1
    free_vids: np.ndarray     # (n,) vertex ids of the free rows
    mask_vids: np.ndarray     # (m,) vertex ids of the mask slots

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


def _check_mask(N: int, mask_idx) -> np.ndarray:
    mask_idx = np.asarray(mask_idx, dtype=np.int64).ravel()
    if mask_idx.size and (mask_idx.min() < 0 or mask_idx.max() >= N * N):
        raise ValueError("mask index out of range")
    if mask_idx.size > 1 and np.any(np.diff(mask_idx) <= 0):
        raise ValueError("mask indices must be strictly ascending")
    return mask_idx


def build_mesh(N: int, mask_idx) -> Mesh:
    mask_idx = _check_mask(N, mask_idx)
    lev = quadtree.balanced_levels(N, mask_idx)
    leaves = quadtree.leaves_from_levels(lev)
    return mesh_from_leaves(N, mask_idx, leaves)


def mesh_from_leaves(N: int, mask_idx: np.ndarray, leaves: np.ndarray) -> Mesh:
    N1 = N + 1
    x0 = leaves[:, 0]
    y0 = leaves[:, 1]
    s = np.left_shift(1, leaves[:, 2])
    h = s // 2

    def lat(x, y):
        return y * N1 + x

    corner = np.zeros(N1 * N1, dtype=bool)
    for cx, cy in ((x0, y0), (x0 + s, y0), (x0 + s, y0 + s), (x0, y0 + s)):
        corner[lat(cx, cy)] = True

    big = s >= 2
    # Midpoints of the bottom, right, top and left edges; hanging if a corner.
    mids = [(x0 + h, y0), (x0 + s, y0 + h), (x0 + h, y0 + s), (x0, y0 + h)]
    hang = np.zeros((leaves.shape[0], 4), dtype=bool)
    for e, (mx, my) in enumerate(mids):
        hang[:, e] = big & corner[lat(np.where(big, mx, 0), np.where(big, my, 0))]
    has_hang = hang.any(axis=1)

    is_vertex = corner.copy()
    is_vertex[lat(x0[has_hang] + h[has_hang], y0[has_hang] + h[has_hang])] = True
    vid_lattice = np.full(N1 * N1, -1, dtype=np.int64)
    lat_ids = np.nonzero(is_vertex)[0]           # ascending = (y, x) row-major
    vid_lattice[lat_ids] = np.arange(lat_ids.size)
    vxy = np.stack([lat_ids % N1, lat_ids // N1], axis=1).astype(np.int64)

    tris = []
    tri_leaf = []
    start = np.zeros(leaves.shape[0] + 1, dtype=np.int64)
    for i in range(leaves.shape[0]):
        X, Y, S, Hh = int(x0[i]), int(y0[i]), int(s[i]), int(h[i])
        if not has_hang[i]:
            a = vid_lattice[lat(X, Y)]
            b = vid_lattice[lat(X + S, Y)]
            c = vid_lattice[lat(X + S, Y + S)]
            d = vid_lattice[lat(X, Y + S)]
            tris.append((a, b, c))
            tris.append((a, c, d))
            tri_leaf += [i, i]
        else:
            ring = [(X, Y)]
            if hang[i, 0]:
                ring.append((X + Hh, Y))
            ring.append((X + S, Y))
            if hang[i, 1]:
                ring.append((X + S, Y + Hh))
            ring.append((X + S, Y + S))
            if hang[i, 2]:
                ring.append((X + Hh, Y + S))
            ring.append((X, Y + S))
            if hang[i, 3]:
                ring.append((X, Y + Hh))
            cen = vid_lattice[lat(X + Hh, Y + Hh)]
            ids = [vid_lattice[lat(px, py)] for px, py in ring]
            for k in range(len(ids)):
                tris.append((cen, ids[k], ids[(k + 1) % len(ids)]))
                tri_leaf.append(i)
        start[i + 1] = len(tris)
    tri = np.asarray(tris, dtype=np.int64).reshape(-1, 3)

    V = vxy.shape[0]
    mask_x = mask_idx % N
    mask_y = mask_idx // N
    mask_vids = vid_lattice[lat(mask_x, mask_y)]
    if np.any(mask_vids < 0):
        raise AssertionError("a mask pixel is not a mesh vertex")
    dirichlet = np.zeros(V, dtype=bool)
    dirichlet[mask_vids] = True
    slot = np.full(V, -1, dtype=np.int64)
    slot[mask_vids] = np.arange(mask_vids.size)
    free_vids = np.nonzero(~dirichlet)[0]
    free = np.full(V, -1, dtype=np.int64)
    free[free_vids] = np.arange(free_vids.size)
    return Mesh(N=N, mask_idx=mask_idx, leaves=leaves, vxy=vxy, tri=tri,
                tri_leaf=np.asarray(tri_leaf, dtype=np.int64), leaf_tri_start=start,
                vid_lattice=vid_lattice, dirichlet=dirichlet, slot=slot, free=free,
                free_vids=free_vids, mask_vids=mask_vids.astype(np.int64))


def orient(ax, ay, bx, by, cx, cy):
    """Twice the signed area of (a, b, c); positive for counter-clockwise order."""
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax)
