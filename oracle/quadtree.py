"""Balanced quadtree over the pixel lattice, refined to unit cells at mask pixels.

Reading used throughout (Section 2.2 requires every mask pixel to be a mesh
vertex): pixel (r, c) sits at the lattice point (x = c, y = r); the root cell is
[0, N]^2 for an N x N image (N a power of two), so the lattice has (N+1)^2
points and its last row and column carry no pixel. A cell of level l has side
2^l and is aligned to multiples of 2^l. The unit cell refined at mask pixel
(r, c) is [c, c+1] x [r, r+1], the one whose lower-left corner is the pixel.

Refinement: a cell of level l >= 1 is split when its half-open box
[x0, x0+2^l) x [y0, y0+2^l) contains a mask pixel. Balance: a leaf is split
while some leaf sharing an edge with it is smaller than half its side (edge
2:1 balance). The smallest tree with both properties is unique; both
functions below compute it, by different means.

The leaf level map ``lev[r, c]`` is the level of the leaf covering the unit
cell whose lower-left corner is (x = c, y = r). Leaves tile [0, N)^2 in unit
cells, so every pixel lies in exactly one leaf's half-open box.
"""
from __future__ import annotations

import numpy as np


def log2_side(N: int) -> int:
    if N < 2 or N & (N - 1):
        raise ValueError("image side must be a power of two >= 2")
    return N.bit_length() - 1


def _block_reduce(a: np.ndarray, l: int, fn) -> np.ndarray:
    n = a.shape[0] >> l
    return fn(a.reshape(n, 1 << l, n, 1 << l), axis=(1, 3))


def _expand(a: np.ndarray, l: int) -> np.ndarray:
    return np.repeat(np.repeat(a, 1 << l, axis=0), 1 << l, axis=1)


def refined_levels(N: int, mask_idx: np.ndarray) -> np.ndarray:
    """Leaf level map after refinement only (before balancing).

    A cell is a node when every larger cell containing it holds a mask pixel;
    its leaf is the largest mask-free node, i.e. the cell one level below the
    smallest mask-holding cell (level 0 when the pixel itself is a mask pixel;
    the root when the mask is empty).
    """
    L = log2_side(N)
    M = np.zeros(N * N, dtype=bool)
    M[np.asarray(mask_idx, dtype=np.int64)] = True
    M = M.reshape(N, N)
    lev = np.full((N, N), L, dtype=np.int16)
    for l in range(L, -1, -1):
        has = _expand(_block_reduce(M, l, np.any), l) if l > 0 else M
        lev = np.where(has, max(l - 1, 0), lev)
    return lev


def _neighbour_min(lev: np.ndarray) -> np.ndarray:
    """Minimum leaf level among the four edge-adjacent unit cells (inside the domain)."""
    big = np.iinfo(np.int16).max
    nb = np.full(lev.shape, big, dtype=np.int16)
    nb[:, :-1] = np.minimum(nb[:, :-1], lev[:, 1:])
    nb[:, 1:] = np.minimum(nb[:, 1:], lev[:, :-1])
    nb[:-1, :] = np.minimum(nb[:-1, :], lev[1:, :])
    nb[1:, :] = np.minimum(nb[1:, :], lev[:-1, :])
    return nb


def balanced_levels(N: int, mask_idx: np.ndarray) -> np.ndarray:
    """Leaf level map of the 2:1 edge-balanced refinement.

    Fixed point: every leaf of level l that touches (across an edge) a unit
    cell whose leaf has level below l - 1 is split into its four children;
    repeat until no leaf needs splitting. Each split is forced in any balanced
    refinement, so the fixed point is the smallest balanced tree.
    """
    L = log2_side(N)
    lev = refined_levels(N, mask_idx)
    while True:
        nb = _neighbour_min(lev)
        new = lev.copy()
        changed = False
        for l in range(2, L + 1):
            corner = lev[:: 1 << l, :: 1 << l]
            bmin = _block_reduce(nb, l, np.min)
            split = (corner == l) & (bmin < l - 1)
            if split.any():
                changed = True
                new = np.where(_expand(split, l), np.int16(l - 1), new)
        if not changed:
            return lev
        lev = new


def morton_key(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Z-order key: x bits in even positions, y bits in odd positions.

    For aligned quadtree cells this is depth-first order with children taken
    as lower-left, lower-right, upper-left, upper-right.
    """
    x = np.asarray(x, dtype=np.uint64)
    y = np.asarray(y, dtype=np.uint64)
    key = np.zeros(np.broadcast(x, y).shape, dtype=np.uint64)
    for b in range(32):
        key |= ((x >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
        key |= ((y >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b + 1)
    return key


def leaves_from_levels(lev: np.ndarray) -> np.ndarray:
    """Leaves as int64 rows (x0, y0, level), in Morton order of (x0, y0)."""
    N = lev.shape[0]
    rows = []
    ys, xs = np.mgrid[0:N, 0:N]
    for l in np.unique(lev):
        s = 1 << int(l)
        sel = (lev == l) & (xs % s == 0) & (ys % s == 0)
        yy, xx = np.nonzero(sel)
        rows.append(np.stack([xx, yy, np.full_like(xx, l)], axis=1))
    leaves = np.concatenate(rows, axis=0).astype(np.int64)
    order = np.argsort(morton_key(leaves[:, 0], leaves[:, 1]), kind="stable")
    return leaves[order]


# ---------------------------------------------------------------------------
# Naive pointer-free recursive builder, for tiny inputs only. It states the
# definition directly (refine from the root; split violating leaves one at a
# time by scanning all pairs of leaves) and serves as a brute-force pin of the
# vectorised fixed point above.
# ---------------------------------------------------------------------------

def naive_leaves(N: int, mask_idx) -> list[tuple[int, int, int]]:
    L = log2_side(N)
    pts = [(int(i) % N, int(i) // N) for i in mask_idx]

    def contains(x0, y0, s):
        return any(x0 <= x < x0 + s and y0 <= y < y0 + s for x, y in pts)

    leaves = set()

    def refine(x0, y0, l):
        s = 1 << l
        if l >= 1 and contains(x0, y0, s):
            h = s // 2
            for dx, dy in ((0, 0), (h, 0), (0, h), (h, h)):
                refine(x0 + dx, y0 + dy, l - 1)
        else:
            leaves.add((x0, y0, l))

    refine(0, 0, L)

    def edge_adjacent(a, b):
        ax, ay, al = a
        bx, by, bl = b
        sa, sb = 1 << al, 1 << bl
        # share a segment of positive length on a vertical or horizontal line
        if ax + sa == bx or bx + sb == ax:
            return min(ay + sa, by + sb) - max(ay, by) > 0
        if ay + sa == by or by + sb == ay:
            return min(ax + sa, bx + sb) - max(ax, bx) > 0
        return False

    while True:
        victim = None
        for a in sorted(leaves):
            if a[2] < 2:
                continue
            if any(edge_adjacent(a, b) and b[2] < a[2] - 1 for b in leaves):
                victim = a
                break
        if victim is None:
            return sorted(leaves)
        x0, y0, l = victim
        leaves.remove(victim)
        h = 1 << (l - 1)
        for dx, dy in ((0, 0), (h, 0), (0, h), (h, h)):
            leaves.add((x0 + dx, y0 + dy, l - 1))
