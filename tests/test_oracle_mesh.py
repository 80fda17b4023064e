"""Pins of the oracle's quadtree and triangle mesh (Section 2.2 mesh rules).

Pins used: brute force against a naive recursive builder, a hand-derived
small case, and invariants any conforming balanced triangulation must satisfy
(every mask pixel is a vertex; areas add up to the domain; Euler's formula;
each interior edge in two triangles; right isosceles positive triangles; 2:1
balance; minimality of every split).
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import mesh as mesh_mod
from oracle import quadtree


def random_mask(rng, N, k):
    return np.sort(rng.choice(N * N, size=k, replace=False))


@st.composite
def tiny_case(draw):
    N = draw(st.sampled_from([2, 4, 8, 16]))
    k = draw(st.integers(0, min(N * N, 12)))
    seed = draw(st.integers(0, 2**31 - 1))
    rng = np.random.default_rng(seed)
    return N, random_mask(rng, N, k)


@settings(max_examples=80, deadline=None)
@given(tiny_case())
def test_levelmap_matches_naive_builder(case):
    N, m = case
    fast = quadtree.leaves_from_levels(quadtree.balanced_levels(N, m))
    naive = quadtree.naive_leaves(N, m)
    assert sorted(map(tuple, fast.tolist())) == naive


def test_hand_case_hanging_nodes():
    # N = 4, mask pixel (r=0, c=0): the lower-left level-1 cell is split to
    # unit cells; the other three level-1 cells stay leaves. The right
    # neighbour (2,0) sees hanging node (2,1) on its left edge, the upper
    # neighbour (0,2) sees (1,2) on its bottom edge, (2,2) has none.
    M = mesh_mod.build_mesh(4, [0])
    got = sorted(map(tuple, M.leaves.tolist()))
    assert got == sorted([(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0), (2, 0, 1), (0, 2, 1), (2, 2, 1)])
    expect_v = [(0, 0), (1, 0), (2, 0), (4, 0),
                (0, 1), (1, 1), (2, 1), (3, 1),
                (0, 2), (1, 2), (2, 2), (4, 2),
                (1, 3),
                (0, 4), (2, 4), (4, 4)]
    assert [tuple(v) for v in M.vxy.tolist()] == expect_v
    assert M.T == 8 + 5 + 5 + 2
    # fan of leaf (2,0): ring (2,0) (4,0) (4,2) (2,2) (2,1), centre (3,1)
    li = [tuple(l) for l in M.leaves.tolist()].index((2, 0, 1))
    tris = M.tri[M.leaf_tri_start[li]:M.leaf_tri_start[li + 1]]
    xy = [[tuple(M.vxy[v]) for v in t] for t in tris]
    assert xy == [[(3, 1), (2, 0), (4, 0)], [(3, 1), (4, 0), (4, 2)], [(3, 1), (4, 2), (2, 2)],
                  [(3, 1), (2, 2), (2, 1)], [(3, 1), (2, 1), (2, 0)]]
    assert M.mask_vids.tolist() == [0]
    assert M.n == 15


def check_invariants(N, m):
    M = mesh_mod.build_mesh(N, m)
    # every mask pixel is a vertex, in ascending index order
    xy = M.vxy[M.mask_vids]
    assert np.array_equal(xy[:, 1] * N + xy[:, 0], np.asarray(m, dtype=np.int64))
    # vertex ids follow (y, x) order
    key = M.vxy[:, 1] * (N + 1) + M.vxy[:, 0]
    assert np.all(np.diff(key) > 0)
    p = M.vxy[M.tri]
    ex1 = p[:, 1] - p[:, 0]
    ex2 = p[:, 2] - p[:, 0]
    twoA = ex1[:, 0] * ex2[:, 1] - ex1[:, 1] * ex2[:, 0]
    assert np.all(twoA > 0)
    assert twoA.sum() == 2 * N * N
    # right isosceles: squared side lengths are (a, a, 2a) in some order
    sides = np.stack([((p[:, 1] - p[:, 0]) ** 2).sum(1), ((p[:, 2] - p[:, 1]) ** 2).sum(1),
                      ((p[:, 0] - p[:, 2]) ** 2).sum(1)], axis=1)
    ss = np.sort(sides, axis=1)
    assert np.all(ss[:, 0] == ss[:, 1]) and np.all(ss[:, 2] == 2 * ss[:, 0])
    # conformity: each edge in one (boundary) or two (interior) triangles
    e = np.concatenate([M.tri[:, [0, 1]], M.tri[:, [1, 2]], M.tri[:, [2, 0]]])
    e = np.sort(e, axis=1)
    uniq, cnt = np.unique(e, axis=0, return_counts=True)
    assert cnt.max() <= 2
    bd = uniq[cnt == 1]
    a, b = M.vxy[bd[:, 0]], M.vxy[bd[:, 1]]
    on_x = (a[:, 0] == b[:, 0]) & ((a[:, 0] == 0) | (a[:, 0] == N))
    on_y = (a[:, 1] == b[:, 1]) & ((a[:, 1] == 0) | (a[:, 1] == N))
    assert np.all(on_x | on_y)
    # Euler: V - E + T = 1 for a triangulated disc
    assert M.V - uniq.shape[0] + M.T == 1
    # each vertex used by a triangle
    assert np.unique(M.tri).size == M.V
    return M


@settings(max_examples=60, deadline=None)
@given(tiny_case())
def test_invariants_tiny(case):
    N, m = case
    check_invariants(N, m)


@pytest.mark.parametrize("N,k,seed", [(32, 20, 1), (64, 205, 2), (64, 3, 3), (128, 400, 4)])
def test_invariants_medium(N, k, seed):
    check_invariants(N, random_mask(np.random.default_rng(seed), N, k))


def test_balance_and_minimality():
    rng = np.random.default_rng(7)
    for N, k in ((16, 5), (32, 9), (32, 40), (64, 30)):
        m = random_mask(rng, N, k)
        lev = quadtree.balanced_levels(N, m)
        # 2:1 balance across every edge of unit cells
        assert np.all(np.abs(np.diff(lev.astype(int), axis=0)) <= 1)
        assert np.all(np.abs(np.diff(lev.astype(int), axis=1)) <= 1)
        # minimality: merging any four sibling leaves breaks a rule
        leaves = quadtree.leaves_from_levels(lev)
        ref = quadtree.refined_levels(N, m)
        s = {tuple(x) for x in leaves.tolist()}
        for x0, y0, l in leaves.tolist():
            S = 1 << (l + 1)
            px, py = (x0 // S) * S, (y0 // S) * S
            if (px, py) != (x0, y0):
                continue
            h = S // 2
            sib = {(px, py, l), (px + h, py, l), (px, py + h, l), (px + h, py + h, l)}
            if not sib <= s:
                continue
            merged = lev.copy()
            merged[py:py + S, px:px + S] = l + 1
            refine_forces = ref[py:py + S, px:px + S].min() <= l
            nb = quadtree._neighbour_min(merged)[py:py + S, px:px + S].min()
            assert refine_forces or nb < l, (N, k, x0, y0, l)


def test_full_even_mask_gives_unit_leaves():
    N = 16
    ys, xs = np.mgrid[0:N:2, 0:N:2]
    m = np.sort((ys * N + xs).ravel())
    lev = quadtree.balanced_levels(N, m)
    assert np.all(lev == 0)
    M = mesh_mod.build_mesh(N, m)
    assert M.V == (N + 1) ** 2 and M.T == 2 * N * N


def test_empty_mask_is_one_leaf():
    M = mesh_mod.build_mesh(8, [])
    assert M.leaves.tolist() == [[0, 0, 3]]
    assert M.V == 4 and M.T == 2 and M.m == 0


def test_rejects_bad_masks():
    with pytest.raises(ValueError):
        mesh_mod.build_mesh(8, [3, 3])
    with pytest.raises(ValueError):
        mesh_mod.build_mesh(8, [5, 2])
    with pytest.raises(ValueError):
        mesh_mod.build_mesh(8, [64])
    with pytest.raises(ValueError):
        mesh_mod.build_mesh(6, [1])
