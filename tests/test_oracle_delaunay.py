"""Pins of the oracle's Delaunay mesh (Section 2.2: mask pixels plus unknown
vertices, Delaunay-triangulated; ties broken by symbolic perturbation).

* Brute force on tiny point sets full of cocircular quadruples: the
  canonical triangles are exactly the counter-clockwise triples whose
  perturbed circumcircle holds no other vertex.
* scipy's Delaunay (Qhull) on point sets without degeneracies gives the same
  triangles.
* Invariants at the parity-test sizes: every interior edge locally regular,
  areas summing to the square, Euler's formula.
* With every pixel a vertex, the stiffness matrix is the 5-point Laplacian
  with the reflecting boundary, which Section 2.2 names as the limit.
* Owner map against a brute-force minimum over all containing triangles.
* The harmonic solve on this mesh: constants reproduced, mask values kept,
  K_FF symmetric positive definite (Section 2.2), and every interior edge's
  entry non-positive (its two opposite angles sum to at most pi).
"""
import itertools

import numpy as np
import pytest
import scipy.spatial

import synth
from oracle import delaunay as D
from oracle import fem, tonal


def brute_triangles(N, pix):
    P = [(int(p % N), int(p // N)) for p in pix]
    V = len(P)
    out = set()
    for a, b, c in itertools.combinations(range(V), 3):
        o = D.orient(*P[a], *P[b], *P[c])
        if o == 0:
            continue
        if o < 0:
            b, c = c, b
        if all(not D.inside(P, a, b, c, d) for d in range(V) if d not in (a, b, c)):
            k = min(range(3), key=lambda i: (a, b, c)[i])
            t = (a, b, c)[k:] + (a, b, c)[:k]
            out.add(t)
    return out


@pytest.mark.parametrize("N,k,seed", [(4, 3, 0), (5, 6, 1), (6, 9, 2), (7, 14, 3)])
def test_brute_force_tiny(N, k, seed):
    rng = np.random.default_rng(seed)
    sel = rng.choice(N * N, size=k, replace=False)
    mask = np.sort(sel[: k // 2])
    unk = np.sort(sel[k // 2:])
    M = D.build_mesh(N, mask, unk)
    assert set(map(tuple, M.tri.tolist())) == brute_triangles(N, M.pix)


def test_full_grid_brute_force():
    """Every pixel a vertex: every unit square is cocircular; the diagonal of
    each is decided by the perturbation alone."""
    N = 5
    pix = np.arange(N * N)
    M = D.build_mesh(N, pix[:1], pix[1:])
    assert set(map(tuple, M.tri.tolist())) == brute_triangles(N, M.pix)
    assert M.T == 2 * (N - 1) ** 2


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_matches_scipy_without_ties(seed):
    N = 4096
    rng = np.random.default_rng(seed)
    xy = rng.integers(1, N - 1, size=(300, 2))
    pix = np.unique(xy[:, 1] * N + xy[:, 0])
    mask, unk = pix[::2], pix[1::2]
    M = D.build_mesh(N, mask, unk)
    pts = M.vxy.astype(np.float64)
    sp = scipy.spatial.Delaunay(pts)
    assert sp.coplanar.size == 0
    ref = set()
    for a, b, c in sp.simplices.tolist():
        if D.orient(*M.vxy[a], *M.vxy[b], *M.vxy[c]) < 0:
            b, c = c, b
        k = min(range(3), key=lambda i: (a, b, c)[i])
        ref.add(((a, b, c)[k:] + (a, b, c)[:k]))
    assert set(map(tuple, M.tri.tolist())) == ref


@pytest.mark.parametrize("N,dens,seed", [(64, 0.05, 6), (256, 0.02, 7)])
def test_invariants(N, dens, seed):
    mask = synth.make_mask(seed, N * N, dens)
    unk = synth.make_unknowns(seed, N * N, mask, mask.size)
    M = D.build_mesh(N, mask, unk)
    assert D.is_regular(N, M.pix, M.tri)
    x = M.vxy
    t = M.tri
    a2 = ((x[t[:, 1], 0] - x[t[:, 0], 0]) * (x[t[:, 2], 1] - x[t[:, 0], 1])
          - (x[t[:, 1], 1] - x[t[:, 0], 1]) * (x[t[:, 2], 0] - x[t[:, 0], 0]))
    assert a2.min() > 0 and a2.sum() == 2 * (N - 1) ** 2
    on_hull = (x[:, 0] == 0) | (x[:, 0] == N - 1) | (x[:, 1] == 0) | (x[:, 1] == N - 1)
    assert M.T == 2 * M.V - int(on_hull.sum()) - 2
    assert np.array_equal(np.unique(t), np.arange(M.V))
    # canonical listing: lowest id first, lexicographic
    assert np.all(t[:, 0] < t[:, 1]) and np.all(t[:, 0] < t[:, 2])
    assert np.all(np.diff(t[:, 0]) >= 0)
    assert M.m == mask.size and M.n == M.V - mask.size


def test_full_grid_is_five_point_laplacian():
    N = 9
    pix = np.arange(N * N)
    mask = pix[::7]
    unk = np.setdiff1d(pix, mask)
    M = D.build_mesh(N, mask, unk)
    K = fem.assemble(M).K.toarray()
    # vertex id = pixel index here (every pixel is a vertex)
    ref = np.zeros((N * N, N * N))
    for r in range(N):
        for c in range(N):
            i = r * N + c
            for dr, dc in ((0, 1), (1, 0)):
                rr, cc = r + dr, c + dc
                if rr >= N or cc >= N:
                    continue
                j = rr * N + cc
                # an edge on the border belongs to one triangle pair half
                w = 0.5 if (dr == 0 and (r == 0 or r == N - 1)) or \
                    (dc == 0 and (c == 0 or c == N - 1)) else 1.0
                ref[i, j] -= w
                ref[j, i] -= w
                ref[i, i] += w
                ref[j, j] += w
    assert np.array_equal(K, ref)


def test_owner_brute_force():
    N = 24
    mask = synth.make_mask(8, N * N, 0.06)
    unk = synth.make_unknowns(8, N * N, mask, mask.size)
    M = D.build_mesh(N, mask, unk)
    rast = D.rasteriser(M)
    x = M.vxy
    for p in range(N * N):
        px, py = p % N, p // N
        best = None
        for ti, (a, b, c) in enumerate(M.tri.tolist()):
            if (D.orient(*x[a], *x[b], px, py) >= 0 and D.orient(*x[b], *x[c], px, py) >= 0
                    and D.orient(*x[c], *x[a], px, py) >= 0):
                best = ti
                break
        assert rast.owner[p] == best
    # weights reproduce the pixel position and sum to one
    lam = rast.lam
    assert np.allclose(lam.sum(axis=1), 1.0, atol=1e-12)
    pos = np.einsum("pk,pkd->pd", lam, x[M.tri[rast.owner]].astype(np.float64))
    pix = np.arange(N * N)
    assert np.allclose(pos, np.stack([pix % N, pix // N], axis=1), atol=1e-9)


def test_harmonic_solve_on_delaunay():
    N = 64
    mask = synth.make_mask(9, N * N, 0.04)
    unk = synth.make_unknowns(9, N * N, mask, mask.size)
    pr = tonal.Problem(N, mask, unknown_idx=unk)
    K = pr.sys.K.toarray()
    # an interior edge has two opposite angles summing to at most pi, so its
    # entry is <= 0; a hull edge has one, possibly obtuse, so no sign there
    x = pr.mesh.vxy
    count = {}
    for a, b, c in pr.mesh.tri.tolist():
        for u, v in ((a, b), (b, c), (c, a)):
            count[(min(u, v), max(u, v))] = count.get((min(u, v), max(u, v)), 0) + 1
    for (u, v), k in count.items():
        if k == 2:
            assert K[u, v] <= 1e-12
        else:
            assert k == 1
            on = (x[u] == x[v]) & ((x[u] == 0) | (x[u] == N - 1))
            assert on.any()  # a single-triangle edge lies on the square's border
    assert np.allclose(K.sum(axis=1), 0.0, atol=1e-10)
    # symmetric positive definite with a mask pixel (Section 2.2)
    Kff = pr.sys.K_FF.toarray()
    assert np.array_equal(Kff, Kff.T)
    assert np.linalg.eigvalsh(Kff).min() > 0
    u = pr.B(np.full(mask.size, 77.0))
    assert np.max(np.abs(u - 77.0)) <= 1e-9
    g = synth.make_image(9, N, N, 8, 3).ravel()[mask].astype(np.float64)
    u = pr.B(g)
    assert np.array_equal(u[mask], g)
