"""Pins of the oracle's Delaunay mesh (Section 2.2: mask pixels plus unknown
vertices, Delaunay-triangulated; ties broken by symbolic perturbation).

* Brute force on tiny point sets full of cocircular quadruples: the
  canonical triangles are exactly the counter-clockwise triples whose
  perturbed circumcircle holds no other vertex.
* The same sets against a construction that shares nothing with the
  oracle's predicates: the points are lifted to heights x^2 + y^2 + d^(id+1)
  with a concrete d = 2^-64 (all heights scaled to exact integers), and the
  lower convex hull of the lifted points is enumerated face by face with 3-D
  integer cross products. The lower hull of the lifted points is the
  Delaunay triangulation (Section 2.2's criterion); the concrete d stands in
  for the infinitesimal perturbation because every coefficient it multiplies
  is far below 2^64.
* Local convexity of the lifted surface across every interior edge, again by
  3-D cross products, on the oracle mesh of every GPU parity case: a
  triangulation of a convex domain whose lifted surface is locally convex at
  every edge is the lower hull, hence the unique perturbed Delaunay one.
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


# --- lifted lower hull, independent of the oracle's predicates ------------
_DELTA_BITS = 64  # the concrete perturbation d = 2^-64


def _lift(N, pix, ids):
    """Integer lifted points (x, y, H) for the vertices `ids` (ascending
    ranks r = 0, 1, ... among them): H = (x^2 + y^2) 2^(64 (k + 1)) +
    2^(64 (k - r)), i.e. x^2 + y^2 + d^(r+1) scaled by d^-(k+1), k = len(ids).
    A lower id gets the larger perturbation, as e_0 >> e_1 >> ... demands."""
    k = len(ids)
    out = []
    for r, v in enumerate(ids):
        x, y = int(pix[v] % N), int(pix[v] // N)
        h = ((x * x + y * y) << (_DELTA_BITS * (k + 1))) + (1 << (_DELTA_BITS * (k - r)))
        out.append((x, y, h))
    return out


def _sub(p, q):
    return (p[0] - q[0], p[1] - q[1], p[2] - q[2])


def _cross(u, v):
    return (u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0])


def _dot(u, v):
    return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]


def lower_hull_triangles(N, pix):
    """Faces (a, b, c) of the lower convex hull of the lifted vertices, each
    counter-clockwise in the plane and rotated to start at its lowest id."""
    V = len(pix)
    L = _lift(N, pix, list(range(V)))
    out = set()
    for a, b, c in itertools.combinations(range(V), 3):
        nrm = _cross(_sub(L[b], L[a]), _sub(L[c], L[a]))
        if nrm[2] == 0:
            continue  # collinear in the plane: no face
        if nrm[2] < 0:  # orient counter-clockwise: normal pointing up
            b, c = c, b
            nrm = (-nrm[0], -nrm[1], -nrm[2])
        # a lower face: every other lifted point strictly above its plane
        if all(_dot(nrm, _sub(L[d], L[a])) > 0 for d in range(V) if d not in (a, b, c)):
            k = min(range(3), key=lambda i: (a, b, c)[i])
            out.add((a, b, c)[k:] + (a, b, c)[:k])
    return out


def lifted_locally_convex(N, pix, tris):
    """Every interior edge (u, v) with triangles (u, v, w) and (v, u, x): x
    lifted lies strictly above the plane of lifted u, v, w, with the
    perturbation ranks taken among the four ids (only their order matters
    for the sign of the symbolic determinant)."""
    opp = {}
    for a, b, c in np.asarray(tris).tolist():
        for (u, v, w) in ((a, b, c), (b, c, a), (c, a, b)):
            opp[(u, v)] = w
    checked = 0
    for (u, v), w in opp.items():
        x = opp.get((v, u))
        if x is None or u > v:
            continue
        ids = sorted((u, v, w, x))
        L = dict(zip(ids, _lift(N, pix, ids)))
        nrm = _cross(_sub(L[v], L[u]), _sub(L[w], L[u]))
        assert nrm[2] > 0, "triangle not counter-clockwise"
        if not _dot(nrm, _sub(L[x], L[u])) > 0:
            return False
        checked += 1
    return checked > 0


def test_lift_orders_perturbations():
    """The lift itself: heights grow with x^2 + y^2 first, and at equal
    x^2 + y^2 the lower id sits higher by orders of magnitude."""
    L = _lift(8, np.array([0, 1, 8, 9]), [0, 1, 2, 3])
    base = 1 << (_DELTA_BITS * 5)
    assert [h // base for _, _, h in L] == [0, 1, 1, 2]
    e = [h % base for _, _, h in L]
    assert e == [1 << (_DELTA_BITS * (4 - r)) for r in range(4)]


@pytest.mark.parametrize("N,k,seed", [(4, 3, 0), (5, 6, 1), (6, 9, 2), (7, 14, 3), (8, 18, 4)])
def test_lifted_lower_hull_tiny(N, k, seed):
    rng = np.random.default_rng(seed)
    sel = rng.choice(N * N, size=k, replace=False)
    mask = np.sort(sel[: k // 2])
    unk = np.sort(sel[k // 2:])
    M = D.build_mesh(N, mask, unk)
    assert set(map(tuple, M.tri.tolist())) == lower_hull_triangles(N, M.pix)


@pytest.mark.parametrize("N", [4, 5])
def test_lifted_lower_hull_full_grid(N):
    """Every pixel a vertex: all unit squares cocircular, so every diagonal
    is the perturbation's choice, and the lifted hull decides it alone."""
    pix = np.arange(N * N)
    M = D.build_mesh(N, pix[:1], pix[1:])
    assert set(map(tuple, M.tri.tolist())) == lower_hull_triangles(N, M.pix)


def test_lifted_check_rejects_a_flipped_diagonal():
    """The local test is not vacuous: flipping one diagonal of the 4x4 full
    grid's canonical mesh makes it fail."""
    N = 4
    pix = np.arange(N * N)
    M = D.build_mesh(N, pix[:1], pix[1:])
    tris = [tuple(t) for t in M.tri.tolist()]
    assert lifted_locally_convex(N, M.pix, tris)
    # find two triangles sharing an edge and flip it
    opp = {}
    for ti, (a, b, c) in enumerate(tris):
        for (u, v, w) in ((a, b, c), (b, c, a), (c, a, b)):
            opp[(u, v)] = (ti, w)
    for (u, v), (t1, w) in opp.items():
        if (v, u) in opp:
            t2, x = opp[(v, u)]
            break
    flipped = [t for i, t in enumerate(tris) if i not in (t1, t2)]
    flipped += [(w, x, v), (x, w, u)]
    assert not lifted_locally_convex(N, M.pix, flipped)


def _gpu_parity_case(side, dens, seed):
    P = side * side
    mask = synth.make_mask(seed, P, dens)
    unk = synth.make_unknowns(seed, P, mask, mask.size)
    return mask, unk


# the meshes the GPU Delaunay parity tests compare against (side, density, seed)
_PARITY_CASES = {"d16": (16, 0.10, 21), "d64": (64, 0.05, 22), "d256": (256, 0.03, 23),
                 "d512": (512, 0.04, 2)}


@pytest.mark.parametrize("name", list(_PARITY_CASES))
def test_parity_meshes_regular_and_valid(name):
    side, dens, seed = _PARITY_CASES[name]
    mask, unk = _gpu_parity_case(side, dens, seed)
    M = D.build_mesh(side, mask, unk)
    assert lifted_locally_convex(side, M.pix, M.tri)
    assert D.is_regular(side, M.pix, M.tri)
    x = M.vxy.astype(np.int64)
    t = M.tri
    a2 = ((x[t[:, 1], 0] - x[t[:, 0], 0]) * (x[t[:, 2], 1] - x[t[:, 0], 1])
          - (x[t[:, 1], 1] - x[t[:, 0], 1]) * (x[t[:, 2], 0] - x[t[:, 0], 0]))
    assert a2.min() > 0 and a2.sum() == 2 * (side - 1) ** 2
    # Euler: V - E + T = 1 for a triangulated disc
    edges = set()
    for a, b, c in t.tolist():
        edges.update({(min(a, b), max(a, b)), (min(b, c), max(b, c)), (min(c, a), max(c, a))})
    assert M.V - len(edges) + M.T == 1
    # every edge in one or two triangles, the single ones on the border
    on_hull = (x[:, 0] == 0) | (x[:, 0] == side - 1) | (x[:, 1] == 0) | (x[:, 1] == side - 1)
    assert M.T == 2 * M.V - int(on_hull.sum()) - 2


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
