"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and its host-side mesh builder matches the oracle bit for bit."""
import os
import re

import numpy as np
import pytest

import paper_2105_01586_amd as fi
import synth
from oracle import mesh as om

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            text = open(os.path.join(inc, f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(fi_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = fi.library()
    decl = declared_symbols()
    assert len(decl) >= 20
    for name in decl:
        assert hasattr(lib, name), name
    assert set(decl) == set(fi.EXPORTED_SYMBOLS)


def test_version_and_defaults():
    lib = fi.library()
    assert b"gfx950" in lib.fi_version()
    o = fi._SolveOpts()
    lib.fi_solve_opts_default(o)
    assert o.rtol == 1e-10 and o.atol == 3e-6 and o.precision == fi.PREC_FP32_IR
    t = fi._TonalOpts()
    lib.fi_tonal_opts_default(t)
    assert t.rtol == 1e-8 and t.inner.rtol == 1e-10
    t.cold_adjoint = 7
    lib.fi_tonal_opts_default(t)
    assert t.cold_adjoint == 0 and t.start_from_g == 0


def rand_mask(N, k, seed):
    return np.sort(np.random.default_rng(seed).choice(N * N, size=k, replace=False))


CASES = [(2, 1, 0), (2, 4, 1), (4, 1, 2), (8, 3, 3), (16, 10, 4), (32, 1, 5), (64, 205, 6),
         (128, 655, 7), (256, 2621, 8)]


@pytest.mark.parametrize("N,k,seed", CASES)
def test_host_mesh_bit_exact(N, k, seed):
    m = rand_mask(N, k, seed)
    h = fi.host_mesh(N, m)
    o = om.build_mesh(N, m)
    assert np.array_equal(h["leaves"], o.leaves)
    assert np.array_equal(h["vxy"], o.vxy)
    assert np.array_equal(h["tri"], o.tri)
    assert np.array_equal(h["free_vids"], o.free_vids)
    assert np.array_equal(h["mask_vids"], o.mask_vids)


def _child_tri(N, m):
    return fi.host_mesh(N, m)["tri"]


def test_host_mesh_in_forked_child():
    # the host builders' worker threads are not copied by fork: a forked
    # child builds on its own thread and gets the same mesh
    import multiprocessing as mp
    m = rand_mask(256, 2621, 8)
    h = fi.host_mesh(256, m)  # starts the workers in this process
    with mp.get_context("fork").Pool(1) as pool:
        tri = pool.apply_async(_child_tri, (256, m)).get(timeout=120)
    assert np.array_equal(tri, h["tri"])


def test_host_mesh_workload_512():
    w = synth.WORKLOADS["tonal512"]
    m = w.mask()
    h = fi.host_mesh(w.side, m)
    o = om.build_mesh(w.side, m)
    assert np.array_equal(h["tri"], o.tri) and np.array_equal(h["vxy"], o.vxy)


def test_host_mesh_full_and_edge_masks():
    N = 16
    for m in (np.arange(N * N), np.array([0]), np.array([N * N - 1]), np.array([N - 1, N * (N - 1)])):
        h = fi.host_mesh(N, m)
        o = om.build_mesh(N, m)
        assert np.array_equal(h["tri"], o.tri)


def _neighbour_counts(h):
    """Distinct neighbours and incident triangles of every vertex."""
    tri = h["tri"].astype(np.int64)
    V = h["vxy"].shape[0]
    edges = np.concatenate([tri[:, [a, b]] for a in range(3) for b in range(3) if a != b])
    edges = np.unique(edges, axis=0)
    nbrs = np.bincount(edges[:, 0], minlength=V)
    tris = np.bincount(tri.ravel(), minlength=V)
    return nbrs, tris


@pytest.mark.parametrize("N,seed,kind", [(64, 1, "random"), (128, 2, "random"), (128, 3, "border"),
                                         (256, 4, "clusters"), (64, 5, "border")])
def test_quadtree_neighbour_bound(N, seed, kind):
    # The device assembly keeps 8 neighbour slots per quadtree row: a vertex
    # inside the square has a closed fan (neighbours = triangles <= 8), one on
    # its border an open fan (neighbours = triangles + 1), so the builder must
    # keep border vertices to 7 triangles.
    rng = np.random.default_rng(seed)
    if kind == "random":
        m = np.sort(rng.choice(N * N, size=N * N // 20, replace=False))
    elif kind == "border":
        b = np.concatenate([np.arange(N), (N - 1) * N + np.arange(N), np.arange(N) * N,
                            np.arange(N) * N + N - 1])
        m = np.unique(rng.choice(b, size=N, replace=False))
    else:
        c = rng.integers(0, N, size=(6, 2))
        pts = (c[:, None, :] + rng.integers(-3, 4, size=(6, 40, 2))).reshape(-1, 2) % N
        m = np.unique(pts[:, 0] * N + pts[:, 1])
    h = fi.host_mesh(N, m)
    nbrs, tris = _neighbour_counts(h)
    x, y = h["vxy"][:, 0], h["vxy"][:, 1]
    border = (x == 0) | (y == 0) | (x == N) | (y == N)
    assert nbrs.max() <= 8
    assert np.array_equal(nbrs[~border], tris[~border])
    assert np.array_equal(nbrs[border], tris[border] + 1)
    assert tris[border].max() <= 7


@pytest.mark.parametrize("side,mask,code", [
    (16, [], fi.E_EMPTY_MASK),
    (16, [3, 3], fi.E_INVALID),
    (16, [5, 2], fi.E_INVALID),
    (16, [256], fi.E_INVALID),
    (16, [-1], fi.E_INVALID),
    (12, [1], fi.E_INVALID),
    (1, [0], fi.E_INVALID),
])
def test_host_mesh_errors(side, mask, code):
    with pytest.raises(fi.FIError) as ei:
        fi.host_mesh(side, mask)
    assert ei.value.code == code


def test_footprint_bound_host_only():
    """The server's admission bound is computed on the host from the mesh:
    positive, growing with the mesh, and rejecting bad masks."""
    side = 128
    small = synth.make_mask(7, side * side, 0.02)
    large = synth.make_mask(7, side * side, 0.10)
    b_small = fi.footprint_bound(side, small)
    b_large = fi.footprint_bound(side, large)
    P = side * side
    assert b_small > 2 * 8 * P + P      # at least r, q (float64) and f per pixel
    assert b_large > b_small
    with pytest.raises(fi.FIError):
        fi.footprint_bound(side, small[::-1].copy())
    with pytest.raises(fi.FIError):
        fi.footprint_bound(100, small)


@pytest.mark.parametrize("N,dens,seed", [(2, 0.5, 1), (8, 0.2, 2), (64, 0.05, 3), (256, 0.03, 4),
                                         (512, 0.04, 2)])
def test_host_delaunay_mesh_bit_exact(N, dens, seed):
    """The library's Delaunay builder (host C++) against the oracle's: the
    same canonical triangles, vertices and free / mask split."""
    from oracle import delaunay
    P = N * N
    mask = synth.make_mask(seed, P, dens)
    unk = synth.make_unknowns(seed, P, mask, min(mask.size, P - mask.size))
    h = fi.host_mesh(N, mask, unk)
    o = delaunay.build_mesh(N, mask, unk)
    assert np.array_equal(h["vxy"], o.vxy)
    assert np.array_equal(h["tri"], o.tri)
    assert np.array_equal(h["free_vids"], o.free_vids)
    assert np.array_equal(h["mask_vids"], o.mask_vids)
    assert h["L"] == 0


def test_host_delaunay_full_grid():
    """Every pixel a vertex: each unit square is cocircular, the diagonal is
    the perturbation's choice on both sides."""
    from oracle import delaunay
    N = 32
    pix = np.arange(N * N, dtype=np.int32)
    mask, unk = pix[::5], np.setdiff1d(pix, pix[::5])
    h = fi.host_mesh(N, mask, unk)
    assert np.array_equal(h["tri"], delaunay.build_mesh(N, mask, unk).tri)
    assert h["T"] == 2 * (N - 1) ** 2


@pytest.mark.parametrize("side,mask,unk,code", [
    (16, [], [3], fi.E_EMPTY_MASK),
    (16, [3], [3], fi.E_INVALID),
    (16, [3], [9, 5], fi.E_INVALID),
    (16, [3], [256], fi.E_INVALID),
    (12, [1], [2], fi.E_INVALID),
])
def test_host_delaunay_errors(side, mask, unk, code):
    with pytest.raises(fi.FIError) as ei:
        fi.host_mesh(side, mask, unk)
    assert ei.value.code == code
