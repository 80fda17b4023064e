"""Pins of the oracle's interpolation to pixels and error measures (Sections 2.2, 3, 5).

Pins: linear functions of (x, y) at the vertices are reproduced exactly at
every pixel (a P1 interpolant is exact on linear data); weights are
non-negative and sum to one; mask pixels get their stored value exactly; the
owner rule is re-derived by a global scan over all triangles; error sums, and
each triangle's error total against errors planted at pixels with one
geometric owner.
"""
import math

import numpy as np
import pytest

from oracle import error as err
from oracle import mesh as mesh_mod, raster, tonal


def random_mask(rng, N, k):
    return np.sort(rng.choice(N * N, size=k, replace=False))


CASES = [(4, 1, 0), (8, 3, 1), (16, 12, 2), (32, 15, 3), (64, 205, 4)]


@pytest.mark.parametrize("N,k,seed", CASES)
def test_linear_reproduction_and_weights(N, k, seed):
    rng = np.random.default_rng(seed)
    M = mesh_mod.build_mesh(N, random_mask(rng, N, k))
    R = raster.rasteriser(M)
    a, b, c = rng.integers(-9, 9, size=3)
    uv = a + b * M.vxy[:, 0] + c * M.vxy[:, 1]
    u = raster.rasterise(R, uv.astype(np.float64))
    pix = np.arange(N * N)
    assert np.array_equal(u, (a + b * (pix % N) + c * (pix // N)).astype(np.float64))
    assert np.all(R.lam >= 0)
    assert np.array_equal(R.lam.sum(axis=1), np.ones(N * N))
    # weights are dyadic: scaled by 2A they are integers
    assert np.array_equal(R.lam * 2 ** 20, np.round(R.lam * 2 ** 20))


@pytest.mark.parametrize("N,k,seed", CASES[:4])
def test_owner_rule_by_global_scan(N, k, seed):
    rng = np.random.default_rng(seed)
    M = mesh_mod.build_mesh(N, random_mask(rng, N, k))
    R = raster.rasteriser(M)
    p = M.vxy[M.tri]
    lv = M.leaves[M.tri_leaf]
    s = 1 << lv[:, 2]
    for pix in range(N * N):
        x, y = pix % N, pix // N
        inbox = (lv[:, 0] <= x) & (x < lv[:, 0] + s) & (lv[:, 1] <= y) & (y < lv[:, 1] + s)
        o = []
        for i in range(3):
            A, B = p[:, i], p[:, (i + 1) % 3]
            o.append((B[:, 0] - A[:, 0]) * (y - A[:, 1]) - (B[:, 1] - A[:, 1]) * (x - A[:, 0]))
        inside = (o[0] >= 0) & (o[1] >= 0) & (o[2] >= 0)
        cands = np.nonzero(inbox & inside)[0]
        assert R.owner[pix] == cands.min()


@pytest.mark.parametrize("N,k,seed", CASES)
def test_mask_pixels_exact(N, k, seed):
    rng = np.random.default_rng(seed)
    pr = tonal.Problem(N, random_mask(rng, N, k))
    g = rng.uniform(0, 255, size=pr.mesh.m)
    u = pr.B(g)
    assert np.array_equal(u[pr.mesh.mask_idx], g)


def test_error_measures():
    rng = np.random.default_rng(5)
    N = 32
    pr = tonal.Problem(N, random_mask(rng, N, 30))
    f = np.full(N * N, 93.0)
    u = pr.inpaint(f)
    assert pr.mse(u, f) <= 1e-20   # constants are reproduced up to solver rounding
    f = rng.integers(0, 256, size=N * N).astype(np.float64)
    u = pr.inpaint(f)
    e = err.pixel_error(u, f)
    ET = pr.triangle_error(u, f)
    assert ET.shape == (pr.mesh.T,)
    assert math.isclose(ET.sum(), N * N * pr.mse(u, f), rel_tol=1e-12)
    # hand case: u - f = 1 on half the pixels, 3 on the other half
    uu = np.zeros(16)
    ff = np.concatenate([np.ones(8), np.full(8, 3.0)])
    assert err.mse(uu, ff) == 5.0


@pytest.mark.parametrize("N,k,seed", CASES[1:4])
def test_triangle_error_per_triangle(N, k, seed):
    """Each triangle's error total (Section 3's local error) pinned one by one:
    errors planted at pixels that lie in exactly one triangle (found by a
    geometric scan, not by the rasteriser's owner map) land on that triangle
    alone, and every other triangle reads zero."""
    rng = np.random.default_rng(seed + 100)
    pr = tonal.Problem(N, random_mask(rng, N, k))
    M = pr.mesh
    p = M.vxy[M.tri]
    one_owner = {}
    for pix in range(N * N):
        x, y = pix % N, pix // N
        o = []
        for i in range(3):
            A, B = p[:, i], p[:, (i + 1) % 3]
            o.append((B[:, 0] - A[:, 0]) * (y - A[:, 1]) - (B[:, 1] - A[:, 1]) * (x - A[:, 0]))
        cands = np.nonzero((o[0] >= 0) & (o[1] >= 0) & (o[2] >= 0))[0]
        if len(cands) == 1:
            one_owner[pix] = int(cands[0])
    assert len(one_owner) > 0
    picked = rng.choice(sorted(one_owner), size=min(12, len(one_owner)), replace=False)
    u = np.zeros(N * N)
    f = np.zeros(N * N)
    want = np.zeros(M.T)
    for j, pix in enumerate(picked):
        d = 2.0 ** (j % 5) * (1 if j % 2 else -1)
        f[pix] = d
        want[one_owner[int(pix)]] += d * d
    assert np.array_equal(pr.triangle_error(u, f), want)
