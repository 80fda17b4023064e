"""Pins of the oracle's B, adjoint and tonal optimisation (Section 4, eqs. (4), (5)).

Pins: the dense least-squares solution by a different library routine
(``numpy.linalg.lstsq`` on B formed column by column); the normal-equation
residual; MSE after optimisation never above MSE of f on the mask (Table 1's
qualitative claim); a full mask gives g* = f; B^T B >= I because every mask
pixel is a vertex with weight one; B is entrywise non-negative with rows
summing to one (constants are harmonic); the adjoint dot-product identity;
central finite differences of the quadratic MSE.
"""
import numpy as np
import pytest

import synth
from oracle import tonal


def random_mask(rng, N, k):
    return np.sort(rng.choice(N * N, size=k, replace=False))


TINY = [(8, 4, 0), (8, 9, 1), (16, 12, 2), (16, 30, 3)]


@pytest.mark.parametrize("N,k,seed", TINY)
def test_dense_B_properties(N, k, seed):
    pr = tonal.Problem(N, random_mask(np.random.default_rng(seed), N, k))
    B = pr.dense_B()
    assert B.min() >= -1e-13
    assert np.allclose(B.sum(axis=1), 1.0, atol=1e-12)
    ev = np.linalg.eigvalsh(B.T @ B)
    assert ev.min() >= 1.0 - 1e-10
    # the mask rows are identity rows
    assert np.allclose(B[pr.mesh.mask_idx], np.eye(pr.mesh.m), atol=1e-14)


@pytest.mark.parametrize("N,k,seed", TINY)
def test_cgls_matches_lstsq(N, k, seed):
    rng = np.random.default_rng(seed)
    pr = tonal.Problem(N, random_mask(rng, N, k))
    f = synth.make_image(seed, N, N, bumps=2, edges=1).astype(np.float64).ravel()
    g_ls = pr.tonal_lstsq(f)
    g_cg, it, rel = pr.tonal_cgls(f)
    assert rel <= 1e-13
    assert np.allclose(g_cg, g_ls, rtol=1e-9, atol=1e-8)
    nr = pr.normal_residual(g_cg, f)
    assert np.linalg.norm(nr) <= 1e-10 * np.linalg.norm(pr.BT(f))
    assert pr.mse_of_g(g_cg, f) <= pr.mse_of_g(pr.default_g(f), f) + 1e-12


def test_full_mask_gives_identity():
    N = 8
    pr = tonal.Problem(N, np.arange(N * N))
    f = np.random.default_rng(1).integers(0, 256, size=N * N).astype(np.float64)
    g, it, rel = pr.tonal_cgls(f)
    assert np.allclose(g, f, atol=1e-10)
    assert pr.mse_of_g(g, f) < 1e-20


@pytest.mark.parametrize("N,k,seed", [(16, 12, 0), (32, 40, 1), (64, 205, 2)])
def test_adjoint_dot_product(N, k, seed):
    rng = np.random.default_rng(seed)
    pr = tonal.Problem(N, random_mask(rng, N, k))
    g = rng.normal(size=pr.mesh.m)
    r = rng.normal(size=N * N)
    lhs = float(pr.B(g) @ r)
    rhs = float(g @ pr.BT(r))
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + np.linalg.norm(g) * np.linalg.norm(r))


@pytest.mark.parametrize("N,k,seed", [(16, 12, 0), (32, 40, 1)])
def test_gradient_finite_differences(N, k, seed):
    rng = np.random.default_rng(seed)
    pr = tonal.Problem(N, random_mask(rng, N, k))
    f = synth.make_image(seed, N, N, bumps=3, edges=1).astype(np.float64).ravel()
    g = pr.default_g(f) + rng.normal(scale=3.0, size=pr.mesh.m)
    grad = pr.mse_grad(g, f)
    eps = 1e-3
    for j in rng.integers(0, pr.mesh.m, size=8):
        e = np.zeros(pr.mesh.m)
        e[j] = eps
        fd = (pr.mse_of_g(g + e, f) - pr.mse_of_g(g - e, f)) / (2 * eps)
        assert abs(fd - grad[j]) <= 1e-8 * max(1.0, abs(grad[j]))


def test_tonal_lowers_mse_plain64():
    w = synth.WORKLOADS["plain64"]
    f = w.image().astype(np.float64).ravel()
    pr = tonal.Problem(w.side, w.mask())
    g, it, rel = pr.tonal_cgls(f, rtol=1e-12)
    before = pr.mse_of_g(pr.default_g(f), f)
    after = pr.mse_of_g(g, f)
    assert after < before
