"""Pins of the oracle's colour form (Section 5: the method per channel, on
one shared mesh; planar (3, P) arrays; colour MSE over all 3P values).

Each pin follows from the mathematics, not from the oracle's code: B is
linear and reproduces constants (its rows sum to one), so for channels
f1 = 255 - f0 and f2 = const the results obey u1 = 255 - u0, u2 = const,
and CGLS, started from f on the mask, is equivariant under the same affine
maps (r, s, p, q change sign; the step lengths do not). The colour MSE of
such an image is two thirds of the grey MSE. A permutation of the channels
permutes the results, and a full mask reproduces every channel exactly.
"""
import numpy as np
import pytest

import synth
from oracle import colour, tonal


def affine_image(seed, side):
    f0 = synth.make_image(seed, side, side, 8, 3).ravel()
    return np.stack([f0, (255 - f0).astype(np.uint8), np.full_like(f0, 77)])


@pytest.mark.parametrize("side,density,seed", [(16, 0.10, 1), (32, 0.05, 2), (64, 0.04, 3)])
def test_affine_channels(side, density, seed):
    f = affine_image(seed, side)
    mask = synth.make_mask(seed, side * side, density)
    pr = tonal.Problem(side, mask)
    u = colour.inpaint(pr, f)
    assert u.shape == (3, side * side)
    assert np.max(np.abs(u[1] - (255.0 - u[0]))) <= 1e-10
    assert np.max(np.abs(u[2] - 77.0)) <= 1e-10
    # mask pixels hold their data in every channel
    assert np.array_equal(u[:, mask], f[:, mask].astype(np.float64))
    e0 = (u[0] - f[0]) ** 2
    assert colour.mse(u, f) == pytest.approx(2.0 * e0.mean() / 3.0, rel=1e-12)


@pytest.mark.parametrize("side,density,seed", [(16, 0.10, 4), (32, 0.05, 5)])
def test_tonal_affine_channels(side, density, seed):
    f = affine_image(seed, side)
    mask = synth.make_mask(seed, side * side, density)
    pr = tonal.Problem(side, mask)
    g, its, _ = colour.tonal_cgls(pr, f, rtol=0.0, maxit=12)
    assert g.shape == (3, mask.size)
    assert its[0] == its[1] == 12
    assert np.max(np.abs(g[1] - (255.0 - g[0]))) <= 1e-8
    # a constant channel is already optimal (its residual is rounding only)
    assert np.max(np.abs(g[2] - 77.0)) <= 1e-8
    u = colour.inpaint(pr, f, g)
    assert colour.mse(u, f) <= colour.mse(colour.inpaint(pr, f), f)


def test_channel_permutation():
    side = 32
    f = synth.make_image_rgb(6, side, side, 8, 3).reshape(3, -1)
    mask = synth.make_mask(6, side * side, 0.06)
    pr = tonal.Problem(side, mask)
    u = colour.inpaint(pr, f)
    perm = [2, 0, 1]
    up = colour.inpaint(pr, f[perm])
    assert np.array_equal(up, u[perm])
    g = np.stack([np.linspace(0, 255, mask.size) * (c + 1) / 3 for c in range(3)])
    ug = colour.inpaint(pr, f, g)
    assert np.array_equal(colour.inpaint(pr, f[perm], g[perm]), ug[perm])


def test_full_mask_reproduces():
    side = 16
    f = synth.make_image_rgb(8, side, side, 4, 2).reshape(3, -1)
    pr = tonal.Problem(side, np.arange(side * side, dtype=np.int32))
    u = colour.inpaint(pr, f)
    assert np.array_equal(u, f.astype(np.float64))
    assert colour.mse(u, f) == 0.0
