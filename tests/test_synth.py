"""Seeded input generators: determinism, counts and the fast half-plane fill."""
import numpy as np
import pytest

import synth


def test_counts_from_density():
    assert synth.count_from_density(0.05, 64 * 64) == 205
    assert synth.count_from_density(0.04, 512 * 512) == 10486
    assert synth.count_from_density(0.01, 1024 * 1024) == 10486
    assert synth.count_from_density(0.001, 1024 * 1024) == 1049
    assert synth.count_from_density(0.02, 8192 * 8192) == 1342177


@pytest.mark.parametrize("seed", [1, 2, 3, 11, 12])
def test_fast_edges_equal_direct(seed):
    a = synth.make_image(seed, 48, 40, bumps=4, edges=6)
    b = synth.make_image(seed, 48, 40, bumps=4, edges=6, _direct_edges=True)
    assert np.array_equal(a, b)


def test_deterministic_and_typed():
    a = synth.WORKLOADS["plain64"].image()
    b = synth.WORKLOADS["plain64"].image()
    assert a.dtype == np.uint8 and a.shape == (64, 64)
    assert np.array_equal(a, b)
    m = synth.WORKLOADS["plain64"].mask()
    assert m.dtype == np.int32 and m.size == 205
    assert np.all(np.diff(m) > 0) and m.min() >= 0 and m.max() < 4096
    assert np.array_equal(m, synth.WORKLOADS["plain64"].mask())


def test_serving_trace():
    tr = synth.serving_trace()
    assert len(tr) == 256
    t = [r.arrival_s for r in tr]
    assert all(b > a for a, b in zip(t, t[1:]))
    assert {r.side for r in tr} <= {128, 256, 512, 1024, 2048}
    assert all(0.02 <= r.density <= 0.10 for r in tr)
    assert tr[5].image_seed == 1005


def test_colour_image():
    a = synth.make_image_rgb(7, 64, 48, bumps=8, edges=3)
    b = synth.make_image_rgb(7, 64, 48, bumps=8, edges=3)
    assert a.dtype == np.uint8 and a.shape == (3, 48, 64)
    assert np.array_equal(a, b)
    # the channels share the luminance layout but are not copies of each other
    x = a.reshape(3, -1).astype(np.float64)
    for i in range(3):
        for j in range(i + 1, 3):
            assert not np.array_equal(a[i], a[j])
            assert np.corrcoef(x[i], x[j])[0, 1] > 0.3
