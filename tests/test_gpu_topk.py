"""GPU top-k mask growth against the oracle's selection on identical errors.

Both sides select from the same float64 error map, so the selection (an
integer result) must match bit for bit, ties included.
"""
import numpy as np
import pytest
import torch

import paper_2105_01586_amd as fi
from oracle import densify
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = fi.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("side,k_mask,k_new,seed,ties", [
    (64, 41, 4, 0, False), (128, 164, 16, 1, True), (256, 655, 66, 2, False),
    (1024, 10486, 1049, 3, False), (256, 655, 0, 4, False), (64, 41, 4096 - 41, 5, True),
])
def test_topk_matches_oracle(ctx, side, k_mask, k_new, seed, ties):
    print(f"case side {side} k {k_new} ties {ties}", flush=True)
    mask = synth.make_mask(seed, side * side, k=k_mask)
    M = fi.Mesh(ctx, side, mask)
    rng = np.random.default_rng(seed)
    if ties:
        e = rng.integers(0, 5, size=side * side).astype(np.float64)
    else:
        e = rng.exponential(10.0, size=side * side)
    got = M.topk_new_pixels(torch.from_numpy(e).cuda(), k_new).cpu().numpy()
    want = densify.topk_new_pixels(e, mask, k_new)
    assert np.array_equal(got, want)
    M.close()


def test_topk_rejects_too_many(ctx):
    mask = synth.make_mask(9, 256, k=10)
    M = fi.Mesh(ctx, 16, mask)
    with pytest.raises(fi.FIError):
        M.topk_new_pixels(torch.zeros(256, dtype=torch.float64, device="cuda:0"), 247)
    M.close()
