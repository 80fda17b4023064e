"""The allocation-free top-k entry point against fi_topk_new_pixels.

fi_topk_new_pixels_noalloc takes its workspace from a fixed device array in
the library instead of memory the mesh allocates; its result must be the
same, bit for bit. Two calls in a row share that array, the second on a
smaller image, and each must match; so must a third at the full size again
after the smaller one. Meshes above 2^20 pixels are refused.
"""
import numpy as np
import pytest
import torch

import paper_2105_01586_amd as fi
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = fi.Context(0)
    yield c
    c.close()


def _case(ctx, side, k_mask, seed, ties):
    mask = synth.make_mask(seed, side * side, k=k_mask)
    M = fi.Mesh(ctx, side, mask)
    rng = np.random.default_rng(seed)
    if ties:
        e = rng.integers(0, 5, size=side * side).astype(np.float64)
    else:
        e = rng.exponential(10.0, size=side * side)
    return M, torch.from_numpy(e).cuda()


def test_noalloc_topk_matches_allocating_path(ctx):
    cases = [(1024, 10486, 1049, 3, False), (256, 655, 66, 2, True), (1024, 20000, 5000, 4, True)]
    for side, k_mask, k_new, seed, ties in cases:
        print(f"case side {side} k {k_new} ties {ties}", flush=True)
        M, e = _case(ctx, side, k_mask, seed, ties)
        out = torch.full((k_new,), -7, dtype=torch.int32, device="cuda:0")
        M.topk_new_pixels_noalloc(e, out)
        want = M.topk_new_pixels(e, k_new)
        assert torch.equal(out, want)
        M.close()


def test_noalloc_topk_limits(ctx):
    print("case limits", flush=True)
    M, e = _case(ctx, 16, 10, 9, False)
    with pytest.raises(fi.FIError):  # more pixels than there are candidates
        M.topk_new_pixels_noalloc(e, torch.zeros(247, dtype=torch.int32, device="cuda:0"))
    M.topk_new_pixels_noalloc(e, torch.zeros(0, dtype=torch.int32, device="cuda:0"))
    M.close()
    big = fi.Mesh(ctx, 2048, synth.make_mask(10, 2048 * 2048, k=1000))
    with pytest.raises(fi.FIError):  # above the 2^20-pixel limit
        big.topk_new_pixels_noalloc(torch.zeros(2048 * 2048, dtype=torch.float64,
                                                device="cuda:0"),
                                    torch.zeros(4, dtype=torch.int32, device="cuda:0"))
    big.close()
