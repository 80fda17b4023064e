"""Colour images on the GPU (Section 5: the method per channel on one shared
mesh), through the multi-right-hand-side step.

* Bit-exact equality with the grey path, channel by channel: each channel's
  u (and its iteration counts) equals what fi_inpaint returns for that
  channel's data on the same mesh, in FP32+refinement and in FP64, with the
  in-kernel and the separate partial-sum reduction, and when the channels
  end their solves at different launches (a zero channel ends at once).
* Parity with the oracle: pixels within 1e-6 on the 0-255 scale, the colour
  MSE within 1e-6 relative.
* Tonal optimisation: g and the statistics of every channel equal
  fi_tonal_opt's on that channel, bit for bit, for a fixed number of
  iterations and when the channels stop at different iterations (rtol > 0);
  30 iterations agree with the oracle's per-channel CGLS (tonal MSE within
  1e-6 relative, g within 1e-3).
"""
import numpy as np
import pytest
import torch

import paper_2105_01586_amd as fi
import synth
from oracle import colour, tonal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = fi.Context(0)
    yield c
    c.close()


# (side, density, seed); the last spans several blocks with a ragged tail
CASES = [(16, 0.10, 1), (64, 0.05, 2), (256, 0.04, 3), (512, 0.02, 4)]


def rgb_case(side, density, seed):
    f = synth.make_image_rgb(seed, side, side, max(8, side // 16), max(3, side // 64))
    mask = synth.make_mask(seed, side * side, density)
    return f.reshape(3, -1), mask


def grey_channels(M, f, opts=None):
    out = []
    for c in range(3):
        u, st = M.inpaint(f=torch.from_numpy(f[c].copy()).cuda(), opts=opts)
        out.append((u.cpu().numpy(), st))
    return out


def check_same_bits(u_rgb, st_rgb, grey, P):
    u_rgb = u_rgb.cpu().numpy().reshape(3, P)
    for c in range(3):
        assert np.array_equal(u_rgb[c], grey[c][0]), f"channel {c}"
        assert st_rgb[c]["iterations"] == grey[c][1]["iterations"]
        assert st_rgb[c]["refinements"] == grey[c][1]["refinements"]


@pytest.mark.parametrize("side,density,seed", CASES)
def test_rgb_equals_grey_channels(ctx, side, density, seed):
    f, mask = rgb_case(side, density, seed)
    M = fi.Mesh(ctx, side, mask)
    u, st = M.inpaint_rgb(f=torch.from_numpy(f.ravel().copy()).cuda())
    grey = grey_channels(M, f)
    print(f"  {side}^2: iterations {[s['iterations'] for s in st]}", flush=True)
    check_same_bits(u, st, grey, side * side)
    M.close()


@pytest.mark.parametrize("side,density,seed", CASES[:3])
def test_rgb_vs_oracle(ctx, side, density, seed):
    f, mask = rgb_case(side, density, seed)
    M = fi.Mesh(ctx, side, mask)
    fd = torch.from_numpy(f.ravel().copy()).cuda()
    u, _ = M.inpaint_rgb(f=fd)
    mse, mse_ch = M.error_rgb(u, fd)
    M.close()
    pr = tonal.Problem(side, mask)
    want = colour.inpaint(pr, f)
    got = u.cpu().numpy().reshape(3, -1)
    err = np.max(np.abs(got - want))
    mse_ref = colour.mse(want, f)
    print(f"  {side}^2: max |u - oracle| {err:.2e}; mse {mse:.9f} / {mse_ref:.9f}", flush=True)
    assert err <= 1e-6
    assert abs(mse - mse_ref) <= 1e-6 * mse_ref
    for c in range(3):
        ref_c = pr.mse(want[c], f[c])
        assert abs(mse_ch[c] - ref_c) <= 1e-6 * ref_c
    assert mse == pytest.approx(sum(mse_ch) / 3, rel=1e-14)


def test_rgb_separate_reduction(ctx, monkeypatch):
    side, density, seed = 256, 0.04, 5
    f, mask = rgb_case(side, density, seed)
    monkeypatch.setenv("FI_CG_LARGE", "1")
    M = fi.Mesh(ctx, side, mask)
    monkeypatch.delenv("FI_CG_LARGE")
    assert M.large_mode()
    u, st = M.inpaint_rgb(f=torch.from_numpy(f.ravel().copy()).cuda())
    check_same_bits(u, st, grey_channels(M, f), side * side)
    want = colour.inpaint(tonal.Problem(side, mask), f)
    assert np.max(np.abs(u.cpu().numpy().reshape(3, -1) - want)) <= 1e-6
    M.close()


def test_rgb_fp64(ctx):
    side, density, seed = 128, 0.05, 6
    f, mask = rgb_case(side, density, seed)
    M = fi.Mesh(ctx, side, mask)
    o = fi.SolveOpts(precision=fi.PREC_FP64)
    u, st = M.inpaint_rgb(f=torch.from_numpy(f.ravel().copy()).cuda(), opts=o)
    check_same_bits(u, st, grey_channels(M, f, o), side * side)
    M.close()


def test_channels_ending_at_different_launches(ctx):
    """A zero channel ends its solve in its first launch, a constant one
    after a few iterations; the third runs on. Each keeps its own bits."""
    side, density, seed = 256, 0.03, 7
    f, mask = rgb_case(side, density, seed)
    f = f.copy()
    f[1] = 0
    f[2] = 90
    M = fi.Mesh(ctx, side, mask)
    u, st = M.inpaint_rgb(f=torch.from_numpy(f.ravel().copy()).cuda())
    grey = grey_channels(M, f)
    print(f"  iterations {[s['iterations'] for s in st]}", flush=True)
    check_same_bits(u, st, grey, side * side)
    ur = u.cpu().numpy().reshape(3, -1)
    assert st[1]["iterations"] == 0 and np.all(ur[1] == 0.0)
    assert np.max(np.abs(ur[2] - 90.0)) <= 1e-6
    M.close()


def test_rgb_given_g_and_full_mask(ctx):
    side = 64
    f, mask = rgb_case(side, 0.05, 8)
    M = fi.Mesh(ctx, side, mask)
    rng = np.random.default_rng(8)
    g = rng.uniform(0, 255, size=3 * mask.size)
    u, _ = M.inpaint_rgb(g=torch.from_numpy(g).cuda())
    M.close()
    want = colour.inpaint(tonal.Problem(side, mask), f, g.reshape(3, -1))
    assert np.max(np.abs(u.cpu().numpy().reshape(3, -1) - want)) <= 1e-6
    # every pixel in the mask (only the lattice's last row and column, which
    # carry no pixel, stay free): u = f exactly in every channel
    full = np.arange(16 * 16, dtype=np.int32)
    f16 = synth.make_image_rgb(9, 16, 16, 4, 2).reshape(3, -1)
    M = fi.Mesh(ctx, 16, full)
    assert M.n == 2 * 16 + 1
    u, st = M.inpaint_rgb(f=torch.from_numpy(f16.ravel().copy()).cuda())
    assert np.array_equal(u.cpu().numpy(), f16.ravel().astype(np.float64))
    check_same_bits(u, st, grey_channels(M, f16), 16 * 16)
    M.close()


def tonal_grey(M, f, opts):
    out = []
    for c in range(3):
        g, ts = M.tonal_opt(torch.from_numpy(f[c].copy()).cuda(), opts=opts)
        out.append((g.cpu().numpy(), ts))
    return out


@pytest.mark.parametrize("side,density,seed,rtol,iters", [(64, 0.05, 10, 0.0, 30),
                                                           (128, 0.04, 11, 1e-6, 500),
                                                           (256, 0.03, 12, 0.0, 8)])
def test_tonal_rgb_equals_grey_channels(ctx, side, density, seed, rtol, iters):
    f, mask = rgb_case(side, density, seed)
    M = fi.Mesh(ctx, side, mask)
    opts = fi.TonalOpts(rtol=rtol, max_outer=iters)
    g, st = M.tonal_opt_rgb(torch.from_numpy(f.ravel().copy()).cuda(), opts=opts)
    grey = tonal_grey(M, f, opts)
    M.close()
    g = g.cpu().numpy().reshape(3, -1)
    print(f"  outer {[s['outer_iterations'] for s in st]}, inner "
          f"{[s['inner_iterations'] for s in st]}", flush=True)
    for c in range(3):
        assert np.array_equal(g[c], grey[c][0]), f"channel {c}"
        for k in ("outer_iterations", "inner_iterations", "mse_initial", "mse_final",
                  "rel_normal_residual", "status"):
            assert st[c][k] == grey[c][1][k], (c, k)


def test_tonal_rgb_vs_oracle(ctx):
    side, density, seed, iters = 64, 0.06, 13, 30
    f, mask = rgb_case(side, density, seed)
    M = fi.Mesh(ctx, side, mask)
    g, st = M.tonal_opt_rgb(torch.from_numpy(f.ravel().copy()).cuda(),
                            opts=fi.TonalOpts(rtol=0.0, max_outer=iters))
    M.close()
    pr = tonal.Problem(side, mask)
    g_ref, its, _ = colour.tonal_cgls(pr, f, rtol=0.0, maxit=iters)
    assert its == [iters] * 3
    g = g.cpu().numpy().reshape(3, -1)
    assert np.max(np.abs(g - g_ref)) <= 1e-3
    for c in range(3):
        ref = pr.mse_of_g(g_ref[c], f[c])
        assert abs(st[c]["mse_final"] - ref) <= 1e-6 * ref
    u_ref = colour.inpaint(pr, f, g_ref)
    assert colour.mse(u_ref, f) < colour.mse(colour.inpaint(pr, f), f)


def test_multi_kernel_timing_and_bytes(ctx):
    side, density, seed = 256, 0.04, 14
    f, mask = rgb_case(side, density, seed)
    M = fi.Mesh(ctx, side, mask)
    b1 = M.cg_kernel_bytes()
    b3 = M.cg_multi_kernel_bytes(3)
    nnz_off = M.info["nnz_ff"] - M.n
    # the three-iteration launch: 2 bytes per matrix entry (once for all
    # solves) and 76 per row and solve (basis records read and written,
    # correction read and written, diagonal); one iteration per launch: 4 per
    # entry and 44 per row and solve
    if M.info["cg_iters_per_launch"] == 3:
        assert b3 == 2 * nnz_off + 3 * 76 * M.n and b1 == 2 * nnz_off + 76 * M.n
    else:
        assert b3 == 4 * nnz_off + 3 * 44 * M.n and b1 == 4 * nnz_off + 44 * M.n
    for nrhs in (1, 2, 3):
        assert M.time_cg_multi_kernel(nrhs, reps=20) > 0
    assert M.device_bytes() > M.info["device_bytes"]  # channel state now exists
    # the channel states are left undefined by timing; a solve starts afresh
    u, st = M.inpaint_rgb(f=torch.from_numpy(f.ravel().copy()).cuda())
    check_same_bits(u, st, grey_channels(M, f), side * side)
    M.close()


def test_rgb512_workload_vs_oracle(ctx):
    """The colour workload as timed: the 512^2, 4% image in three channels,
    inpainted and tonally optimised to 1e-8 on the GPU, against the oracle's
    inpainting and its CGLS (exact inner solves) to 1e-12."""
    w = synth.WORKLOADS["tonal512"]
    side = w.side
    f = synth.make_image_rgb(w.seed, side, side, w.bumps, w.edges, w.sigma_lo,
                             w.sigma_hi).reshape(3, -1)
    mask = w.mask()
    M = fi.Mesh(ctx, side, mask)
    fd = torch.from_numpy(f.ravel().copy()).cuda()
    u, _ = M.inpaint_rgb(f=fd)
    mse, _ = M.error_rgb(u, fd)
    g, st = M.tonal_opt_rgb(fd, opts=fi.TonalOpts(rtol=1e-8))
    M.close()
    pr = tonal.Problem(side, mask)
    want = colour.inpaint(pr, f)
    err = np.max(np.abs(u.cpu().numpy().reshape(3, -1) - want))
    mse_ref = colour.mse(want, f)
    print(f"  inpainting: max |u - oracle| {err:.2e}; mse {mse:.9f} / {mse_ref:.9f}", flush=True)
    assert err <= 1e-6
    assert abs(mse - mse_ref) <= 1e-6 * mse_ref
    g_ref, _, _ = colour.tonal_cgls(pr, f, rtol=1e-12, maxit=2000)
    for c in range(3):
        ref = pr.mse_of_g(g_ref[c], f[c])
        print(f"  channel {c}: tonal mse {st[c]['mse_final']:.9f} / {ref:.9f}, "
              f"{st[c]['outer_iterations']} outer", flush=True)
        assert st[c]["status"] == 0
        assert abs(st[c]["mse_final"] - ref) <= 1e-6 * ref
