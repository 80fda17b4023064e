"""GPU tests of the batched server (requests: inpaint, then 30 CGLS
iterations of tonal optimisation, on images of uneven size and density).

* Bit-exact equality with the single-request path (fi_tonal_opt with
  max_outer = 30, rtol = 0: g, both MSEs, inner iterations) for every
  request of a mix.
* Batch invariance: a request alone and amid others gives the same bits.
* Parity with the oracle: its CGLS, 30 iterations from g0 = f on the mask,
  with exact (Cholesky) solves: tonal MSE within 1e-6 relative, inpainting
  MSE within 1e-6 relative, g within 1e-3.
* Admission by footprint: with a budget for about three requests, no more
  are resident at once, the arena never exceeds its size, each request's
  bytes stay within its bound, and a request larger than the budget fails
  with FI_E_NOMEM without disturbing the others.
"""
import numpy as np
import pytest
import torch

import paper_2105_01586_amd as fi
import synth
from oracle import tonal

pytestmark = pytest.mark.gpu

ITERS = 30


@pytest.fixture(scope="module")
def ctx():
    c = fi.Context(0)
    yield c
    c.close()


def request(side, density, seed):
    f = synth.make_image(seed, side, side, max(8, side // 16), max(3, side // 64))
    mask = synth.make_mask(seed, side * side, density)
    return f.ravel(), mask


# (side, density, seed): uneven sizes and densities; the 1024^2 / 10%
# request has more rows than one launch re-reduces (the separate reduction).
MIX = [(64, 0.05, 101), (128, 0.10, 102), (256, 0.02, 103), (128, 0.03, 104), (512, 0.04, 105),
       (64, 0.08, 106), (256, 0.06, 107), (1024, 0.10, 108), (32, 0.10, 109), (128, 0.02, 110)]


def single_path(ctx, f, mask):
    """fi_inpaint + fi_tonal_opt(max_outer = 30, rtol = 0) on one mesh."""
    side = int(round(f.size ** 0.5))
    M = fi.Mesh(ctx, side, mask)
    fd = torch.from_numpy(f.copy()).cuda()
    u, _ = M.inpaint(f=fd)
    mse_inp, _, _ = M.error(u, fd)
    g, ts = M.tonal_opt(fd, opts=fi.TonalOpts(rtol=0.0, max_outer=ITERS))
    # the MSE of u = B g0 by the error kernel and by the CGLS residual: two
    # summation orders of the same squares
    assert abs(ts["mse_initial"] - mse_inp) <= 1e-12 * mse_inp
    out = (ts["mse_initial"], g.cpu().numpy(), ts["mse_final"], ts["inner_iterations"],
           M.large_mode())
    M.close()
    return out


@pytest.fixture(scope="module")
def singles(ctx):
    return [single_path(ctx, *request(*r)) for r in MIX]


def test_mix_matches_single_path(ctx, singles):
    assert any(s[4] for s in singles), "the mix should hold a large-mode request"
    with fi.Server(ctx, fi.ServerOpts(max_slots=16)) as S:
        tickets = [S.submit(*request(*r), tonal_iters=ITERS) for r in MIX]
        res = [S.poll(t) for t in tickets]
        st = S.stats()
    print(f"  peak resident {st['peak_resident']}, mean batch "
          f"{st['slot_steps'] / max(st['step_rounds'], 1):.2f}", flush=True)
    assert st["jobs_done"] == len(MIX) and st["jobs_failed"] == 0
    assert st["peak_resident"] > 1
    for r, s, (side, dens, seed) in zip(res, singles, MIX):
        assert r["status"] == 0, r["error"]
        assert r["mse_inpaint"] == s[0], (side, dens)
        assert np.array_equal(r["g"], s[1]), (side, dens)
        assert r["mse_tonal"] == s[2], (side, dens)
        assert r["inner_iterations"] == s[3]
        assert r["device_bytes"] <= r["footprint_bound"]
        assert r["t_submit"] <= r["t_admit"] <= r["t_start"] <= r["t_done"]


def test_alone_and_in_a_mix(ctx):
    probe = (256, 0.05, 201)
    with fi.Server(ctx, fi.ServerOpts(max_slots=8)) as S:
        alone = S.poll(S.submit(*request(*probe), tonal_iters=ITERS))
    with fi.Server(ctx, fi.ServerOpts(max_slots=8, chunk=4)) as S:
        others = [S.submit(*request(*r), tonal_iters=ITERS) for r in MIX[:5]]
        t = S.submit(*request(*probe), tonal_iters=ITERS)
        others += [S.submit(*request(*r), tonal_iters=ITERS) for r in MIX[5:7]]
        mixed = S.poll(t)
        for o in others:
            assert S.poll(o)["status"] == 0
    assert alone["status"] == 0 and mixed["status"] == 0
    assert np.array_equal(alone["g"], mixed["g"])
    assert alone["mse_tonal"] == mixed["mse_tonal"]
    assert alone["mse_inpaint"] == mixed["mse_inpaint"]


@pytest.mark.parametrize("r", [(64, 0.05, 301), (128, 0.10, 302), (256, 0.03, 303)])
def test_server_vs_oracle(ctx, r):
    f, mask = request(*r)
    with fi.Server(ctx, fi.ServerOpts(max_slots=4)) as S:
        res = S.poll(S.submit(f, mask, tonal_iters=ITERS))
    assert res["status"] == 0
    pr = tonal.Problem(r[0], mask)
    f64 = f.astype(np.float64)
    mse_inp = pr.mse(pr.inpaint(f), f)
    g, it, _ = pr.tonal_cgls(f64, rtol=0.0, maxit=ITERS)
    assert it == ITERS
    mse_ton = pr.mse_of_g(g, f)
    print(f"  {r}: mse inpaint {res['mse_inpaint']:.9f} / {mse_inp:.9f}, tonal "
          f"{res['mse_tonal']:.9f} / {mse_ton:.9f}, max |dg| {np.max(np.abs(res['g'] - g)):.2e}")
    assert abs(res["mse_inpaint"] - mse_inp) <= 1e-6 * mse_inp
    assert abs(res["mse_tonal"] - mse_ton) <= 1e-6 * mse_ton
    assert np.max(np.abs(res["g"] - g)) <= 1e-3


def test_sequential_fp64_matches_single_path(ctx):
    f, mask = request(128, 0.05, 401)
    M = fi.Mesh(ctx, 128, mask)
    fd = torch.from_numpy(f.copy()).cuda()
    inner = fi.SolveOpts(precision=fi.PREC_FP64)
    g_ref, ts = M.tonal_opt(fd, opts=fi.TonalOpts(inner=inner, rtol=0.0, max_outer=ITERS))
    M.close()
    with fi.Server(ctx, fi.ServerOpts(precision=fi.PREC_FP64)) as S:
        res = S.poll(S.submit(f, mask, tonal_iters=ITERS))
        assert S.stats()["step_rounds"] == 0  # no batched stepping in this mode
    assert res["status"] == 0
    assert np.array_equal(res["g"], g_ref.cpu().numpy())
    assert res["mse_tonal"] == ts["mse_final"]


def test_admission_by_footprint(ctx):
    reqs = [request(256, 0.05, 500 + i) for i in range(9)]
    bounds = [fi.footprint_bound(256, m, ITERS) for _, m in reqs]
    budget = int(3.2 * max(bounds))
    big_f, big_m = request(1024, 0.05, 599)
    assert fi.footprint_bound(1024, big_m, ITERS) > budget
    with fi.Server(ctx, fi.ServerOpts(max_slots=16, hbm_budget=budget, build_threads=4)) as S:
        ts = [S.submit(f, m, tonal_iters=ITERS) for f, m in reqs[:4]]
        tb = S.submit(big_f, big_m, tonal_iters=ITERS)
        ts += [S.submit(f, m, tonal_iters=ITERS) for f, m in reqs[4:]]
        res = [S.poll(t) for t in ts]
        big = S.poll(tb)
        st = S.stats()
    print(f"  budget {budget / 1e6:.1f} MB, arena peak {st['arena_peak_bytes'] / 1e6:.1f} MB, "
          f"peak resident {st['peak_resident']}")
    assert big["status"] == fi.E_NOMEM
    assert all(r["status"] == 0 for r in res)
    assert st["arena_peak_bytes"] <= st["arena_bytes"] <= budget
    assert st["peak_resident"] <= 3
    for r, b in zip(res, bounds):
        assert r["device_bytes"] <= r["footprint_bound"] == b


def test_submit_rejects_bad_requests(ctx):
    with fi.Server(ctx, fi.ServerOpts(max_slots=2)) as S:
        f, m = request(64, 0.05, 601)
        with pytest.raises(fi.FIError):
            S.submit(np.zeros(48 * 48, np.uint8), np.array([3, 5], np.int32))  # side 48
        with pytest.raises(fi.FIError):
            S.submit(f, m[::-1].copy())
        with pytest.raises(fi.FIError):
            S.submit(f, np.array([], np.int32))
        with pytest.raises(fi.FIError):
            S.submit(f, np.array([0, 64 * 64], np.int32))
        r = S.poll(S.submit(f, m, tonal_iters=0))
        assert r["status"] == 0 and r["mse_tonal"] == r["mse_inpaint"]
        assert np.array_equal(r["g"], f[m].astype(np.float64))


def test_largest_request_class(ctx):
    """A request of the trace's largest class (2048^2; the separate
    partial-sum reduction) beside a small one: the same bits as the
    single-request path."""
    big = request(2048, 0.06, 501)
    small = request(128, 0.05, 502)
    want_big = single_path(ctx, *big)
    want_small = single_path(ctx, *small)
    assert want_big[4]  # large mode
    with fi.Server(ctx, fi.ServerOpts(max_slots=4)) as S:
        tb = S.submit(*big, tonal_iters=ITERS)
        ts_ = S.submit(*small, tonal_iters=ITERS)
        rb, rs = S.poll(tb), S.poll(ts_)
    for r, s in ((rb, want_big), (rs, want_small)):
        assert r["status"] == 0
        assert r["mse_inpaint"] == s[0]
        assert np.array_equal(r["g"], s[1])
        assert r["mse_tonal"] == s[2]
        assert r["inner_iterations"] == s[3]


def test_one_slot_fp32_matches_single_path(ctx):
    """max_slots = 1 runs requests one at a time through the single-mesh FP32
    solver: the same bits as fi_inpaint + fi_tonal_opt, and no batched steps."""
    reqs = [request(128, 0.05, 601), request(256, 0.03, 602)]
    want = [single_path(ctx, *r) for r in reqs]
    with fi.Server(ctx, fi.ServerOpts(max_slots=1)) as S:
        tickets = [S.submit(*r, tonal_iters=ITERS) for r in reqs]
        got = [S.poll(t) for t in tickets]
        assert S.stats()["step_rounds"] == 0
    for r, s in zip(got, want):
        assert r["status"] == 0
        assert r["mse_inpaint"] == s[0]
        assert np.array_equal(r["g"], s[1])
        assert r["mse_tonal"] == s[2]
