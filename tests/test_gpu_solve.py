"""The harmonic-extension system K_FF x = b on the GPU (fi_solve), against
the oracle's direct Cholesky solve and the definition of the residual:

* ||b - K_FF x|| <= 1e-10 ||b|| recomputed on the host in FP64 from the
  oracle's K_FF (the GPU's matrix equals it; see test_gpu_inpaint), and x
  close to the Cholesky solution;
* starts: an exact start is returned as it is with no iteration; a perturbed
  start meets the same bar in fewer iterations; b = 0 gives x = 0 exactly,
  from any start; x may overwrite its own start;
* the quadtree (ELL) and Delaunay (CSR) layouts, the large-system launch
  shape, FP32 with FP64 refinement and plain FP64.
"""
import numpy as np
import pytest
import torch

import paper_2105_01586_amd as fi
import synth
from gpu_common import case, oracle_problem
from oracle import tonal

pytestmark = pytest.mark.gpu
RES_TOL = 1.2e-10  # the solver's 1e-10, plus host re-summation rounding


@pytest.fixture(scope="module")
def ctx():
    c = fi.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rel_residual(pr, b, x):
    return np.linalg.norm(b - pr.sys.K_FF @ x) / np.linalg.norm(b)


def quadtree(ctx, name):
    side, mask, _ = case(name)
    return fi.Mesh(ctx, side, mask), oracle_problem(name)


_DEL = {}


def delaunay(ctx):
    if "pr" not in _DEL:
        side = 64
        mask = synth.make_mask(22, side * side, 0.05)
        unk = synth.make_unknowns(22, side * side, mask, mask.size)
        _DEL.update(side=side, mask=mask, unk=unk,
                    pr=tonal.Problem(side, mask, unknown_idx=unk))
    return fi.Mesh(ctx, _DEL["side"], _DEL["mask"], unknowns=_DEL["unk"]), _DEL["pr"]


def get(ctx, name):
    return delaunay(ctx) if name == "delaunay64" else quadtree(ctx, name)


@pytest.mark.parametrize("precision", [fi.PREC_FP32_IR, fi.PREC_FP64])
@pytest.mark.parametrize("name", ["n16_k7", "n256_k2000", "c2", "delaunay64"])
def test_solve_vs_cholesky(ctx, name, precision):
    print(f"case {name} precision {precision}", flush=True)
    M, pr = get(ctx, name)
    b = np.random.default_rng(31).normal(size=M.n)
    x, st = M.solve(dev(b), opts=fi.SolveOpts(precision=precision))
    M.close()
    x = x.cpu().numpy()
    x_ref = pr.factor.solve(b)
    res = rel_residual(pr, b, x)
    print(f"  n={b.size}: {st['iterations']} iterations, residual {res:.2e} "
          f"(device {st['rel_residual']:.2e})", flush=True)
    assert st["status"] == 0 and res <= RES_TOL and st["rel_residual"] <= 1e-10
    assert np.max(np.abs(x - x_ref)) <= 1e-6 * np.max(np.abs(x_ref))


@pytest.mark.parametrize("precision", [fi.PREC_FP32_IR, fi.PREC_FP64])
@pytest.mark.parametrize("name", ["n256_k2000", "delaunay64"])
def test_solve_starts(ctx, name, precision):
    print(f"case {name} precision {precision}", flush=True)
    M, pr = get(ctx, name)
    o = fi.SolveOpts(precision=precision)
    rng = np.random.default_rng(32)
    b = rng.normal(size=M.n)
    x_ref = pr.factor.solve(b)
    _, st_cold = M.solve(dev(b), opts=o)
    # an exact start: returned unchanged, no iteration
    x, st = M.solve(dev(b), x0=dev(x_ref), opts=o)
    assert st["iterations"] == 0 and np.array_equal(x.cpu().numpy(), x_ref)
    # a start 1e-4 off: the same bar, fewer iterations
    x0 = x_ref + 1e-4 * np.max(np.abs(x_ref)) * rng.normal(size=M.n)
    x, st = M.solve(dev(b), x0=dev(x0), opts=o)
    assert rel_residual(pr, b, x.cpu().numpy()) <= RES_TOL
    assert st["iterations"] < st_cold["iterations"]
    # the output may overwrite its start
    xx = dev(x0)
    M.solve(dev(b), x0=xx, x=xx, opts=o)
    assert rel_residual(pr, b, xx.cpu().numpy()) <= RES_TOL
    # b = 0: x = 0 exactly, from 0 and from a non-zero start
    zero = torch.zeros(M.n, dtype=torch.float64, device="cuda:0")
    x, st = M.solve(zero, opts=o)
    assert st["status"] == 0 and st["iterations"] == 0 and not x.any()
    x, st = M.solve(zero, x0=dev(rng.normal(size=M.n)), opts=o)
    assert st["status"] == 0 and not x.any()
    M.close()


def test_solve_large_launch_shape(ctx, monkeypatch):
    """The separate partial-sum reduction launch (large systems) with starts."""
    side, mask, _ = case("n256_k2000")
    monkeypatch.setenv("FI_CG_LARGE", "1")
    M = fi.Mesh(ctx, side, mask)
    monkeypatch.delenv("FI_CG_LARGE")
    assert M.large_mode()
    pr = oracle_problem("n256_k2000")
    rng = np.random.default_rng(33)
    b = rng.normal(size=M.n)
    x_ref = pr.factor.solve(b)
    x, st_cold = M.solve(dev(b))
    assert rel_residual(pr, b, x.cpu().numpy()) <= RES_TOL
    x0 = x_ref + 1e-4 * np.max(np.abs(x_ref)) * rng.normal(size=M.n)
    x, st = M.solve(dev(b), x0=dev(x0))
    assert rel_residual(pr, b, x.cpu().numpy()) <= RES_TOL
    assert st["iterations"] < st_cold["iterations"]
    zero = torch.zeros(M.n, dtype=torch.float64, device="cuda:0")
    x, st = M.solve(zero, x0=dev(rng.normal(size=M.n)))
    assert st["status"] == 0 and not x.any()
    M.close()


def test_solve_rejects_non_finite(ctx):
    M, _ = quadtree(ctx, "n16_k7")
    b = np.zeros(M.n)
    b[0] = np.nan
    with pytest.raises(fi.FIError) as ei:
        M.solve(dev(b))
    assert ei.value.code == fi.E_INVALID
    M.close()
