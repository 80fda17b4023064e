"""GPU parity of the adjoint, the autograd gradient and tonal optimisation.

Adjoint B^T r against the oracle (relative 1e-8) and the dot-product
identity; d(MSE)/dg from autograd against the oracle gradient and central
finite differences on 16 random mask coordinates (eps = 1e-3); tonal MSE
within 1e-6 relative of the oracle's least-squares optimum, whose normal
residual the GPU result also drives near zero.
"""
import numpy as np
import pytest
import torch

import paper_2105_01586_amd as fi
from paper_2105_01586_amd import autograd as fa
from gpu_common import case, oracle_problem, oracle_tonal

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = fi.Context(0)
    yield c
    c.close()


_meshes = {}


def gpu_mesh(ctx, name):
    if name not in _meshes:
        side, mask, _ = case(name)
        _meshes[name] = fi.Mesh(ctx, side, mask)
    return _meshes[name]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("precision", [fi.PREC_FP32_IR, fi.PREC_FP64])
@pytest.mark.parametrize("name", ["n16_k7", "n64_c1", "n256_k2000", "c2"])
def test_adjoint_parity(ctx, name, precision):
    print(f"case {name} precision {precision}", flush=True)
    M = gpu_mesh(ctx, name)
    pr = oracle_problem(name)
    rng = np.random.default_rng(5)
    r = rng.normal(size=M.P)
    s, st = M.adjoint(dev(r), opts=fi.SolveOpts(precision=precision))
    s = s.cpu().numpy()
    ref = pr.BT(r)
    rel = np.linalg.norm(s - ref) / np.linalg.norm(ref)
    print(f"  rel err {rel:.3e}, iters {st['iterations']}")
    assert rel <= 1e-8
    g = rng.normal(size=M.m)
    u, _ = M.inpaint(g=dev(g), opts=fi.SolveOpts(precision=precision))
    lhs = float(u.cpu().numpy() @ r)
    rhs = float(g @ s)
    assert abs(lhs - rhs) <= 1e-8 * (np.linalg.norm(g) * np.linalg.norm(r))


@pytest.mark.parametrize("name", ["n64_c1", "c2"])
def test_autograd_gradient_and_fd(ctx, name):
    print(f"case {name}", flush=True)
    M = gpu_mesh(ctx, name)
    pr = oracle_problem(name)
    _, _, f = case(name)
    rng = np.random.default_rng(7)
    g0 = pr.default_g(f) + rng.normal(scale=2.0, size=M.m)
    g = dev(g0).requires_grad_(True)
    fd_t = dev(f)
    loss = fa.mse_loss(g, fd_t, M)
    loss.backward()
    grad = g.grad.cpu().numpy()
    ref = pr.mse_grad(g0, f)
    rel = np.linalg.norm(grad - ref) / np.linalg.norm(ref)
    print(f"  gradient rel err vs oracle {rel:.3e}")
    assert rel <= 1e-8
    # The MSE is quadratic in g, so central differences carry no truncation
    # error: what is left is the rounding of the two losses and the error of
    # their solves, divided by 2 eps. The losses are solved tightly (1e-12).
    eps = 1e-3
    tight = fi.SolveOpts(rtol=1e-12)
    scale = np.max(np.abs(grad))
    worst = 0.0
    for j in rng.integers(0, M.m, size=16):
        gp = g0.copy()
        gm = g0.copy()
        gp[j] += eps
        gm[j] -= eps
        with torch.no_grad():
            lp = fa.mse_loss(dev(gp), fd_t, M, tight).item()
            lm = fa.mse_loss(dev(gm), fd_t, M, tight).item()
        fd = (lp - lm) / (2 * eps)
        dev_j = abs(fd - grad[j])
        worst = max(worst, dev_j / (abs(grad[j]) + 1e-3 * scale))
        assert dev_j <= 1e-4 * abs(grad[j]) + 1e-6 * scale, (j, fd, grad[j])
    print(f"  worst FD deviation (relative) {worst:.3e}")


@pytest.mark.parametrize("name", ["n16_k7", "n64_c1", "c2"])
def test_mse_and_backward_in_library(ctx, name):
    """The MSE on the device equals fi_error's MSE bit for bit; the library's
    MSE backward, s (2 / P) B^T (B g - f), matches the oracle gradient times s
    (s = 1 and s = -3.5) and the loss's autograd gradient under a scale."""
    print(f"case {name}", flush=True)
    M = gpu_mesh(ctx, name)
    pr = oracle_problem(name)
    _, _, f = case(name)
    rng = np.random.default_rng(11)
    g0 = pr.default_g(f) + rng.normal(scale=3.0, size=M.m)
    fd_t = dev(f)
    u, _ = M.inpaint(g=dev(g0))
    mse_host, _, _ = M.error(u, fd_t)
    mse_dev = M.mse_dev(u, fd_t).item()
    assert mse_dev == mse_host
    ref = pr.mse_grad(g0, f)
    for s in (1.0, -3.5):
        scale = None if s == 1.0 else dev(np.array([s]))
        grad, st = M.mse_backward(u, fd_t, scale=scale)
        grad = grad.cpu().numpy()
        rel = np.linalg.norm(grad - s * ref) / np.linalg.norm(s * ref)
        print(f"  s = {s}: rel err vs oracle {rel:.3e}, {st['iterations']} CG iterations")
        assert st["status"] == 0 and rel <= 1e-8
    g = dev(g0).requires_grad_(True)
    (-3.5 * fa.mse_loss(g, fd_t, M)).backward()
    rel = np.linalg.norm(g.grad.cpu().numpy() + 3.5 * ref) / np.linalg.norm(3.5 * ref)
    assert rel <= 1e-8


@pytest.mark.parametrize("precision", [fi.PREC_FP32_IR, fi.PREC_FP64])
@pytest.mark.parametrize("name", ["n16_k7", "n64_c1", "n256_k2000", "c2"])
def test_tonal_parity(ctx, name, precision):
    print(f"case {name} precision {precision}", flush=True)
    M = gpu_mesh(ctx, name)
    pr = oracle_problem(name)
    _, _, f = case(name)
    g, st = M.tonal_opt(dev(f), opts=fi.TonalOpts(inner=fi.SolveOpts(precision=precision)))
    g = g.cpu().numpy()
    g_ref, it_ref, _ = oracle_tonal(name)
    mse_gpu_by_oracle = pr.mse_of_g(g, f)
    mse_ref = pr.mse_of_g(g_ref, f)
    mse0 = pr.mse_of_g(pr.default_g(f), f)
    print(f"  outer {st['outer_iterations']} (oracle {it_ref}), inner {st['inner_iterations']}, "
          f"mse {st['mse_final']:.9f} oracle {mse_ref:.9f} (untuned {mse0:.6f})")
    assert st["status"] == 0 and st["rel_normal_residual"] <= 1e-8
    assert abs(st["mse_final"] - mse_ref) <= 1e-6 * mse_ref
    assert abs(mse_gpu_by_oracle - mse_ref) <= 1e-6 * mse_ref
    assert mse_ref <= mse0 + 1e-12 and st["mse_final"] <= st["mse_initial"]
    s0 = np.linalg.norm(pr.normal_residual(pr.default_g(f), f))
    assert np.linalg.norm(pr.normal_residual(g, f)) <= 1e-6 * s0


@pytest.mark.parametrize("name", ["n256_k2000", "c2"])
def test_adjoint_warm_start(ctx, name):
    """Each adjoint solve of the CGLS loop starts from the previous one's
    solution (the default) or from 0: the same stopping test, so the same
    result to the parity bar, and fewer CG iterations warm."""
    print(f"case {name}", flush=True)
    M = gpu_mesh(ctx, name)
    pr = oracle_problem(name)
    _, _, f = case(name)
    g_w, st_w = M.tonal_opt(dev(f), opts=fi.TonalOpts())
    g_c, st_c = M.tonal_opt(dev(f), opts=fi.TonalOpts(cold_adjoint=True))
    g_ref, _, _ = oracle_tonal(name)
    mse_ref = pr.mse_of_g(g_ref, f)
    print(f"  inner iterations warm {st_w['inner_iterations']} cold {st_c['inner_iterations']}, "
          f"outer {st_w['outer_iterations']} / {st_c['outer_iterations']}", flush=True)
    for st, g in ((st_w, g_w), (st_c, g_c)):
        assert st["status"] == 0
        assert abs(st["mse_final"] - mse_ref) <= 1e-6 * mse_ref
        assert abs(pr.mse_of_g(g.cpu().numpy(), f) - mse_ref) <= 1e-6 * mse_ref
    assert st_w["inner_iterations"] < st_c["inner_iterations"]


@pytest.mark.parametrize("name", ["n64_c1", "n256_k2000"])
def test_tonal_from_given_g(ctx, name):
    """start_from_g: CGLS from a given g (f on the mask plus seeded noise)
    against the oracle's CGLS from the same g, 20 iterations."""
    M = gpu_mesh(ctx, name)
    pr = oracle_problem(name)
    _, _, f = case(name)
    g0 = pr.default_g(f) + np.random.default_rng(17).normal(scale=5.0, size=M.m)
    g = dev(g0.copy())
    g, st = M.tonal_opt(dev(f), g=g, opts=fi.TonalOpts(rtol=0.0, max_outer=20, start_from_g=True))
    g_ref, it, _ = pr.tonal_cgls(f.astype(np.float64), g0=g0, rtol=0.0, maxit=20)
    assert it == 20
    mse0 = pr.mse_of_g(g0, f)
    ref = pr.mse_of_g(g_ref, f)
    print(f"  mse from g0 {mse0:.6f} -> {st['mse_final']:.9f} (oracle {ref:.9f})", flush=True)
    assert abs(st["mse_initial"] - mse0) <= 1e-6 * mse0
    assert abs(st["mse_final"] - ref) <= 1e-6 * ref
