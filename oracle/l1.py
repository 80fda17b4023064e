"""Tonal optimisation for the L1 error (Section 5, the large colour example).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper optimises one result for the L1 error without stating how. The
reading taken here is iteratively reweighted least squares (IRLS), built on
the same operator B and adjoint as the L2 tonal optimisation of Section 4:

* objective E1(g) = sum_i |(B g)_i - f_i|, reported as the mean absolute
  error E1 / P;
* start g_0 = f on the mask (or given values);
* IRLS step k: residual r = f - B g_k, weights w_i = 1 / max(|r_i|, eps),
  then g_{k+1} from J iterations of CGLS on the weighted least-squares
  problem min sum_i w_i ((B g)_i - f_i)^2, i.e. CGLS on W^(1/2) B with right
  side W^(1/2) f, started from g_k;
* defaults eps = 0.5 grey levels, K = 8 IRLS steps, J = 20 CGLS iterations.

With w from g_k, the weighted objective sum_i (w_i r_i^2 + 1 / w_i) / 2
majorises the Huber function H(g) = sum_i rho(r_i), rho(r) = |r| for
|r| >= eps and r^2 / (2 eps) + eps / 2 below, and touches it at g_k. CGLS
lowers the weighted residual at every iteration, so H never increases from
one IRLS step to the next, however small J is; and E1 <= H <= E1 + P eps / 2.
"""
from __future__ import annotations

import math

import numpy as np

from .tonal import Problem


def weighted_cgls(pr: Problem, f, wsqrt, g0, iters: int, rtol: float = 0.0):
    """CGLS on min || W^(1/2) (B g - f) ||^2 from g0, `iters` iterations (or
    until ||s|| <= rtol ||s_0||). Returns (g, iterations)."""
    f = np.asarray(f, dtype=np.float64).ravel()
    wsqrt = np.asarray(wsqrt, dtype=np.float64).ravel()
    g = np.array(g0, dtype=np.float64)
    r = wsqrt * (f - pr.B(g))
    s = pr.BT(wsqrt * r)
    p = s.copy()
    gamma = float(s @ s)
    s0 = math.sqrt(gamma)
    if s0 == 0.0:
        return g, 0
    it = 0
    while it < iters:
        q = wsqrt * pr.B(p)
        alpha = gamma / float(q @ q)
        g += alpha * p
        r -= alpha * q
        s = pr.BT(wsqrt * r)
        gnew = float(s @ s)
        it += 1
        if math.sqrt(gnew) <= rtol * s0:
            break
        p = s + (gnew / gamma) * p
        gamma = gnew
    return g, it


def mae(pr: Problem, g, f) -> float:
    """Mean absolute error of B g against f, correctly rounded sum."""
    d = pr.B(g) - np.asarray(f, dtype=np.float64).ravel()
    return math.fsum(np.abs(d).tolist()) / d.size


def huber(pr: Problem, g, f, eps: float) -> float:
    r = np.abs(pr.B(g) - np.asarray(f, dtype=np.float64).ravel())
    rho = np.where(r >= eps, r, r * r / (2.0 * eps) + eps / 2.0)
    return math.fsum(rho.tolist())


def irls(pr: Problem, f, eps: float = 0.5, K: int = 8, J: int = 20, g0=None):
    """Returns (g, [MAE after each step, the start first])."""
    f = np.asarray(f, dtype=np.float64).ravel()
    g = pr.default_g(f) if g0 is None else np.array(g0, dtype=np.float64)
    hist = [mae(pr, g, f)]
    for _ in range(K):
        r = f - pr.B(g)
        w = 1.0 / np.maximum(np.abs(r), eps)
        g, _ = weighted_cgls(pr, f, np.sqrt(w), g, J)
        hist.append(mae(pr, g, f))
    return g, hist
