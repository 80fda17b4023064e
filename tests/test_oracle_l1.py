"""Pins of the oracle's L1 tonal optimisation (IRLS over weighted CGLS; the
paper states no method, see oracle/l1.py for the reading).

* Weighted CGLS with unit weights is the L2 CGLS of Section 4, bit for bit.
* A weighted least-squares step run to convergence equals the dense
  weighted solution by numpy.linalg.lstsq.
* IRLS reaches the exact L1 minimum from linear programming
  (scipy.optimize.linprog) within the smoothing bound P eps / 2.
* The Huber objective never increases over IRLS steps, and the MAE falls.
"""
import numpy as np
import pytest
import scipy.optimize

import synth
from oracle import l1, tonal


def tiny(N, k, seed):
    rng = np.random.default_rng(seed)
    mask = np.sort(rng.choice(N * N, size=k, replace=False))
    f = synth.make_image(seed, N, N, 2, 1).ravel().astype(np.float64)
    return tonal.Problem(N, mask), f


@pytest.mark.parametrize("N,k,seed", [(8, 5, 1), (16, 12, 2)])
def test_unit_weights_equal_l2_cgls(N, k, seed):
    pr, f = tiny(N, k, seed)
    g2, it2, _ = pr.tonal_cgls(f, rtol=0.0, maxit=7)
    g1, it1 = l1.weighted_cgls(pr, f, np.ones(N * N), pr.default_g(f), 7)
    assert it1 == it2 == 7
    assert np.array_equal(g1, g2)


@pytest.mark.parametrize("N,k,seed", [(8, 5, 3), (16, 12, 4)])
def test_weighted_step_matches_lstsq(N, k, seed):
    pr, f = tiny(N, k, seed)
    w = np.random.default_rng(seed).uniform(0.2, 3.0, size=N * N)
    sw = np.sqrt(w)
    g, _ = l1.weighted_cgls(pr, f, sw, pr.default_g(f), 500, rtol=1e-14)
    B = pr.dense_B()
    ref, *_ = np.linalg.lstsq(sw[:, None] * B, sw * f, rcond=None)
    assert np.max(np.abs(g - ref)) <= 1e-8 * max(1.0, np.max(np.abs(ref)))


def test_irls_reaches_linear_programming_minimum():
    N, k, seed = 8, 6, 5
    pr, f = tiny(N, k, seed)
    B = pr.dense_B()
    P, m = B.shape
    # min sum t  s.t.  B g - f <= t,  f - B g <= t
    c = np.concatenate([np.zeros(m), np.ones(P)])
    A = np.block([[B, -np.eye(P)], [-B, -np.eye(P)]])
    b = np.concatenate([f, -f])
    lp = scipy.optimize.linprog(c, A_ub=A, b_ub=b, bounds=[(None, None)] * (m + P),
                                method="highs")
    assert lp.status == 0
    e1_star = lp.fun
    eps = 1e-3
    g, hist = l1.irls(pr, f, eps=eps, K=300, J=60)
    e1 = hist[-1] * P
    assert e1 >= e1_star - 1e-7
    assert e1 <= e1_star + P * eps / 2 + 1e-7


def test_huber_monotone_and_mae_falls():
    N = 64
    mask = synth.make_mask(6, N * N, 0.05)
    f = synth.make_image(6, N, N, 8, 3).ravel()
    pr = tonal.Problem(N, mask)
    eps = 0.5
    g = pr.default_g(f)
    H = [l1.huber(pr, g, f, eps)]
    for _ in range(6):
        r = f - pr.B(g)
        w = 1.0 / np.maximum(np.abs(r), eps)
        g, _ = l1.weighted_cgls(pr, f, np.sqrt(w), g, 5)
        H.append(l1.huber(pr, g, f, eps))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(H, H[1:]))
    _, hist = l1.irls(pr, f, eps=eps, K=4, J=10)
    assert hist[-1] < hist[0]
