"""Colour images: the method applied channel by channel (Section 5).

TEST INFRASTRUCTURE ONLY (see the package header).

Section 5 calls the extension to colour images straightforward without
spelling it out; the reading here treats each channel as its own grey-value
problem. The channels share the mask, so they
share the mesh, the stiffness matrix and the operator B = R_D - R_F K_FF^-1
K_FD of Section 4; only the data differ. Arrays here are planar: channel c
of a per-pixel array is row c of a (3, P) array, and the stored values are a
(3, m) array.

Readings (the paper states none of these for colour):
* the colour MSE is the mean squared error over all 3P channel values, i.e.
  the mean of the three channel MSEs;
* tonal optimisation is three independent least-squares problems, one per
  channel, each solved by the grey CGLS of ``tonal.Problem``.
"""
from __future__ import annotations

import math

import numpy as np

from .tonal import Problem

C = 3


def planar(x, n: int) -> np.ndarray:
    """A planar colour array as (3, n) float64."""
    a = np.asarray(x, dtype=np.float64).reshape(C, n)
    return a


def inpaint(pr: Problem, f, g=None) -> np.ndarray:
    """u = B g_c for every channel c; g defaults to f on the mask. (3, P)."""
    f3 = planar(f, pr.P)
    g3 = None if g is None else planar(g, pr.mesh.m)
    return np.stack([pr.inpaint(f3[c], None if g3 is None else g3[c]) for c in range(C)])


def mse(u, f) -> float:
    """Mean over all 3P channel values of (u - f)^2, correctly rounded sum."""
    d = np.asarray(u, dtype=np.float64).ravel() - np.asarray(f, dtype=np.float64).ravel()
    return math.fsum((d * d).tolist()) / d.size


def tonal_cgls(pr: Problem, f, rtol: float = 1e-13, maxit: int = 5000):
    """Per channel: CGLS from g0 = f on the mask. Returns (g (3, m),
    iterations per channel, relative normal residual per channel)."""
    f3 = planar(f, pr.P)
    out = [pr.tonal_cgls(f3[c], rtol=rtol, maxit=maxit) for c in range(C)]
    return (np.stack([o[0] for o in out]), [o[1] for o in out], [o[2] for o in out])
