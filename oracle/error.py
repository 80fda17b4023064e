"""Error measures of a reconstruction (Section 3 and Section 5).

Section 3 defines the pointwise error e_i = (u_i - f_i)^2 and the total L2
error of each triangle (the sum of e_i over the pixels it owns). The mean
squared error reported in Section 5 is the mean of e_i over all pixels, mask
pixels included; u is neither clipped nor rounded.
"""
from __future__ import annotations

import math

import numpy as np


def pixel_error(u: np.ndarray, f: np.ndarray) -> np.ndarray:
    d = np.asarray(u, dtype=np.float64).ravel() - np.asarray(f, dtype=np.float64).ravel()
    return d * d


def mse(u: np.ndarray, f: np.ndarray) -> float:
    """Mean squared error, summed with correct rounding (math.fsum)."""
    e = pixel_error(u, f)
    return math.fsum(e.tolist()) / e.size


def triangle_error(e: np.ndarray, owner: np.ndarray, T: int) -> np.ndarray:
    """Per-triangle total squared error over the pixels each triangle owns."""
    return np.bincount(np.asarray(owner), weights=np.asarray(e, dtype=np.float64), minlength=T)
