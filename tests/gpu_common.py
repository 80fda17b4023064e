"""Shared helpers of the GPU parity tests: seeded cases and cached oracle runs."""
from __future__ import annotations

import functools

import numpy as np

import synth
from oracle import tonal

# (name, side, mask size or density, seed, bumps, edges)
SMALL_CASES = [
    ("n2_k1", 2, 1, 10, 1, 1),
    ("n4_corner", 4, 1, 11, 1, 1),
    ("n16_k7", 16, 7, 12, 2, 1),
    ("n32_k1", 32, 1, 13, 2, 1),
    ("n64_c1", 64, 205, 1, 8, 3),        # the 64x64, 5% plain workload
    ("n128_k300", 128, 300, 14, 8, 3),
    ("n256_k2000", 256, 2000, 15, 16, 4),
]


@functools.lru_cache(maxsize=None)
def case(name: str):
    if name == "c2":
        w = synth.WORKLOADS["tonal512"]
        return w.side, w.mask(), w.image().ravel()
    for nm, side, k, seed, b, e in SMALL_CASES:
        if nm == name:
            if name == "n64_c1":
                w = synth.WORKLOADS["plain64"]
                return w.side, w.mask(), w.image().ravel()
            if name == "n4_corner":
                mask = np.array([side * side - 1], dtype=np.int32)
            else:
                mask = synth.make_mask(seed, side * side, k=k)
            return side, mask, synth.make_image(seed, side, side, b, e).ravel()
    raise KeyError(name)


@functools.lru_cache(maxsize=None)
def oracle_problem(name: str) -> tonal.Problem:
    side, mask, _ = case(name)
    return tonal.Problem(side, mask)


@functools.lru_cache(maxsize=None)
def oracle_inpaint(name: str) -> np.ndarray:
    _, _, f = case(name)
    return oracle_problem(name).inpaint(f)


@functools.lru_cache(maxsize=None)
def oracle_tonal(name: str, rtol: float = 1e-12):
    _, _, f = case(name)
    return oracle_problem(name).tonal_cgls(f.astype(np.float64), rtol=rtol)
