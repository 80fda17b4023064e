"""Pins of the oracle's mask-growth selection rules (Section 3), by brute force."""
import numpy as np

from oracle import densify


def test_topk_brute_force():
    rng = np.random.default_rng(0)
    for _ in range(20):
        P = int(rng.integers(10, 200))
        e = rng.integers(0, 6, size=P).astype(np.float64)   # many ties
        mask = np.sort(rng.choice(P, size=int(rng.integers(0, P // 2)), replace=False))
        k = int(rng.integers(0, P - mask.size + 1))
        cand = sorted((-e[i], i) for i in range(P) if i not in set(mask.tolist()))
        want = sorted(i for _, i in cand[:k])
        assert densify.topk_new_pixels(e, mask, k).tolist() == want


def test_paper_step_brute_force():
    rng = np.random.default_rng(1)
    for _ in range(20):
        P = int(rng.integers(20, 120))
        T = int(rng.integers(3, 15))
        owner = rng.integers(0, T, size=P)
        e = rng.integers(0, 5, size=P).astype(np.float64)
        mask = np.sort(rng.choice(P, size=int(rng.integers(0, P // 3)), replace=False))
        k = int(rng.integers(0, T + 2))
        ET = [sum(e[i] for i in range(P) if owner[i] == t) for t in range(T)]
        order = sorted(range(T), key=lambda t: (-ET[t], t))
        ms = set(mask.tolist())
        want = []
        for t in order:
            if len(want) == k:
                break
            empty = [i for i in range(P) if owner[i] == t and i not in ms]
            if empty:
                want.append(min(empty, key=lambda i: (-e[i], i)))
        got = densify.paper_densify_step(e, owner, T, mask, k)
        assert got.tolist() == sorted(want)
