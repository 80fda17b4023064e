"""Error-driven mask growth (Section 3).

``topk_new_pixels`` is the global variant used by the mask-selection loop:
add the k non-mask pixels of largest pointwise error e_i = (u_i - f_i)^2,
breaking ties by the lower linear index.

``paper_densify_step`` follows Section 3 as written: compute the total L2
error of every triangle, visit triangles in descending order of that error
and insert one mask pixel per triangle, at the empty pixel (not yet in the
mask) of largest pointwise error among the pixels it owns, until the
requested number has been added. Ties are broken by the lower triangle index
and the lower pixel index.
"""
from __future__ import annotations

import numpy as np


def topk_new_pixels(e: np.ndarray, mask_idx: np.ndarray, k: int) -> np.ndarray:
    e = np.asarray(e, dtype=np.float64).ravel()
    P = e.size
    cand = np.ones(P, dtype=bool)
    cand[np.asarray(mask_idx, dtype=np.int64)] = False
    idx = np.nonzero(cand)[0]
    order = np.lexsort((idx, -e[idx]))   # primary: -e, secondary: index
    return np.sort(idx[order[:k]])


def paper_densify_step(e: np.ndarray, owner: np.ndarray, T: int, mask_idx: np.ndarray,
                       k: int) -> np.ndarray:
    e = np.asarray(e, dtype=np.float64).ravel()
    owner = np.asarray(owner, dtype=np.int64).ravel()
    P = e.size
    in_mask = np.zeros(P, dtype=bool)
    in_mask[np.asarray(mask_idx, dtype=np.int64)] = True
    ET = np.bincount(owner, weights=e, minlength=T)
    tri_order = np.lexsort((np.arange(T), -ET))
    # best empty pixel per triangle: largest e, then lowest index
    pix = np.nonzero(~in_mask)[0]
    order = np.lexsort((pix, -e[pix], owner[pix]))
    pix_sorted = pix[order]
    tri_sorted = owner[pix_sorted]
    first = np.ones(pix_sorted.size, dtype=bool)
    first[1:] = tri_sorted[1:] != tri_sorted[:-1]
    best = np.full(T, -1, dtype=np.int64)
    best[tri_sorted[first]] = pix_sorted[first]
    added = []
    for t in tri_order:
        if len(added) == k:
            break
        if best[t] >= 0:
            added.append(best[t])
    return np.sort(np.asarray(added, dtype=np.int64))
