"""Direct sparse Cholesky for large systems (test infrastructure only).

Wraps the plain C factorisation in ``oracle/csrc/sparse_chol.c`` (built by
``oracle/cbuild.py``) behind the same ``solve(b)`` interface as
``BandedCholesky``. The fill-reducing order is geometric nested dissection
on the quadtree's dyadic boxes: the vertices on the two centre lines of a
box form its separator (no leaf of the box's children straddles those lines,
so they separate the four quadrants up to the box's own leaf), and are
numbered after the four quadrants, recursively. Without coordinates the
order falls back to reverse Cuthill-McKee.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee

from . import cbuild

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = cbuild.lib_path("sparse_chol")
        if not os.path.exists(path):
            cbuild.build()
        L = ctypes.CDLL(path)
        L.chol_factor.restype = ctypes.c_int
        L.chol_factor.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_void_p)]
        L.chol_solve.restype = None
        L.chol_solve.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        L.chol_free.restype = None
        L.chol_free.argtypes = [ctypes.c_void_p]
        L.chol_nnz.restype = ctypes.c_int64
        L.chol_nnz.argtypes = [ctypes.c_void_p]
        _lib = L
    return _lib


def nested_dissection(xy: np.ndarray, side: int, leaf: int = 64) -> np.ndarray:
    """Order of the points ``xy`` (integer lattice coordinates in [0, side])."""
    xs = np.asarray(xy[:, 0], dtype=np.int64)
    ys = np.asarray(xy[:, 1], dtype=np.int64)
    out = []

    def rec(idx, x0, y0, S):
        if idx.size <= leaf or S <= 1:
            out.append(idx)
            return
        xm, ym = x0 + S // 2, y0 + S // 2
        x, y = xs[idx], ys[idx]
        sep = (x == xm) | (y == ym)
        h = S // 2
        for qx, qy, sel in ((x0, y0, (x < xm) & (y < ym)), (xm, y0, (x > xm) & (y < ym)),
                            (x0, ym, (x < xm) & (y > ym)), (xm, ym, (x > xm) & (y > ym))):
            sub = idx[sel & ~sep]
            if sub.size:
                rec(sub, qx, qy, h)
        out.append(idx[sep])

    rec(np.arange(xs.size, dtype=np.int64), 0, 0, side)
    order = np.concatenate(out) if out else np.zeros(0, dtype=np.int64)
    assert order.size == xs.size
    return order


class SparseCholesky:
    """A = L L^T with a nested-dissection (or RCM) order; ``solve(b)``."""

    def __init__(self, A: sp.spmatrix, coords: np.ndarray | None = None, side: int | None = None):
        A = sp.csc_matrix(A)
        n = A.shape[0]
        self.n = n
        if coords is not None:
            perm = nested_dissection(coords, side)
        else:
            perm = np.asarray(reverse_cuthill_mckee(sp.csr_matrix(A), symmetric_mode=True),
                              dtype=np.int64)
        self.perm = perm
        Ap = A[perm][:, perm].tocsc()
        Ap.sort_indices()
        self._Ap = np.ascontiguousarray(Ap.indptr.astype(np.int64))
        self._Ai = np.ascontiguousarray(Ap.indices.astype(np.int32))
        self._Ax = np.ascontiguousarray(Ap.data.astype(np.float64))
        h = ctypes.c_void_p()
        rc = _load().chol_factor(n, self._Ap.ctypes.data, self._Ai.ctypes.data,
                                 self._Ax.ctypes.data, ctypes.byref(h))
        if rc == 1:
            raise np.linalg.LinAlgError("matrix is not positive definite")
        if rc != 0:
            raise MemoryError("sparse Cholesky: allocation failed")
        self._h = h
        self.nnz_L = int(_load().chol_nnz(h))

    def solve(self, b: np.ndarray) -> np.ndarray:
        b = np.asarray(b, dtype=np.float64)
        if self.n == 0:
            return np.zeros_like(b)
        y = np.ascontiguousarray(b[self.perm])
        _load().chol_solve(self._h, y.ctypes.data, 1)
        x = np.empty_like(y)
        x[self.perm] = y
        return x

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.chol_free(h)
            self._h = None
