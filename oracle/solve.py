"""Direct solve of the SPD system K_FF u_F = -K_FD g (Section 2.2).

Section 2.2 notes that with at least one mask pixel the FEM matrix is
symmetric positive definite; the paper then approximates the solution with
CG. The oracle instead computes the exact discrete solution with a direct
Cholesky factorisation, so that an iterative GPU answer can be measured
against it.

Two factorisations are provided:

* ``BandedCholesky``: reverse Cuthill-McKee ordering, then LAPACK's banded
  Cholesky (``scipy.linalg.cholesky_banded``), a library step. Used up to
  20,000 unknowns.
* ``SparseCholesky`` (in ``oracle.sparse_chol``): a plain C left-looking
  sparse Cholesky with a geometric nested-dissection order, for larger
  systems, where the band is wide.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee


class BandedCholesky:
    """Cholesky factor of a sparse SPD matrix in RCM-ordered banded storage."""

    def __init__(self, A: sp.spmatrix):
        A = sp.csr_matrix(A)
        n = A.shape[0]
        self.n = n
        if n == 0:
            self.perm = np.zeros(0, dtype=np.int64)
            self.cb = None
            self.bandwidth = 0
            return
        perm = np.asarray(reverse_cuthill_mckee(A, symmetric_mode=True), dtype=np.int64)
        Ap = A[perm][:, perm].tocoo()
        low = Ap.row >= Ap.col
        r = Ap.row[low]
        c = Ap.col[low]
        v = Ap.data[low]
        bw = int((r - c).max()) if r.size else 0
        ab = np.zeros((bw + 1, n), dtype=np.float64)
        ab[r - c, c] = v
        self.cb = sla.cholesky_banded(ab, lower=True, check_finite=False)
        self.perm = perm
        self.bandwidth = bw

    def solve(self, b: np.ndarray) -> np.ndarray:
        b = np.asarray(b, dtype=np.float64)
        if self.n == 0:
            return np.zeros_like(b)
        y = sla.cho_solve_banded((self.cb, True), b[self.perm], check_finite=False)
        x = np.empty_like(y)
        x[self.perm] = y
        return x


def factorise(A: sp.spmatrix, method: str = "auto", coords: np.ndarray | None = None,
              side: int | None = None):
    """Direct Cholesky factor object with a ``solve(b)`` method.

    ``auto`` takes the banded factorisation up to 20,000 unknowns and the
    sparse one (nested dissection on ``coords`` when given) above.
    """
    n = A.shape[0]
    if method == "auto":
        method = "banded" if n <= 20_000 else "sparse"
    if method == "banded":
        return BandedCholesky(A)
    if method == "sparse":
        from .sparse_chol import SparseCholesky
        return SparseCholesky(A, coords, side)
    raise ValueError(method)
