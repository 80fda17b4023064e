"""Linear (P1) finite-element stiffness matrix and Dirichlet split (Section 2.2).

The weak form of -Laplace(u) = 0 with the reflecting boundary of Section 2.1
eq. (3) is the natural (Neumann) condition, so the boundary adds no terms.
For a triangle with vertices p_i = (x_i, y_i), area A and (i, j, k) cyclic,
grad(phi_i) = (b_i, c_i) / (2A) with b_i = y_j - y_k and c_i = x_k - x_j, so the
element matrix is K^e_ij = A grad(phi_i).grad(phi_j) = (b_i b_j + c_i c_j) / (4A).

Mask vertices carry prescribed values (Section 2.1 eq. (2)), so the unknowns
are the free vertices: K_FF u_F = -K_FD g. Exact zeros (couplings across the
hypotenuse of right triangles) are dropped from the sparse pattern.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .mesh import Mesh


def element_matrices(vxy: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """(T, 3, 3) float64 element stiffness matrices."""
    p = vxy[tri].astype(np.float64)           # (T, 3, 2)
    x = p[:, :, 0]
    y = p[:, :, 1]
    j = [1, 2, 0]
    k = [2, 0, 1]
    b = y[:, j] - y[:, k]
    c = x[:, k] - x[:, j]
    twoA = (x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (y[:, 1] - y[:, 0]) * (x[:, 2] - x[:, 0])
    if np.any(twoA <= 0):
        raise AssertionError("degenerate or negatively oriented triangle")
    return (b[:, :, None] * b[:, None, :] + c[:, :, None] * c[:, None, :]) / (2.0 * twoA)[:, None, None]


@dataclass
class System:
    K: sp.csr_matrix      # (V, V) full stiffness matrix
    K_FF: sp.csr_matrix   # (n, n)
    K_FD: sp.csr_matrix   # (n, m)
    K_DF: sp.csr_matrix   # (m, n)


def assemble(mesh: Mesh) -> System:
    Ke = element_matrices(mesh.vxy, mesh.tri)
    rows = np.repeat(mesh.tri, 3, axis=1).ravel()
    cols = np.tile(mesh.tri, (1, 3)).ravel()
    K = sp.coo_matrix((Ke.ravel(), (rows, cols)), shape=(mesh.V, mesh.V)).tocsr()
    K.sum_duplicates()
    K.eliminate_zeros()
    K.sort_indices()
    F = mesh.free_vids
    D = mesh.mask_vids
    K_FF = K[F][:, F].tocsr()
    K_FD = K[F][:, D].tocsr()
    K_DF = K[D][:, F].tocsr()
    for A in (K_FF, K_FD, K_DF):
        A.eliminate_zeros()
        A.sort_indices()
    return System(K=K, K_FF=K_FF, K_FD=K_FD, K_DF=K_DF)
