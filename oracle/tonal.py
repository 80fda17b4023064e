"""Inpainting as a linear map u = B g, its adjoint, and tonal optimisation (Section 4).

For mask values g (m of them, in ascending mask pixel order) the inpainted
image is u = B g (Section 4): the harmonic extension to the free vertices,
u_F = -K_FF^{-1} K_FD g with u_D = g, followed by linear interpolation to the
pixels, u = R_F u_F + R_D g. So B = R_D - R_F K_FF^{-1} K_FD; it is dense and
never formed here except on tiny inputs.

Its transpose follows by transposing each factor (K_FF is symmetric and
K_DF = K_FD^T): B^T r = t_D - K_DF K_FF^{-1} t_F with t = R^T r.

Tonal optimisation solves min_g ||B g - f||^2 (eq. (4)) through the normal
equations B^T B g = B^T f (eq. (5)) by conjugate gradients, with B and B^T
applied through exact (Cholesky) inner solves; the paper's nested CG uses CG
for those inner solves. The gradient of MSE(g) = ||B g - f||^2 / P is
(2 / P) B^T (B g - f).
"""
from __future__ import annotations

import math

import numpy as np

from . import delaunay
from . import error as err
from . import fem, mesh as mesh_mod, raster, solve


class Problem:
    """Everything the oracle derives from one (image side, mask) pair."""

    def __init__(self, N: int, mask_idx, factor_method: str = "auto", unknown_idx=None):
        """unknown_idx: None for the quadtree mesh; else the unknown vertices
        (pixel indices) of the paper's Delaunay mesh (``delaunay``)."""
        if unknown_idx is None:
            self.mesh = mesh_mod.build_mesh(N, mask_idx)
        else:
            self.mesh = delaunay.build_mesh(N, mask_idx, unknown_idx)
        if self.mesh.m == 0:
            raise ValueError("empty mask: the system is singular (Section 2.2 needs a mask pixel)")
        self.sys = fem.assemble(self.mesh)
        self.rast = (raster.rasteriser(self.mesh) if unknown_idx is None
                     else delaunay.rasteriser(self.mesh))
        R = self.rast.R.tocsc()
        self.R_F = R[:, self.mesh.free_vids].tocsr()
        self.R_D = R[:, self.mesh.mask_vids].tocsr()
        self.R_FT = self.R_F.T.tocsr()
        self.R_DT = self.R_D.T.tocsr()
        self.factor = solve.factorise(self.sys.K_FF, factor_method,
                                      self.mesh.vxy[self.mesh.free_vids], N)
        self.N = N
        self.P = N * N

    # -- the harmonic extension and its rasterisation ------------------------
    def vertex_solution(self, g: np.ndarray) -> np.ndarray:
        """u at every vertex: u_D = g, u_F = K_FF^{-1} (-K_FD g)."""
        g = np.asarray(g, dtype=np.float64)
        u = np.empty(self.mesh.V, dtype=np.float64)
        u[self.mesh.mask_vids] = g
        u[self.mesh.free_vids] = self.factor.solve(-(self.sys.K_FD @ g))
        return u

    def B(self, g: np.ndarray) -> np.ndarray:
        """Inpainted pixels u = B g (flattened, row-major)."""
        return raster.rasterise(self.rast, self.vertex_solution(g))

    def BT(self, r: np.ndarray) -> np.ndarray:
        """Adjoint B^T r = t_D - K_DF K_FF^{-1} t_F with t = R^T r."""
        r = np.asarray(r, dtype=np.float64).ravel()
        tF = self.R_FT @ r
        tD = self.R_DT @ r
        y = self.factor.solve(tF)
        return tD - self.sys.K_DF @ y

    def default_g(self, f: np.ndarray) -> np.ndarray:
        """Stored values at the mask pixels: g = f restricted to K."""
        return np.asarray(f, dtype=np.float64).ravel()[self.mesh.mask_idx]

    def inpaint(self, f: np.ndarray, g: np.ndarray | None = None) -> np.ndarray:
        if g is None:
            g = self.default_g(f)
        return self.B(g)

    def mse(self, u: np.ndarray, f: np.ndarray) -> float:
        return err.mse(u, f)

    def mse_of_g(self, g: np.ndarray, f: np.ndarray) -> float:
        return err.mse(self.B(g), f)

    def mse_grad(self, g: np.ndarray, f: np.ndarray) -> np.ndarray:
        f = np.asarray(f, dtype=np.float64).ravel()
        return (2.0 / self.P) * self.BT(self.B(g) - f)

    def triangle_error(self, u: np.ndarray, f: np.ndarray) -> np.ndarray:
        return err.triangle_error(err.pixel_error(u, f), self.rast.owner, self.mesh.T)

    # -- tonal optimisation ---------------------------------------------------
    def dense_B(self) -> np.ndarray:
        """B column by column (B e_j); tiny inputs only."""
        m = self.mesh.m
        cols = [self.B(np.eye(1, m, j).ravel()) for j in range(m)]
        return np.stack(cols, axis=1)

    def tonal_lstsq(self, f: np.ndarray) -> np.ndarray:
        f = np.asarray(f, dtype=np.float64).ravel()
        g, *_ = np.linalg.lstsq(self.dense_B(), f, rcond=None)
        return g

    def tonal_cgls(self, f: np.ndarray, g0: np.ndarray | None = None, rtol: float = 1e-13,
                   maxit: int = 5000):
        """CG on B^T B g = B^T f in least-squares form (CGLS).

        Residual r = f - B g, normal residual s = B^T r. Stops when
        ||s|| <= rtol ||s_0||. Returns (g, iterations, ||s|| / ||s_0||).
        """
        f = np.asarray(f, dtype=np.float64).ravel()
        g = self.default_g(f) if g0 is None else np.array(g0, dtype=np.float64)
        r = f - self.B(g)
        s = self.BT(r)
        p = s.copy()
        gamma = float(s @ s)
        s0 = math.sqrt(gamma)
        if s0 == 0.0:
            return g, 0, 0.0
        it = 0
        rel = 1.0
        while it < maxit:
            q = self.B(p)
            alpha = gamma / float(q @ q)
            g += alpha * p
            r -= alpha * q
            s = self.BT(r)
            gnew = float(s @ s)
            it += 1
            rel = math.sqrt(gnew) / s0
            if rel <= rtol:
                break
            beta = gnew / gamma
            p = s + beta * p
            gamma = gnew
        return g, it, rel

    def normal_residual(self, g: np.ndarray, f: np.ndarray) -> np.ndarray:
        f = np.asarray(f, dtype=np.float64).ravel()
        return self.BT(f - self.B(g))
