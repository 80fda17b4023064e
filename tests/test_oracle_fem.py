"""Pins of the oracle's P1 stiffness matrix and direct solve (Section 2.2).

Pins: an independent gradient computation (inverting the 3x3 Vandermonde
matrix of each triangle); the closed form on an all-unit mesh, where the FEM
matrix equals the 5-point finite-difference Laplacian with halved boundary
couplings, as Section 2.2 states for a mesh whose vertices are all pixels;
symmetry, zero row sums, non-positive off-diagonals, integer 2K; positive
definiteness exactly when the mask is non-empty; dense brute-force solves;
constants reproduced; the discrete maximum principle.
"""
import numpy as np
import pytest

from oracle import fem, mesh as mesh_mod, solve, tonal


def random_mask(rng, N, k):
    return np.sort(rng.choice(N * N, size=k, replace=False))


def test_element_matrix_matches_vandermonde_gradients():
    rng = np.random.default_rng(0)
    for _ in range(50):
        p = rng.integers(-20, 20, size=(3, 2))
        twoA = (p[1, 0] - p[0, 0]) * (p[2, 1] - p[0, 1]) - (p[1, 1] - p[0, 1]) * (p[2, 0] - p[0, 0])
        if twoA == 0:
            continue
        if twoA < 0:
            p = p[[0, 2, 1]]
            twoA = -twoA
        Vm = np.column_stack([np.ones(3), p[:, 0], p[:, 1]]).astype(float)
        C = np.linalg.inv(Vm)          # phi_i = C[0,i] + C[1,i] x + C[2,i] y
        G = C[1:, :].T                 # (3, 2) gradients
        ref = 0.5 * twoA * G @ G.T
        got = fem.element_matrices(p.astype(np.int64), np.array([[0, 1, 2]]))[0]
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


def five_point_neumann(N):
    """FEM on the all-unit mesh: -1 per interior lattice edge, -1/2 per boundary edge."""
    V = (N + 1) ** 2
    K = np.zeros((V, V))

    def vid(x, y):
        return y * (N + 1) + x
    for y in range(N + 1):
        for x in range(N + 1):
            for dx, dy in ((1, 0), (0, 1)):
                X, Y = x + dx, y + dy
                if X > N or Y > N:
                    continue
                on_boundary = (dy == 0 and y in (0, N)) or (dx == 0 and x in (0, N))
                w = -0.5 if on_boundary else -1.0
                a, b = vid(x, y), vid(X, Y)
                K[a, b] += w
                K[b, a] += w
    K[np.diag_indices(V)] = -K.sum(axis=1)
    return K


@pytest.mark.parametrize("N", [2, 4, 8])
def test_all_unit_mesh_is_five_point_fdm(N):
    ys, xs = np.mgrid[0:N:2, 0:N:2]
    m = np.sort((ys * N + xs).ravel())
    M = mesh_mod.build_mesh(N, m)
    S = fem.assemble(M)
    assert M.V == (N + 1) ** 2
    assert np.array_equal(S.K.toarray(), five_point_neumann(N))


@pytest.mark.parametrize("N,k,seed", [(8, 3, 0), (16, 7, 1), (32, 30, 2), (64, 205, 3), (64, 1, 4)])
def test_matrix_invariants(N, k, seed):
    M = mesh_mod.build_mesh(N, random_mask(np.random.default_rng(seed), N, k))
    S = fem.assemble(M)
    K = S.K.toarray()
    assert np.array_equal(K, K.T)
    assert np.allclose(K.sum(axis=1), 0.0, atol=0)          # exact: dyadic values
    off = K - np.diag(np.diag(K))
    assert off.max() <= 0
    assert np.array_equal(2 * K, np.round(2 * K))
    assert set(np.unique(2 * off)) <= {0.0, -1.0, -2.0}
    # no explicit zeros stored
    assert np.all(S.K_FF.data != 0) and np.all(S.K_FD.data != 0)
    assert np.array_equal(S.K_DF.toarray(), S.K_FD.toarray().T)


@pytest.mark.parametrize("N,k,seed", [(8, 1, 0), (8, 4, 1), (16, 9, 2)])
def test_spd_iff_mask_nonempty(N, k, seed):
    M = mesh_mod.build_mesh(N, random_mask(np.random.default_rng(seed), N, k))
    S = fem.assemble(M)
    ev = np.linalg.eigvalsh(S.K_FF.toarray())
    assert ev.min() > 1e-10
    # the full matrix is singular, with the constants as its null space
    evk = np.linalg.eigvalsh(S.K.toarray())
    assert abs(evk[0]) < 1e-10 and evk[1] > 1e-8


@pytest.mark.parametrize("N,k,seed", [(8, 3, 0), (16, 10, 1), (32, 25, 2)])
def test_banded_cholesky_matches_dense_solve(N, k, seed):
    rng = np.random.default_rng(seed)
    M = mesh_mod.build_mesh(N, random_mask(rng, N, k))
    S = fem.assemble(M)
    b = rng.normal(size=M.n)
    x_dense = np.linalg.solve(S.K_FF.toarray(), b)
    x_chol = solve.BandedCholesky(S.K_FF).solve(b)
    assert np.allclose(x_chol, x_dense, rtol=1e-12, atol=1e-10)
    assert np.linalg.norm(S.K_FF @ x_chol - b) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("N,k,seed", [(16, 6, 0), (32, 40, 1), (64, 205, 2)])
def test_constant_and_maximum_principle(N, k, seed):
    rng = np.random.default_rng(seed)
    pr = tonal.Problem(N, random_mask(rng, N, k))
    u = pr.vertex_solution(np.full(pr.mesh.m, 37.25))
    assert np.allclose(u, 37.25, rtol=0, atol=1e-11)
    g = rng.uniform(-50, 200, size=pr.mesh.m)
    u = pr.vertex_solution(g)
    assert u.min() >= g.min() - 1e-9 and u.max() <= g.max() + 1e-9
    assert np.array_equal(u[pr.mesh.mask_vids], g)


@pytest.mark.parametrize("N,k,seed", [(8, 3, 0), (16, 10, 1), (32, 25, 2), (64, 205, 3)])
def test_sparse_cholesky_matches_dense(N, k, seed):
    from oracle.sparse_chol import SparseCholesky, nested_dissection
    rng = np.random.default_rng(seed)
    M = mesh_mod.build_mesh(N, random_mask(rng, N, k))
    S = fem.assemble(M)
    b = rng.normal(size=M.n)
    x_dense = np.linalg.solve(S.K_FF.toarray(), b)
    for c in (SparseCholesky(S.K_FF, M.vxy[M.free_vids], N), SparseCholesky(S.K_FF)):
        assert np.allclose(c.solve(b), x_dense, rtol=1e-12, atol=1e-11)
    order = nested_dissection(M.vxy[M.free_vids], N)
    assert np.array_equal(np.sort(order), np.arange(M.n))
    # the factor itself: L L^T reproduces the permuted matrix
    c = SparseCholesky(S.K_FF, M.vxy[M.free_vids], N)
    e = np.zeros(M.n)
    e[3] = 1.0
    assert np.allclose(S.K_FF @ c.solve(e), e, atol=1e-12)


def test_sparse_cholesky_rejects_indefinite():
    from oracle.sparse_chol import SparseCholesky
    import scipy.sparse as sp
    A = sp.csc_matrix(np.array([[1.0, 2.0], [2.0, 1.0]]))
    with pytest.raises(np.linalg.LinAlgError):
        SparseCholesky(A)


def test_sparse_and_banded_agree_on_workload():
    import synth
    from oracle.sparse_chol import SparseCholesky
    w = synth.WORKLOADS["plain64"]
    M = mesh_mod.build_mesh(w.side, w.mask())
    S = fem.assemble(M)
    b = np.random.default_rng(1).normal(size=M.n)
    x1 = SparseCholesky(S.K_FF, M.vxy[M.free_vids], w.side).solve(b)
    x2 = solve.BandedCholesky(S.K_FF).solve(b)
    assert np.allclose(x1, x2, rtol=1e-12, atol=1e-11)
