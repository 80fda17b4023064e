"""Row blocks with halos for the s-step CG launch (csrc/ss_plan.h), compiled
with g++ and run on the oracle's K_FF (CPU only).

Checks, per block: the own rows are the block's slice of a Hilbert-order numbering
of the free rows (last lattice row and column clamped onto the one before); the region holds exactly the rows within S hops of them,
in rings of increasing distance; every local matrix row decodes to that
row's entries of K_FF (neighbour slot and weight -1/2 or -1, padding pointing
at the zero slot). Then the Chebyshev basis the launch builds from region data
alone (rho_0 = v, rho_1 = D^-1 A_off v, rho_k+1 = 2 D^-1 A_off rho_k - rho_k-1)
is compared, on every block's own rows, with the same basis computed on the
whole system: S levels must agree to rounding.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import fem, mesh as om

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2105_01586_amd", "csrc")
SLOTS = 6  # local matrix entries per row (the plan's kPlanSlots)
PAD, M1 = 1 << 14, 1 << 15


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    out = str(tmp_path_factory.mktemp("ssplan") / "ss_plan_check")
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-pthread", "-I", CSRC,
                    os.path.join(HERE, "ss_plan_check.cpp"), "-o", out], check=True)
    return out


def ell_of(K_FF, W):
    """The library's ELL layout of the off-diagonal part (natural order)."""
    A = sp.csr_matrix(K_FF)
    n = A.shape[0]
    n_pad = (n + 63) // 64 * 64
    ell = np.empty((W, n_pad), dtype=np.int64)
    for i in range(n_pad):
        ell[:, i] = (1 << 30) | (i if i < n else 0)
    for i in range(n):
        cols = [c for c in A.indices[A.indptr[i]:A.indptr[i + 1]] if c != i]
        vals = [A[i, c] for c in cols]
        assert len(cols) <= W
        for k, (c, v) in enumerate(zip(cols, vals)):
            assert v in (-0.5, -1.0)
            ell[k, i] = int(c) | ((1 << 31) if v == -1.0 else 0)
    return ell.astype(np.uint32).view(np.int32), n_pad


def run_plan(exe, tmp_path, xy, ell, n, n_pad, W, S, BS, tasks=4):
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(fin, "wb") as f:
        np.array([n, n_pad], dtype=np.int64).tofile(f)
        np.array([W, S, BS, tasks], dtype=np.int32).tofile(f)
        np.ascontiguousarray(xy, dtype=np.int32).tofile(f)
        np.ascontiguousarray(ell, dtype=np.int32).tofile(f)
    subprocess.run([exe, fin, fout], check=True, timeout=300)
    raw = open(fout, "rb").read()
    ok, grid, maxreg = np.frombuffer(raw[:12], dtype=np.int32)
    plan = {"ok": int(ok), "grid": int(grid), "max_region": int(maxreg)}
    if not ok:
        return plan
    o = 12
    plan["perm"] = np.frombuffer(raw, dtype=np.int32, count=n, offset=o); o += 4 * n
    plan["blocks"] = np.frombuffer(raw, dtype=np.int32, count=8 * grid, offset=o).reshape(grid, 8)
    o += 32 * grid
    nh = int(np.frombuffer(raw, dtype=np.int64, count=1, offset=o)[0]); o += 8
    plan["region"] = np.frombuffer(raw, dtype=np.int32, count=nh, offset=o); o += 4 * nh
    nl = int(np.frombuffer(raw, dtype=np.int64, count=1, offset=o)[0]); o += 8
    plan["lmat"] = np.frombuffer(raw, dtype=np.uint16, count=nl, offset=o).reshape(-1, SLOTS)
    return plan


def hilbert(x, y, order):
    """Position along the Hilbert curve over [0, 2^order)^2 (quadrant digits
    from the top level down, the frame turned at each level)."""
    x = np.asarray(x, np.int64).copy()
    y = np.asarray(y, np.int64).copy()
    side = 1 << order
    d = np.zeros_like(x)
    s = side >> 1
    while s > 0:
        rx = (x & s) > 0
        ry = (y & s) > 0
        d += s * s * ((3 * rx.astype(np.int64)) ^ ry.astype(np.int64))
        turn = ~ry
        flip = turn & rx
        x[flip] = side - 1 - x[flip]
        y[flip] = side - 1 - y[flip]
        x[turn], y[turn] = y[turn].copy(), x[turn].copy()
        s >>= 1
    return d


@pytest.mark.parametrize("order", [0, 1, 2, 3, 5])
def test_hilbert_reference(order):
    # the test's own curve: every cell once, consecutive cells edge neighbours
    side = 1 << order
    xs, ys = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    d = hilbert(xs.ravel(), ys.ravel(), order)
    assert np.array_equal(np.sort(d), np.arange(side * side))
    at = np.empty((side * side, 2), np.int64)
    at[d] = np.stack([xs.ravel(), ys.ravel()], axis=1)
    assert np.all(np.abs(np.diff(at, axis=0)).sum(axis=1) == 1)


def check_plan(plan, K_FF, xy, S, BS):
    A = sp.csr_matrix(K_FF)
    n = A.shape[0]
    perm = plan["perm"].astype(np.int64)
    assert np.array_equal(np.sort(perm), np.arange(n))
    top = 1 << int(np.floor(np.log2(max(int(xy.max()), 1))))
    c = top - 1 if xy.max() > 1 else int(xy.max())
    order = int(c).bit_length()
    keys = hilbert(np.minimum(xy[perm, 0], c), np.minimum(xy[perm, 1], c), order)
    assert np.all((keys[1:] > keys[:-1]) | ((keys[1:] == keys[:-1]) & (perm[1:] > perm[:-1])))
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    Ap = A[perm][:, perm].tocsr()
    Aoff = Ap.copy()
    Aoff.setdiag(0)
    Aoff.eliminate_zeros()
    grid = plan["grid"]
    assert grid % 8 == 0 and grid >= (n + BS - 1) // BS
    regions = []
    for b in range(grid):
        reg_off, lmat_off, nown, n1, ninner, nreg = plan["blocks"][b][:6]
        r0, r1 = min(n, b * BS), min(n, (b + 1) * BS)
        assert nown == r1 - r0
        if nown == 0:
            assert nreg == 0 and reg_off == 0 and lmat_off == 0
            regions.append(np.zeros(0, np.int64))
            continue
        reg = plan["region"][reg_off:reg_off + nreg].astype(np.int64)
        assert np.array_equal(reg[:nown], np.arange(r0, r1))
        assert len(np.unique(reg)) == nreg
        # rings by BFS distance
        dist = np.full(n, -1)
        dist[r0:r1] = 0
        front = np.arange(r0, r1)
        for d in range(1, S + 1):
            nb = np.unique(Aoff[front].indices)
            nb = nb[dist[nb] < 0]
            dist[nb] = d
            front = nb
        assert set(reg.tolist()) == set(np.nonzero(dist >= 0)[0].tolist())
        dreg = dist[reg]
        assert np.all(np.diff(dreg) >= 0)
        for d in range(1, S + 1):
            ring = reg[dreg == d]
            assert np.all(np.diff(ring) > 0)
        assert n1 == np.count_nonzero(dreg <= 1)
        assert ninner == (np.count_nonzero(dreg <= S - 1) if S > 1 else nown)
        lm = plan["lmat"][lmat_off:lmat_off + ninner]
        for l in range(ninner):
            i = reg[l]
            cols = Aoff.indices[Aoff.indptr[i]:Aoff.indptr[i + 1]]
            vals = Aoff.data[Aoff.indptr[i]:Aoff.indptr[i + 1]]
            want = {int(c): float(v) for c, v in zip(cols, vals)}
            got = {}
            for e in lm[l]:
                e = int(e)
                if e & PAD:
                    assert e & 0x3FFF == 0 and not e & M1
                    continue
                assert e & 0x3FFF >= 1
                got[int(reg[(e & 0x3FFF) - 1])] = -1.0 if e & M1 else -0.5
            assert got == want, (b, l)
        regions.append(reg)
    return Aoff, regions


def check_basis(plan, Aoff, regions, d, S, seed=0):
    """The launch's local Chebyshev basis against the global one."""
    n = Aoff.shape[0]
    dinv = 1.0 / d
    v = np.random.default_rng(seed).normal(size=n)
    glob = [v]
    for k in range(S):
        t = dinv * (Aoff @ glob[-1])
        glob.append(t if k == 0 else 2.0 * t - glob[-2])
    for b, reg in enumerate(regions):
        if reg.size == 0:
            continue
        _, lmat_off, nown, _, ninner, nreg = plan["blocks"][b][:6]
        lm = plan["lmat"][lmat_off:lmat_off + ninner].astype(np.int64)
        # as the launch evaluates it: every entry one load from the slot
        # array (slot 0 a zero, slot l + 1 region row l), weight from bit 15
        idx = lm & 0x3FFF
        w = np.where(lm & M1, -1.0, -0.5)
        lev = [v[reg]]
        for k in range(S):
            prev = np.concatenate([[0.0], lev[-1]])
            nxt = np.full(nreg, np.nan)
            t = dinv[reg[:ninner]] * (w * prev[idx]).sum(axis=1)
            nxt[:ninner] = t if k == 0 else 2.0 * t - lev[-2][:ninner]
            lev.append(nxt)
        for k in range(S + 1):
            assert np.allclose(lev[k][:nown], glob[k][reg[:nown]], rtol=1e-12, atol=1e-12), (b, k)


@pytest.mark.parametrize("side,k,S,BS", [(16, 7, 3, 64), (32, 40, 2, 64), (64, 205, 3, 128),
                                         (64, 205, 1, 512), (128, 500, 4, 256)])
def test_plan_small(exe, tmp_path, side, k, S, BS):
    mask = synth.make_mask(side, side * side, k=k)
    M = om.build_mesh(side, mask)
    K = fem.assemble(M).K_FF
    xy = M.vxy[M.free_vids]
    ell, n_pad = ell_of(K, SLOTS)
    plan = run_plan(exe, tmp_path, xy, ell, K.shape[0], n_pad, SLOTS, S, BS)
    assert plan["ok"]
    Aoff, regions = check_plan(plan, K, xy, S, BS)
    check_basis(plan, Aoff, regions, K.diagonal()[plan["perm"]], S)


def test_plan_refuses_rows_wider_than_its_slots(exe, tmp_path):
    # the library's ELL is 8 wide only when a row has more than 6 entries;
    # such a mesh keeps the one-iteration launch
    mask = synth.make_mask(32, 32 * 32, k=40)
    M = om.build_mesh(32, mask)
    K = fem.assemble(M).K_FF
    ell, n_pad = ell_of(K, 8)
    plan = run_plan(exe, tmp_path, M.vxy[M.free_vids], ell, K.shape[0], n_pad, 8, 3, 64)
    assert plan["ok"] == 0


def test_plan_independent_of_task_count(exe, tmp_path):
    # every pass is split into tasks on the host pool; the plan is the same
    # for any split
    mask = synth.make_mask(128, 128 * 128, k=500)
    M = om.build_mesh(128, mask)
    K = fem.assemble(M).K_FF
    xy = M.vxy[M.free_vids]
    ell, n_pad = ell_of(K, SLOTS)
    plans = [run_plan(exe, tmp_path, xy, ell, K.shape[0], n_pad, SLOTS, 3, 256, tasks=t)
             for t in (1, 3, 16)]
    for p in plans[1:]:
        assert plans[0]["ok"] and p["ok"] and p["grid"] == plans[0]["grid"]
        for key in ("perm", "blocks", "region", "lmat"):
            assert np.array_equal(p[key], plans[0][key]), key


@pytest.mark.slow
def test_plan_workload_512(exe, tmp_path):
    w = synth.WORKLOADS["tonal512"]
    M = om.build_mesh(w.side, w.mask())
    K = fem.assemble(M).K_FF
    xy = M.vxy[M.free_vids]
    ell, n_pad = ell_of(K, 6)
    plan = run_plan(exe, tmp_path, xy, ell, K.shape[0], n_pad, 6, 3, 512)
    assert plan["ok"]
    print("grid", plan["grid"], "largest region", plan["max_region"],
          "halo rows per own row", round(plan["region"].size / K.shape[0] - 1, 3))
    # no block is a thin strip: the largest region stays under twice the block
    assert plan["max_region"] < 2 * 512
    Aoff, regions = check_plan(plan, K, xy, 3, 512)
    check_basis(plan, Aoff, regions, K.diagonal()[plan["perm"]], 3)
