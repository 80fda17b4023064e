"""The S-iteration launch's plan built on the device against the host builder
(csrc/ss_plan.h, itself checked against the definition of the plan in
test_ss_plan.py): the Hilbert-order permutation, the block table, every
region list and every local matrix row, bit for bit. The host builder runs
on the library's own matrix (exported CSR, repacked into the ELL layout) and
coordinates, compiled with g++ from tests/ss_plan_check.cpp."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import torch

import paper_2105_01586_amd as fi
import synth
from gpu_common import case
from test_ss_plan import CSRC, HERE, SLOTS, run_plan

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = fi.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def host_exe(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    out = str(tmp_path_factory.mktemp("ssplan_gpu") / "ss_plan_check")
    subprocess.run(["g++", "-std=c++17", "-O2", "-Wall", "-pthread", "-I", CSRC,
                    os.path.join(HERE, "ss_plan_check.cpp"), "-o", out], check=True)
    return out


def ell_from_csr(c, n, W=SLOTS):
    """The library's ELL (off-diagonal entries in CSR order, padding pointing
    at the row itself, bit 31 for weight -1) from the exported K_FF."""
    rp, col, val = c["ff_rowptr"], c["ff_col"], c["ff_val"]
    rows = np.repeat(np.arange(n), np.diff(rp))
    off = col != rows
    r, cc, v = rows[off], col[off].astype(np.int64), val[off]
    assert np.all((v == -0.5) | (v == -1.0))
    starts = np.concatenate([[0], np.cumsum(np.bincount(r, minlength=n))[:-1]])
    slot = np.arange(r.size) - starts[r]
    assert slot.size == 0 or slot.max() < W
    n_pad = (n + 63) // 64 * 64
    pad_row = np.concatenate([np.arange(n), np.zeros(n_pad - n, np.int64)])
    ell = np.broadcast_to((1 << 30) | pad_row, (W, n_pad)).copy()
    ell[slot, r] = cc | np.where(v == -1.0, 1 << 31, 0)
    return ell.astype(np.uint32).view(np.int32), n_pad


def masks():
    out = []
    for name in ("n16_k7", "n256_k2000", "c2"):
        side, mask, _ = case(name)
        out.append((name, side, np.asarray(mask)))
    # a 1024^2 mesh of about 900 blocks (the reduction-launch shape), and a
    # clustered mask whose blocks have wide halos
    out.append(("r1024", 1024, synth.make_mask(21, 1024 * 1024, k=31466)))
    rng = np.random.default_rng(22)
    cx, cy = 300, 700
    pts = np.unique(((cy + rng.integers(-90, 90, 20000)) % 1024) * 1024
                    + (cx + rng.integers(-90, 90, 20000)) % 1024)
    out.append(("cluster1024", 1024, np.sort(pts).astype(np.int32)))
    return out


CASES = masks()


@pytest.mark.parametrize("name,side,mask", CASES, ids=[c[0] for c in CASES])
def test_device_plan_equals_host_plan(ctx, host_exe, tmp_path, name, side, mask):
    print(f"case {name}: side {side}, {mask.size} mask pixels", flush=True)
    M = fi.Mesh(ctx, side, mask.astype(np.int32))
    try:
        info = M.info
        assert info["cg_iters_per_launch"] == 3
        dev = M.export_ss_plan()
        geo = M.export_geometry()
        n = M.n
        ell, n_pad = ell_from_csr(M.export_csr(), n)
    finally:
        M.close()
    xy = geo["vxy"][geo["free_vids"]]
    host = run_plan(host_exe, tmp_path, xy, ell, n, n_pad, SLOTS, 3, 512, tasks=16)
    assert host["ok"]
    print(f"  {host['grid']} blocks, largest region {host['max_region']}, "
          f"{host['region'].size} region rows", flush=True)
    assert np.array_equal(dev["perm"], host["perm"])
    assert dev["blocks"].shape == host["blocks"].shape
    assert np.array_equal(dev["blocks"][:, :6], host["blocks"][:, :6])
    assert dev["blocks"][0, 6] == host["max_region"] == info["cg_max_region"]
    assert np.array_equal(dev["region"], host["region"])
    assert np.array_equal(dev["lmat"], host["lmat"])


def test_host_planned_solve_same_bits(ctx, monkeypatch):
    """A mesh planned on the host (FI_SS_PLAN=host, as server requests are)
    solves to the same bits as one planned on the device."""
    side, mask, f = case("c2")
    fd = torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0")
    M = fi.Mesh(ctx, side, mask)
    u_dev, _ = M.inpaint(f=fd)
    M.close()
    monkeypatch.setenv("FI_SS_PLAN", "host")
    H = fi.Mesh(ctx, side, mask)
    monkeypatch.delenv("FI_SS_PLAN")
    u_host, _ = H.inpaint(f=fd)
    H.close()
    assert torch.equal(u_dev, u_host)
