"""The quadtree mesh built on the device (fi_mesh_build) against the host
builder (fi_host_mesh_build, itself bit-exact against the oracle's mesh in the
CPU tests): coordinates, triangles, leaves, free and mask vertex ids, bit for
bit, on masks of every kind; and a solve on a device-built mesh gives the
same bits as on the host-built one (FI_MESH_HOST=1)."""
import numpy as np
import pytest
import torch

import paper_2105_01586_amd as fi
import synth
from gpu_common import case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = fi.Context(0)
    yield c
    c.close()


def masks():
    rng = np.random.default_rng(31)
    out = [("n2_one", 2, np.array([3])), ("n2_full", 2, np.arange(4)),
           ("n4_corner", 4, np.array([15])), ("n16_full", 16, np.arange(256)),
           ("n16_edges", 16, np.array([0, 15, 240, 255])),
           ("n64_border", 64, np.unique(np.concatenate([np.arange(64), 63 * 64 + np.arange(64),
                                                         64 * np.arange(64)])))]
    for name in ("n128_k300", "n256_k2000", "c2"):
        side, mask, _ = case(name)
        out.append((name, side, np.asarray(mask)))
    out.append(("r1024", 1024, synth.make_mask(41, 1024 * 1024, k=10486)))
    pts = np.unique(((700 + rng.integers(-60, 60, 15000)) % 1024) * 1024
                    + (300 + rng.integers(-60, 60, 15000)) % 1024)
    out.append(("cluster1024", 1024, pts))
    out.append(("r2048", 2048, synth.make_mask(42, 2048 * 2048, k=2048 * 2048 // 20)))
    out.append(("dense1024", 1024, synth.make_mask(43, 1024 * 1024, k=1024 * 1024 * 7 // 10)))
    out.append(("r4096", 4096, synth.make_mask(44, 4096 * 4096, k=4096 * 4096 // 50)))
    return out


CASES = masks()


@pytest.mark.parametrize("name,side,mask", CASES, ids=[c[0] for c in CASES])
def test_device_mesh_equals_host_mesh(ctx, name, side, mask):
    mask = np.sort(np.asarray(mask)).astype(np.int32)
    print(f"case {name}: side {side}, {mask.size} mask pixels", flush=True)
    h = fi.host_mesh(side, mask)
    M = fi.Mesh(ctx, side, mask)
    try:
        info = M.info
        g = M.export_geometry()
    finally:
        M.close()
    for k in ("V", "T", "L", "n", "m"):
        assert info[k] == h[k], k
    for k in ("vxy", "tri", "leaves", "free_vids", "mask_vids"):
        assert np.array_equal(g[k], h[k]), k


def test_device_mesh_solves_to_host_mesh_bits(ctx, monkeypatch):
    side, mask, f = case("c2")
    fd = torch.from_numpy(np.ascontiguousarray(f)).to("cuda:0")
    M = fi.Mesh(ctx, side, mask)
    u_dev, _ = M.inpaint(f=fd)
    M.close()
    monkeypatch.setenv("FI_MESH_HOST", "1")
    H = fi.Mesh(ctx, side, mask)
    monkeypatch.delenv("FI_MESH_HOST")
    u_host, _ = H.inpaint(f=fd)
    H.close()
    assert torch.equal(u_dev, u_host)


@pytest.mark.parametrize("side,mask,code", [(2, [], "empty"), (100, [1], "side"),
                                            (8, [5, 3], "order"), (8, [64], "range")])
def test_device_mesh_rejects_bad_input(ctx, side, mask, code):
    with pytest.raises(fi.FIError):
        fi.Mesh(ctx, side, np.asarray(mask, dtype=np.int32))
