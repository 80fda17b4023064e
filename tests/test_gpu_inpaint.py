"""GPU parity of the inpainting path against the FP64 oracle.

Integer work (mesh, CSR pattern, 2K values, owner triangles) must match
bit for bit; inpainted pixels within 1e-6 absolute on the 0-255 scale in both
FP32+refinement and plain FP64 modes; error measures within rounding.
"""
import numpy as np
import pytest
import torch

import paper_2105_01586_amd as fi
import synth
from gpu_common import SMALL_CASES, case, oracle_inpaint, oracle_problem

pytestmark = pytest.mark.gpu

NAMES = [c[0] for c in SMALL_CASES] + ["c2"]
PIX_TOL = 1e-6


@pytest.fixture(scope="module")
def ctx():
    c = fi.Context(0)
    yield c
    c.close()


_meshes = {}


def gpu_mesh(ctx, name):
    if name not in _meshes:
        side, mask, _ = case(name)
        _meshes[name] = fi.Mesh(ctx, side, mask)
    return _meshes[name]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("name", NAMES)
def test_geometry_and_matrices_bit_exact(ctx, name):
    print(f"case {name}", flush=True)
    M = gpu_mesh(ctx, name)
    pr = oracle_problem(name)
    g = M.export_geometry()
    assert np.array_equal(g["vxy"], pr.mesh.vxy)
    assert np.array_equal(g["tri"], pr.mesh.tri)
    assert np.array_equal(g["leaves"], pr.mesh.leaves)
    c = M.export_csr()
    K = pr.sys.K_FF
    assert np.array_equal(c["ff_rowptr"], K.indptr)
    assert np.array_equal(c["ff_col"], K.indices)
    assert np.array_equal(c["ff_val"], K.data)          # exact dyadic values
    assert np.array_equal((2 * c["ff_val"]).astype(np.int64), 2 * K.data)
    KD = pr.sys.K_FD
    assert np.array_equal(c["fd_rowptr"], KD.indptr)
    assert np.array_equal(c["fd_col"], KD.indices)
    assert np.array_equal(c["fd_val"], KD.data)


@pytest.mark.parametrize("name", NAMES)
def test_owner_map_bit_exact(ctx, name):
    print(f"case {name}", flush=True)
    M = gpu_mesh(ctx, name)
    own = M.owner_map().cpu().numpy()
    assert np.array_equal(own, oracle_problem(name).rast.owner)


@pytest.mark.parametrize("precision", [fi.PREC_FP32_IR, fi.PREC_FP64])
@pytest.mark.parametrize("name", NAMES)
def test_inpaint_parity(ctx, name, precision):
    print(f"case {name} precision {precision}", flush=True)
    M = gpu_mesh(ctx, name)
    _, _, f = case(name)
    u, st = M.inpaint(f=dev(f), opts=fi.SolveOpts(precision=precision))
    u = u.cpu().numpy()
    ref = oracle_inpaint(name)
    err = np.max(np.abs(u - ref))
    print(f"  max abs err {err:.3e}, iters {st['iterations']}, refinements {st['refinements']}, "
          f"rel residual {st['rel_residual']:.3e}")
    assert st["status"] == 0 and st["rel_residual"] <= 1e-10
    assert err <= PIX_TOL
    # mask pixels carry g exactly
    _, mask, _ = case(name)
    assert np.array_equal(u[mask], f[mask].astype(np.float64))


@pytest.mark.parametrize("name", NAMES)
def test_error_measures(ctx, name):
    print(f"case {name}", flush=True)
    M = gpu_mesh(ctx, name)
    _, _, f = case(name)
    pr = oracle_problem(name)
    ref = oracle_inpaint(name)
    u = dev(ref)   # same pixels on both sides: compare the error kernels alone
    mse, e, E = M.error(u, dev(f), pixel=True, triangle=True)
    e_ref = (ref - f.astype(np.float64)) ** 2
    assert np.array_equal(e.cpu().numpy(), e_ref)
    E_ref = pr.triangle_error(ref, f)
    assert np.allclose(E.cpu().numpy(), E_ref, rtol=1e-12, atol=1e-12)
    mse_ref = pr.mse(ref, f)
    assert abs(mse - mse_ref) <= 1e-12 * max(mse_ref, 1e-300) + 1e-300


def test_determinism(ctx):
    M = gpu_mesh(ctx, "c2")
    _, _, f = case("c2")
    u1, _ = M.inpaint(f=dev(f))
    u2, _ = M.inpaint(f=dev(f))
    assert torch.equal(u1, u2)
    m1 = M.error(u1, dev(f))[0]
    m2 = M.error(u2, dev(f))[0]
    assert m1 == m2


def test_given_g_and_constant(ctx):
    M = gpu_mesh(ctx, "n256_k2000")
    g = torch.full((M.m,), 77.5, dtype=torch.float64, device="cuda:0")
    u, _ = M.inpaint(g=g)
    # constants are harmonic: exact up to the solve tolerance
    assert torch.max(torch.abs(u - 77.5)).item() <= PIX_TOL
    pr = oracle_problem("n256_k2000")
    rng = np.random.default_rng(3)
    gv = rng.uniform(-100, 300, size=M.m)
    u, _ = M.inpaint(g=dev(gv))
    assert np.max(np.abs(u.cpu().numpy() - pr.B(gv))) <= PIX_TOL


def test_inpaint_image_one_shot(ctx):
    """fi_inpaint_image (mask as a bitmap, mesh built and freed inside) gives
    the mesh path's bits."""
    side, mask, f = case("n256_k2000")
    bitmap = np.zeros(side * side, np.uint8)
    bitmap[mask] = 1
    u1, st1 = fi.inpaint_image(ctx, dev(f), bitmap)
    M = gpu_mesh(ctx, "n256_k2000")
    u2, st2 = M.inpaint(f=dev(f))
    assert torch.equal(u1, u2) and st1["iterations"] == st2["iterations"]


def test_reassemble_is_identical(ctx):
    M = gpu_mesh(ctx, "n128_k300")
    before = M.export_csr()
    M.assemble()
    after = M.export_csr()
    for k in before:
        assert np.array_equal(before[k], after[k])


def test_error_paths(ctx):
    with pytest.raises(fi.FIError) as ei:
        fi.Mesh(ctx, 16, [])
    assert ei.value.code == fi.E_EMPTY_MASK
    with pytest.raises(fi.FIError) as ei:
        fi.Mesh(ctx, 16, [9, 3])
    assert ei.value.code == fi.E_INVALID
    M = gpu_mesh(ctx, "n16_k7")
    g = torch.zeros(M.m, dtype=torch.float64, device="cuda:0")
    g[0] = float("nan")
    with pytest.raises(fi.FIError) as ei:
        M.inpaint(g=g)
    assert ei.value.code == fi.E_INVALID
    with pytest.raises(ValueError):
        M.inpaint(g=torch.zeros(M.m + 1, dtype=torch.float64, device="cuda:0"))
    # iteration cap forced from the host: one CG iteration, one refinement
    Mc = gpu_mesh(ctx, "c2")
    _, _, f = case("c2")
    with pytest.raises(fi.NoConvergence):
        Mc.inpaint(f=dev(f), opts=fi.SolveOpts(max_inner=1, max_refine=1))


@pytest.mark.parametrize("precision", [fi.PREC_FP32_IR, fi.PREC_FP64])
def test_large_launch_shape_parity(ctx, precision, monkeypatch):
    """The launch shape used above 524288 unknowns (a one-block reduction
    launch between solver steps), forced on the 512^2 case for the oracle."""
    monkeypatch.setenv("FI_CG_LARGE", "1")
    side, mask, f = case("c2")
    M = fi.Mesh(ctx, side, mask)
    monkeypatch.delenv("FI_CG_LARGE")
    u, st = M.inpaint(f=dev(f), opts=fi.SolveOpts(precision=precision))
    err = np.max(np.abs(u.cpu().numpy() - oracle_inpaint("c2")))
    print(f"  large shape: max abs err {err:.3e}, iters {st['iterations']}")
    assert st["status"] == 0 and err <= PIX_TOL
    r = np.random.default_rng(9).normal(size=M.P)
    s, _ = M.adjoint(dev(r), opts=fi.SolveOpts(precision=precision))
    ref = oracle_problem("c2").BT(r)
    assert np.linalg.norm(s.cpu().numpy() - ref) <= 1e-8 * np.linalg.norm(ref)
    M.close()


def test_three_iterations_per_launch(ctx, monkeypatch):
    """The FP32 solve on the quadtree mesh advances three CG iterations per
    launch: the 512^2 solve takes at least 1.8 times fewer launches than
    the one-iteration launch (FI_CG_SSTEP=0), both within the pixel bar."""
    side, mask, f = case("c2")
    ref = oracle_inpaint("c2")
    M3 = gpu_mesh(ctx, "c2")
    monkeypatch.setenv("FI_CG_SSTEP", "0")
    M1 = fi.Mesh(ctx, side, mask)
    monkeypatch.delenv("FI_CG_SSTEP")
    assert M3.info["cg_iters_per_launch"] == 3 and M1.info["cg_iters_per_launch"] == 1
    u3, st3 = M3.inpaint(f=dev(f))
    u1, st1 = M1.inpaint(f=dev(f))
    M1.close()
    print(f"  launches {st3['launches']} (3 per launch) against {st1['launches']}; "
          f"iterations {st3['iterations']} / {st1['iterations']}")
    for u in (u3, u1):
        assert np.max(np.abs(u.cpu().numpy() - ref)) <= PIX_TOL
    assert st3["launches"] > 0 and 1.8 * st3["launches"] <= st1["launches"]


def test_kept_device_blocks_give_the_same_bits():
    """A context keeps a destroyed mesh's device blocks for the meshes built
    after it; meshes built in turn on such blocks (as a mask-growth loop
    builds them, each larger than the last) give the same bits as on a fresh
    context."""
    side, mask, f = case("c2")
    rng = np.random.default_rng(11)
    extra = np.setdiff1d(rng.choice(side * side, 3000, replace=False), mask)
    masks = [np.asarray(mask), np.union1d(mask, extra[:1000]), np.union1d(mask, extra)]
    fd = dev(f)

    def run(c, m):
        M = fi.Mesh(c, side, m.astype(np.int32))
        u, _ = M.inpaint(f=fd)
        out = u.cpu().numpy()
        M.close()
        return out

    c1 = fi.Context(0)
    reused = [run(c1, m) for m in masks]
    c1.close()
    for k, (m, u) in enumerate(zip(masks, reused)):
        print(f"  mesh {k}: {m.size} mask pixels", flush=True)
        c2 = fi.Context(0)
        fresh = run(c2, m)
        c2.close()
        assert np.array_equal(u, fresh)


def test_reduction_launch_same_bits_up_to_256_blocks(ctx, monkeypatch):
    """Up to 256 blocks the reduction launch (used by batched and multi-solve
    launches) sums the Gram partials in the order the blocks themselves use,
    so a solve gives the same bits either way."""
    side, mask, f = case("c2")
    M = gpu_mesh(ctx, "c2")
    assert M.info["cg_blocks"] <= 256 and not M.large_mode()
    monkeypatch.setenv("FI_CG_LARGE", "1")
    ML = fi.Mesh(ctx, side, mask)
    monkeypatch.delenv("FI_CG_LARGE")
    assert ML.large_mode()
    u, st = M.inpaint(f=dev(f))
    uL, stL = ML.inpaint(f=dev(f))
    ML.close()
    assert torch.equal(u, uL) and st["iterations"] == stL["iterations"]


@pytest.mark.parametrize("bs", ["256", "512"])
def test_block_sizes_agree(ctx, bs, monkeypatch):
    monkeypatch.setenv("FI_CG_BLOCK", bs)
    side, mask, f = case("n256_k2000")
    M = fi.Mesh(ctx, side, mask)
    monkeypatch.delenv("FI_CG_BLOCK")
    u, _ = M.inpaint(f=dev(f))
    assert np.max(np.abs(u.cpu().numpy() - oracle_inpaint("n256_k2000"))) <= PIX_TOL
    M.close()


@pytest.mark.parametrize("name,kind", [("n128_k300", "ell"), ("c2", "ell"), ("n256_k2000", "large"),
                                       ("n256_k2000", "delaunay")])
def test_reassembly_keeps_every_bit(ctx, name, kind, monkeypatch):
    """Later assemblies recompute every value (free and mask rows and the ELL
    slots) in one launch: the matrices and a solve afterwards are the same
    bits as after the first assembly. Also with the large-system launch shape
    and on the Delaunay mesh (CSR, up to 32 neighbours per row)."""
    side, mask, f = case(name)
    if kind == "large":
        monkeypatch.setenv("FI_CG_LARGE", "1")
        M = fi.Mesh(ctx, side, mask)
        monkeypatch.delenv("FI_CG_LARGE")
        assert M.large_mode()
    elif kind == "delaunay":
        unk = synth.make_unknowns(15, side * side, mask, mask.size)
        M = fi.Mesh(ctx, side, mask, unknowns=unk)
    else:
        M = gpu_mesh(ctx, name)
    before = M.export_csr()
    u1, st1 = M.inpaint(f=dev(f))
    for _ in range(2):
        M.assemble()
    after = M.export_csr()
    u2, st2 = M.inpaint(f=dev(f))
    if kind != "ell":
        M.close()
    for k in before:
        assert np.array_equal(before[k], after[k]), k
    assert torch.equal(u1, u2) and st1["iterations"] == st2["iterations"]


def test_error_dev_matches_error(ctx):
    """fi_error_dev leaves the squared-error sum on the device: the same bits
    as fi_error's MSE times P."""
    M = gpu_mesh(ctx, "c2")
    _, _, f = case("c2")
    fd = dev(f)
    u, _ = M.inpaint(f=fd)
    mse, _, _ = M.error(u, fd)
    sse = M.error_dev(u, fd)
    assert sse.item() / M.P == mse
