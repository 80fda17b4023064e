"""Benchmark of the inpainting hot path on one MI355X.

One step = one pass of the hot path over the 512 x 512 synthetic image with a
4% random mask (the mixed-precision + tonal-optimisation workload; the
default; ``--workload large8192`` runs the 8192 x 8192 / 2% image instead,
``--workload serving`` the batched-serving trace, see ``serving_main``):
  assembly of the stiffness matrix, inpainting u = B g with FP32 Jacobi-PCG +
  FP64 iterative refinement to relative residual 1e-10, interpolation to
  pixels and the squared-error sum of the MSE, kept on the device until the
  timing ends (the "inpainting" phase), then tonal optimisation by CGLS to
  relative normal residual 1e-8 (the "tonal" phase).
Inputs sit in device memory before timing starts; the mesh is built once
(it depends on the mask only).

Prints ONE JSON line. ``value`` is inpainted Mpixel/s (P / inpainting-phase
time); tonal-optimisation solves/s and the full step time are reported
beside it. ``roofline`` covers the dominant kernel (the fused FP32 CG
iteration), timed with HIP events on the library's stream; ``cpu_baseline``
times the FP64 CPU oracle on the same workload (repeated inpaintings for about
10 s), and the untimed checks beside it compare the results with the oracle.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("solver.hip", "sstep.hip", "ss_plan.h", "cg_common.h", "reduce.h", "internal.h")


def kernel_source_hash() -> str:
    """sha256 over the sources of the CG step kernel."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2105_01586_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def cg_kernel_name(info, nrhs: int = 1) -> str:
    """The FP32 CG step kernel a mesh uses, for the roofline label."""
    mode = "summed by a second launch" if info["large_mode"] else "block re-reduce"
    if info["cg_iters_per_launch"] > 1:
        what = "k_ss_multi" if nrhs > 1 else "k_ss_step"
        return (f"{what}<3 iterations per launch, {mode}, 512 rows + 3-hop halo per block"
                + (f", {nrhs} right-hand sides" if nrhs > 1 else "") + ">")
    what = "k_step_multi" if nrhs > 1 else "k_step"
    return f"{what}<float, {mode}, 512>"


def ss_layout_bytes(info):
    """Bytes the three-iteration launch moves by its layout, with no cache
    help: per own row the 32-byte basis record read and written, the
    correction read and written, the diagonal; per region row a 12-byte
    local matrix row (which only rows within two hops have: an upper bound)
    and its row index (halo rows only in the large-system launch, which
    takes own rows from the block's position); per halo row the record read
    again. None for the one-iteration kernel."""
    if info["cg_iters_per_launch"] <= 1:
        return None
    n, reg = info["n"], info["cg_region_rows"]
    idx_rows = reg - n if info["large_mode"] else reg
    return n * (32 + 32 + 8 + 4) + reg * 12 + idx_rows * 4 + (reg - n) * 32


def launch_rates(info, nrhs, kms):
    """Extra fields of a roofline line for the three-iteration launch: the
    byte rate of its layout, and the rate three one-iteration launches (4
    bytes per matrix entry and 44 per row and solve each) would need to take
    the same time, a time-to-solution figure, not HBM traffic."""
    k = info["cg_iters_per_launch"]
    if k <= 1:
        return {}
    nnz_off = int(info["nnz_ff"]) - int(info["n"])
    equiv = k * (4 * nnz_off + 44 * nrhs * int(info["n"]))
    out = {"iteration_equivalent_bytes": equiv,
           "iteration_equivalent_GBs": equiv / (kms * 1e-3) / 1e9}
    lay = ss_layout_bytes(info)
    if lay is not None and nrhs == 1:
        out["layout_bytes_per_launch"] = lay
        out["layout_GBs"] = lay / (kms * 1e-3) / 1e9
    return out


def recorded_traffic(workload: str):
    """HBM bytes per launch of the dominant kernel from the counter runs in
    profiles/traffic.json (FETCH_SIZE and WRITE_SIZE, scaled by a plain
    copy), or None when they were taken on other kernel sources."""
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
            rec = json.load(fh)[workload]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 5; 1 for the 8192^2 workload)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps (default 2; 0 for the 8192^2 workload)")
    ap.add_argument("--workload", default="tonal512",
                    help="tonal512 (default), large8192, serving, densify, rgb512 or l1512")
    ap.add_argument("--requests", type=int, default=256, help="serving: requests in the trace")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="serving: arrivals per second (default 0.7 x FP64 capacity)")
    ap.add_argument("--capacity-sample", type=int, default=64,
                    help="serving: requests timed to measure the FP64 capacity")
    ap.add_argument("--max-slots", type=int, default=16)
    ap.add_argument("--build-threads", type=int, default=8)
    ap.add_argument("--hbm-budget-gb", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=300)
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run one 256 MiB device-to-device copy (a kernel of known "
                         "traffic, to scale hardware byte counters)")
    return ap.parse_args()


def cpu_cores_used(t_wall0, t_cpu0):
    """Threads the oracle actually kept busy over a sample: this process's
    CPU time (all its threads) over the wall time."""
    wall = time.perf_counter() - t_wall0
    return round((time.process_time() - t_cpu0) / wall, 2) if wall > 0 else None


def cpu_baseline(side, f_np, mask, u_gpu, what, grad_at=None, tonal_rtol=None, runs=3):
    """The oracle, as it stands, timed part by part over ``runs`` full runs on
    ``what``; each part reports its median. One run is: mesh, assembly,
    owner map and interpolation matrix, sparse Cholesky factorisation, the
    inpainting solve, interpolation and MSE, and (with ``tonal_rtol``) the
    oracle's CGLS tonal optimisation to that tolerance on a prepared problem.
    ``value`` is pixels over the median of assembly + factorisation + solve +
    interpolation and error: the scope of the GPU's inpainting step (the mesh
    and the owner map are per-mesh set-up on both sides and reported apart).
    The oracle's sparse Cholesky is plain single-threaded C; ``cores`` is the
    process CPU time over wall time (BLAS threads included).

    Also returns the GPU result's agreement with the oracle: max |u - u_oracle|
    and, with ``grad_at`` = (g, GPU gradient of the MSE at g), the oracle's MSE
    and the gradient's relative error against the oracle's."""
    from oracle import error as oerr, fem, mesh as omesh, raster, solve, tonal
    f = f_np.ravel()
    keys = ("mesh", "assembly", "owner_map", "factorisation", "solve", "interpolation_error")
    parts = {k: [] for k in keys}
    tonal_s = []
    pr = None
    t0, c0 = time.perf_counter(), time.process_time()
    for _ in range(runs):
        t = [time.perf_counter()]
        M = omesh.build_mesh(side, mask)
        t.append(time.perf_counter())
        S = fem.assemble(M)
        t.append(time.perf_counter())
        R = raster.rasteriser(M)
        t.append(time.perf_counter())
        fac = solve.factorise(S.K_FF, "auto", M.vxy[M.free_vids], side)
        t.append(time.perf_counter())
        g = f[M.mask_idx].astype(np.float64)
        uv = np.empty(M.V, dtype=np.float64)
        uv[M.mask_vids] = g
        uv[M.free_vids] = fac.solve(-(S.K_FD @ g))
        t.append(time.perf_counter())
        u_ref = raster.rasterise(R, uv)
        mse_ref = oerr.mse(u_ref, f)
        t.append(time.perf_counter())
        for k, a, b in zip(keys, t[:-1], t[1:]):
            parts[k].append(b - a)
        if tonal_rtol is not None:
            if pr is None:
                pr = tonal.Problem(side, mask)
            ts0 = time.perf_counter()
            g_t, it_t, _ = pr.tonal_cgls(f.astype(np.float64), rtol=tonal_rtol)
            tonal_s.append(time.perf_counter() - ts0)
    el = time.perf_counter() - t0
    cores = cpu_cores_used(t0, c0)
    med = {k: float(np.median(v)) for k, v in parts.items()}
    step = med["assembly"] + med["factorisation"] + med["solve"] + med["interpolation_error"]
    P = side * side
    err = float(np.max(np.abs(u_gpu - u_ref))) if u_gpu is not None else None
    if grad_at is not None:
        if pr is None:
            pr = tonal.Problem(side, mask)
        g0, grad = grad_at
        ref = pr.mse_grad(g0, f)
        err = {"max_abs_pixel_err": err, "mse_oracle": mse_ref,
               "grad_rel_err_vs_oracle": float(np.linalg.norm(grad - ref) / np.linalg.norm(ref))}
        if tonal_rtol is not None:
            err["mse_tonal_oracle"] = pr.mse_of_g(g_t, f)
            err["tonal_iterations_oracle"] = it_t
    out = {"value": P / step / 1e6, "unit": "Mpixel/s", "cores": cores,
           "host_cores": len(os.sched_getaffinity(0)), "kind": "oracle",
           "sample": f"{runs} full oracle runs on {what} (each part: median of {runs}); value = "
                     f"pixels / (assembly + factorisation + solve + interpolation and error); "
                     f"sparse Cholesky single-threaded; {el:.1f} s in all",
           "median_s": med}
    if tonal_s:
        tm = float(np.median(tonal_s))
        out["tonal_s"] = tm
        out["tonal_solves_per_s"] = 1.0 / tm
        out["tonal_iterations"] = it_t
    return out, err


def crop_check(fi, ctx, f_np, mask):
    """The final MSEs on the 2048^2 crop the oracle can solve (inpainting,
    and tonal optimisation to 1e-8), against the oracle's values stored in
    tests/golden/large8192_crop.json (written by the script beside it, which
    calls only the oracle)."""
    import torch
    import synth
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests",
                                       "golden", "large8192_crop.json")))
    r0, c0 = synth.busiest_block(f_np, 2048)
    cf, cm = synth.crop(f_np, mask, r0, c0, 2048)
    M = fi.Mesh(ctx, 2048, cm)
    fd = torch.from_numpy(cf.ravel().copy()).cuda()
    u, _ = M.inpaint(f=fd)
    mse, _, _ = M.error(u, fd)
    _, ts = M.tonal_opt(fd, opts=fi.TonalOpts(rtol=1e-8))
    M.close()
    return {"crop_origin": [r0, c0], "mse_inpaint": mse, "mse_inpaint_oracle": gold["mse_inpaint"],
            "mse_tonal": ts["mse_final"], "mse_tonal_oracle": gold["mse_tonal"],
            "rel_diff_inpaint": abs(mse - gold["mse_inpaint"]) / gold["mse_inpaint"],
            "rel_diff_tonal": abs(ts["mse_final"] - gold["mse_tonal"]) / gold["mse_tonal"]}


def fd_check(fi, mesh, f, f_np, mask, n_dir=16, eps=1e-3, seed=7):
    """The gradient of MSE(g) = ||B g - f||^2 / P from the adjoint,
    (2 / P) B^T (B g - f), against central differences along 16 random
    coordinates of g (eps = 1e-3), at g = f on the mask plus N(0, 2) noise.
    The MSE is quadratic in g, so the differences carry only the rounding and
    solve error of the two losses (solved to 1e-12). All on the GPU. Returns
    (g, gradient) and the report."""
    import torch
    rng = np.random.default_rng(seed)
    g0 = f_np.ravel()[mask].astype(np.float64) + rng.normal(scale=2.0, size=mask.size)
    g = torch.from_numpy(g0).cuda()
    u, _ = mesh.inpaint(g=g)
    grad = mesh.mse_backward(u, f)[0].cpu().numpy()
    tight = fi.SolveOpts(rtol=1e-12)
    scale = float(np.max(np.abs(grad)))
    worst = 0.0
    for j in rng.integers(0, mask.size, size=n_dir):
        loss = []
        for sign in (1.0, -1.0):
            gj = g.clone()
            gj[j] += sign * eps
            uj, _ = mesh.inpaint(g=gj, opts=tight)
            loss.append(mesh.error(uj, f)[0])
        fd = (loss[0] - loss[1]) / (2 * eps)
        worst = max(worst, abs(fd - grad[j]) / (abs(grad[j]) + 1e-3 * scale))
    return (g0, grad), {"directions": n_dir, "eps": eps,
                        "max_rel_dev": worst, "scale": "|fd - grad| / (|grad| + 1e-3 max|grad|)"}


def _gen(req):
    return req.image().ravel(), req.mask()


def serving_main(args):
    """The batched-serving workload: a Poisson trace of requests (side
    uniform over 128..2048, mask density U[2%, 10%]), each one inpainting +
    30 CGLS iterations (FP32 inner solves, FP64 residuals).

    1. Plain FP64 GPU server, one request at a time, all requests of the first
       ``--capacity-sample`` queued at once: its capacity mu (requests/s).
    2. The arrival rate is 0.7 mu (a load the sequential FP64 server can
       sustain); the trace is drawn at that rate.
    3. The batched FP32 server on the whole trace queued at once (throughput:
       ``value``), then replayed at the trace's arrival times and at twice the
       rate (p50 / p99 latency), and the FP64 server replayed at the trace's
       arrival times (its p50 / p99)."""
    import concurrent.futures as cf
    import torch
    import paper_2105_01586_amd as fi
    from paper_2105_01586_amd import serving
    import synth

    iters = 30
    trace = synth.serving_trace(seed=4, n=args.requests)
    t = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        reqs = list(ex.map(_gen, trace, chunksize=4))
    print(f"generated {len(reqs)} requests in {time.perf_counter() - t:.1f} s", file=sys.stderr,
          flush=True)
    ctx = fi.Context(0)
    budget = args.hbm_budget_gb << 30
    base = dict(hbm_budget=budget, build_threads=args.build_threads)
    # 1. FP64 sequential capacity
    k = min(args.capacity_sample, len(reqs))
    with fi.Server(ctx, fi.ServerOpts(max_slots=1, precision=fi.PREC_FP64, **base)) as S:
        cap = serving.summarize(serving.replay(S, reqs[:k], np.zeros(k), iters))
    mu = cap["requests_per_s"]
    rate = args.rate if args.rate else 0.7 * mu
    print(f"FP64 sequential capacity {mu:.2f} req/s; rate {rate:.2f} req/s", file=sys.stderr,
          flush=True)
    # the same trace drawn at that rate: identical sides, densities and
    # images; the exponential gaps scale with 1 / rate
    arr = np.array([r.arrival_s for r in synth.serving_trace(seed=4, n=len(reqs), rate_hz=rate)])
    out = {}
    bopts = fi.ServerOpts(max_slots=args.max_slots, **base)
    with fi.Server(ctx, bopts) as S:
        closed = serving.summarize(serving.replay(S, reqs, np.zeros(len(reqs)), iters))
        st_closed = S.stats()
    print(f"batched closed loop {closed['mpixel_per_s']:.1f} Mpixel/s", file=sys.stderr,
          flush=True)
    with fi.Server(ctx, bopts) as S:
        at1 = serving.summarize(serving.replay(S, reqs, arr, iters))
        st1 = S.stats()
    print(f"batched at rate: p50 {at1['p50_ms']:.0f} ms p99 {at1['p99_ms']:.0f} ms",
          file=sys.stderr, flush=True)
    with fi.Server(ctx, bopts) as S:
        at2 = serving.summarize(serving.replay(S, reqs, arr / 2.0, iters))
    print(f"batched at 2x rate: p50 {at2['p50_ms']:.0f} ms p99 {at2['p99_ms']:.0f} ms",
          file=sys.stderr, flush=True)
    fp64 = None
    if not args.skip_fp64:
        with fi.Server(ctx, fi.ServerOpts(max_slots=1, precision=fi.PREC_FP64, **base)) as S:
            fp64 = serving.summarize(serving.replay(S, reqs, arr, iters))
        print(f"FP64 sequential at rate: p50 {fp64['p50_ms']:.0f} ms p99 {fp64['p99_ms']:.0f} ms",
              file=sys.stderr, flush=True)
    # dominant kernel: the CG step on the largest request class (2048^2, 10%)
    big = max(range(len(trace)), key=lambda i: (trace[i].side, trace[i].density))
    f_big, m_big = reqs[big]
    M = fi.Mesh(ctx, trace[big].side, m_big)
    fd = torch.from_numpy(f_big.copy()).cuda()
    M.inpaint(f=fd)
    kms = M.time_cg_kernel(fi.PREC_FP32_IR, args.kernel_reps)
    kbytes = M.cg_kernel_bytes(fi.PREC_FP32_IR)
    achieved = kbytes / (kms * 1e-3) / 1e9
    M.close()
    pix = sum(f.size for f, _ in reqs)
    out = {
        "metric": "inpainted Mpixel/s + tonal-opt solves/s at <=1e-6 err vs FP64; p50/p99 latency",
        "value": closed["mpixel_per_s"],
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": closed["makespan_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (CG) + f64 (residual, refinement, CGLS)",
        "data": "synthetic",
        "config": {"workload": f"serving: {len(reqs)} requests, side U{{128..2048}}, mask "
                               f"U[2%,10%], inpainting + {iters} CGLS iterations each",
                   "requests": len(reqs), "total_pixels": pix, "rate_req_s": rate,
                   "max_slots": args.max_slots, "hbm_budget_gb": args.hbm_budget_gb},
        "batched_closed_loop": closed,
        "batched_at_rate": at1,
        "batched_at_2x_rate": at2,
        "fp64_sequential_at_rate": fp64,
        "fp64_sequential_capacity": cap,
        "speedup_throughput_vs_fp64": closed["mpixel_per_s"] / cap["mpixel_per_s"],
        "server_stats": {"closed_loop": st_closed, "at_rate": st1},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic("serving"),
                     "kernel": f"{cg_kernel_name(M.info)} on the {trace[big].side}^2 / "
                               f"{trace[big].density:.1%} request",
                     "iterations_per_launch": M.info["cg_iters_per_launch"],
                     "bytes_per_launch": kbytes, "us_per_launch": kms * 1e3,
                     **launch_rates(M.info, 1, kms)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = serving_cpu_baseline(trace, reqs, iters)
    print(json.dumps(out))
    ctx.close()


def serving_cpu_baseline(trace, reqs, iters):
    """The oracle on the first requests of side <= 256 until about 15 s:
    inpainting plus the same CGLS iterations with exact Cholesky solves."""
    from oracle import tonal
    t0, c0 = time.perf_counter(), time.process_time()
    pix, n = 0, 0
    for r, (f, m) in zip(trace, reqs):
        if r.side > 256:
            continue
        pr = tonal.Problem(r.side, m)
        pr.mse(pr.inpaint(f), f)
        pr.tonal_cgls(f.astype(np.float64), rtol=0.0, maxit=iters)
        pix += f.size
        n += 1
        if time.perf_counter() - t0 > 15.0:
            break
    el = time.perf_counter() - t0
    return {"value": pix / el / 1e6, "unit": "Mpixel/s", "cores": cpu_cores_used(t0, c0),
            "host_cores": len(os.sched_getaffinity(0)), "kind": "oracle",
            "sample": f"{n} requests of side <= 256 from the trace (inpainting + {iters} CGLS "
                      f"iterations, direct Cholesky), {el:.1f} s"}


def densify_main(args):
    """Error-driven mask selection (Section 3), timed end to end: every round
    builds the mesh on the host, inpaints, computes the error map and picks
    the next pixels on the GPU.

    * densify1024: the global top-k rule, 1024^2, 1% -> 3% in 20 rounds of
      +0.1% (21 inpaintings);
    * the paper's own per-triangle rule at 512^2 and 1024^2: final density
      4% introduced in n = 10 inpaintings, m/n pixels each (first m/n at
      random), as in its Table 2 (context only: the paper's CPU and image);
    * the same at 512^2 on the paper's own Delaunay mesh, with m unknown
      vertices drawn once.

    ``value`` is inpainted Mpixel/s over all the loops with the time the
    workload defines: the solves, interpolation and error of every round
    (HIP events around them; the host mesh builds and the pixel selection
    between rounds excluded). ``mpixel_per_s_wall`` is the same over wall
    time, mesh builds included."""
    import torch
    import paper_2105_01586_amd as fi
    import synth

    ctx = fi.Context(0)
    runs = {}

    def run(name, side, f_np, mask0, k, rounds, rule, unknowns=None):
        f = torch.from_numpy(f_np.ravel().copy()).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        order, mse, ms = fi.densify(ctx, side, f, mask0, k, rounds, rule=rule, unknowns=unknowns)
        wall = time.perf_counter() - t0
        runs[name] = {"side": side, "rule": "top-k" if rule == fi.DENSIFY_TOPK else "per-triangle",
                      "mesh": "quadtree" if unknowns is None else
                              f"Delaunay, {len(unknowns)} unknown vertices",
                      "inpaintings": rounds + 1, "final_mask": int(order.size),
                      "wall_s": wall, "gpu_ms_total": float(np.sum(ms)),
                      "mse_first": float(mse[0]), "mse_last": float(mse[-1]),
                      "mpixel_per_s": (rounds + 1) * side * side / (float(np.sum(ms)) * 1e3),
                      "mpixel_per_s_wall": (rounds + 1) * side * side / wall / 1e6}
        print(f"{name}: {wall:.2f} s, device {np.sum(ms):.1f} ms", file=sys.stderr, flush=True)
        return order

    w = synth.WORKLOADS["densify1024"]
    f1024 = w.image()
    P = w.side * w.side
    run("densify1024_topk", w.side, f1024, w.mask(), synth.count_from_density(0.001, P), 20,
        fi.DENSIFY_TOPK)
    f512 = synth.WORKLOADS["tonal512"].image()
    for side, f_np, seed in ((512, f512, 2), (1024, f1024, 3)):
        Pn = side * side
        m = synth.count_from_density(0.04, Pn)
        k = m // 10
        order = run(f"paper_{side}", side, f_np, synth.make_mask(seed, Pn, k=k), k, 9,
                    fi.DENSIFY_TRIANGLES)
        if side == 1024:
            last_mask = np.sort(order)
    # the paper's whole method: its own Delaunay mesh, unknown vertices drawn
    # once (as many as the final mask), the per-triangle rule, 4% in n = 10
    Pn = 512 * 512
    m = synth.count_from_density(0.04, Pn)
    mask0 = synth.make_mask(2, Pn, k=m // 10)
    run("paper_delaunay_512", 512, f512, mask0, m // 10, 9, fi.DENSIFY_TRIANGLES,
        unknowns=synth.make_unknowns(2, Pn, mask0, m))
    total_pix = sum(r["inpaintings"] * r["side"] ** 2 for r in runs.values())
    total_wall = sum(r["wall_s"] for r in runs.values())
    total_dev_ms = sum(r["gpu_ms_total"] for r in runs.values())
    # dominant kernel on the final 1024^2 mesh of the per-triangle run
    M = fi.Mesh(ctx, 1024, last_mask)
    fd = torch.from_numpy(f1024.ravel().copy()).cuda()
    M.inpaint(f=fd)
    kms = M.time_cg_kernel(fi.PREC_FP32_IR, args.kernel_reps)
    kbytes = M.cg_kernel_bytes(fi.PREC_FP32_IR)
    achieved = kbytes / (kms * 1e-3) / 1e9
    M.close()
    out = {
        "metric": "inpainted Mpixel/s + tonal-opt solves/s at <=1e-6 err vs FP64; p50/p99 latency",
        "value": total_pix / (total_dev_ms * 1e3),
        "unit": "Mpixel/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": total_dev_ms,
        "mpixel_per_s_wall": total_pix / total_wall / 1e6,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (CG) + f64 (residual, refinement, error)", "data": "synthetic",
        "config": {"workload": "densify: 1024^2 top-k 1%->3% x20 rounds; paper per-triangle "
                               "rule at 512^2 and 1024^2, 4% in n=10 inpaintings; the same "
                               "at 512^2 on the Delaunay mesh"},
        "runs": runs,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic("densify"),
                     "kernel": f"{cg_kernel_name(M.info)} on the final 1024^2 mesh",
                     "iterations_per_launch": M.info["cg_iters_per_launch"],
                     "bytes_per_launch": kbytes, "us_per_launch": kms * 1e3,
                     **launch_rates(M.info, 1, kms)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = densify_cpu_baseline(f512)
    print(json.dumps(out))
    ctx.close()


def densify_cpu_baseline(f512):
    """The oracle running the paper's per-triangle loop at 512^2 (4%, n = 10),
    started over until about 10 s have passed: mesh, Cholesky, inpainting,
    error, selection."""
    from oracle import densify, tonal
    import synth
    side = 512
    P = side * side
    k = synth.count_from_density(0.04, P) // 10
    mask0 = synth.make_mask(2, P, k=k)
    f = f512.ravel()
    t0, c0 = time.perf_counter(), time.process_time()
    n = 0
    while time.perf_counter() - t0 <= 10.0 and n < 100:
        mask = mask0
        for r in range(10):
            pr = tonal.Problem(side, mask)
            u = pr.inpaint(f)
            e = (u - f.astype(np.float64)) ** 2
            n += 1
            if r == 9 or time.perf_counter() - t0 > 10.0:
                break
            add = densify.paper_densify_step(e, pr.rast.owner, pr.mesh.T, mask, k)
            mask = np.sort(np.concatenate([mask, add]))
    el = time.perf_counter() - t0
    return {"value": n * P / el / 1e6, "unit": "Mpixel/s", "cores": cpu_cores_used(t0, c0),
            "host_cores": len(os.sched_getaffinity(0)), "kind": "oracle",
            "sample": f"{n} rounds of the per-triangle loop at 512^2 (mesh, direct Cholesky, "
                      f"inpainting, error, selection), {el:.1f} s"}


def colour_main(args):
    """Colour (Section 5: the method per channel on one shared mesh): the
    512^2 image of the tonal512 recipe in three correlated channels
    (synth.make_image_rgb), 4% mask. One step = assembly, inpainting of all
    three channels (one multi-right-hand-side solve), colour MSE, then tonal
    optimisation of every channel to relative normal residual 1e-8.

    ``value`` is inpainted colour Mpixel/s (P / inpainting-phase time, three
    channels per pixel). The same work done channel after channel with the
    grey calls is timed beside it (``grey_by_channel``)."""
    import torch
    import paper_2105_01586_amd as fi
    import synth

    w = synth.WORKLOADS["tonal512"]
    side = w.side
    P = side * side
    f_np = synth.make_image_rgb(w.seed, side, side, w.bumps, w.edges, w.sigma_lo,
                                w.sigma_hi).reshape(3, -1)
    mask = w.mask()
    steps = args.steps or 5
    warmup = 2 if args.warmup is None else args.warmup
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(0)
    ctx = fi.Context(0, stream)
    mesh = fi.Mesh(ctx, side, mask)
    f = torch.from_numpy(f_np.ravel().copy()).to(dev)
    fch = [torch.from_numpy(f_np[c].copy()).to(dev) for c in range(3)]
    u = torch.empty(3 * P, dtype=torch.float64, device=dev)
    g = torch.empty(3 * mesh.m, dtype=torch.float64, device=dev)
    inner = fi.SolveOpts(precision=fi.PREC_FP32_IR)
    topts = fi.TonalOpts(inner=inner, rtol=1e-8)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def step_rgb(rec):
        e0, e1, e2 = ev(), ev(), ev()
        e0.record(stream)
        mesh.assemble()
        _, st = mesh.inpaint_rgb(f=f, u=u, opts=inner)
        mse, _ = mesh.error_rgb(u, f)
        e1.record(stream)
        _, ts = mesh.tonal_opt_rgb(f, g=g, opts=topts)
        e2.record(stream)
        rec.append((e0, e1, e2, st, ts, mse))

    def step_grey(rec):
        e0, e1, e2 = ev(), ev(), ev()
        e0.record(stream)
        mesh.assemble()
        for c in range(3):
            mesh.inpaint(f=fch[c], u=u[c * P:(c + 1) * P], opts=inner)
            mesh.error(u[c * P:(c + 1) * P], fch[c])
        e1.record(stream)
        for c in range(3):
            mesh.tonal_opt(fch[c], g=g[c * mesh.m:(c + 1) * mesh.m], opts=topts)
        e2.record(stream)
        rec.append((e0, e1, e2))

    def timed(fn):
        for _ in range(warmup):
            fn([])
        torch.cuda.synchronize()
        rec = []
        t0 = time.perf_counter()
        for _ in range(steps):
            fn(rec)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        inp = float(np.mean([r[0].elapsed_time(r[1]) for r in rec]))
        ton = float(np.mean([r[1].elapsed_time(r[2]) for r in rec]))
        return rec, wall, inp, ton

    rec, wall, inp, ton = timed(step_rgb)
    st, ts, mse = rec[-1][3], rec[-1][4], rec[-1][5]
    _, wall_g, inp_g, ton_g = timed(step_grey)
    _, st = mesh.inpaint_rgb(f=f, u=u, opts=inner)  # leave the colour result in u
    kms = mesh.time_cg_multi_kernel(3, fi.PREC_FP32_IR, args.kernel_reps)
    kbytes = mesh.cg_multi_kernel_bytes(3, fi.PREC_FP32_IR)
    k1 = mesh.time_cg_kernel(fi.PREC_FP32_IR, args.kernel_reps)
    achieved = kbytes / (kms * 1e-3) / 1e9
    torch.cuda.synchronize()
    out = {
        "metric": "inpainted Mpixel/s + tonal-opt solves/s at <=1e-6 err vs FP64; p50/p99 latency",
        "value": P / (inp * 1e3),
        "unit": "Mpixel/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (CG) + f64 (residual, refinement, tonal)", "data": "synthetic",
        "config": {"workload": f"rgb512: 512x512 colour (3 channels), {w.bumps} bumps, "
                               f"{w.edges} edges, 4% random mask (m={mesh.m})",
                   "side": side, "channels": 3, "mask_pixels": mesh.m, "unknowns": mesh.n},
        "inpaint_ms": inp, "tonal_ms": ton, "tonal_solves_per_s": 1000.0 / ton,
        "cg_iterations_inpaint": [x["iterations"] for x in st],
        "tonal_outer_iterations": [x["outer_iterations"] for x in ts],
        "tonal_inner_iterations": [x["inner_iterations"] for x in ts],
        "mse_inpaint": mse, "mse_tonal": float(np.mean([x["mse_final"] for x in ts])),
        "grey_by_channel": {"inpaint_ms": inp_g, "tonal_ms": ton_g,
                            "ms_per_step": wall_g * 1e3 / steps,
                            "inpaint_speedup": inp_g / inp, "tonal_speedup": ton_g / ton},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic("rgb512"),
                     "kernel": cg_kernel_name(mesh.info, 3),
                     "iterations_per_launch": mesh.info["cg_iters_per_launch"],
                     "bytes_per_launch": kbytes, "us_per_launch": kms * 1e3,
                     "one_rhs_step_us": k1 * 1e3, **launch_rates(mesh.info, 3, kms)},
    }
    if not args.no_cpu_baseline:
        from oracle import colour, tonal
        t0, c0 = time.perf_counter(), time.process_time()
        reps = 0
        while True:
            pr = tonal.Problem(side, mask)
            u_ref = colour.inpaint(pr, f_np)
            colour.mse(u_ref, f_np)
            reps += 1
            el = time.perf_counter() - t0
            if el > 10.0 or reps >= 100:
                break
        cores = cpu_cores_used(t0, c0)
        out["max_abs_err_vs_fp64_oracle"] = float(np.max(np.abs(u.cpu().numpy().reshape(3, -1)
                                                                - u_ref)))
        out["cpu_baseline"] = {"value": reps * P / el / 1e6, "unit": "Mpixel/s", "cores": cores,
                               "host_cores": len(os.sched_getaffinity(0)), "kind": "oracle",
                               "sample": f"{reps} colour inpainting(s) of the 512^2 image (mesh, "
                                         f"assembly, one direct Cholesky, three solves, "
                                         f"interpolation, MSE), {el:.1f} s"}
    print(json.dumps(out))
    mesh.close()
    ctx.close()


def l1_main(args):
    """L1 tonal optimisation (IRLS: eps 0.5, K = 8 reweighting steps of
    J = 20 CGLS iterations) on the tonal512 image, quadtree and Delaunay
    meshes. ``value``: inpainted Mpixel/s of the inpainting phase as in the
    default workload; the L1 phase's time, MAE before and after, beside it."""
    import torch
    import paper_2105_01586_amd as fi
    import synth

    w = synth.WORKLOADS["tonal512"]
    f_np = w.image().ravel()
    mask = w.mask()
    P = w.side * w.side
    ctx = fi.Context(0, torch.cuda.current_stream(0))
    f = torch.from_numpy(f_np.copy()).cuda()
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    runs = {}
    for name, unk in (("quadtree", None),
                      ("delaunay", synth.make_unknowns(w.seed, P, mask, mask.size))):
        M = fi.Mesh(ctx, w.side, mask, unknowns=unk)
        u = torch.empty(P, dtype=torch.float64, device="cuda")
        M.inpaint(f=f, u=u)
        a, b, c = ev(), ev(), ev()
        a.record()
        M.inpaint(f=f, u=u)
        b.record()
        g, st, hist = M.tonal_opt_l1(f)
        c.record()
        torch.cuda.synchronize()
        runs[name] = {"vertices": M.V, "unknowns": M.n, "inpaint_ms": a.elapsed_time(b),
                      "l1_ms": b.elapsed_time(c), "mae_initial": st["mae_initial"],
                      "mae_final": st["mae_final"], "mse_final": st["mse_final"],
                      "irls_steps": st["irls_iters"], "inner_iterations": st["inner_iterations"],
                      "mae_per_step": [float(x) for x in hist]}
        if name == "quadtree":
            kms = M.time_cg_kernel(fi.PREC_FP32_IR, args.kernel_reps)
            kbytes = M.cg_kernel_bytes(fi.PREC_FP32_IR)
            qinfo = M.info
        M.close()
    q = runs["quadtree"]
    achieved = kbytes / (kms * 1e-3) / 1e9
    out = {
        "metric": "inpainted Mpixel/s + tonal-opt solves/s at <=1e-6 err vs FP64; p50/p99 latency",
        "value": P / (q["inpaint_ms"] * 1e3), "unit": "Mpixel/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": q["inpaint_ms"] + q["l1_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (CG) + f64 (residual, refinement, IRLS)", "data": "synthetic",
        "config": {"workload": "l1512: tonal512 image and mask, L1 tonal optimisation by IRLS "
                               "(eps 0.5, 8 steps x 20 CGLS iterations), quadtree and Delaunay"},
        "runs": runs,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic("tonal512"),
                     "kernel": f"{cg_kernel_name(qinfo)} on the quadtree mesh",
                     "iterations_per_launch": qinfo["cg_iters_per_launch"],
                     "bytes_per_launch": kbytes, "us_per_launch": kms * 1e3,
                     **launch_rates(qinfo, 1, kms)},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"], _ = cpu_baseline(w.side, f_np, mask, None, "the 512^2 image")
    print(json.dumps(out))
    ctx.close()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus above 1 is not "
                                   "supported (the path has no multi-GPU sharding)"}))
        sys.exit(2)
    import torch
    if args.copy_calibration:
        # a 256 MiB device copy whose counter readings scale FETCH_SIZE and
        # WRITE_SIZE in profiles
        a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.workload == "serving":
        serving_main(args)
        return
    if args.workload == "densify":
        densify_main(args)
        return
    if args.workload == "rgb512":
        colour_main(args)
        return
    if args.workload == "l1512":
        l1_main(args)
        return
    import paper_2105_01586_amd as fi
    import synth

    t_start = time.perf_counter()

    def progress(what):
        print(f"[{time.perf_counter() - t_start:7.1f} s] {what}", file=sys.stderr, flush=True)

    w = synth.WORKLOADS[args.workload]
    big = w.side > 2048
    if args.steps is None:
        args.steps = 1 if big else 5
    if args.warmup is None:
        args.warmup = 0 if big else 2
    f_np = w.image()
    mask = w.mask()
    P = w.side * w.side
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(0)
    ctx = fi.Context(0, stream)
    mesh = fi.Mesh(ctx, w.side, mask)
    progress(f"mesh built: {mesh.n} unknowns")
    f = torch.from_numpy(f_np.ravel().copy()).to(dev)
    u = torch.empty(P, dtype=torch.float64, device=dev)
    g = torch.empty(mesh.m, dtype=torch.float64, device=dev)
    inner = fi.SolveOpts(precision=fi.PREC_FP32_IR)
    topts = fi.TonalOpts(inner=inner, rtol=1e-8)
    # The default stop (relative 1e-10 and absolute 3e-6) keeps every pixel
    # within 1e-6 of the exact solution at every size; the error is measured
    # below against a 1e-13 FP64 solve.
    inner_inp = fi.SolveOpts(precision=fi.PREC_FP32_IR)

    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    peak_used = [0]

    def note_memory():
        free, total = torch.cuda.mem_get_info(0)
        peak_used[0] = max(peak_used[0], total - free)

    # the error sum stays on the device inside the timed step (no host wait);
    # the MSE is read after the timing
    sse = torch.empty(1, dtype=torch.float64, device=dev)

    def step(record):
        e0, e1, e2 = ev(), ev(), ev()
        e0.record(stream)
        mesh.assemble()
        _, st = mesh.inpaint(f=f, u=u, opts=inner_inp)
        mesh.error_dev(u, f, sse=sse)
        e1.record(stream)
        _, ts = mesh.tonal_opt(f, g=g, opts=topts)
        e2.record(stream)
        note_memory()
        record.append((e0, e1, e2, st, ts, None))

    warm = []
    for _ in range(args.warmup):
        step(warm)
    torch.cuda.synchronize()
    progress(f"{args.warmup} warm-up steps done")
    recs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(recs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    progress(f"{args.steps} timed steps done")
    inp_ms = [a.elapsed_time(b) for a, b, *_ in recs]
    ton_ms = [b.elapsed_time(c) for _, b, c, *_ in recs]
    st, ts = recs[-1][3], recs[-1][4]
    mse = float(sse.item()) / P
    ms_step = wall * 1000.0 / args.steps
    inp_mean = float(np.mean(inp_ms))
    ton_mean = float(np.mean(ton_ms))

    # plain FP64 GPU comparator on the same inpainting
    fp64 = None
    if not args.skip_fp64:
        o64 = fi.SolveOpts(precision=fi.PREC_FP64)
        t64 = []
        for k in range(args.steps + 1):
            a, b = ev(), ev()
            a.record(stream)
            mesh.assemble()
            _, st64 = mesh.inpaint(f=f, u=u, opts=o64)
            mesh.error_dev(u, f, sse=sse)
            b.record(stream)
            torch.cuda.synchronize()
            if k:
                t64.append(a.elapsed_time(b))
        fp64 = {"inpaint_mpix_s": P / (np.mean(t64) * 1e3), "iterations": st64["iterations"]}
        _, st = mesh.inpaint(f=f, u=u, opts=inner_inp)   # leave the FP32 result in u
        progress("plain FP64 comparator done")

    # every pixel against a tight FP64 solve on the GPU
    u_tight, st_t = mesh.inpaint(f=f, opts=fi.SolveOpts(precision=fi.PREC_FP64, rtol=1e-13))
    err_tight = float((u - u_tight).abs().max())
    del u_tight
    progress("tight FP64 check done")

    # checks that launch solves of their own run before the kernel timing,
    # so that the timed launches are the last of the run (profiles pick them
    # from the trace's end)
    g_fd = fd_res = crop_res = None
    if w.side <= 1024:
        g_fd, fd_res = fd_check(fi, mesh, f, f_np, mask)
        progress("finite-difference check done")
    if big:
        crop_res = crop_check(fi, ctx, f_np, mask)
        progress("crop check done")

    # dominant kernel: the FP32 CG launch, timed on the library's stream
    kms = mesh.time_cg_kernel(fi.PREC_FP32_IR, args.kernel_reps)
    kbytes = mesh.cg_kernel_bytes(fi.PREC_FP32_IR)
    achieved = kbytes / (kms * 1e-3) / 1e9
    torch.cuda.synchronize()
    progress("kernel timing done")

    out = {
        "metric": "inpainted Mpixel/s + tonal-opt solves/s at <=1e-6 err vs FP64; p50/p99 latency",
        "value": P / (inp_mean * 1e3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (CG) + f64 (residual, refinement, tonal)",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {w.side}x{w.side}, {w.bumps} bumps, {w.edges} edges, "
                               f"{w.density:.0%} random mask (m={mesh.m})",
                   "side": w.side, "mask_pixels": mesh.m, "vertices": mesh.V,
                   "unknowns": mesh.n, "triangles": mesh.T, "nnz_ff": int(mesh.info["nnz_ff"])},
        "inpaint_ms": inp_mean,
        "tonal_ms": ton_mean,
        "tonal_solves_per_s": 1000.0 / ton_mean,
        "cg_iterations_inpaint": st["iterations"],
        "launches_inpaint": st["launches"],
        "refinements_inpaint": st["refinements"],
        "rel_residual_inpaint": st["rel_residual"],
        "rtol_inpaint": inner_inp.rtol, "residual_inpaint": st["residual"],
        "max_abs_err_vs_tight_fp64_gpu": err_tight,
        "tight_fp64_rel_residual": st_t["rel_residual"],
        "tonal_outer_iterations": ts["outer_iterations"],
        "tonal_inner_iterations": ts["inner_iterations"],
        "mse_inpaint": mse,
        "mse_tonal": ts["mse_final"],
        "fp64_gpu": fp64,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(args.workload),
                     "kernel": cg_kernel_name(mesh.info),
                     "iterations_per_launch": mesh.info["cg_iters_per_launch"],
                     "bytes_per_launch": kbytes, "us_per_launch": kms * 1e3,
                     **launch_rates(mesh.info, 1, kms)},
    }
    # the mesh's memory after assembly, and after the run (state the first
    # FP64 solve and the first tonal optimisation allocate included)
    out["device_memory_gb"] = {"mesh_and_solver": mesh.info["device_bytes"] / 1e9,
                               "mesh_and_solver_after_run": mesh.device_bytes() / 1e9,
                               "torch_peak": torch.cuda.max_memory_allocated() / 1e9,
                               "device_used_peak": peak_used[0] / 1e9}
    if fd_res is not None:
        out["gradient_fd_check"] = fd_res
    if not args.no_cpu_baseline:
        if w.side <= 1024:
            cb, acc = cpu_baseline(w.side, f_np, mask, u.cpu().numpy(), f"the {w.side}^2 image",
                                   grad_at=g_fd, tonal_rtol=1e-8)
            out["max_abs_err_vs_fp64_oracle"] = acc["max_abs_pixel_err"]
            out["mse_inpaint_oracle"] = acc["mse_oracle"]
            out["mse_tonal_oracle"] = acc["mse_tonal_oracle"]
            out["tonal_outer_iterations_oracle"] = acc["tonal_iterations_oracle"]
            out["gradient_fd_check"]["rel_err_vs_oracle_gradient"] = acc["grad_rel_err_vs_oracle"]
        else:
            # the oracle on the whole image is out of reach; it runs on the
            # 2048^2 crop that the parity tests use
            r0, c0 = synth.busiest_block(f_np, 2048)
            cf, cm = synth.crop(f_np, mask, r0, c0, 2048)
            cb, _ = cpu_baseline(2048, cf, cm, None, f"the 2048^2 crop at ({r0}, {c0})")
        out["cpu_baseline"] = cb
    if big:
        out["crop_vs_oracle"] = crop_res
    print(json.dumps(out))
    mesh.close()
    ctx.close()


if __name__ == "__main__":
    main()
