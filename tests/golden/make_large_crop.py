"""Writes tests/golden/large8192_crop.json: oracle results on a 2048^2 crop
of the 8192^2 / 2% workload (test infrastructure: calls the oracle only).

The crop is the 2048-aligned block with the most unclipped pixels
(synth.busiest_block); its mask is the workload mask restricted to the
crop. Stored: the inpainting MSE, u at 4096 seeded sample pixels, and the
tonal optimum's MSE (CGLS to relative normal residual 1e-10) with g at 1024
seeded sample mask slots.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import tonal  # noqa: E402


def main():
    t0 = time.time()
    w = synth.WORKLOADS["large8192"]
    img = w.image()
    mask = w.mask()
    r0, c0 = synth.busiest_block(img, 2048)
    f, m = synth.crop(img, mask, r0, c0, 2048)
    f = f.ravel()
    pr = tonal.Problem(2048, m)
    u = pr.inpaint(f)
    rng = np.random.default_rng(2048)
    pix = np.sort(rng.choice(f.size, 4096, replace=False))
    out = {"crop_origin": [int(r0), int(c0)], "side": 2048, "mask_pixels": int(m.size),
           "mse_inpaint": pr.mse(u, f), "sample_pixels": pix.tolist(),
           "sample_u": u[pix].tolist()}
    print("inpainting done", time.time() - t0, flush=True)
    g, it, rel = pr.tonal_cgls(f.astype(np.float64), rtol=1e-10)
    slots = np.sort(rng.choice(m.size, 1024, replace=False))
    out.update({"mse_tonal": pr.mse_of_g(g, f), "tonal_iterations": int(it),
                "tonal_rel_normal_residual": float(rel), "sample_slots": slots.tolist(),
                "sample_g": g[slots].tolist(),
                "mse_untuned": out["mse_inpaint"]})
    with open(os.path.join(HERE, "large8192_crop.json"), "w") as fh:
        json.dump(out, fh)
    print("done", time.time() - t0, it, rel, out["mse_inpaint"], out["mse_tonal"])


if __name__ == "__main__":
    main()
