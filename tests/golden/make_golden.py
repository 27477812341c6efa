"""Writes the stored oracle results used by the full-size GPU parity tests.

Runs only the FP64 oracle (oracle/bilateral.py) on the seeded workloads of
workloads.py and stores small samples of its outputs as JSON:

    python tests/golden/make_golden.py

depthsr2048x1536.json: the depth super-resolution workload (2048x1536,
sigma (8,4,4), lambda 64, hierarchical init, Jacobi PCG to relative residual
1e-5): vertex count, pyramid sizes, bistochastization and PCG iteration counts,
and the solution x at 1024 pixels drawn with numpy.random.default_rng(2024).

mixed64_image{4,7,10}.json: images 4 (1920x419, one channel, sigma_xy 16: the
widest image, next to the packed neighbour table's 16-bit bound), 7 (1871x645,
21 channels, sigma_xy 16) and 10 (1731x997, one channel, sigma_xy 8: the most
pixels) of the 64-image mixed batch (workloads.mixed_batch(seed=0)), solved
forward and backward as bench.py runs them (lambda 128, hierarchical init,
Jacobi PCG to 1e-5 both ways, upstream gradient workloads.random_grad(i, ...)):
x and dL/dt at 1024 (channel, pixel) pairs and dL/dc at 1024 pixels, drawn
with numpy.random.default_rng(2025 + i).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as WL  # noqa: E402
from oracle import bilateral as O  # noqa: E402


def depth_golden(path):
    p = WL.depth_superres()
    prm = O.Params(p.sigma_xy, p.sigma_l, p.sigma_uv, p.lam, max_iters=p.max_iters,
                   rel_tol=p.rel_tol)
    t0 = time.time()
    sol = O.solve(p.ref, p.target, p.conf, prm)
    rng = np.random.default_rng(2024)
    pix = np.sort(rng.choice(p.pixels, size=1024, replace=False))
    x = sol.x[0].reshape(-1)
    out = {
        "workload": "depthsr2048x1536", "seed": 0, "sigma": [p.sigma_xy, p.sigma_l, p.sigma_uv],
        "lambda": p.lam, "rel_tol": p.rel_tol, "init": "hier",
        "V": int(sol.grid.V), "pyramid_sizes": [int(s) for s in sol.pyr.sizes],
        "bist_iters": int(sol.bist.iters), "pcg_iters": int(sol.runs[0].iters),
        "true_rel_residual": sol.runs[0].true_rel_residual,
        "pixels": [int(i) for i in pix], "x": [float(v) for v in x[pix]],
        "oracle_seconds": round(time.time() - t0, 1),
    }
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, "V", out["V"], "pcg iters", out["pcg_iters"])


def mixed64_golden(i, path):
    p = WL.mixed_batch(seed=0, count=64)[i]
    prm = O.Params(p.sigma_xy, p.sigma_l, p.sigma_uv, p.lam, max_iters=20000, rel_tol=1e-5)
    t0 = time.time()
    sol = O.solve(p.ref, p.target, p.conf, prm)
    gx = WL.random_grad(i, p.C, p.H, p.W)
    og = O.solve_backward(sol, p.target, p.conf, gx, prm)
    rng = np.random.default_rng(2025 + i)
    ch = rng.integers(0, p.C, size=1024)
    pix = rng.choice(p.pixels, size=1024, replace=False)
    pc = rng.choice(p.pixels, size=1024, replace=False)
    x = sol.x.reshape(p.C, -1)
    gt = og.grad_t.reshape(p.C, -1)
    out = {
        "workload": "mixed64", "image": i, "W": p.W, "H": p.H, "C": p.C,
        "sigma": [p.sigma_xy, p.sigma_l, p.sigma_uv], "lambda": p.lam, "rel_tol": 1e-5,
        "init": "hier", "V": int(sol.grid.V),
        "pcg_iters": [int(r.iters) for r in sol.runs],
        "adjoint_iters": [int(r.iters) for r in og.runs],
        "channels": [int(c) for c in ch], "pixels": [int(v) for v in pix],
        "x": [float(x[c, q]) for c, q in zip(ch, pix)],
        "grad_t": [float(gt[c, q]) for c, q in zip(ch, pix)],
        "grad_c_pixels": [int(v) for v in pc],
        "grad_c": [float(og.grad_c.reshape(-1)[q]) for q in pc],
        "conf_at_grad_c_pixels": [float(p.conf.reshape(-1)[q]) for q in pc],
        "oracle_seconds": round(time.time() - t0, 1),
    }
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, "V", out["V"], "pcg iters", max(out["pcg_iters"]),
          "adjoint", max(out["adjoint_iters"]), "seconds", out["oracle_seconds"])


if __name__ == "__main__":
    which = sys.argv[1:] or ["depth", "mixed64"]
    if "depth" in which:
        depth_golden(os.path.join(HERE, "depthsr2048x1536.json"))
    if "mixed64" in which:
        for i in (4, 7, 10):
            mixed64_golden(i, os.path.join(HERE, f"mixed64_image{i}.json"))
