"""Writes the stored oracle results used by the full-size GPU parity tests.

Runs only the FP64 oracle (oracle/bilateral.py) on the seeded workloads of
workloads.py and stores small samples of its outputs as JSON:

    python tests/golden/make_golden.py

depthsr2048x1536.json: the depth super-resolution workload (2048x1536,
sigma (8,4,4), lambda 64, hierarchical init, Jacobi PCG to relative residual
1e-5): vertex count, pyramid sizes, bistochastization and PCG iteration counts,
and the solution x at 1024 pixels drawn with numpy.random.default_rng(2024).
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


if __name__ == "__main__":
    depth_golden(os.path.join(HERE, "depthsr2048x1536.json"))
