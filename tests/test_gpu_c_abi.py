"""The C ABI used directly from a host program (paper_1511_03296_amd/
examples/solve_c.cpp, built by build()): grid, bistochastization, solve,
slice and the domain-transform post-process through include/bsolve.h alone.
Its output must match the FP64 oracle and, bit for bit, the Python binding,
which makes the same calls."""
import os
import subprocess

import numpy as np
import pytest
import torch

import workloads as WL
from oracle import bilateral as O
from oracle import domain_transform as DT
from tests.gpu_helpers import gpu_grid, params, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXAMPLE = os.path.join(ROOT, "paper_1511_03296_amd", "examples", "solve_c")


def test_c_program_matches_oracle_and_binding(tmp_path):
    if not os.path.exists(EXAMPLE):
        pytest.skip("C example not built (run __graft_entry__.build())")
    p = WL.tiny_ramp(seed=31, channels=2)
    prm = params(p)
    inp = tmp_path / "in.bin"
    out = tmp_path / "out.bin"
    np.concatenate([p.ref.reshape(-1), p.target.reshape(-1), p.conf.reshape(-1)]).astype(
        np.float32).tofile(inp)
    say("C-ABI example program: ramp64x48 C=2")
    args = [EXAMPLE, str(p.H), str(p.W), str(p.C), str(p.sigma_xy), str(p.sigma_l),
            str(p.sigma_uv), repr(float(p.lam)), str(prm.max_iters), repr(prm.rel_tol),
            str(inp), str(out)]
    res = subprocess.run(args, capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    raw = np.fromfile(out, dtype=np.uint8)
    n = p.C * p.H * p.W
    x = raw[: 4 * n].view(np.float32).reshape(p.C, p.H, p.W)
    iters = raw[4 * n: 4 * n + 4 * p.C].view(np.int32)
    xd = raw[4 * n + 4 * p.C:].view(np.float32).reshape(p.C, p.H, p.W)
    sol = O.solve(p.ref, p.target, p.conf, prm)
    assert rel_l2(x, sol.x) <= 1e-4
    assert all(abs(int(i) - r.iters) <= 3 for i, r in zip(iters, sol.runs))
    G = gpu_grid(p)
    y, _ = G.solve(to_dev(p.target), to_dev(p.conf), p.lam, max_iters=prm.max_iters,
                   rel_tol=prm.rel_tol)
    xb = G.slice(y, p.C)
    torch.cuda.synchronize()
    assert np.array_equal(xb.cpu().numpy(), x)
    # the post-process of the program's own x: the float64 filter, and the
    # binding's call bit for bit
    want = DT.domain_transform(p.ref, x, 4.0, 8.0, 3)
    assert rel_l2(xd, want) <= 1e-5
    from paper_1511_03296_amd import domain_transform
    xdb = domain_transform(to_dev(p.ref), xb, 4.0, 8.0, 3)
    torch.cuda.synchronize()
    assert np.array_equal(xdb.cpu().numpy(), xd)
