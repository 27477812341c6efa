"""Graph capture of the single-image solve: with check_every = 0, bs_solve
and bs_slice only enqueue kernels on the caller's stream (no host wait, no
memset), so they can be recorded into a HIP graph.  Every replay must equal
the eager result bit for bit (the reductions run in a fixed order), with the
program's own eager work and synchronisations between the replays."""
import numpy as np
import pytest
import torch

import workloads as WL
from oracle import bilateral as O
from tests.gpu_helpers import gpu_grid, params, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu


def test_solve_and_slice_replay_from_a_graph():
    p = WL.tiny_ramp(seed=33, H=48, W=64, regions=8, channels=2)
    say("graph: capture solve + slice (64x48, two channels), replay 3 times")
    G = gpu_grid(p)                       # grid and bistochastization run eagerly
    t, c = to_dev(p.target), to_dev(p.conf)
    kw = dict(max_iters=200, rel_tol=1e-6, check_every=0)
    ws = G.solve_workspace(2)
    y0, _ = G.solve(t, c, p.lam, ws=ws, **kw)
    x0 = G.slice(y0, 2).clone()
    torch.cuda.synchronize()
    exact = O.solve(p.ref, p.target, p.conf, params(p, rel_tol=1e-12, max_iters=20000))
    assert rel_l2(x0.cpu().numpy(), exact.x) <= 1e-4

    y = torch.empty_like(y0)
    x = torch.empty_like(x0)
    stats = torch.empty(2 * 24, dtype=torch.uint8, device="cuda")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        G.solve(t, c, p.lam, ws=ws, y=y, stats=stats, **kw)
        G.slice(y, 2, out=x)
    ws2 = G.solve_workspace(2)
    for r in range(3):
        x.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, x0), r
        # eager work between replays, on its own workspace
        ye, _ = G.solve(t * 0.5, c, p.lam, ws=ws2, **kw)
        xe = G.slice(ye, 2)
        torch.cuda.synchronize()
        assert rel_l2(xe.cpu().numpy(), 0.5 * x0.cpu().numpy()) <= 1e-5, r
