"""The solve without a workspace argument (bs_solve_noalloc), called through
the C ABI: its result must equal bs_solve's, bit for bit (same kernels, same
launch shapes), on two calls in a row, the second on a smaller image, since
the library's one scratch array per GPU keeps the previous call's contents.
Also: the size limit and the no-polling rule are enforced before any launch,
and the call can be recorded into a HIP graph."""
import ctypes as ct

import numpy as np
import pytest
import torch

import workloads as WL
from oracle import bilateral as O
from tests.gpu_helpers import gpu_grid, params, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(G, t, c, C, opts, y, stats):
    from paper_1511_03296_amd import _lib as L
    p = opts.struct()
    return L.lib.bs_solve_noalloc(ct.byref(G.handle), t.data_ptr(), c.data_ptr(), C,
                                  ct.byref(p), y.data_ptr(),
                                  stats.data_ptr() if stats is not None else None,
                                  torch.cuda.current_stream().cuda_stream)


def _case(seed, H, W, C, regions):
    from paper_1511_03296_amd import SolveOptions, _lib as L, read_stats
    p = WL.tiny_ramp(seed=seed, H=H, W=W, regions=regions, channels=C)
    say(f"noalloc: {W}x{H} C={C} seed={seed}")
    G = gpu_grid(p)
    t, c = to_dev(p.target), to_dev(p.conf)
    opts = SolveOptions(p.lam, max_iters=400, rel_tol=1e-6, check_every=0)
    y_ref, st_ref = G.solve(t, c, p.lam, max_iters=400, rel_tol=1e-6, check_every=0)
    y = torch.full_like(y_ref, float("nan"))
    stats = torch.zeros_like(st_ref)
    L.check(_noalloc(G, t, c, C, opts, y, stats), "bs_solve_noalloc")
    torch.cuda.synchronize()
    V = G.vertex_count()
    assert torch.equal(y[:V], y_ref[:V])
    assert np.array_equal(read_stats(stats), read_stats(st_ref))
    exact = O.solve(p.ref, p.target, p.conf, params(p, rel_tol=1e-12, max_iters=20000))
    x = G.slice(y, C)
    assert rel_l2(x.cpu().numpy(), exact.x) <= 1e-4
    return G, p


def test_noalloc_equals_solve_on_two_calls_second_smaller():
    _case(seed=71, H=120, W=160, C=2, regions=20)
    _case(seed=72, H=48, W=64, C=1, regions=8)


def test_noalloc_rejects_before_launch():
    from paper_1511_03296_amd import SolveOptions, _lib as L
    p = WL.tiny_ramp(seed=73, H=48, W=64, regions=8, channels=1)
    say("noalloc: argument checks")
    G = gpu_grid(p)
    t, c = to_dev(p.target), to_dev(p.conf)
    y = torch.full((G.vcap, 1), 7.0, device="cuda")
    st = _noalloc(G, t, c, 1, SolveOptions(p.lam, 50, 1e-5, check_every=8), y, None)
    assert st == L.BS_EINVAL and "check_every" in L.lib.bs_last_error().decode()
    # a 512 x 512 image with 21 channels needs more than the scratch array
    big = WL.tiny_ramp(seed=74, H=512, W=512, regions=30, channels=1)
    Gb = gpu_grid(big)
    need = L.lib.bs_solve_workspace_bytes(ct.byref(Gb.handle), 21)
    assert need > L.BS_NOALLOC_SCRATCH_BYTES
    tb = torch.zeros((21, 512, 512), device="cuda")
    cb = to_dev(big.conf)
    yb = torch.full((Gb.vcap, 21), 7.0, device="cuda")
    st = _noalloc(Gb, tb, cb, 21, SolveOptions(big.lam, 50, 1e-5, check_every=0), yb, None)
    assert st == L.BS_EUNSUPPORTED
    torch.cuda.synchronize()
    assert bool((y == 7.0).all()) and bool((yb == 7.0).all())


def test_noalloc_replays_from_a_graph():
    from paper_1511_03296_amd import SolveOptions, _lib as L
    G, p = _case(seed=75, H=96, W=128, C=2, regions=12)
    say("noalloc: capture solve + slice, replay 3 times")
    t, c = to_dev(p.target), to_dev(p.conf)
    opts = SolveOptions(p.lam, max_iters=400, rel_tol=1e-6, check_every=0)
    y0, _ = G.solve(t, c, p.lam, max_iters=400, rel_tol=1e-6, check_every=0)
    x0 = G.slice(y0, 2).clone()
    y = torch.empty_like(y0)
    x = torch.empty_like(x0)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        L.check(_noalloc(G, t, c, 2, opts, y, None), "bs_solve_noalloc")
        G.slice(y, 2, out=x)
    for r in range(3):
        x.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, x0), r
        # eager use of the same scratch array between replays, on another image
        _case(seed=76 + r, H=48, W=64, C=1, regions=8)
