"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Integer outputs (vertex keys and ids, pixel->vertex index, pixel CSR,
neighbour table, pyramid maps and P(1)) must match bit for bit; the float64
bistochastization vector to 1e-12 relative; the float32 solution to relative
L2 <= 1e-4 (the bound the solver is specified to) against the oracle running
the same algorithm in float64.
"""
import numpy as np
import pytest
import torch

import workloads as WL
from oracle import bilateral as O
from tests.gpu_helpers import (check_grad_c, grid_arrays, gpu_grid, oracle_level_keys, params, rel_l2, say,
                               to_dev)

pytestmark = pytest.mark.gpu

TOL_X = 1e-4


def _grid_cases():
    return [
        ("ramp64x48", lambda: WL.tiny_ramp()),
        ("ramp64x48_s3_5_7", lambda: WL.tiny_ramp(seed=1, sigma=(3, 5, 7))),
        ("stereo256x192", lambda: WL.stereo_refine(H=192, W=256, regions=40)),
        ("depth320x240", lambda: WL.depth_superres(H=240, W=320, regions=60)),
        ("odd61x37_s1", lambda: WL.tiny_ramp(seed=2, H=37, W=61, sigma=(1, 16, 16))),
        ("seg96x80_s9", lambda: WL.tiny_ramp(seed=3, H=80, W=96, sigma=(9, 2, 3))),
        ("row1x50", lambda: WL.tiny_ramp(seed=4, H=1, W=50, regions=3)),
        ("col50x1", lambda: WL.tiny_ramp(seed=5, H=50, W=1, regions=3)),
        ("pixel1x1", lambda: WL.tiny_ramp(seed=6, H=1, W=1, regions=1)),
        ("flat_colour", lambda: _constant_ref(WL.tiny_ramp(seed=7, H=40, W=56))),
        ("s32_bigcells", lambda: WL.tiny_ramp(seed=8, H=100, W=130, regions=30, sigma=(32, 8, 8))),
    ]


def _constant_ref(p):
    p.ref = np.full_like(p.ref, 0.25)
    return p


@pytest.mark.parametrize("name,make", _grid_cases(), ids=[c[0] for c in _grid_cases()])
def test_grid_bit_exact(name, make):
    p = make()
    say(f"grid case {name} {p.W}x{p.H} sigma=({p.sigma_xy},{p.sigma_l},{p.sigma_uv})")
    G = gpu_grid(p)
    torch.cuda.synchronize()
    got = grid_arrays(G)
    g = O.build_grid(p.ref, p.sigma_xy, p.sigma_l, p.sigma_uv)
    pyr = O.build_pyramid(g)
    bs = O.bistochastize(g, 1e-10, 200)
    assert got["V"] == g.V
    assert np.array_equal(got["key"], g.keys)
    assert np.array_equal(got["idx"], g.idx)
    assert np.array_equal(got["m"], g.m)
    assert np.array_equal(got["nbr"], g.nbr)
    assert got["nb_packed"] == 1 and got["nb_wide"] == 0 and np.array_equal(got["nb16"], g.nbr)
    ptr = np.concatenate([[0], np.cumsum(g.m)])
    assert np.array_equal(got["pix_ptr"], ptr)
    assert np.array_equal(got["pix_list"], np.argsort(g.idx, kind="stable"))
    # pyramid
    assert got["K"] == pyr.K
    assert got["sizes"][: pyr.K + 1] == pyr.sizes
    assert all(s == 0 for s in got["sizes"][pyr.K + 1:])
    okeys = oracle_level_keys(g, pyr)
    for k in range(pyr.K):
        assert np.array_equal(got["parents"][k], pyr.parents[k]), f"parents level {k}"
        assert np.array_equal(got["level_keys"][k], okeys[k]), f"keys level {k + 1}"
        assert np.array_equal(got["ones"][k], pyr.ones[k + 1].astype(np.int64)), f"ones {k + 1}"
    # bistochastization: same number of updates, n to 1e-12
    assert got["bist_iters"] == bs.iters
    assert np.max(np.abs(got["n"] - bs.n) / bs.n) <= 1e-12
    nn = bs.n * O.neighbour_sum(g, bs.n)
    assert np.max(np.abs(got["nn"] - nn) / np.maximum(nn, 1e-300)) <= 1e-11
    assert np.array_equal(got["nf"], bs.n.astype(np.float32))


def test_grid_deterministic():
    p = WL.stereo_refine(H=192, W=256, regions=40)
    say("determinism stereo256x192")
    a = grid_arrays(gpu_grid(p))
    b = grid_arrays(gpu_grid(p))
    for k in ("key", "idx", "nbr", "pix_list", "n"):
        assert np.array_equal(a[k], b[k])


def _solve_both(p, init="hier", max_iters=None, rel_tol=None, C=None, lam=None):
    prm = params(p, init=init, max_iters=p.max_iters if max_iters is None else max_iters,
                 rel_tol=p.rel_tol if rel_tol is None else rel_tol,
                 lam=p.lam if lam is None else lam)
    G = gpu_grid(p)
    t, c = to_dev(p.target), to_dev(p.conf)
    ws = G.solve_workspace(p.C)
    y, st = G.solve(t, c, prm.lam, max_iters=prm.max_iters, rel_tol=prm.rel_tol, init=init, ws=ws)
    x = G.slice(y, p.C)
    torch.cuda.synchronize()
    sol = O.solve(p.ref, p.target, p.conf, prm)
    return G, ws, y, x, st, sol, prm


@pytest.mark.parametrize("init", ["flat", "hier"])
def test_splat_diag_and_init(init):
    p = WL.tiny_ramp(seed=11, channels=2)
    say(f"splat/init ramp64x48 C=2 init={init}")
    G, ws, y, x, st, sol, prm = _solve_both(p, init=init, max_iters=0)
    V = sol.grid.V
    b, sc, dg, mi = [a.cpu().numpy() for a in G.solve_ws_arrays(ws, 2)]
    assert rel_l2(b[:V], sol.b) <= 1e-7
    assert rel_l2(sc[:V], sol.sc) <= 1e-7
    assert rel_l2(dg[:V], sol.A.diag()) <= 1e-6
    assert rel_l2(mi[:V], sol.minv) <= 1e-6
    assert rel_l2(y.cpu().numpy()[:V], sol.y0) <= 1e-6


@pytest.mark.parametrize("init", ["flat", "hier"])
def test_solve_tiny_to_tolerance(init):
    p = WL.tiny_ramp()
    say(f"solve ramp64x48 init={init} tol=1e-5")
    G, ws, y, x, st, sol, prm = _solve_both(p, init=init)
    from paper_1511_03296_amd import read_stats
    s = read_stats(st)[0]
    assert s["reason"] == 1 and s["rel_residual"] <= 1e-5
    assert abs(int(s["iters"]) - sol.runs[0].iters) <= 3
    assert rel_l2(x.cpu().numpy(), sol.x) <= TOL_X
    # against the exact minimiser too
    exact = O.solve(p.ref, p.target, p.conf, params(p, rel_tol=1e-12, max_iters=5000))
    assert rel_l2(x.cpu().numpy(), exact.x) <= TOL_X
    tr = O.true_relative_residual(sol.A, sol.b, y.cpu().numpy()[: sol.grid.V])
    assert tr[0] <= 2e-5


def test_solve_fixed_iterations_stereo_shape():
    p = WL.stereo_refine(H=384, W=512, regions=120)
    say("solve stereo512x384 25 iterations")
    G, ws, y, x, st, sol, prm = _solve_both(p)
    from paper_1511_03296_amd import read_stats
    s = read_stats(st)[0]
    assert s["iters"] == 25 and s["reason"] == 2
    assert rel_l2(x.cpu().numpy(), sol.x) <= TOL_X


@pytest.mark.parametrize("C", [3, 21])
def test_solve_multichannel(C):
    p = WL.segmentation(H=96, W=128, regions=20, C=C, rel_tol=1e-5)
    say(f"solve seg128x96 C={C}")
    G, ws, y, x, st, sol, prm = _solve_both(p)
    from paper_1511_03296_amd import read_stats
    s = read_stats(st)
    assert np.all(s["reason"] == 1)
    for ch in range(C):
        assert abs(int(s["iters"][ch]) - sol.runs[ch].iters) <= 3
    assert rel_l2(x.cpu().numpy(), sol.x) <= TOL_X


def test_lambda_zero_closed_form_on_gpu():
    p = WL.tiny_ramp(seed=9)
    say("solve lambda=0")
    G, ws, y, x, st, sol, prm = _solve_both(p, lam=0.0, rel_tol=1e-6, max_iters=50)
    g = sol.grid
    c = p.conf.reshape(-1).astype(float)
    t = p.target[0].reshape(-1).astype(float)
    want = np.bincount(g.idx, c * t, g.V) / np.bincount(g.idx, c, g.V)
    assert rel_l2(y.cpu().numpy()[: g.V, 0], want) <= 1e-6


def test_zero_confidence_is_finite():
    p = WL.tiny_ramp(seed=10)
    p.conf = np.zeros_like(p.conf)
    say("solve zero confidence")
    G, ws, y, x, st, sol, prm = _solve_both(p)
    from paper_1511_03296_amd import read_stats
    s = read_stats(st)[0]
    assert s["reason"] == 5 and s["iters"] == 0
    assert np.all(x.cpu().numpy() == 0.0)


def test_backward_parity():
    p = WL.segmentation(H=64, W=80, regions=12, C=3, rel_tol=1e-6)
    say("backward seg80x64 C=3")
    G, ws, y, x, st, sol, prm = _solve_both(p)
    gx = WL.random_grad(3, p.C, p.H, p.W)
    gt, gc, gb, bst = G.backward(to_dev(p.target), to_dev(p.conf), y, to_dev(gx), prm.lam,
                                 max_iters=prm.max_iters, rel_tol=prm.rel_tol, want_g=True,
                                 ws=ws)
    torch.cuda.synchronize()
    V = sol.grid.V
    # given the kernel's own solution (the adjoint and scatter alone) ...
    og = O.solve_backward(sol, p.target, p.conf, gx, prm, y_hat=y.cpu().numpy()[:V])
    u = G.solve_ws_arrays(ws, p.C)[0].cpu().numpy()[:V]
    assert rel_l2(u, og.u) <= 1e-6
    assert rel_l2(gb.cpu().numpy()[:V], og.gb) <= TOL_X
    assert rel_l2(gt.cpu().numpy(), og.grad_t) <= TOL_X
    assert rel_l2(gc.cpu().numpy(), og.grad_c) <= TOL_X
    # ... and end to end, on the oracle's own solution
    og = O.solve_backward(sol, p.target, p.conf, gx, prm)
    assert rel_l2(gt.cpu().numpy(), og.grad_t) <= TOL_X
    check_grad_c(gc.cpu().numpy(), og.grad_c, p.conf)


def test_autograd_function_matches_backward():
    from paper_1511_03296_amd import bilateral_solve
    p = WL.segmentation(H=48, W=64, regions=8, C=2, rel_tol=1e-6)
    say("autograd seg64x48 C=2")
    G = gpu_grid(p)
    t = to_dev(p.target).requires_grad_(True)
    c = to_dev(p.conf).requires_grad_(True)
    x = bilateral_solve(G, t, c, p.lam, max_iters=5000, rel_tol=1e-6)
    onehot = to_dev(p.extra["onehot"])
    loss = ((x - onehot) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    prm = params(p, max_iters=5000, rel_tol=1e-6)
    sol = O.solve(p.ref, p.target, p.conf, prm)
    gx = 2.0 * (x.detach().cpu().numpy() - p.extra["onehot"])
    og = O.solve_backward(sol, p.target, p.conf, gx, prm)
    assert rel_l2(t.grad.cpu().numpy(), og.grad_t) <= TOL_X
    assert rel_l2(c.grad.cpu().numpy(), og.grad_c) <= TOL_X


def test_full_size_stereo_1024x768():
    """The stereo workload at full size, 25 iterations: every pixel compared."""
    p = WL.stereo_refine()
    say("full stereo1024x768")
    G, ws, y, x, st, sol, prm = _solve_both(p)
    got = grid_arrays(G)
    assert got["V"] == sol.grid.V and np.array_equal(got["idx"], sol.grid.idx)
    assert np.array_equal(got["nbr"], sol.grid.nbr)
    assert got["nb_packed"] == 1 and got["nb_wide"] == 0 and np.array_equal(got["nb16"], sol.grid.nbr)
    assert rel_l2(x.cpu().numpy(), sol.x) <= TOL_X


def test_full_size_stereo_backward():
    """Stereo workload at full size: the backward pass, every pixel compared."""
    p = WL.stereo_refine()
    say("full stereo1024x768 backward")
    G, ws, y, x, st, sol, prm = _solve_both(p)
    gx = WL.random_grad(0, p.C, p.H, p.W)
    gt, gc, gb, bst = G.backward(to_dev(p.target), to_dev(p.conf), y, to_dev(gx), prm.lam,
                                 max_iters=prm.max_iters, rel_tol=prm.rel_tol, ws=ws)
    torch.cuda.synchronize()
    og = O.solve_backward(sol, p.target, p.conf, gx, prm, y_hat=y.cpu().numpy()[: sol.grid.V])
    assert rel_l2(gt.cpu().numpy(), og.grad_t) <= TOL_X
    assert rel_l2(gc.cpu().numpy(), og.grad_c) <= TOL_X
    og = O.solve_backward(sol, p.target, p.conf, gx, prm)    # end to end
    assert rel_l2(gt.cpu().numpy(), og.grad_t) <= TOL_X
    check_grad_c(gc.cpu().numpy(), og.grad_c, p.conf)


@pytest.mark.parametrize("h,w", [(240, 320), (480, 640)])
def test_depth_backward_crop(h, w):
    """The depth workload's backward pass as bench.py runs it: a centre crop
    (on the 16-pixel sample grid, so 1 pixel in 256 keeps confidence 1 and
    the rest 0), forward and adjoint PCG to 1e-5, and the confidence-weighted
    upstream gradient, for which the singular adjoint system is consistent:
    x, dL/dt and dL/dc against the oracle's same-algorithm solves."""
    full = WL.depth_superres()
    y0 = (full.H - h) // 2 // 16 * 16
    x0 = (full.W - w) // 2 // 16 * 16
    p = WL.crop(full, y0, x0, h, w)
    say(f"depth backward crop {w}x{h} at ({x0}, {y0})")
    G, ws, y, x, st, sol, prm = _solve_both(p)
    gx = WL.random_grad(0, 1, h, w) * p.conf[None]
    gt, gc, _, bst = G.backward(to_dev(p.target), to_dev(p.conf), y, to_dev(gx), prm.lam,
                                max_iters=prm.max_iters, rel_tol=prm.rel_tol, ws=ws)
    torch.cuda.synchronize()
    from paper_1511_03296_amd import read_stats
    assert read_stats(st)[0]["reason"] == 1 and read_stats(bst)[0]["reason"] == 1
    og = O.solve_backward(sol, p.target, p.conf, gx, prm)
    assert rel_l2(x.cpu().numpy(), sol.x) <= TOL_X
    assert rel_l2(gt.cpu().numpy(), og.grad_t) <= TOL_X
    check_grad_c(gc.cpu().numpy(), og.grad_c, p.conf)


def test_full_size_depth_2048x1536():
    """Depth super-resolution workload at full size (V ~ 1.6M): grid and
    bistochastization bit-exact / 1e-12 against the oracle; the solution at
    1024 sampled pixels against the oracle's FP64 solve stored by
    tests/golden/make_golden.py (the oracle's own PCG needs minutes here)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "depthsr2048x1536.json")))
    p = WL.depth_superres()
    say("full depth2048x1536")
    G = gpu_grid(p)
    t, c = to_dev(p.target), to_dev(p.conf)
    y, st = G.solve(t, c, p.lam, max_iters=p.max_iters, rel_tol=p.rel_tol)
    x = G.slice(y, 1)
    torch.cuda.synchronize()
    got = grid_arrays(G)
    g = O.build_grid(p.ref, p.sigma_xy, p.sigma_l, p.sigma_uv)
    assert got["V"] == g.V == gold["V"] and np.array_equal(got["key"], g.keys)
    assert np.array_equal(got["idx"], g.idx) and np.array_equal(got["nbr"], g.nbr)
    assert got["nb_packed"] == 1 and got["nb_wide"] == 0 and np.array_equal(got["nb16"], g.nbr)
    pyr = O.build_pyramid(g)
    assert got["K"] == pyr.K and got["sizes"][: pyr.K + 1] == pyr.sizes == gold["pyramid_sizes"]
    bs = O.bistochastize(g, 1e-10, 200)
    assert got["bist_iters"] == bs.iters == gold["bist_iters"]
    assert np.max(np.abs(got["n"] - bs.n) / bs.n) <= 1e-12
    from paper_1511_03296_amd import read_stats
    s = read_stats(st)[0]
    assert s["reason"] == 1 and s["rel_residual"] <= p.rel_tol
    xs = x.cpu().numpy().reshape(-1)[np.array(gold["pixels"])]
    err = rel_l2(xs, np.array(gold["x"]))
    say(f"depth: GPU iterations {int(s['iters'])} (oracle {gold['pcg_iters']}), "
        f"sampled rel-L2 vs oracle {err:.3e}")
    assert err <= TOL_X
