"""GPU edge cases of the solve: every lane width and channel padding (C = 4,
5, 6, 9, 64), degenerate images (one pixel, one row, one column), the
largest grid scale, neighbour offsets at the limit of the packed 16-bit
table and beyond it, a batch mixing them, and invalid inputs rejected on the
host before anything is launched."""
import numpy as np
import pytest
import torch

import workloads as WL
from oracle import bilateral as O
from tests.gpu_helpers import grid_arrays, gpu_grid, params, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu

TOL_X = 1e-4


def _solve_vs_oracle(p, init="hier", rel_tol=1e-6, max_iters=3000):
    G = gpu_grid(p)
    t, c = to_dev(p.target), to_dev(p.conf)
    y, st = G.solve(t, c, p.lam, max_iters=max_iters, rel_tol=rel_tol, init=init)
    x = G.slice(y, p.C)
    torch.cuda.synchronize()
    exact = O.solve(p.ref, p.target, p.conf, params(p, rel_tol=1e-12, max_iters=20000,
                                                   init=init))
    return x.cpu().numpy(), exact, st


@pytest.mark.parametrize("C", [4, 5, 6, 9, 64])
def test_channel_counts(C):
    # 4: float4 lanes, no padding; 5: float4 lanes padded to 8; 6, 9: 3-float
    # lanes; 64: 16 lanes per vertex (the widest)
    p = WL.segmentation(H=40, W=56, regions=10, C=C, rel_tol=1e-6)
    say(f"edge: channels C={C}")
    x, exact, st = _solve_vs_oracle(p)
    assert rel_l2(x, exact.x) <= TOL_X
    from paper_1511_03296_amd import read_stats
    s = read_stats(st)
    assert len(s) == C and np.all(s["reason"] == 1)


@pytest.mark.parametrize("H,W", [(1, 1), (1, 50), (50, 1), (2, 3)])
def test_degenerate_images(H, W):
    p = WL.tiny_ramp(seed=21, H=H, W=W, regions=min(3, H * W), channels=2)
    say(f"edge: image {W}x{H}")
    x, exact, _ = _solve_vs_oracle(p)
    assert np.all(np.isfinite(x))
    assert rel_l2(x, exact.x) <= TOL_X


def test_largest_grid_scale():
    # sigma_xy = 128 and colour scales 255: a handful of vertices in one cell
    p = WL.tiny_ramp(seed=22, H=90, W=120, regions=8, sigma=(128, 255, 255))
    say("edge: sigma (128, 255, 255)")
    x, exact, _ = _solve_vs_oracle(p, init="flat")
    assert rel_l2(x, exact.x) <= TOL_X


@pytest.mark.parametrize("W,packed,wide", [(32767, 1, 0), (32800, 0, 1)])
def test_neighbour_offsets_at_16_bit_limit(W, packed, wide):
    # sigma_xy = 1 and a reference constant down each column: every pixel is a
    # vertex and its neighbour one row down is W ids away.  W = 32767 is the
    # widest strip the packed table holds (the host bound admits it exactly);
    # at 32800 the host keeps the 32-bit table and the grid reports the
    # offset that does not fit.  Forward and backward against the oracle.
    p = WL.strip(seed=27, H=3, W=W)
    say(f"edge: strip {W}x3, sigma_xy 1 (packed table {packed})")
    G = gpu_grid(p)
    t, c = to_dev(p.target), to_dev(p.conf)
    y, st = G.solve(t, c, p.lam, max_iters=p.max_iters, rel_tol=p.rel_tol)
    x = G.slice(y, 1)
    gx = WL.random_grad(28, 1, 3, W)
    gt, gc, _, _ = G.backward(t, c, y, to_dev(gx), p.lam, max_iters=p.max_iters,
                           rel_tol=p.rel_tol)
    torch.cuda.synchronize()
    got = grid_arrays(G)
    g = O.build_grid(p.ref, p.sigma_xy, p.sigma_l, p.sigma_uv)
    assert got["V"] == g.V == 3 * W
    assert got["nb_packed"] == packed and got["nb_wide"] == wide
    assert np.array_equal(got["nbr"], g.nbr)
    assert int(np.max(np.abs(np.where(g.nbr >= 0, g.nbr - np.arange(g.V), 0)))) == W
    if packed:
        assert np.array_equal(got["nb16"], g.nbr)
    bs = O.bistochastize(g, 1e-10, 200)
    assert got["bist_iters"] == bs.iters
    assert np.max(np.abs(got["n"] - bs.n) / bs.n) <= 1e-12
    prm = params(p, rel_tol=1e-12, max_iters=20000)
    sol = O.solve(p.ref, p.target, p.conf, prm)
    og = O.solve_backward(sol, p.target, p.conf, gx, prm)
    assert rel_l2(x.cpu().numpy(), sol.x) <= TOL_X
    assert rel_l2(gt.cpu().numpy(), og.grad_t) <= TOL_X


@pytest.mark.parametrize("H,W", [(1, 65535), (65535, 1)])
def test_largest_image_side(H, W):
    # the longest side the 16-bit key fields hold; at sigma_xy = 1 every pixel
    # has its own cell, so the cell coordinate reaches 65534
    p = WL.tiny_ramp(seed=31, H=H, W=W, regions=40, sigma=(1, 8, 8))
    say(f"edge: image {W}x{H}, sigma_xy 1")
    G = gpu_grid(p)
    t, c = to_dev(p.target), to_dev(p.conf)
    y, _ = G.solve(t, c, p.lam, max_iters=3000, rel_tol=1e-6)
    x = G.slice(y, 1)
    torch.cuda.synchronize()
    got = grid_arrays(G)
    g = O.build_grid(p.ref, p.sigma_xy, p.sigma_l, p.sigma_uv)
    assert got["V"] == g.V and np.array_equal(got["key"], g.keys)
    assert np.array_equal(got["idx"], g.idx) and np.array_equal(got["nbr"], g.nbr)
    assert int(np.max(g.coords[:, 0 if H > 1 else 1])) == max(H, W) - 1
    exact = O.solve(p.ref, p.target, p.conf, params(p, rel_tol=1e-12, max_iters=20000))
    assert rel_l2(x.cpu().numpy(), exact.x) <= TOL_X


def test_batch_mixing_packed_and_wide_tables():
    # one launch group (C = 1) holding a grid with the packed table and one
    # without: the group reads the 32-bit ids of both
    from paper_1511_03296_amd import BatchState, SolveOptions
    probs = [WL.strip(seed=29, H=3, W=32800),
             WL.tiny_ramp(seed=30, H=48, W=64, regions=6)]
    say("edge: batch of a wide strip and a packed image")
    st = BatchState([to_dev(p.ref) for p in probs], [to_dev(p.target) for p in probs],
                    [to_dev(p.conf) for p in probs],
                    [(p.sigma_xy, p.sigma_l, p.sigma_uv) for p in probs], 2)
    xs, _ = st.forward(SolveOptions(128.0, 3000, 1e-6))
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        exact = O.solve(p.ref, p.target, p.conf,
                        params(p, lam=128.0, rel_tol=1e-12, max_iters=20000))
        assert rel_l2(xs[i].cpu().numpy(), exact.x) <= TOL_X, i


def test_batch_of_extremes():
    from paper_1511_03296_amd import BatchState, SolveOptions
    probs = [WL.tiny_ramp(seed=23, H=1, W=1, regions=1),
             WL.segmentation(seed=24, H=30, W=44, regions=6, C=64, rel_tol=1e-6),
             WL.tiny_ramp(seed=25, H=50, W=1, regions=3, channels=2),
             WL.segmentation(seed=26, H=33, W=47, regions=6, C=5, rel_tol=1e-6)]
    say("edge: batch of extremes")
    refs = [to_dev(p.ref) for p in probs]
    ts = [to_dev(p.target) for p in probs]
    cs = [to_dev(p.conf) for p in probs]
    sig = [(p.sigma_xy, p.sigma_l, p.sigma_uv) for p in probs]
    st = BatchState(refs, ts, cs, sig, 2)
    xs, _ = st.forward(SolveOptions(128.0, 3000, 1e-6))
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        exact = O.solve(p.ref, p.target, p.conf,
                        params(p, lam=128.0, rel_tol=1e-12, max_iters=20000))
        assert rel_l2(xs[i].cpu().numpy(), exact.x) <= TOL_X, i


def test_non_finite_input_stops_only_its_channels():
    # device data are not scanned: a NaN target value stops its own channel
    # after one iteration (reason 4, non-finite residual); the other channel
    # is solved as if alone.  A NaN confidence stops every channel.
    from paper_1511_03296_amd import read_stats
    p = WL.tiny_ramp(seed=32, H=40, W=56, regions=6, channels=2)
    say("edge: NaN target in channel 0, NaN confidence")
    G = gpu_grid(p)
    t = p.target.copy()
    t[0, 7, 9] = np.nan
    y, st = G.solve(to_dev(t), to_dev(p.conf), p.lam, max_iters=3000, rel_tol=1e-6)
    x = G.slice(y, 2)
    torch.cuda.synchronize()
    s = read_stats(st)
    assert s["reason"][0] == 4 and s["iters"][0] <= 1 and not np.isfinite(s["rel_residual"][0])
    assert s["reason"][1] == 1
    one = O.solve(p.ref, p.target[1:2], p.conf, params(p, rel_tol=1e-12, max_iters=20000))
    assert rel_l2(x[1:2].cpu().numpy(), one.x) <= TOL_X
    c = p.conf.copy()
    c[3, 4] = np.nan
    y, st = G.solve(to_dev(p.target), to_dev(c), p.lam, max_iters=3000, rel_tol=1e-6)
    torch.cuda.synchronize()
    s = read_stats(st)
    assert np.all(s["reason"] == 4) and np.all(s["iters"] <= 1)


def test_invalid_inputs_rejected():
    from paper_1511_03296_amd import BilateralGrid
    from paper_1511_03296_amd import _lib as L
    say("edge: invalid inputs")
    p = WL.tiny_ramp(seed=27)
    ref = to_dev(p.ref)
    with pytest.raises(ValueError):
        BilateralGrid(ref[:, :0, :], 8, 4, 4)        # empty image
    with pytest.raises(ValueError):
        BilateralGrid(ref, 0, 4, 4)                  # zero grid scale
    G = BilateralGrid(ref, 8, 4, 4)
    t65 = torch.zeros((65, p.H, p.W), device="cuda")
    with pytest.raises(ValueError):
        G.solve(t65, to_dev(p.conf), 128.0)          # more than 64 channels
    with pytest.raises(ValueError):
        G.solve(to_dev(p.target), to_dev(p.conf), -1.0)   # negative lambda
    assert L.lib.bs_solve_workspace_bytes(None, 1) == 0
