"""GPU parity of the low-rank reduction of many right-hand sides
(supplement Section Multiple Output Channels) through the C ABI against the
FP64 oracle: the same rank, and the reduced solution to the solver's
tolerance."""
import numpy as np
import pytest
import torch

import workloads as WL
from oracle import bilateral as O
from tests.gpu_helpers import gpu_grid, params, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu

TOL_X = 1e-4


def test_lowrank_class_probabilities():
    p = WL.segmentation_probs(H=192, W=256, regions=30)
    say("lowrank segprob256x192 C=21 eps=0.01")
    prm = params(p)
    G = gpu_grid(p)
    y, st, t = G.solve_lowrank(to_dev(p.target), to_dev(p.conf), p.lam, 0.01,
                               max_iters=prm.max_iters, rel_tol=prm.rel_tol)
    x = G.slice(y, p.C)
    torch.cuda.synchronize()
    Y, xo, lr, runs = O.solve_lowrank(p.ref, p.target, p.conf, prm, 0.01)
    say(f"  rank {t} (oracle {lr.rank})")
    assert t == lr.rank and 1 <= t <= 5
    from paper_1511_03296_amd import read_stats
    s = read_stats(st)[:t]
    assert np.all(s["reason"] == 1)
    V = Y.shape[0]
    assert rel_l2(y.cpu().numpy()[:V], Y) <= TOL_X
    assert rel_l2(x.cpu().numpy(), xo) <= TOL_X
    # what the reduction drops: small next to the full solve
    full = O.solve(p.ref, p.target, p.conf, prm)
    assert rel_l2(x.cpu().numpy(), full.x) <= 0.1


def test_lowrank_eps_zero_is_the_full_solve():
    p = WL.segmentation(H=96, W=128, regions=20, C=5, rel_tol=1e-6)
    say("lowrank eps=0 seg128x96 C=5")
    G = gpu_grid(p)
    t_, c_ = to_dev(p.target), to_dev(p.conf)
    y, st, t = G.solve_lowrank(t_, c_, p.lam, 0.0, max_iters=p.max_iters, rel_tol=p.rel_tol)
    yf, _ = G.solve(t_, c_, p.lam, max_iters=p.max_iters, rel_tol=p.rel_tol)
    torch.cuda.synchronize()
    V = G.vertex_count()
    assert t == 5
    assert rel_l2(y.cpu().numpy()[:V], yf.cpu().numpy()[:V]) <= TOL_X


def test_lowrank_zero_target_and_invalid_eps():
    p = WL.segmentation(H=40, W=48, regions=6, C=4)
    G = gpu_grid(p)
    z = torch.zeros((4, p.H, p.W), device="cuda")
    y, _, t = G.solve_lowrank(z, to_dev(p.conf), p.lam, 0.01)
    torch.cuda.synchronize()
    assert t == 0 and torch.count_nonzero(y) == 0
    with pytest.raises(ValueError):
        G.solve_lowrank(to_dev(p.target), to_dev(p.conf), p.lam, 1.0)


@pytest.mark.slow
def test_lowrank_full_size_in_bench_configuration():
    """One image of segprob16x512x512 as bench.py runs it (eps = 0.01, PCG to
    1e-6): the rank and the solution against the oracle."""
    p = WL.segmentation_probs(seed=0)
    say("lowrank full size segprob512x512")
    prm = params(p)
    G = gpu_grid(p)
    y, st, t = G.solve_lowrank(to_dev(p.target), to_dev(p.conf), p.lam, 0.01,
                               max_iters=prm.max_iters, rel_tol=prm.rel_tol)
    x = G.slice(y, p.C)
    torch.cuda.synchronize()
    Y, xo, lr, _ = O.solve_lowrank(p.ref, p.target, p.conf, prm, 0.01)
    say(f"  rank {t} (oracle {lr.rank})")
    assert t == lr.rank
    assert rel_l2(x.cpu().numpy(), xo) <= TOL_X


def test_batch_lowrank_matches_single_image():
    """The batched low-rank forward against the single-image one on a batch
    of class-probability maps of different sizes, a full-rank five-channel
    image and a zero target (rank 0)."""
    from paper_1511_03296_amd import BatchState, SolveOptions
    probs = [WL.segmentation_probs(seed=s, H=h, W=w, regions=20)
             for s, (h, w) in enumerate([(120, 160), (192, 256), (300, 200)])]
    five = WL.segmentation(H=96, W=128, regions=20, C=5, rel_tol=1e-6)
    zero = WL.segmentation_probs(seed=9, H=64, W=80, regions=8)
    zero.target = np.zeros_like(zero.target)
    batch = probs + [five, zero]
    say("batch lowrank: 5 images")
    st = BatchState([to_dev(p.ref) for p in batch], [to_dev(p.target) for p in batch],
                    [to_dev(p.conf) for p in batch],
                    [(p.sigma_xy, p.sigma_l, p.sigma_uv) for p in batch], 3)
    opts = SolveOptions(128.0, 20000, 1e-6)
    xs, _, ranks = st.forward_lowrank(opts, 0.01)
    torch.cuda.synchronize()
    for i, p in enumerate(batch):
        G = gpu_grid(p)
        y, _, t = G.solve_lowrank(to_dev(p.target), to_dev(p.conf), 128.0, 0.01,
                                  max_iters=20000, rel_tol=1e-6)
        x = G.slice(y, p.C)
        torch.cuda.synchronize()
        say(f"  image {i}: rank {ranks[i]} (single image {t})")
        assert ranks[i] == t
        if t == 0:
            assert torch.count_nonzero(xs[i]) == 0
        else:
            assert rel_l2(xs[i].cpu().numpy(), x.cpu().numpy()) <= TOL_X
    assert ranks[-1] == 0 and ranks[3] == 5
    p = probs[1]
    prm = params(p, max_iters=20000, rel_tol=1e-6)
    _, xo, lr, _ = O.solve_lowrank(p.ref, p.target, p.conf, prm, 0.01)
    assert ranks[1] == lr.rank and rel_l2(xs[1].cpu().numpy(), xo) <= TOL_X


@pytest.mark.parametrize("case", ["C1", "C64", "rank2of8"])
def test_lowrank_edge_channel_counts(case):
    """One channel (t = 1), the largest channel count (64, lanes of 4) and
    an exactly rank-2 B of 8 channels: rank and solution against the
    oracle."""
    if case == "C1":
        p = WL.tiny_ramp(seed=21, H=60, W=80, regions=8)
    elif case == "C64":
        p = WL.segmentation(seed=22, H=48, W=64, regions=8, C=64, rel_tol=1e-6)
    else:
        p = WL.segmentation(seed=23, H=60, W=80, regions=8, C=2, rel_tol=1e-6)
        mix = np.random.default_rng(5).normal(size=(8, 2))
        p.target = np.einsum("kc,chw->khw", mix, p.target).astype(np.float32)
    say(f"lowrank edge {case}: C={p.C}")
    prm = params(p, max_iters=5000, rel_tol=1e-6)
    G = gpu_grid(p)
    y, st, t = G.solve_lowrank(to_dev(p.target), to_dev(p.conf), p.lam, 0.01,
                               max_iters=prm.max_iters, rel_tol=prm.rel_tol)
    x = G.slice(y, p.C)
    torch.cuda.synchronize()
    Y, xo, lr, _ = O.solve_lowrank(p.ref, p.target, p.conf, prm, 0.01)
    say(f"  rank {t} (oracle {lr.rank})")
    assert t == lr.rank
    if case == "C1":
        assert t == 1
    if case == "rank2of8":
        assert t == 2
    assert rel_l2(x.cpu().numpy(), xo) <= TOL_X
