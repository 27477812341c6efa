"""GPU parity of the robust bilateral solver (supplement Algorithm RBS)
through the C ABI against the FP64 oracle: Geman-McClure IRLS rounds of
solve, slice and reweight."""
import numpy as np
import pytest
import torch

import workloads as WL
from oracle import bilateral as O
from tests.gpu_helpers import gpu_grid, params, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu

TOL_X = 1e-4


def _outliers(p, frac, size, seed):
    rng = np.random.default_rng(seed)
    t = p.target.copy()
    t[:, rng.random(t.shape[1:]) < frac] += size
    return t


def _both(p, t, c, sigma_gm, n, **kw):
    prm = params(p, **kw)
    G = gpu_grid(p)
    y, x, st = G.robust_solve(to_dev(t), to_dev(c), prm.lam, sigma_gm, n,
                              max_iters=prm.max_iters, rel_tol=prm.rel_tol)
    torch.cuda.synchronize()
    o = O.robust_solve(p.ref, t, c, prm, sigma_gm, n)
    return G, y, x, st, o, prm


def test_robust_stereo_shape_with_outliers():
    """The stereo-refinement shape (10 % outlier disparities) at 512x384,
    8 IRLS rounds of 25 PCG iterations each, sigma_gm = 4 disparities."""
    p = WL.stereo_refine(H=384, W=512, regions=120)
    say("robust stereo512x384 n=8")
    G, y, x, st, o, prm = _both(p, p.target, p.conf, 4.0, 8)
    err = rel_l2(x.cpu().numpy(), o.solution.x)
    say(f"  rel-L2 vs oracle {err:.2e}")
    assert err <= TOL_X


def test_robust_tolerance_three_channels():
    p = WL.tiny_ramp(seed=12, H=120, W=160, regions=10, channels=3)
    t = _outliers(p, 0.05, 2.0, seed=3)
    say("robust ramp160x120 C=3 n=6 tol=1e-6")
    G, y, x, st, o, prm = _both(p, t, p.conf, 0.2, 6, max_iters=2000, rel_tol=1e-6)
    from paper_1511_03296_amd import read_stats
    s = read_stats(st)
    assert np.all(s["reason"] == 1)
    assert rel_l2(x.cpu().numpy(), o.solution.x) <= TOL_X


def test_robust_one_round_is_the_solve():
    p = WL.tiny_ramp(seed=13)
    say("robust one round vs bs_solve")
    prm = params(p)
    G = gpu_grid(p)
    t, c = to_dev(p.target), to_dev(p.conf)
    y1, x1, _ = G.robust_solve(t, c, prm.lam, 0.5, 1, max_iters=prm.max_iters,
                               rel_tol=prm.rel_tol)
    y2, _ = G.solve(t, c, prm.lam, max_iters=prm.max_iters, rel_tol=prm.rel_tol)
    x2 = G.slice(y2, 1)
    torch.cuda.synchronize()
    V = G.vertex_count()
    assert torch.equal(y1[:V], y2[:V]) and torch.equal(x1, x2)


def test_robust_rejects_invalid_arguments():
    p = WL.tiny_ramp(seed=14)
    G = gpu_grid(p)
    t, c = to_dev(p.target), to_dev(p.conf)
    for sigma, n in ((0.0, 4), (float("nan"), 4), (1.0, 0)):
        with pytest.raises(ValueError):
            G.robust_solve(t, c, p.lam, sigma, n)


@pytest.mark.slow
def test_robust_full_size_in_bench_configuration():
    """robust_stereo1024x768 as bench.py runs it: 8 rounds of 25 iterations,
    sigma_gm = 4, on the full stereo input with its outliers."""
    p = WL.stereo_refine()
    say("robust full size stereo1024x768 n=8")
    G, y, x, st, o, prm = _both(p, p.target, p.conf, 4.0, 8)
    err = rel_l2(x.cpu().numpy(), o.solution.x)
    say(f"  rel-L2 vs oracle {err:.2e}")
    assert err <= TOL_X
