"""GPU tests of the batch engine: a batch of images of uneven size, channel
count and grid scale must reproduce the single-image path bit for bit (same
deterministic kernels), forward and backward, and the batched autograd
Function must agree with the per-image one."""
import numpy as np
import pytest
import torch

import workloads as WL
from oracle import bilateral as O
from tests.gpu_helpers import params, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu


def small_batch(n=7, seed=3):
    return WL.mixed_batch(seed=seed, count=n, wmin=40, wmax=200, hmin=30, hmax=150,
                          rel_tol=1e-5, max_iters=3000)


def test_batch_forward_backward_matches_single_image():
    from paper_1511_03296_amd import BilateralGrid, BatchState, SolveOptions
    probs = small_batch()
    say("batch forward/backward " + " ".join(f"{p.W}x{p.H}c{p.C}s{p.sigma_xy}" for p in probs))
    refs = [to_dev(p.ref) for p in probs]
    ts = [to_dev(p.target) for p in probs]
    cs = [to_dev(p.conf) for p in probs]
    gxs = [to_dev(WL.random_grad(i, p.C, p.H, p.W)) for i, p in enumerate(probs)]
    sig = [(p.sigma_xy, p.sigma_l, p.sigma_uv) for p in probs]
    opts = SolveOptions(probs[0].lam, 3000, 1e-5)
    for streams in (1, 3):
        st = BatchState(refs, ts, cs, sig, streams)
        xs, _ = st.forward(opts)
        gts, gcs, _ = st.backward(gxs, opts)
        torch.cuda.synchronize()
        for i, p in enumerate(probs):
            G = BilateralGrid(refs[i], *sig[i])
            y, _ = G.solve(ts[i], cs[i], p.lam, max_iters=3000, rel_tol=1e-5)
            x = G.slice(y, p.C)
            gt, gc, _, _ = G.backward(ts[i], cs[i], y, gxs[i], p.lam, max_iters=3000,
                                      rel_tol=1e-5)
            torch.cuda.synchronize()
            assert torch.equal(x, xs[i]), (streams, i)
            assert torch.equal(gt, gts[i]) and torch.equal(gc, gcs[i]), (streams, i)
    # and the batch against the oracle's minimiser on two of its images
    for i in (0, len(probs) - 1):
        p = probs[i]
        sol = O.solve(p.ref, p.target, p.conf, params(p, rel_tol=1e-10, max_iters=5000))
        assert rel_l2(xs[i].cpu().numpy(), sol.x) <= 1e-4, i


def test_batched_autograd_matches_single():
    from paper_1511_03296_amd import BilateralGrid, bilateral_solve, bilateral_solve_batch
    probs = small_batch(n=4, seed=5)
    say("batched autograd")
    refs = [to_dev(p.ref) for p in probs]
    ts = [to_dev(p.target).requires_grad_(True) for p in probs]
    cs = [to_dev(p.conf).requires_grad_(True) for p in probs]
    sig = [(p.sigma_xy, p.sigma_l, p.sigma_uv) for p in probs]
    xs = bilateral_solve_batch(refs, ts, cs, sig, probs[0].lam, max_iters=3000, rel_tol=1e-6)
    loss = sum((x * x).sum() for x in xs)
    loss.backward()
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        t1 = to_dev(p.target).requires_grad_(True)
        c1 = to_dev(p.conf).requires_grad_(True)
        x1 = bilateral_solve(BilateralGrid(refs[i], *sig[i]), t1, c1, p.lam, max_iters=3000,
                             rel_tol=1e-6)
        (x1 * x1).sum().backward()
        torch.cuda.synchronize()
        assert torch.equal(x1.detach(), xs[i].detach())
        assert torch.equal(t1.grad, ts[i].grad) and torch.equal(c1.grad, cs[i].grad)


def test_batch_rejects_bad_items():
    from paper_1511_03296_amd import BatchState
    p = small_batch(n=1)[0]
    with pytest.raises(ValueError):
        BatchState([to_dev(p.ref)], [to_dev(p.target)], [to_dev(p.conf)],
                   [(0, 4, 4)], 2)
    with pytest.raises(ValueError):
        BatchState([to_dev(p.ref)], [to_dev(p.target)], [to_dev(p.conf)],
                   [(8, 4, 4)], 17)
