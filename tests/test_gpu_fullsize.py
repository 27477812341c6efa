"""Full-size parity of the batched benchmark workloads, in the launch
configuration bench.py times: the 64-image mixed batch (43 Mpix, C in
{1, 2, 21}) and the 16-image 21-channel segmentation batch, through the
batch engine on 4 streams, forward and backward with the bench's tolerances
and upstream gradients.  Every image's channels must stop on the tolerance;
images the oracle can solve in seconds (the smallest of each channel count,
or the first) are compared with it, forward and backward."""
import json
import os

import numpy as np
import pytest
import torch

import bench
import workloads as WL
from oracle import bilateral as O
from tests.gpu_helpers import check_grad_c, rel_l2, say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL = 1e-4
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_mixed64_batch_in_bench_configuration():
    from paper_1511_03296_amd import BatchState, SolveOptions, read_stats
    spec = bench.WORKLOADS["mixed64"]
    probs = bench.make_problems("mixed64")
    say(f"full size mixed64: {len(probs)} images, {sum(p.pixels for p in probs)} pixels")
    inputs = bench.gpu_inputs(probs, spec, torch.device("cuda:0"))
    (fi, ft), (bi, bt) = spec["fwd"], spec["bwd"]
    lam = probs[0].lam
    state = BatchState([d["ref"] for d in inputs], [d["t"] for d in inputs],
                       [d["c"] for d in inputs],
                       [(p.sigma_xy, p.sigma_l, p.sigma_uv) for p in probs], 4)
    xs, fst = state.forward(SolveOptions(lam, fi, ft, check_every=8), stats=True)
    gts, gcs, bst = state.backward([d["gx"] for d in inputs],
                                   SolveOptions(lam, bi, bt, check_every=8), stats=True)
    torch.cuda.synchronize()
    for i in range(len(probs)):
        f, b = read_stats(fst[i]), read_stats(bst[i])
        assert np.all(f["reason"] == 1) and np.all(f["rel_residual"] <= ft), i
        assert np.all(b["reason"] == 1) and np.all(b["rel_residual"] <= bt), i
        assert torch.isfinite(xs[i]).all() and torch.isfinite(gts[i]).all(), i
    by_c = {}
    for i, p in enumerate(probs):
        if p.C not in by_c or p.pixels < probs[by_c[p.C]].pixels:
            by_c[p.C] = i
    for C, i in sorted(by_c.items()):
        p = probs[i]
        say(f"  oracle check image {i}: {p.W}x{p.H} C={C} sigma_xy={p.sigma_xy}")
        prm = O.Params(p.sigma_xy, p.sigma_l, p.sigma_uv, lam, max_iters=fi, rel_tol=ft)
        sol = O.solve(p.ref, p.target, p.conf, prm)
        gx = inputs[i]["gx"].cpu().numpy()
        prmb = O.Params(p.sigma_xy, p.sigma_l, p.sigma_uv, lam, max_iters=bi, rel_tol=bt)
        og = O.solve_backward(sol, p.target, p.conf, gx, prmb)
        assert rel_l2(xs[i].cpu().numpy(), sol.x) <= TOL, i
        assert rel_l2(gts[i].cpu().numpy(), og.grad_t) <= TOL, i
        # confidences U[0, 1]: dL/dc through c o dL/dc (check_grad_c)
        plain, weighted = check_grad_c(gcs[i].cpu().numpy(), og.grad_c, p.conf, TOL)
        say(f"    dL/dc rel-L2 {plain:.2e}, c o dL/dc {weighted:.2e}")
    # the largest image, the widest (next to the packed table's 16-bit bound)
    # and the widest 21-channel image against the oracle's stored samples
    # (tests/golden/make_golden.py, the same solves in float64)
    for i in (4, 7, 10):
        with open(os.path.join(GOLDEN, f"mixed64_image{i}.json")) as f:
            gold = json.load(f)
        p = probs[i]
        assert (gold["W"], gold["H"], gold["C"]) == (p.W, p.H, p.C)
        ch, px = np.array(gold["channels"]), np.array(gold["pixels"])
        x = xs[i].cpu().numpy().reshape(p.C, -1)[ch, px]
        gt = gts[i].cpu().numpy().reshape(p.C, -1)[ch, px]
        pc = np.array(gold["grad_c_pixels"])
        gc = gcs[i].cpu().numpy().reshape(-1)[pc]
        ex, et = rel_l2(x, gold["x"]), rel_l2(gt, gold["grad_t"])
        ec = rel_l2(np.array(gold["conf_at_grad_c_pixels"]) * gc,
                    np.array(gold["conf_at_grad_c_pixels"]) * np.array(gold["grad_c"]))
        say(f"  golden image {i} ({p.W}x{p.H} C={p.C}): x {ex:.2e}, dL/dt {et:.2e}, "
            f"c o dL/dc {ec:.2e} on 1024 samples")
        assert ex <= TOL and et <= TOL and ec <= TOL, (i, ex, et, ec)


def test_seg16_batch_in_bench_configuration():
    """The 16-image 21-channel segmentation batch (512x512 each) as bench.py
    runs it: batch engine on 4 streams, forward and adjoint PCG to 1e-6,
    upstream gradient 2 (x - onehot label).  Every channel must stop on the
    tolerance; image 0 is compared with the oracle, forward and backward."""
    from paper_1511_03296_amd import BatchState, SolveOptions, read_stats
    spec = bench.WORKLOADS["seg16x512x512"]
    probs = bench.make_problems("seg16x512x512")
    say(f"full size seg16x512x512: {len(probs)} images")
    inputs = bench.gpu_inputs(probs, spec, torch.device("cuda:0"))
    (fi, ft), (bi, bt) = spec["fwd"], spec["bwd"]
    lam = probs[0].lam
    state = BatchState([d["ref"] for d in inputs], [d["t"] for d in inputs],
                       [d["c"] for d in inputs],
                       [(p.sigma_xy, p.sigma_l, p.sigma_uv) for p in probs], 4)
    xs, fst = state.forward(SolveOptions(lam, fi, ft, check_every=8), stats=True)
    gts, gcs, bst = state.backward([d["gx"] for d in inputs],
                                   SolveOptions(lam, bi, bt, check_every=8), stats=True)
    torch.cuda.synchronize()
    for i in range(len(probs)):
        f, b = read_stats(fst[i]), read_stats(bst[i])
        assert np.all(f["reason"] == 1) and np.all(f["rel_residual"] <= ft), i
        assert np.all(b["reason"] == 1) and np.all(b["rel_residual"] <= bt), i
    p = probs[0]
    say("  oracle check image 0 (21 channels, forward and backward)")
    prm = O.Params(p.sigma_xy, p.sigma_l, p.sigma_uv, lam, max_iters=fi, rel_tol=ft)
    sol = O.solve(p.ref, p.target, p.conf, prm)
    gx = inputs[0]["gx"].cpu().numpy()
    prmb = O.Params(p.sigma_xy, p.sigma_l, p.sigma_uv, lam, max_iters=bi, rel_tol=bt)
    og = O.solve_backward(sol, p.target, p.conf, gx, prmb)
    assert rel_l2(xs[0].cpu().numpy(), sol.x) <= TOL
    assert rel_l2(gts[0].cpu().numpy(), og.grad_t) <= TOL
    # confidences U[0.2, 1]: dL/dc itself within the bar
    plain, weighted = check_grad_c(gcs[0].cpu().numpy(), og.grad_c, p.conf, TOL)
    say(f"    dL/dc rel-L2 {plain:.2e}, c o dL/dc {weighted:.2e}")
