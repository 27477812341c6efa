"""The hierarchical preconditioner M_hier^-1 (Section 4, Eq. hier_precond)
on the GPU, against the oracle's HierPrecond: the solution and gradients of
a solve preconditioned by it against the oracle's exact minimiser, and its
iteration count against the oracle's float64 PCG with the same
preconditioner (a wrong level scale or a missing level would change the
count, not the minimiser).  Jacobi runs on the same inputs give the A/B."""
import numpy as np
import pytest
import torch

import workloads as WL
from oracle import bilateral as O
from tests.gpu_helpers import check_grad_c, gpu_grid, params, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _iters(stats):
    from paper_1511_03296_amd import read_stats
    st = read_stats(stats)
    assert set(st["reason"].tolist()) <= {1, 5}, st
    return [int(i) for i in st["iters"]]


CASES = [
    ("ramp64x48 C=2", lambda: WL.tiny_ramp(seed=5, channels=2), 1e-6),
    ("seg96x80 C=21", lambda: WL.segmentation(H=80, W=96, regions=12, C=21, rel_tol=1e-6), 1e-6),
    ("depth crop 256x192", lambda: WL.crop(WL.depth_superres(), 672, 896, 192, 256), 1e-5),
]


@pytest.mark.parametrize("name,make,tol", CASES, ids=[c[0] for c in CASES])
def test_hier_precond_solve_and_backward(name, make, tol):
    p = make()
    say(f"hierarchical preconditioner: {name}")
    G = gpu_grid(p)
    t, c = to_dev(p.target), to_dev(p.conf)
    gx = WL.random_grad(1, p.C, p.H, p.W)
    if "depth" in name:
        gx = gx * p.conf[None]        # consistent adjoint on the unconfident components
    out = {}
    for pre in ("jacobi", "hier"):
        ws = G.solve_workspace(p.C)
        y, st = G.solve(t, c, p.lam, max_iters=5000, rel_tol=tol, precond=pre, ws=ws)
        x = G.slice(y, p.C)
        gt, gc, _, bst = G.backward(t, c, y, to_dev(gx), p.lam, max_iters=5000, rel_tol=tol,
                                    precond=pre, ws=ws)
        torch.cuda.synchronize()
        out[pre] = (x.cpu().numpy(), gt.cpu().numpy(), gc.cpu().numpy(), _iters(st), _iters(bst))
    prm = params(p, max_iters=5000, rel_tol=tol)
    prm_h = O.Params(**{**prm.__dict__, "precond": "hier"})
    # the oracle with the same preconditioner: its iteration counts, and the
    # reference wherever the minimiser is not unique (components of the grid
    # without confidence keep what the initial state and the preconditioned
    # directions give them, which differs between preconditioners)
    sol_h = O.solve(p.ref, p.target, p.conf, prm_h)
    og = O.solve_backward(sol_h, p.target, p.conf, gx, prm_h)
    x, gt, gc, fi, bi = out["hier"]
    assert rel_l2(x, sol_h.x) <= TOL
    assert rel_l2(gt, og.grad_t) <= TOL
    check_grad_c(gc, og.grad_c, p.conf)
    if np.all(p.conf > 0):
        # a unique minimiser: the same as the Jacobi solve's
        assert rel_l2(out["jacobi"][0], sol_h.x) <= TOL
    oi = [r.iters for r in sol_h.runs]
    say(f"  iterations forward: GPU hier {max(fi)}, oracle hier {max(oi)}, "
        f"GPU Jacobi {max(out['jacobi'][3])}; backward: GPU hier {max(bi)}, "
        f"GPU Jacobi {max(out['jacobi'][4])}")
    for g_it, o_it in zip(fi, oi):
        assert abs(g_it - o_it) <= max(3, 0.1 * o_it), (fi, oi)


def test_hier_precond_large_alpha_is_jacobi_counts():
    """With alpha -> infinity every coarse scale vanishes and M_hier^-1 is the
    Jacobi inverse: the iteration counts equal a Jacobi solve's."""
    p = WL.tiny_ramp(seed=8, channels=1)
    say("hierarchical preconditioner, alpha = 1e30")
    G = gpu_grid(p)
    t, c = to_dev(p.target), to_dev(p.conf)
    _, sj = G.solve(t, c, p.lam, max_iters=2000, rel_tol=1e-6)
    yh, sh = G.solve(t, c, p.lam, max_iters=2000, rel_tol=1e-6, precond="hier", pre_alpha=1e30)
    x = G.slice(yh, 1)
    torch.cuda.synchronize()
    assert abs(_iters(sj)[0] - _iters(sh)[0]) <= 2
    exact = O.solve(p.ref, p.target, p.conf, params(p, rel_tol=1e-12, max_iters=20000))
    assert rel_l2(x.cpu().numpy(), exact.x) <= TOL


def test_hier_precond_rejected_where_unsupported():
    from paper_1511_03296_amd import BatchState, SolveOptions
    p = WL.tiny_ramp(seed=9, channels=2)
    st = BatchState([to_dev(p.ref)], [to_dev(p.target)], [to_dev(p.conf)],
                    [(p.sigma_xy, p.sigma_l, p.sigma_uv)], 1)
    with pytest.raises(Exception, match="Jacobi"):
        st.forward(SolveOptions(p.lam, 100, 1e-6, precond="hier"))
