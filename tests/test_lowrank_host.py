"""The host factorisation of the low-rank reduction (bs_lowrank_factor, a
pure host call of the library) against the oracle's column-pivoted QR
(supplement Section Multiple Output Channels): the same rank t, a Q-tilde
with orthonormal columns and the same reduced approximation Q-tilde R-tilde
of B."""
import ctypes as ct

import numpy as np
import pytest

import workloads as WL
from oracle import bilateral as O


def _splat_b(p):
    prm = O.Params(p.sigma_xy, p.sigma_l, p.sigma_uv, p.lam)
    g, _, _ = O.prepare(p.ref, prm)
    c = p.conf.reshape(-1).astype(np.float64)
    return np.stack([O.splat(g, c * p.target[ch].reshape(-1)) for ch in range(p.C)], axis=1)


def _factor(B, eps):
    from paper_1511_03296_amd import _lib as L
    C = B.shape[1]
    G = np.ascontiguousarray(B.T @ B, dtype=np.float64)
    M = np.zeros(C * C, np.float32)
    Rt = np.zeros(C * C, np.float32)
    t = ct.c_int32(-1)
    L.check(L.lib.bs_lowrank_factor(G.ctypes.data, C, eps, M.ctypes.data, Rt.ctypes.data,
                                    ct.byref(t)), "bs_lowrank_factor")
    t = t.value
    return t, M[: C * t].reshape(C, t), Rt[: t * C].reshape(t, C)


def _cases():
    rng = np.random.default_rng(7)
    seg = WL.segmentation(H=48, W=64, regions=8, C=8)
    low = WL.segmentation(H=48, W=64, regions=8, C=3)
    low.target = np.einsum("kc,chw->khw", rng.normal(size=(7, 3)), low.target).astype(np.float32)
    e = np.exp(seg.target - seg.target.max(0))
    prob = WL.segmentation(H=48, W=64, regions=8, C=8)
    prob.target = (e / e.sum(0)).astype(np.float32)
    return [("seg C=8", _splat_b(seg)), ("rank 3 of 7", _splat_b(low)),
            ("softmax C=8", _splat_b(prob))]


@pytest.mark.parametrize("eps", [0.0, 1e-9, 0.01, 0.2])
def test_factor_matches_pivoted_qr(eps):
    for name, B in _cases():
        if eps == 0.0 and name.startswith("rank"):
            # eps = 0 on a rank-deficient B: the QR keeps rows of rounding
            # noise (relative mass 1e-16) until its sum reaches the total,
            # the factorisation stops at the numerical rank
            continue
        lr = O.lowrank_reduce(B, eps)
        t, M, Rt = _factor(B, eps)
        assert t == lr.rank, (name, t, lr.rank)
        Qt = B @ M.astype(np.float64)
        assert np.allclose(Qt.T @ Qt, np.eye(t), atol=2e-5), name
        approx = Qt @ Rt.astype(np.float64)
        want = lr.Q @ lr.R
        assert np.linalg.norm(approx - want) <= 1e-5 * np.linalg.norm(B), name


def test_factor_of_zero_and_invalid_input():
    from paper_1511_03296_amd import _lib as L
    t, _, _ = _factor(np.zeros((50, 4)), 0.01)
    assert t == 0
    G = np.eye(3)
    M = np.zeros(9, np.float32)
    r = ct.c_int32(0)
    assert L.lib.bs_lowrank_factor(G.ctypes.data, 3, 1.0, M.ctypes.data, M.ctypes.data,
                                   ct.byref(r)) == L.BS_EINVAL
    assert L.lib.bs_lowrank_factor(G.ctypes.data, 0, 0.1, M.ctypes.data, M.ctypes.data,
                                   ct.byref(r)) == L.BS_EINVAL
