"""Pins of the FP64 domain-transform oracle (oracle/domain_transform.py)
against what the filter's definition and mathematics fix: a pass written out
as an explicit matrix of products of feedback coefficients, the closed-form
impulse response of a pass on a flat guide, the variances of the iterations
adding up to sigma_s^2, the exact equivalence of a constant-gradient guide
with a flat guide at a smaller sigma_s, edge stopping, and the invariants of
the variance confidence (supplement Section Robustness)."""
import math

import numpy as np

import workloads as WL
from oracle import domain_transform as DT


def flat_ref(H, W, value=0.5):
    return np.full((3, H, W), value, np.float32)


def pass_matrix(d, sigma):
    """The 1-D pass (causal, then anti-causal) on a line of len(d) samples
    as a dense matrix, built from products of the feedback coefficients
    w[x] = a^d[x] of the edges (x-1, x): the causal output at x weighs
    input k < x by (1 - w[k]) w[k+1] ... w[x] (the first sample by the
    product alone), the anti-causal output likewise to the right."""
    a = math.exp(-math.sqrt(2.0) / sigma)
    L = len(d)
    w = a ** np.asarray(d, np.float64)
    Lc = np.zeros((L, L))
    for x in range(L):
        for k in range(x + 1):
            prod = np.prod(w[k + 1:x + 1])
            Lc[x, k] = prod if k == 0 else (1.0 - w[k]) * prod
    U = np.zeros((L, L))
    for x in range(L):
        for k in range(x, L):
            prod = np.prod(w[x + 1:k + 1])          # edges (x, x+1) .. (k-1, k)
            U[x, k] = prod if k == L - 1 else (1.0 - w[k + 1]) * prod
    return U @ Lc


def test_constant_signal_passes_unchanged():
    rng = np.random.default_rng(0)
    ref = rng.uniform(0, 1, (3, 9, 11)).astype(np.float32)
    x = np.full((2, 9, 11), 3.25)
    y = DT.domain_transform(ref, x, 8.0, 4.0)
    assert np.max(np.abs(y - 3.25)) < 1e-13


def test_pass_equals_its_matrix_of_coefficient_products():
    rng = np.random.default_rng(1)
    for L in (1, 2, 7, 23):
        d = np.concatenate([[0.0], rng.uniform(1.0, 30.0, L - 1)])
        u = rng.normal(size=L)
        got = DT.recursive_pass(u[None, None, :], d[None, :], 5.0, axis=-1)[0, 0]
        assert np.allclose(got, pass_matrix(d, 5.0) @ u, rtol=0, atol=1e-13)
        # the same pass along columns
        gotc = DT.recursive_pass(u[None, :, None], d[:, None], 5.0, axis=-2)[0, :, 0]
        assert np.allclose(gotc, got, rtol=0, atol=1e-14)


def test_two_d_filter_equals_product_of_pass_matrices():
    """N iterations of (horizontal, vertical) passes on a 5x6 image with a
    random guide, as one dense operator built from the 1-D matrices."""
    rng = np.random.default_rng(2)
    H, W, N, ss, sr = 5, 6, 3, 6.0, 40.0
    ref = rng.uniform(0, 1, (3, H, W)).astype(np.float32)
    dh, dv = DT.domain_steps(DT.guide_codes(ref), ss, sr)
    M = np.eye(H * W)
    idx = np.arange(H * W).reshape(H, W)
    for s in DT.iteration_sigmas(ss, N):
        Hm = np.zeros((H * W, H * W))
        for y in range(H):
            Hm[np.ix_(idx[y], idx[y])] = pass_matrix(dh[y], s)
        Vm = np.zeros((H * W, H * W))
        for x in range(W):
            Vm[np.ix_(idx[:, x], idx[:, x])] = pass_matrix(dv[:, x], s)
        M = Vm @ Hm @ M
    u = rng.normal(size=(H, W))
    got = DT.domain_transform(ref, u[None], ss, sr, N)[0]
    assert np.allclose(got.reshape(-1), M @ u.reshape(-1), rtol=0, atol=1e-12)


def test_flat_guide_impulse_response_closed_form():
    """Far from the ends, one pass on a flat guide answers a unit impulse with
    ((1 - a) / (1 + a)) a^|n|."""
    L, c, sigma = 401, 200, 7.0
    a = math.exp(-math.sqrt(2.0) / sigma)
    d = np.ones(L)
    d[0] = 0.0
    u = np.zeros(L)
    u[c] = 1.0
    got = DT.recursive_pass(u[None, None], d[None], sigma, axis=-1)[0, 0]
    n = np.arange(L) - c
    want = (1 - a) / (1 + a) * a ** np.abs(n)
    assert np.max(np.abs(got - want)) < 1e-15


def test_iteration_variances_add_up_to_sigma_s_squared():
    """Three iterations on a flat 1-row image: the impulse response's
    variance is sigma_s^2 (to the discretisation of each exponential
    kernel, whose variance 2a / (1 - a)^2 is sigma_i^2 to O(1))."""
    ss = 24.0
    sig = DT.iteration_sigmas(ss, 3)
    assert abs(sum(s * s for s in sig) - ss * ss) < 1e-9
    assert sig[0] > sig[1] > sig[2] and abs(sig[0] / sig[1] - 2.0) < 1e-12
    W, c = 2001, 1000
    u = np.zeros((1, 1, W))
    u[0, 0, c] = 1.0
    h = DT.domain_transform(flat_ref(1, W), u, ss, 10.0, 3)[0, 0]
    n = np.arange(W) - c
    assert abs(h.sum() - 1.0) < 1e-12
    var = float(np.sum(h * n * n))
    exact = sum(2 * math.exp(-math.sqrt(2) / s) / (1 - math.exp(-math.sqrt(2) / s)) ** 2
                for s in sig)
    assert abs(var - exact) < 1e-6 * exact
    assert abs(var - ss * ss) < 0.01 * ss * ss


def test_constant_gradient_guide_is_a_flat_guide_with_smaller_sigma():
    """A guide whose red code rises by g per pixel puts every neighbour
    1 + (s_s / s_r) g apart: on a single row (or column) that is the flat-guide
    filter with sigma_s / (1 + (s_s / s_r) g)."""
    rng = np.random.default_rng(3)
    W, g, ss, sr = 64, 3, 12.0, 20.0
    ref = np.zeros((3, 1, W), np.float32)
    ref[0, 0] = (np.arange(W) * g) / 255.0
    ref[1] = 0.3
    u = rng.normal(size=(1, 1, W))
    got = DT.domain_transform(ref, u, ss, sr)
    flat = DT.domain_transform(flat_ref(1, W), u, ss / (1 + ss / sr * g), sr)
    assert np.max(np.abs(got - flat)) < 1e-12
    # the same along a column
    refc = np.ascontiguousarray(ref.transpose(0, 2, 1))
    uc = np.ascontiguousarray(u.transpose(0, 2, 1))
    gotc = DT.domain_transform(refc, uc, ss, sr)
    assert np.max(np.abs(gotc - got.transpose(0, 2, 1))) < 1e-12


def test_strong_edges_stop_the_filter():
    """With s_s / s_r large, a guide edge separates the two sides: a signal
    constant on each side of the same edge is left unchanged."""
    H, W = 12, 14
    for axis in (1, 2):
        ref = np.zeros((3, H, W), np.float32)
        x = np.zeros((1, H, W))
        if axis == 2:
            ref[:, :, W // 2:] = 1.0
            x[:, :, W // 2:] = 5.0
        else:
            ref[:, H // 2:, :] = 1.0
            x[:, H // 2:, :] = 5.0
        y = DT.domain_transform(ref, x + 1.0, 16.0, 0.1)
        assert np.max(np.abs(y - (x + 1.0))) < 1e-12


def test_variance_confidence_invariants():
    rng = np.random.default_rng(4)
    p = WL.stereo_refine(seed=3, H=40, W=56, regions=12)
    z = p.target[0].astype(np.float64)
    m1 = DT.domain_transform(p.ref, z[None], 32.0, 32.0)[0]
    m2 = DT.domain_transform(p.ref, (z * z)[None], 32.0, 32.0)[0]
    # a normalised filter with non-negative weights: DT(z^2) >= DT(z)^2
    assert np.min(m2 - m1 * m1) > -1e-9 * np.max(z * z)
    c = DT.dt_confidence(p.ref, z, 32.0, 32.0, 2.0, zero_cols=5)
    assert np.all(c[:, :5] == 0.0)
    assert np.all((c[:, 5:] >= 0.0) & (c[:, 5:] <= 1.0)) and np.any(c[:, 5:] > 0.5)
    V = np.maximum(m2 - m1 * m1, 0.0)
    assert np.allclose(c[:, 5:], np.exp(-V[:, 5:] / 8.0), rtol=0, atol=1e-15)
    # a constant depth has no variance; a shift of the depth changes nothing
    assert np.max(np.abs(DT.dt_confidence(p.ref, np.full_like(z, 7.0), 32, 32, 2.0) - 1)) < 1e-12
    c2 = DT.dt_confidence(p.ref, z + 100.0, 32.0, 32.0, 2.0, zero_cols=5)
    assert np.max(np.abs(c2 - c)) < 1e-8
    # the filter is linear in the signal
    u, v = rng.normal(size=(2, 1, 40, 56))
    lhs = DT.domain_transform(p.ref, 2.0 * u - 3.0 * v, 8.0, 16.0)
    rhs = 2.0 * DT.domain_transform(p.ref, u, 8.0, 16.0) - 3.0 * DT.domain_transform(
        p.ref, v, 8.0, 16.0)
    assert np.max(np.abs(lhs - rhs)) < 1e-12
