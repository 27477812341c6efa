"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: the paper's
dense equations built independently (oracle/dense.py), brute force on tiny
inputs, closed forms, limits and invariants.  Citations name the paper's
sections and equations.
"""
from fractions import Fraction

import numpy as np
import pytest

import workloads as WL
from oracle import bilateral as O
from oracle import dense as D


def tiny(seed=0, H=10, W=12, regions=3, sigma=(4, 24, 24), lam=2.0, C=1):
    return WL.tiny_ramp(seed=seed, H=H, W=W, regions=regions, sigma=sigma, lam=lam,
                        channels=C)


def params_of(p, **kw):
    base = dict(sigma_xy=p.sigma_xy, sigma_l=p.sigma_l, sigma_uv=p.sigma_uv, lam=p.lam,
                max_iters=5000, rel_tol=1e-13, bist_tol=1e-13, bist_max_iters=2000)
    base.update(kw)
    return O.Params(**base)


def dense_problem(p, prm):
    """Dense S, B-bar (brute force), W-hat and literal A for a tiny problem."""
    g, bs, pyr = O.prepare(p.ref, prm)
    S = D.splat_matrix(g.idx, g.V)
    B = D.blur_matrix_bruteforce(g.coords)
    m = g.m.astype(np.float64)
    c = p.conf.reshape(-1).astype(np.float64)
    Wh = D.w_hat(S, m, bs.n, B)
    Alit = D.a_literal(m, bs.n, B, S @ c, p.lam)
    return g, bs, pyr, S, B, Wh, Alit


# --------------------------------------------------------------------------
# Colour, coordinates, vertex set (Section 2, Eq. bilateral_affinity, Eq. equiv)
# --------------------------------------------------------------------------

def test_quantise8_values():
    v = np.array([0.0, 1.0, 0.5, 1.0 / 255.0, -0.1, 1.5, np.nan, 0.00197, 0.00195, 0.998],
                 np.float32)
    got = O.quantise8(v)
    # floor(255 v + 1/2) clamped; NaN -> 0
    assert got.tolist() == [0, 255, 128, 1, 0, 255, 0, 1, 0, 254]


def test_yuv_fixed_point_against_jfif_float_formula():
    """Fixed-point YCbCr within 1 code of the JFIF real-valued definition for all
    2^24 colours, and equal for nearly all of them."""
    r, g, b = np.meshgrid(np.arange(256), np.arange(256), np.arange(256), indexing="ij")
    r, g, b = r.ravel(), g.ravel(), b.ravel()
    y, u, v = O.rgb8_to_yuv8(r, g, b)
    fy = 0.299 * r + 0.587 * g + 0.114 * b
    fu = 128.0 - 0.168736 * r - 0.331264 * g + 0.5 * b
    fv = 128.0 + 0.5 * r - 0.418688 * g - 0.081312 * b
    ref = [np.clip(np.floor(f + 0.5), 0, 255) for f in (fy, fu, fv)]
    for got, want in zip((y, u, v), ref):
        diff = np.abs(got - want)
        assert diff.max() <= 1
        assert np.mean(diff == 0) > 0.99
    # primaries: black, white, red, green, blue
    probe = np.array([[0, 0, 0], [255, 255, 255], [255, 0, 0], [0, 255, 0], [0, 0, 255]])
    yy, uu, vv = O.rgb8_to_yuv8(probe[:, 0], probe[:, 1], probe[:, 2])
    assert yy.tolist() == [0, 255, 76, 150, 29]
    assert uu.tolist() == [128, 128, 85, 44, 255]
    assert vv.tolist() == [128, 128, 255, 21, 107]


def test_grid_coord_is_round_half_up():
    for s in range(1, 41):
        v = np.arange(0, 700)
        want = [int(np.floor(Fraction(int(x), s) + Fraction(1, 2))) for x in v]
        assert O.grid_coord(v, s).tolist() == want


@pytest.mark.parametrize("seed,sigma", [(0, (4, 24, 24)), (1, (3, 16, 8)), (2, (5, 40, 12))])
def test_vertex_set_bruteforce(seed, sigma):
    """Each pixel lies on exactly one vertex (S S^T = D_m, Eq. SS); vertices in
    lexicographic (y, x, l, u, v) order; m counts pixels."""
    p = tiny(seed=seed, sigma=sigma)
    g = O.build_grid(p.ref, *sigma)
    coords = O.pixel_coords(p.ref, *sigma)
    table = {}
    for i, c in enumerate(map(tuple, coords.tolist())):
        table.setdefault(c, []).append(i)
    order = sorted(table)
    assert [tuple(c) for c in g.coords.tolist()] == order
    for v, c in enumerate(order):
        assert g.m[v] == len(table[c])
        assert all(g.idx[i] == v for i in table[c])
    S = D.splat_matrix(g.idx, g.V)
    assert np.array_equal(S @ S.T, np.diag(g.m.astype(float)))
    assert g.m.sum() == p.pixels


@pytest.mark.parametrize("seed", [0, 3])
def test_neighbour_table_bruteforce(seed):
    p = tiny(seed=seed, H=14, W=16, sigma=(4, 16, 16))
    g = O.build_grid(p.ref, p.sigma_xy, p.sigma_l, p.sigma_uv)
    B = D.blur_matrix_bruteforce(g.coords)
    Bo = np.zeros((g.V, g.V))
    Bo[np.arange(g.V), np.arange(g.V)] = 10.0
    for j in range(10):
        ok = g.nbr[j] >= 0
        Bo[np.nonzero(ok)[0], g.nbr[j][ok]] += 1.0
    assert np.array_equal(B, Bo)
    # direction semantics: slot 2d is -1 and 2d+1 is +1 along dim d
    for d in range(5):
        for j, step in enumerate((-1, 1)):
            ok = g.nbr[2 * d + j] >= 0
            delta = g.coords[g.nbr[2 * d + j][ok]] - g.coords[ok]
            want = np.zeros(5, int)
            want[d] = step
            assert np.all(delta == want)


# --------------------------------------------------------------------------
# Bistochastization (supplement Algorithm 1, Eq. equiv)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bistochastization_fixed_point(seed):
    p = tiny(seed=seed)
    prm = params_of(p)
    g, bs, _, S, B, Wh, _ = dense_problem(p, prm)
    m = g.m.astype(float)
    # D_n B D_n 1 = D_m 1
    assert np.max(np.abs(bs.n * (B @ bs.n) - m) / m) <= 1e-12
    # W-hat is symmetric, non-negative and row-stochastic
    assert np.allclose(Wh, Wh.T, atol=1e-15)
    assert Wh.min() >= 0
    assert np.max(np.abs(Wh.sum(axis=1) - 1.0)) <= 1e-12
    assert bs.residual <= 1e-13 and bs.iters > 0


def test_bistochastization_stopping_rule():
    p = tiny(seed=4, H=20, W=24, sigma=(4, 16, 16))
    g = O.build_grid(p.ref, p.sigma_xy, p.sigma_l, p.sigma_uv)
    loose = O.bistochastize(g, 1e-3, 200)
    tight = O.bistochastize(g, 1e-10, 200)
    capped = O.bistochastize(g, 0.0, 3)
    assert loose.residual <= 1e-3 and tight.residual <= 1e-10
    assert loose.iters < tight.iters
    assert capped.iters == 3 and capped.residual > 0
    # one more update from the loose answer reduces the residual (contraction)
    m = g.m.astype(float)
    n1 = np.sqrt(loose.n * m / O.blur(g, loose.n))
    r1 = np.max(np.abs(n1 * O.blur(g, n1) - m) / m)
    assert r1 < loose.residual


# --------------------------------------------------------------------------
# The bilateral-space quadratic (Eq. pixel_loss, Eq. quad_min, Eq. solution)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_quadratic_equals_pixel_loss(seed):
    """f(S^T y) = y^T A y - 2 b^T y + (c o t)^T t for the pixel loss f, A, b of Eq. quad_min."""
    p = tiny(seed=seed)
    prm = params_of(p)
    g, bs, _, S, B, Wh, Alit = dense_problem(p, prm)
    c = p.conf.reshape(-1).astype(float)
    t = p.target[0].reshape(-1).astype(float)
    sc = O.splat(g, c)
    A = O.Operator(g, bs.n, sc, p.lam)
    b = O.splat(g, c * t)
    rng = np.random.default_rng(seed)
    for _ in range(4):
        y = rng.normal(size=g.V)
        lhs = D.pixel_loss(S.T @ y, t, c, Wh, p.lam)
        rhs = y @ A(y) - 2 * b @ y + (c * t) @ t
        assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))
    # Hessian of the pixel loss, projected, is 2A; the literal A agrees with the operator
    H = D.pixel_loss_hessian(Wh, c, p.lam)
    Aop = np.stack([A(e) for e in np.eye(g.V)], axis=1)
    assert np.allclose(0.5 * S @ H @ S.T, Aop, rtol=0, atol=1e-10 * np.abs(Aop).max())
    assert np.allclose(Alit, Aop, rtol=0, atol=1e-10 * np.abs(Aop).max())
    assert np.allclose(np.diag(Alit), A.diag(), rtol=0, atol=1e-10 * np.abs(Aop).max())


def test_operator_invariants():
    p = WL.tiny_ramp(seed=5)
    prm = params_of(p, bist_tol=1e-10)
    g, bs, _ = O.prepare(p.ref, prm)
    sc = O.splat(g, p.conf.reshape(-1))
    A = O.Operator(g, bs.n, sc, p.lam)
    rng = np.random.default_rng(0)
    u, v = rng.normal(size=g.V), rng.normal(size=g.V)
    assert abs(u @ A(v) - v @ A(u)) <= 1e-10 * abs(u @ A(v))
    assert np.allclose(A(np.ones(g.V)), sc, rtol=0, atol=1e-9 * p.lam)
    assert np.all(A.diag()[sc > 0] > 0)
    # literal formula differs by lam * m * bistochastization residual at most
    z = rng.normal(size=g.V)
    gap = np.abs(A(z) - A.literal(z))
    assert np.all(gap <= 2 * p.lam * g.m * bs.residual * np.abs(z) + 1e-9)
    for _ in range(3):
        z = rng.normal(size=g.V)
        assert z @ A(z) > 0


@pytest.mark.parametrize("seed,init", [(0, "hier"), (1, "flat"), (2, "hier")])
def test_pcg_matches_dense_solve(seed, init):
    """Converged PCG equals the exact minimiser y = A^-1 b (Eq. linear_system, solution)."""
    p = tiny(seed=seed, C=2)
    prm = params_of(p, init=init)
    g, bs, pyr, S, B, Wh, Alit = dense_problem(p, prm)
    sol = O.solve(p.ref, p.target, p.conf, prm, prepared=(g, bs, pyr))
    c = p.conf.reshape(-1).astype(float)
    for ch in range(2):
        y = D.solve_dense(Alit, sol.b[:, ch])
        assert np.linalg.norm(sol.y[:, ch] - y) <= 1e-9 * np.linalg.norm(y)
        # the sliced output is a stationary point of the pixel loss over x = S^T y
        t = p.target[ch].reshape(-1).astype(float)
        x = S.T @ sol.y[:, ch]
        grad_x = D.pixel_loss_hessian(Wh, c, p.lam) @ x - 2 * c * t
        assert np.linalg.norm(S @ grad_x) <= 1e-8 * np.linalg.norm(2 * c * t)
        assert np.allclose(sol.x[ch].reshape(-1), x, rtol=0, atol=1e-12)


def test_lambda_zero_closed_form():
    """lam = 0: y = S(c t) / S(c), the per-vertex confidence-weighted mean of t."""
    p = WL.tiny_ramp(seed=3)
    for init in ("flat", "hier"):
        prm = params_of(p, lam=0.0, init=init, rel_tol=1e-12)
        sol = O.solve(p.ref, p.target, p.conf, prm)
        g = sol.grid
        c = p.conf.reshape(-1).astype(float)
        t = p.target[0].reshape(-1).astype(float)
        want = np.zeros(g.V)
        for v in range(g.V):
            px = np.nonzero(g.idx == v)[0]
            want[v] = np.sum(c[px] * t[px]) / np.sum(c[px])
        assert np.allclose(sol.y[:, 0], want, rtol=1e-12, atol=0)
        assert sol.runs[0].iters <= (0 if init == "flat" else 1)


def test_constant_reference_large_lambda_limit():
    """Constant reference, lam -> inf: x -> the global weighted mean sum(c t)/sum(c), error O(1/lam)."""
    p = WL.tiny_ramp(seed=2, H=24, W=32)
    ref = np.full_like(p.ref, 0.4)
    c = p.conf.astype(float)
    t = p.target[0].astype(float)
    mean = np.sum(c * t) / np.sum(c)
    errs = []
    for lam in (1e4, 1e5, 1e6):
        prm = params_of(p, lam=lam, rel_tol=1e-14, max_iters=20000)
        sol = O.solve(ref, p.target, p.conf, prm)
        errs.append(np.max(np.abs(sol.x[0] - mean)))
    assert errs[2] <= 1e-4 * abs(mean)
    assert 5.0 < errs[1] / errs[2] < 20.0 and 5.0 < errs[0] / errs[1] < 20.0


# --------------------------------------------------------------------------
# Bilateral pyramid and hierarchical initialisation (supplement Section 2; Section 4)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1])
def test_pyramid_bruteforce(seed):
    p = WL.tiny_ramp(seed=seed)
    g = O.build_grid(p.ref, p.sigma_xy, p.sigma_l, p.sigma_uv)
    pyr = O.build_pyramid(g)
    level = [tuple(c) for c in g.coords.tolist()]
    for k in range(pyr.K):
        halves = [tuple(x >> 1 for x in c) for c in level]
        nxt = sorted(set(halves))
        pos = {c: i for i, c in enumerate(nxt)}
        assert pyr.parents[k].tolist() == [pos[h] for h in halves]
        assert pyr.sizes[k + 1] == len(nxt)
        level = nxt
    assert len(level) == 1 and all(s > 1 for s in pyr.sizes[:-1])
    assert pyr.ones[-1].tolist() == [g.V]
    # adjointness <P y, z> = <y, P^T z>
    rng = np.random.default_rng(seed)
    y = rng.normal(size=g.V)
    z = [rng.normal(size=s) for s in pyr.sizes]
    lhs = sum(float(a @ b) for a, b in zip(O.lift(pyr, y), z))
    rhs = float(y @ O.collapse(pyr, z))
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_hier_init_limits():
    p = WL.tiny_ramp(seed=1)
    g = O.build_grid(p.ref, p.sigma_xy, p.sigma_l, p.sigma_uv)
    pyr = O.build_pyramid(g)
    c = p.conf.reshape(-1).astype(float)
    t = p.target[0].reshape(-1).astype(float)
    sc, b = O.splat(g, c), O.splat(g, c * t)
    # alpha -> inf degenerates to the flat init where S c > 0
    big = O.hier_init(pyr, b, sc, alpha=1e30, beta=0.0)
    flat = O.flat_init(b, sc)
    assert np.allclose(big[sc > 0], flat[sc > 0], rtol=1e-12)
    # push-pull of a constant ratio is that constant everywhere
    assert np.allclose(O.hier_init(pyr, 3.25 * sc, sc), 3.25, rtol=1e-13)
    # zero total confidence gives zero
    assert not np.any(O.hier_init(pyr, b, np.zeros_like(sc)))
    # every vertex gets a finite value even where S c = 0
    c2 = c.copy()
    c2[: c2.size // 2] = 0.0
    sc2, b2 = O.splat(g, c2), O.splat(g, c2 * t)
    y0 = O.hier_init(pyr, b2, sc2)
    assert np.all(np.isfinite(y0)) and np.any(sc2 == 0)
    assert y0.min() >= t.min() - 1e-12 and y0.max() <= t.max() + 1e-12


def test_hier_init_reduces_iterations():
    """Hierarchical init reaches 1e-5 in no more iterations than flat init (Section 4, Fig. precon_init)."""
    p = WL.depth_superres(H=192, W=256, regions=30)
    its = {}
    for init in ("flat", "hier"):
        prm = O.Params(p.sigma_xy, p.sigma_l, p.sigma_uv, p.lam, max_iters=20000,
                       rel_tol=1e-5, init=init)
        sol = O.solve(p.ref, p.target, p.conf, prm)
        its[init] = sol.runs[0].iters
        assert sol.runs[0].true_rel_residual <= 2e-5
    assert its["hier"] < its["flat"]


def _hand_grid(coords):
    """A grid whose level-0 vertices have the given (y, x, l, u, v) coordinates
    (ascending key order), one pixel each."""
    coords = np.asarray(coords, np.int64)
    keys = O.pack_key(coords)
    assert np.all(np.diff(keys) > 0)
    V = coords.shape[0]
    return O.Grid(1, V, keys, coords, np.arange(V), np.ones(V, np.int64),
                  O.neighbours(keys, coords))


def test_hier_init_hand_computed_two_levels():
    """Two vertices under one coarse vertex (K = 1), alpha = 4, beta = 0, by hand
    from the Section 4 formula: w_1 = 4^-1, P(1) = (1, 1 | 2),
    y_v = (b_v + w_1 (b_0 + b_1) / 2) / (s_v + w_1 (s_0 + s_1) / 2)."""
    g = _hand_grid([(0, 0, 0, 0, 0), (0, 1, 0, 0, 0)])
    pyr = O.build_pyramid(g)
    assert pyr.sizes == [2, 1]
    b, sc = np.array([2.0, 3.0]), np.array([1.0, 0.5])
    y = O.hier_init(pyr, b, sc, alpha=4.0, beta=0.0)
    # 2 + 5/8 over 1 + 3/16, and 3 + 5/8 over 1/2 + 3/16
    want = [Fraction(21, 8) / Fraction(19, 16), Fraction(29, 8) / Fraction(11, 16)]
    assert np.allclose(y, [float(w) for w in want], rtol=1e-15, atol=0)


def test_hier_init_hand_computed_three_levels():
    """Three vertices: v0, v1 share a level-1 vertex, v2 has its own; level 2
    is the top (K = 2).  alpha = 2, beta = 0: w = (1, 1/2, 1/4); P(1) at level 1
    is (2, 1), at level 2 it is 3.  b = (1, 0, 4), S c = (1, 0, 2), by hand:
    y_0 = (1 + 1/4 + 5/12) / (1 + 1/4 + 1/4)   = 10/9,
    y_1 = (0 + 1/4 + 5/12) / (0 + 1/4 + 1/4)   = 4/3,
    y_2 = (4 + 2 + 5/12)   / (2 + 1 + 1/4)     = 77/39."""
    g = _hand_grid([(0, 0, 0, 0, 0), (0, 1, 0, 0, 0), (0, 2, 0, 0, 0)])
    pyr = O.build_pyramid(g)
    assert pyr.sizes == [3, 2, 1]
    assert pyr.ones[1].tolist() == [2.0, 1.0] and pyr.ones[2].tolist() == [3.0]
    y = O.hier_init(pyr, np.array([1.0, 0.0, 4.0]), np.array([1.0, 0.0, 2.0]), alpha=2.0,
                    beta=0.0)
    want = [Fraction(10, 9), Fraction(4, 3), Fraction(77, 39)]
    assert np.allclose(y, [float(w) for w in want], rtol=1e-15, atol=0)


@pytest.mark.parametrize("seed,alpha,beta", [(0, 4.0, 0.0), (1, 2.0, 1.0), (2, 1.5, 0.0)])
def test_hier_init_equals_the_dense_pyramid_formula(seed, alpha, beta):
    """hier_init (lift and collapse by parent maps) against the Section 4 formula
    evaluated with explicit pyramid matrices built by brute-force halving of
    the vertex coordinates (supplement Section 2), at finite alpha."""
    p = tiny(seed=seed, H=12, W=16, regions=4, sigma=(3, 40, 40))
    g = O.build_grid(p.ref, p.sigma_xy, p.sigma_l, p.sigma_uv)
    pyr = O.build_pyramid(g)
    assert pyr.K >= 3
    c = p.conf.reshape(-1).astype(float)
    c[::5] = 0.0
    t = p.target[0].reshape(-1).astype(float)
    sc, b = O.splat(g, c), O.splat(g, c * t)
    want = D.hier_init_dense(g.coords, b, sc, alpha, beta)
    got = O.hier_init(pyr, b, sc, alpha=alpha, beta=beta)
    assert np.allclose(got, want, rtol=1e-12, atol=0)


def test_hier_precond_hand_computed_and_limits():
    """M_hier^-1 (Section 4, Eq. hier_precond) on the three-vertex pyramid, by
    hand with alpha = 2, beta = 0 (w = 1, 1/2, 1/4), diag(A) = (1, 2, 4),
    r = (1, 1, 1): the level-1 scalings are w_1 P(1)/P(diag) = (1/2)(2/3),
    (1/2)(1/4) and the top's (1/4)(3/7), so
    z_0 = 1 + 2/3 * 2 ... written out below; large alpha gives Jacobi."""
    g = _hand_grid([(0, 0, 0, 0, 0), (0, 1, 0, 0, 0), (0, 2, 0, 0, 0)])
    pyr = O.build_pyramid(g)
    diag = np.array([1.0, 2.0, 4.0])
    r = np.array([1.0, 1.0, 1.0])
    M = O.HierPrecond(pyr, diag, alpha=2.0, beta=0.0)
    s1 = [Fraction(1, 2) * Fraction(2, 3), Fraction(1, 2) * Fraction(1, 4)]
    s2 = Fraction(1, 4) * Fraction(3, 7)
    top = s2 * 3                      # P(r) at the top is 3
    z = [1 + s1[0] * 2 + top,         # P(r) at v0's level-1 vertex is 2
         Fraction(1, 2) + s1[0] * 2 + top,
         Fraction(1, 4) + s1[1] * 1 + top]
    assert np.allclose(M(r), [float(v) for v in z], rtol=1e-15, atol=0)
    big = O.HierPrecond(pyr, diag, alpha=1e30, beta=0.0)
    assert np.allclose(big(np.array([3.0, -1.0, 2.0])), [3.0, -0.5, 0.5], rtol=1e-14)
    # a zero diagonal gives a zero coefficient, not a division by zero (R22)
    Mz = O.HierPrecond(pyr, np.array([0.0, 0.0, 4.0]), alpha=2.0, beta=0.0)
    assert np.all(np.isfinite(Mz(r)))


@pytest.mark.parametrize("seed", [0, 1])
def test_hier_precond_equals_dense_and_is_spd(seed):
    """The matrix-free M_hier^-1 equals P^T D P built from brute-force pyramid
    matrices; it is symmetric positive definite where diag(A) > 0, and PCG with
    it reaches the dense solution."""
    p = tiny(seed=seed, H=12, W=16, regions=4, sigma=(3, 40, 40), C=1)
    prm = params_of(p, precond="hier", pre_alpha=2.0, pre_beta=1.0)
    g, bs, pyr, S, B, Wh, Alit = dense_problem(p, prm)
    sol = O.solve(p.ref, p.target, p.conf, prm, prepared=(g, bs, pyr))
    Md = D.hier_precond_dense(g.coords, sol.A.diag(), 2.0, 1.0)
    rng = np.random.default_rng(seed)
    for _ in range(3):
        r = rng.normal(size=g.V)
        assert np.allclose(sol.pre(r), Md @ r, rtol=1e-12, atol=1e-14)
    assert np.allclose(Md, Md.T, rtol=0, atol=1e-14)
    assert np.linalg.eigvalsh(Md).min() > 0
    y = D.solve_dense(Alit, sol.b[:, 0])
    assert np.linalg.norm(sol.y[:, 0] - y) <= 1e-9 * np.linalg.norm(y)


def test_hier_precond_reduces_iterations():
    """The hierarchical preconditioner (alpha = 2, beta = 5) reaches 1e-5 in
    fewer PCG iterations than Jacobi on a sparse-confidence interpolation
    problem (Section 4, Fig. precon_init), to the same solution."""
    p = WL.depth_superres(H=192, W=256, regions=30)
    its, ys = {}, {}
    for pre in ("jacobi", "hier"):
        prm = O.Params(p.sigma_xy, p.sigma_l, p.sigma_uv, p.lam, max_iters=20000,
                       rel_tol=1e-8, precond=pre)
        sol = O.solve(p.ref, p.target, p.conf, prm)
        its[pre] = sol.runs[0].iters
        ys[pre] = sol.y[:, 0]
    assert its["hier"] < its["jacobi"]
    # the solution is unique on the grid components that carry confidence
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    g = sol.grid
    ok = g.nbr >= 0
    rows = np.concatenate([np.nonzero(ok[j])[0] for j in range(10)])
    cols = np.concatenate([g.nbr[j][ok[j]] for j in range(10)])
    _, lab = connected_components(coo_matrix((np.ones(rows.size), (rows, cols)),
                                             shape=(g.V, g.V)), directed=False)
    live = (np.bincount(lab, weights=sol.sc) > 0)[lab]
    assert live.sum() > 0.5 * g.V
    d = ys["hier"][live] - ys["jacobi"][live]
    assert np.linalg.norm(d) <= 1e-5 * np.linalg.norm(ys["jacobi"][live])


# --------------------------------------------------------------------------
# PCG behaviour (supplement Algorithm 2)
# --------------------------------------------------------------------------

def test_pcg_energy_decreases_and_stops():
    p = WL.tiny_ramp(seed=0)
    prm = O.Params(p.sigma_xy, p.sigma_l, p.sigma_uv, p.lam, max_iters=500, rel_tol=1e-8)
    sol = O.solve(p.ref, p.target, p.conf, prm, track_energy=True)
    e = np.array(sol.runs[0].energy)
    assert np.all(np.diff(e) <= 1e-12 * np.abs(e[:-1]))
    r = sol.runs[0]
    assert r.rel_residual <= 1e-8 and r.history[-2] > 1e-8
    assert abs(r.true_rel_residual - r.rel_residual) <= 1e-9
    fixed = O.solve(p.ref, p.target, p.conf,
                    O.Params(p.sigma_xy, p.sigma_l, p.sigma_uv, p.lam, max_iters=7, rel_tol=0.0))
    assert fixed.runs[0].iters == 7


def test_multichannel_linearity_and_independence():
    p = tiny(seed=6, C=3, H=16, W=20)
    prm = params_of(p)
    joint = O.solve(p.ref, p.target, p.conf, prm)
    for ch in range(3):
        one = O.solve(p.ref, p.target[ch:ch + 1], p.conf, prm)
        assert np.allclose(one.x[0], joint.x[ch], rtol=0, atol=1e-12)
    combo = (p.target[0].astype(float) + 2.0 * p.target[1].astype(float))[None]
    sol = O.solve(p.ref, combo, p.conf, prm)
    assert np.allclose(sol.x[0], joint.x[0] + 2.0 * joint.x[1], rtol=0, atol=1e-9)


# --------------------------------------------------------------------------
# Backpropagation (Section 3)
# --------------------------------------------------------------------------

def _dense_output(p, prm, target, conf, pre):
    g, bs, pyr = pre
    c = conf.reshape(-1).astype(float)
    S = D.splat_matrix(g.idx, g.V)
    B = D.blur_matrix_bruteforce(g.coords)
    A = D.a_literal(g.m.astype(float), bs.n, B, S @ c, prm.lam)
    out = []
    for ch in range(target.shape[0]):
        b = S @ (c * target[ch].reshape(-1))
        out.append(S.T @ D.solve_dense(A, b))
    return np.stack(out).reshape(target.shape)


def test_gradients_against_finite_differences():
    """dL/dt and dL/dc against FP64 central differences of dense solves, L = <w, x_hat>."""
    p = WL.crop(WL.segmentation(H=64, W=64, regions=8, C=2), 20, 24, 12, 16)
    prm = params_of(p, lam=4.0)
    pre = O.prepare(p.ref, prm)
    sol = O.solve(p.ref, p.target, p.conf, prm, prepared=pre)
    w = WL.random_grad(0, p.C, p.H, p.W).astype(float)
    grads = O.solve_backward(sol, p.target, p.conf, w, prm)
    t = p.target.astype(float)
    c = p.conf.astype(float)
    rng = np.random.default_rng(0)
    picks = rng.choice(p.pixels, size=12, replace=False)
    for flat in picks:
        i, j = divmod(int(flat), p.W)
        for ch in range(p.C):
            h = 1e-6
            tp, tm = t.copy(), t.copy()
            tp[ch, i, j] += h
            tm[ch, i, j] -= h
            fd = (np.sum(w * _dense_output(p, prm, tp, c, pre))
                  - np.sum(w * _dense_output(p, prm, tm, c, pre))) / (2 * h)
            assert abs(fd - grads.grad_t[ch, i, j]) <= 1e-6 * max(1.0, abs(fd))
        h = 1e-5
        cp, cm = c.copy(), c.copy()
        cp[i, j] += h
        cm[i, j] -= h
        fd = (np.sum(w * _dense_output(p, prm, t, cp, pre))
              - np.sum(w * _dense_output(p, prm, t, cm, pre))) / (2 * h)
        assert abs(fd - grads.grad_c[i, j]) <= 1e-6 * max(1.0, abs(fd))
    # adjoint identity <w, x(t + delta) - x(t)> = <dL/dt, delta> (x is linear in t)
    delta = rng.normal(size=t.shape)
    lhs = np.sum(w * (_dense_output(p, prm, t + delta, c, pre) - _dense_output(p, prm, t, c, pre)))
    assert abs(lhs - np.sum(grads.grad_t * delta)) <= 1e-8 * max(1.0, abs(lhs))


# --------------------------------------------------------------------------
# Robust bilateral solver (supplement Section Robustness, Algorithm RBS)
# --------------------------------------------------------------------------

def _with_outliers(p, frac, size, seed):
    """The target with a fraction of pixels moved by +size (gross outliers)."""
    rng = np.random.default_rng(seed)
    t = p.target.copy()
    mask = rng.random(t.shape[1:]) < frac
    t[:, mask] += size
    return t, mask


def test_gm_weight_is_the_irls_weight_of_the_printed_loss():
    """IRLS weights are rho'(e) / e; checked against central differences of
    the printed Geman-McClure loss rho(e) = e^2 / (sigma^2 + e^2)."""
    for sigma in (0.1, 1.0, 7.5):
        e = np.linspace(-5 * sigma, 5 * sigma, 41)
        e = e[np.abs(e) > 1e-3 * sigma]
        h = 1e-6 * sigma
        drho = (O.gm_loss((e + h) ** 2, sigma) - O.gm_loss((e - h) ** 2, sigma)) / (2 * h)
        assert np.allclose(O.gm_weight(e ** 2, sigma), drho / e, rtol=1e-6, atol=0)


def test_robust_one_iteration_is_the_solve():
    p = tiny(seed=3)
    prm = params_of(p)
    r = O.robust_solve(p.ref, p.target, p.conf, prm, sigma_gm=0.2, irls_iters=1)
    plain = O.solve(p.ref, p.target, p.conf, prm)
    assert np.array_equal(r.solution.x, plain.x)
    assert np.array_equal(r.weights[0], p.conf.reshape(-1).astype(np.float64))


def test_robust_objective_decreases():
    """Each IRLS step minimises a quadratic majorizer of the Geman-McClure
    objective, so with exact solves the objective never increases.  The
    solve's data term sum c (x - t)^2 carries no 1/2, so the objective
    majorized is (lam / 4) sum W-hat (x_i - x_j)^2 + sum rho(x - t): the
    printed robust loss with lam / 2.  W-hat is the dense matrix of
    Eq. equiv, independent of the matrix-free operator."""
    p = tiny(seed=4, H=12, W=16, regions=4)
    t, _ = _with_outliers(p, 0.08, 2.0, seed=1)
    prm = params_of(p)
    g, bs, _, S, B, Wh, _ = dense_problem(p, prm)
    sigma = 0.15
    r = O.robust_solve(p.ref, t, p.conf, prm, sigma_gm=sigma, irls_iters=8)
    tt = t.reshape(-1).astype(np.float64)
    F = []
    for c in r.weights:
        x = O.solve(p.ref, t, c.reshape(p.conf.shape), prm).x.reshape(-1)
        smooth = 0.5 * D.pixel_loss(x, tt, np.zeros_like(x), Wh, p.lam)
        F.append(smooth + float(np.sum(O.gm_loss((x - tt) ** 2, sigma))))
    F = np.array(F)
    assert np.all(np.diff(F[1:]) <= 1e-9 * np.abs(F[1:-1])), F
    assert F[-1] < F[1]


def test_robust_large_sigma_is_uniform_confidence():
    """sigma_gm -> inf: every weight tends to 2 / sigma^2, so the second solve
    tends to the plain solve with that uniform confidence (relative change
    O(max e^2 / sigma^2))."""
    p = tiny(seed=5)
    prm = params_of(p)
    sigma = 1e3
    r = O.robust_solve(p.ref, p.target, p.conf, prm, sigma_gm=sigma, irls_iters=2)
    uni = O.solve(p.ref, p.target, np.full(p.conf.shape, 2.0 / sigma ** 2), prm)
    assert np.linalg.norm(r.solution.x - uni.x) <= 1e-5 * np.linalg.norm(uni.x)


def test_robust_rejects_outliers():
    """A piecewise ramp with 5 % gross outliers: the robust solve stays close
    to the plain solve of the target without them, from which the plain
    solve of the corrupted target is pulled away."""
    p = WL.tiny_ramp(seed=6, H=32, W=40, regions=4, sigma=(4, 8, 8), lam=0.5)
    t, mask = _with_outliers(p, 0.05, 3.0, seed=2)
    c = np.ones_like(p.conf)
    prm = params_of(p)
    want = O.solve(p.ref, p.target, c, prm).x[0]
    plain = O.solve(p.ref, t, c, prm).x[0]
    rob = O.robust_solve(p.ref, t, c, prm, sigma_gm=0.1, irls_iters=10).solution.x[0]
    keep = ~mask
    err_plain = np.abs(plain[keep] - want[keep]).mean()
    err_rob = np.abs(rob[keep] - want[keep]).mean()
    assert err_rob < 0.2 * err_plain, (err_rob, err_plain)


# --------------------------------------------------------------------------
# Low-rank reduction of many right-hand sides (supplement Section Multiple
# Output Channels)
# --------------------------------------------------------------------------

def _splat_b(p, prm):
    g, bs, pyr = O.prepare(p.ref, prm)
    c = p.conf.reshape(-1).astype(np.float64)
    B = np.stack([O.splat(g, c * p.target[ch].reshape(-1)) for ch in range(p.C)], axis=1)
    return g, B


def test_lowrank_eps_zero_is_the_full_solve():
    """eps = 0 keeps every row: A^-1 (Q-tilde R-tilde) = A^-1 B exactly."""
    p = WL.segmentation(H=40, W=48, regions=6, C=5)
    prm = params_of(p, rel_tol=1e-12)
    Y, x, lr, _ = O.solve_lowrank(p.ref, p.target, p.conf, prm, 0.0)
    full = O.solve(p.ref, p.target, p.conf, prm)
    assert lr.rank == 5
    assert np.linalg.norm(Y - full.y) <= 1e-9 * np.linalg.norm(full.y)
    assert np.linalg.norm(x - full.x) <= 1e-9 * np.linalg.norm(full.x)


def test_lowrank_exact_rank_is_found_and_solved():
    """Six channels spanned by two: t = 2 for a small eps, and the reduced
    solve equals the full one."""
    p = WL.segmentation(H=40, W=48, regions=6, C=2)
    rng = np.random.default_rng(3)
    mix = rng.normal(size=(6, 2))
    p.target = np.einsum("kc,chw->khw", mix, p.target).astype(np.float32)
    prm = params_of(p, rel_tol=1e-12)
    Y, x, lr, _ = O.solve_lowrank(p.ref, p.target, p.conf, prm, 1e-6)
    full = O.solve(p.ref, p.target, p.conf, prm)
    assert lr.rank == 2
    # the float32 targets are rank 2 up to their rounding (~1e-8)
    assert np.linalg.norm(Y - full.y) <= 1e-6 * np.linalg.norm(full.y)


@pytest.mark.parametrize("eps", [0.01, 0.1, 0.5])
def test_lowrank_drops_at_most_eps_and_keeps_the_fewest_rows(eps):
    """R18: ||B - Q-tilde R-tilde||_F^2 <= eps ||B||_F^2, computed from B
    itself, and one row fewer would drop more than eps; Q-tilde has
    orthonormal columns."""
    p = WL.segmentation(H=48, W=64, regions=8, C=8)
    prm = params_of(p)
    g, B = _splat_b(p, prm)
    lr = O.lowrank_reduce(B, eps)
    nb = np.sum(B ** 2)
    assert np.sum((B - lr.Q @ lr.R) ** 2) <= eps * nb * (1 + 1e-12)
    assert np.allclose(lr.Q.T @ lr.Q, np.eye(lr.rank), atol=1e-12)
    if lr.rank > 0:
        fewer = lr.Q[:, :-1] @ lr.R[:-1]
        assert np.sum((B - fewer) ** 2) > eps * nb


def test_unconfident_components_and_the_inconsistent_adjoint():
    """R21: a grid component without confidence.  Three pixels of unrelated
    colours at sigma_xy = 1 are three isolated vertices; with confidence only
    on the first, two components have none.  The adjoint system is solvable
    only where dL/dx vanishes on them, which a confidence-weighted gradient
    does; otherwise solve_backward refuses."""
    ref = np.array([[[0.0, 1.0, 0.0]], [[0.0, 0.0, 1.0]], [[1.0, 0.0, 0.0]]], np.float32)
    conf = np.array([[1.0, 0.0, 0.0]], np.float32)
    t = np.array([[[0.3, 0.7, 0.9]]], np.float32)
    prm = O.Params(1, 8, 8, 10.0, max_iters=100, rel_tol=1e-12)
    sol = O.solve(ref, t, conf, prm)
    g = sol.grid
    assert g.V == 3 and np.all(g.nbr < 0)
    assert O.unconfident_components(g, sol.sc) == 2
    gx = np.ones((1, 1, 3), np.float32)
    assert O.unconfident_components(g, sol.sc, O.splat(g, gx.reshape(-1))[:, None]) == 2
    with pytest.raises(ValueError):
        O.solve_backward(sol, t, conf, gx, prm)
    og = O.solve_backward(sol, t, conf, gx * conf[None], prm)
    # the one confident isolated vertex: x = t there, so dL/dt = 1 and dL/dc = 0
    assert abs(og.grad_t[0, 0, 0] - 1.0) < 1e-12 and abs(og.grad_c[0, 0]) < 1e-12
