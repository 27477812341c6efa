"""FP64 CPU oracle of the fast bilateral solver (Barron & Poole, "The Fast
Bilateral Solver").  TEST INFRASTRUCTURE ONLY: it exists to check the GPU path
and is imported only by the test-suite, the smoke check and the benchmark's
CPU-baseline leg.  It shares no code, table or helper with the HIP library.

Everything is plain NumPy in float64 (integers in int64), written for a reader
to check against the paper by eye.  Library primitives used as single steps:
``np.unique`` (sorted vertex set), ``np.searchsorted`` (key lookup),
``np.bincount`` (splat sums).  No blocking, fusion or reordering.

Readings of passages where the paper is silent or ambiguous:
  R1  colour space: quantise each channel to 8 bits, then JFIF (BT.601 full
      range) YCbCr in 16.16 fixed point; luma l = Y, chroma (u, v) = (Cb, Cr).
  R2  grid coordinate of a value v at scale s: round half up of v/s, computed
      in integers as floor((2v + s) / 2s); pixel positions are 0-based.
  R3  vertex order: ascending packed key (y, x, l, u, v), 16/16/8/8/8 bits.
  R4  B-bar is the SUM over the five grid dimensions of a [1 2 1] blur, so its
      diagonal is 10 and each application is one 11-point stencil.
  R5  a neighbour missing from the sparse grid contributes 0.
  R6  bistochastization stops when max_v |n_v (B n)_v - m_v| / m_v <= tol, or
      after max_iters updates.
  R7  pyramid: coordinates are halved with floor; K is the first level holding
      a single vertex; k = 0 is the finest level (the grid itself).
  R8  P^T(z) = sum_k S_0^T ... S_{k-1}^T z_k, the exact adjoint of P.
  R9  Jacobi inverse is 0 where diag(A) <= 0; flat init is 0 where S c = 0;
      with zero total confidence every init is 0.
  R10 multi-channel PCG runs one independent PCG per channel; a channel stops
      when its recursive ||r|| / ||b|| <= rel_tol (rel_tol = 0: never), after
      max_iters iterations, when r^T s = 0, or when d^T A d <= 0.
  R11 backward: the adjoint solve uses the same A, preconditioner and init
      operator with b replaced by u = S dL/dx; dL/dc sums the per-channel terms.
  R12 the diagonal of the smoothness term, m - 10 n^2, is evaluated as n o N n,
      its value at the bistochastization fixed point (see Operator).
  R17 robust solver with several channels: the Geman-McClure weight of a pixel
      takes e o e summed over the channels (the confidence is shared); with
      one channel this is the printed weight.
  R18 low-rank reduction, the rank t: the number of kept rows is the smallest
      t whose mass reaches (1 - eps) of the total, so that at most eps of B's
      squared norm is dropped (the printed inequality, read literally, keeps
      at most (1 - eps) and contradicts the stated role of eps).
  R19 low-rank reduction, R-tilde: the first t rows of R', which already is
      R P^T with its rows reordered (applying P^T once more would permute the
      columns twice).
  R21 the backward pass on a grid with a connected component of zero total
      confidence: A restricted to it is a singular graph Laplacian.  If dL/dx
      does not vanish on the component, A g = S dL/dx has no solution and the
      printed gradient is not defined (solve_backward raises); if it does
      (e.g. a confidence-weighted upstream gradient), g there is what PCG
      keeps of its initial state.  The forward solve is always defined
      (b = 0 there).
  R22 hierarchical preconditioner: a pyramid coefficient whose P(diag A) is 0
      (every level-0 vertex below it has a zero diagonal: no neighbours and no
      confidence) contributes 0, as the Jacobi inverse does where diag(A) = 0.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------
# Colour and grid coordinates  (Section 2, Eq. bilateral_affinity; R1, R2)
# ----------------------------------------------------------------------------

# BT.601 full-range (JFIF) coefficients scaled by 2^16 and rounded, each row
# adjusted so luma weights sum to 2^16 and chroma weights sum to 0.
_Y_COEF = (19595, 38470, 7471)
_CB_COEF = (-11058, -21710, 32768)
_CR_COEF = (32768, -27439, -5329)


def quantise8(v: np.ndarray) -> np.ndarray:
    """Round [0,1] values to 8-bit codes: clamp(floor(255 v + 1/2), 0, 255).

    Evaluated in float64 (exact for float32 input); NaN maps to 0."""
    s = np.floor(np.asarray(v, np.float32).astype(np.float64) * 255.0 + 0.5)
    s = np.where(np.isnan(s), 0.0, s)
    return np.clip(s, 0.0, 255.0).astype(np.int64)


def rgb8_to_yuv8(r: np.ndarray, g: np.ndarray, b: np.ndarray):
    """JFIF YCbCr of 8-bit RGB in 16.16 fixed point with round-half-up (R1)."""
    half = 1 << 15
    y = (_Y_COEF[0] * r + _Y_COEF[1] * g + _Y_COEF[2] * b + half) >> 16
    u = (_CB_COEF[0] * r + _CB_COEF[1] * g + _CB_COEF[2] * b + (128 << 16) + half) >> 16
    v = (_CR_COEF[0] * r + _CR_COEF[1] * g + _CR_COEF[2] * b + (128 << 16) + half) >> 16
    return np.clip(y, 0, 255), np.clip(u, 0, 255), np.clip(v, 0, 255)


def grid_coord(v: np.ndarray, s: int) -> np.ndarray:
    """Round half up of v / s in integers (R2)."""
    return (2 * np.asarray(v, np.int64) + s) // (2 * s)


# Packed key: y:16 | x:16 | l:8 | u:8 | v:8, most significant first (R3).
_SHIFT = (40, 24, 16, 8, 0)
_WIDTH = (16, 16, 8, 8, 8)


def pack_key(coords: np.ndarray) -> np.ndarray:
    """coords int64 [N][5] in (y, x, l, u, v) order -> uint64-valued int64 keys."""
    k = np.zeros(coords.shape[0], np.int64)
    for d in range(5):
        k |= coords[:, d].astype(np.int64) << _SHIFT[d]
    return k


def unpack_key(keys: np.ndarray) -> np.ndarray:
    out = np.empty((keys.shape[0], 5), np.int64)
    for d in range(5):
        out[:, d] = (keys >> _SHIFT[d]) & ((1 << _WIDTH[d]) - 1)
    return out


def pixel_coords(ref: np.ndarray, sigma_xy: int, sigma_l: int, sigma_uv: int) -> np.ndarray:
    """Bilateral-space coordinates (y, x, l, u, v) of every pixel, raster order."""
    _, H, W = ref.shape
    q = quantise8(ref)
    l, u, v = rgb8_to_yuv8(q[0], q[1], q[2])
    yy, xx = np.mgrid[0:H, 0:W]
    c = np.stack([grid_coord(yy, sigma_xy), grid_coord(xx, sigma_xy),
                  grid_coord(l, sigma_l), grid_coord(u, sigma_uv),
                  grid_coord(v, sigma_uv)], axis=-1)
    return c.reshape(-1, 5)


# ----------------------------------------------------------------------------
# Simplified bilateral grid  (Section 2, Eq. factorization / equiv; R3-R5)
# ----------------------------------------------------------------------------

@dataclass
class Grid:
    H: int
    W: int
    keys: np.ndarray        # int64 [V], ascending
    coords: np.ndarray      # int64 [V][5]
    idx: np.ndarray         # int64 [P]: the vertex of each pixel (S as an index)
    m: np.ndarray           # int64 [V]: m = S 1, pixels per vertex
    nbr: np.ndarray         # int64 [10][V]: neighbour id or -1; slot 2d = -1, 2d+1 = +1 along dim d

    @property
    def V(self) -> int:
        return self.keys.shape[0]

    @property
    def P(self) -> int:
        return self.idx.shape[0]


def neighbours(keys: np.ndarray, coords: np.ndarray) -> np.ndarray:
    """For every vertex and each of the 10 unit steps, the neighbour's id or -1."""
    V = keys.shape[0]
    nbr = np.full((10, V), -1, np.int64)
    for d in range(5):
        for j, step in enumerate((-1, +1)):
            c = coords[:, d] + step
            valid = (c >= 0) & (c < (1 << _WIDTH[d]))
            want = keys + (step << _SHIFT[d])
            pos = np.searchsorted(keys, want)
            pos_c = np.minimum(pos, V - 1)
            hit = valid & (pos < V) & (keys[pos_c] == want)
            nbr[2 * d + j] = np.where(hit, pos_c, -1)
    return nbr


def build_grid(ref: np.ndarray, sigma_xy: int, sigma_l: int, sigma_uv: int) -> Grid:
    """Splat every pixel onto the single grid vertex holding its coordinates."""
    _, H, W = ref.shape
    coords = pixel_coords(ref, sigma_xy, sigma_l, sigma_uv)
    keys_px = pack_key(coords)
    keys, idx = np.unique(keys_px, return_inverse=True)
    m = np.bincount(idx, minlength=keys.shape[0]).astype(np.int64)
    vc = unpack_key(keys)
    return Grid(H, W, keys, vc, idx.reshape(-1).astype(np.int64), m, neighbours(keys, vc))


def neighbour_sum(g: Grid, z: np.ndarray) -> np.ndarray:
    """N z: the sum of z over the (up to 10) grid neighbours of each vertex (R5)."""
    out = np.zeros(g.V)
    for j in range(10):
        nb = g.nbr[j]
        out = out + np.where(nb >= 0, z[np.maximum(nb, 0)], 0.0)
    return out


def blur(g: Grid, z: np.ndarray) -> np.ndarray:
    """B-bar z = sum over 5 dims of [1 2 1] blurs = 10 z + N z (R4)."""
    return 10.0 * z + neighbour_sum(g, z)


# ----------------------------------------------------------------------------
# Bistochastization  (supplement Algorithm 1; R6)
# ----------------------------------------------------------------------------

@dataclass
class Bistoch:
    n: np.ndarray           # float64 [V]
    iters: int              # number of updates applied
    residual: float         # max relative invariant residual of the returned n


def bistochastize(g: Grid, tol: float = 1e-10, max_iters: int = 200) -> Bistoch:
    m = g.m.astype(np.float64)
    n = np.ones(g.V)
    it = 0
    while True:
        bn = blur(g, n)
        res = float(np.max(np.abs(n * bn - m) / m))
        if res <= tol or it >= max_iters:
            return Bistoch(n, it, res)
        n = np.sqrt(n * m / bn)
        it += 1


# ----------------------------------------------------------------------------
# The bilateral-space problem  (Eq. quad_min; Section 4 Jacobi; R9)
# ----------------------------------------------------------------------------

def splat(g: Grid, pixel_values: np.ndarray) -> np.ndarray:
    """S v for per-pixel values [P] -> per-vertex sums [V]."""
    return np.bincount(g.idx, weights=np.asarray(pixel_values, np.float64).reshape(-1),
                       minlength=g.V)


def slice_(g: Grid, y: np.ndarray) -> np.ndarray:
    """S^T y: each pixel takes its vertex's value."""
    return y[g.idx]


class Operator:
    """A = lam (D_m - D_n B D_n) + diag(S c), applied matrix-free (R12).

    With B = 10 I + N, the smoothness part is lam (diag(m - 10 n^2) - D_n N D_n).
    At the bistochastization fixed point m = n o (B n), i.e. m - 10 n^2 = n o N n,
    and that cancellation-free form is the one used for the diagonal, so that
        A = lam (diag(n o N n) - D_n N D_n) + diag(S c),
    a graph Laplacian with edge weights lam n_u n_v plus the data diagonal: exactly
    symmetric positive semi-definite, with an exactly zero row for a vertex that
    has neither neighbours nor confidence.  It differs from the literal formula
    by lam * m * (bistochastization residual)."""

    def __init__(self, g: Grid, n: np.ndarray, sc: np.ndarray, lam: float):
        self.g, self.n, self.sc, self.lam = g, n, sc, float(lam)
        self.m = g.m.astype(np.float64)
        self.nn = n * neighbour_sum(g, n)         # = m - 10 n^2 at the fixed point

    def __call__(self, z: np.ndarray) -> np.ndarray:
        n = self.n
        return self.diag() * z - self.lam * n * neighbour_sum(self.g, n * z)

    def literal(self, z: np.ndarray) -> np.ndarray:
        """The paper's formula as printed: lam (m z - n o B(n o z)) + Sc z."""
        n = self.n
        return self.lam * (self.m * z - n * blur(self.g, n * z)) + self.sc * z

    def diag(self) -> np.ndarray:
        """diag(A) = lam (m - n^2 B_diag) + S c, evaluated as lam n o N n + S c."""
        return self.lam * self.nn + self.sc

    def jacobi_inverse(self) -> np.ndarray:
        d = self.diag()
        return np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)


def flat_init(b: np.ndarray, sc: np.ndarray) -> np.ndarray:
    """y_flat = S(c t) / S(c), 0 where S(c) = 0 (Eq. flat_init; R9)."""
    return np.where(sc > 0, b / np.where(sc > 0, sc, 1.0), 0.0)


# ----------------------------------------------------------------------------
# Bilateral pyramid  (supplement Section 2; Section 4 hierarchical init; R7, R8)
# ----------------------------------------------------------------------------

@dataclass
class Pyramid:
    parents: list           # parents[k]: int64 [V_k] -> id at level k+1
    sizes: list             # V_0 .. V_K
    ones: list              # P(1) per level (float64)

    @property
    def K(self) -> int:
        return len(self.parents)


def build_pyramid(g: Grid) -> Pyramid:
    coords = g.coords
    parents, sizes = [], [g.V]
    while coords.shape[0] > 1:
        half = coords >> 1
        keys, inv = np.unique(pack_key(half), return_inverse=True)
        parents.append(inv.reshape(-1).astype(np.int64))
        coords = unpack_key(keys)
        sizes.append(coords.shape[0])
    pyr = Pyramid(parents, sizes, [])
    pyr.ones = lift(pyr, np.ones(g.V))
    return pyr


def lift(pyr: Pyramid, y: np.ndarray) -> list:
    """P(y) = [y, S_0 y, S_1 S_0 y, ...], finest first, built bottom-up."""
    out = [np.asarray(y, np.float64)]
    for k, par in enumerate(pyr.parents):
        out.append(np.bincount(par, weights=out[-1], minlength=pyr.sizes[k + 1]))
    return out


def collapse(pyr: Pyramid, z: list) -> np.ndarray:
    """P^T(z) = sum_k S_0^T ... S_{k-1}^T z_k, evaluated top-down."""
    acc = np.asarray(z[pyr.K], np.float64)
    for k in range(pyr.K - 1, -1, -1):
        acc = z[k] + acc[pyr.parents[k]]
    return acc


def level_weights(pyr: Pyramid, alpha: float, beta: float) -> list:
    """z_weight: 1 at k = 0, alpha^-(beta + k) at coarser levels k >= 1."""
    return [1.0] + [float(alpha) ** (-(beta + k)) for k in range(1, pyr.K + 1)]


class HierPrecond:
    """M_hier^-1(r) = P^T(w o P(1) o P(r) / P(diag A))  (Section 4,
    Eq. hier_precond): lift r into pyramid space, scale every coefficient by
    its level weight times the number of vertices under it over the sum of
    diag(A) under it, collapse.  At level 0 the scaling is 1 / diag(A), so
    large alpha or beta leave the Jacobi preconditioner.  A coefficient with
    P(diag A) = 0 contributes 0 (R22).  P^T D P with D >= 0 diagonal:
    symmetric positive semi-definite."""

    def __init__(self, pyr: Pyramid, diag: np.ndarray, alpha: float = 2.0, beta: float = 5.0):
        self.pyr = pyr
        w = level_weights(pyr, alpha, beta)
        self.scale = []
        for k, (pd, o) in enumerate(zip(lift(pyr, diag), pyr.ones)):
            self.scale.append(np.where(pd > 0, w[k] * o / np.where(pd > 0, pd, 1.0), 0.0))

    def __call__(self, r: np.ndarray) -> np.ndarray:
        z = [s * pr for s, pr in zip(self.scale, lift(self.pyr, r))]
        return collapse(self.pyr, z)


def hier_init(pyr: Pyramid, b: np.ndarray, sc: np.ndarray, alpha: float = 4.0,
              beta: float = 0.0) -> np.ndarray:
    """Push-pull init  P^T(w P(b) / P(1)) / P^T(w P(Sc) / P(1))  (Section 4)."""
    if not np.sum(sc) > 0:
        return np.zeros_like(b, dtype=np.float64)
    w = level_weights(pyr, alpha, beta)
    den = collapse(pyr, [w[k] * s / o for k, (s, o) in
                         enumerate(zip(lift(pyr, sc), pyr.ones))])
    num = collapse(pyr, [w[k] * s / o for k, (s, o) in
                         enumerate(zip(lift(pyr, b), pyr.ones))])
    return num / den


# ----------------------------------------------------------------------------
# Preconditioned conjugate gradients  (supplement Algorithm 2; R10)
# ----------------------------------------------------------------------------

@dataclass
class PCGResult:
    y: np.ndarray
    iters: int
    rel_residual: float           # recursive ||r|| / ||b|| at exit
    true_rel_residual: float      # ||b - A y|| / ||b|| at exit
    history: list = field(default_factory=list)    # recursive relative residuals
    alphas: list = field(default_factory=list)
    betas: list = field(default_factory=list)
    energy: list = field(default_factory=list)     # 1/2 y^T A y - b^T y per iterate


def pcg(A, b: np.ndarray, y0: np.ndarray, minv, max_iters: int,
        rel_tol: float, track_energy: bool = False) -> PCGResult:
    """Shewchuk's PCG (B3) on one right-hand side, with the stopping rule R10.
    `minv` is the Jacobi inverse (a vector, applied element-wise) or a
    preconditioner applied as a function (HierPrecond)."""
    apply_m = minv if callable(minv) else (lambda r: minv * r)
    y = np.array(y0, np.float64)
    b = np.asarray(b, np.float64)
    bnorm = float(np.sqrt(b @ b))
    if bnorm == 0.0:
        return PCGResult(y, 0, 0.0, 0.0)
    r = b - A(y)
    d = apply_m(r)
    rho = float(r @ d)
    res = float(np.sqrt(r @ r)) / bnorm
    out = PCGResult(y, 0, res, 0.0, [res])
    if track_energy:
        out.energy.append(0.5 * y @ A(y) - b @ y)
    i = 0
    while i < max_iters and res > rel_tol and rho != 0.0:
        q = A(d)
        dq = float(d @ q)
        if not dq > 0.0:
            break
        alpha = rho / dq
        y = y + alpha * d
        r = r - alpha * q
        s = apply_m(r)
        rho_old, rho = rho, float(r @ s)
        beta = rho / rho_old
        d = s + beta * d
        i += 1
        res = float(np.sqrt(r @ r)) / bnorm
        out.history.append(res)
        out.alphas.append(alpha)
        out.betas.append(beta)
        if track_energy:
            out.energy.append(0.5 * y @ A(y) - b @ y)
    tr = b - A(y)
    out.y, out.iters, out.rel_residual = y, i, res
    out.true_rel_residual = float(np.sqrt(tr @ tr)) / bnorm
    return out


# ----------------------------------------------------------------------------
# The solver and its backward pass  (Sections 2-4; R9-R11)
# ----------------------------------------------------------------------------

@dataclass
class Params:
    sigma_xy: int
    sigma_l: int
    sigma_uv: int
    lam: float
    max_iters: int = 25
    rel_tol: float = 0.0
    init: str = "hier"            # "hier" | "flat"
    init_alpha: float = 4.0
    init_beta: float = 0.0
    precond: str = "jacobi"       # "jacobi" | "hier"
    pre_alpha: float = 2.0
    pre_beta: float = 5.0
    bist_tol: float = 1e-10
    bist_max_iters: int = 200


@dataclass
class Solution:
    grid: Grid
    bist: Bistoch
    pyr: Pyramid
    A: Operator
    minv: np.ndarray
    sc: np.ndarray
    b: np.ndarray                 # [V][C]
    y0: np.ndarray                # [V][C]
    y: np.ndarray                 # [V][C]
    x: np.ndarray                 # [C][H][W]
    runs: list                    # PCGResult per channel
    pre: object = None            # the preconditioner PCG applied (minv or a HierPrecond)


def initial_state(sol_pyr: Pyramid, b: np.ndarray, sc: np.ndarray, p: Params) -> np.ndarray:
    cols = []
    for ch in range(b.shape[1]):
        if p.init == "flat":
            cols.append(flat_init(b[:, ch], sc) if np.sum(sc) > 0 else np.zeros(b.shape[0]))
        else:
            cols.append(hier_init(sol_pyr, b[:, ch], sc, p.init_alpha, p.init_beta))
    return np.stack(cols, axis=1)


def prepare(ref: np.ndarray, p: Params):
    """Problem construction shared by the forward and backward passes."""
    g = build_grid(ref, p.sigma_xy, p.sigma_l, p.sigma_uv)
    bs = bistochastize(g, p.bist_tol, p.bist_max_iters)
    pyr = build_pyramid(g)
    return g, bs, pyr


def solve(ref: np.ndarray, target: np.ndarray, conf: np.ndarray, p: Params,
          prepared=None, track_energy: bool = False) -> Solution:
    """x_hat = S^T A^{-1} b with A, b from Eq. quad_min, solved by PCG."""
    g, bs, pyr = prepared if prepared is not None else prepare(ref, p)
    C = target.shape[0]
    c = np.asarray(conf, np.float64).reshape(-1)
    t = np.asarray(target, np.float64).reshape(C, -1)
    sc = splat(g, c)
    b = np.stack([splat(g, c * t[ch]) for ch in range(C)], axis=1)
    A = Operator(g, bs.n, sc, p.lam)
    minv = A.jacobi_inverse()
    pre = preconditioner(pyr, A, minv, p)
    y0 = initial_state(pyr, b, sc, p)
    runs = [pcg(A, b[:, ch], y0[:, ch], pre, p.max_iters, p.rel_tol, track_energy)
            for ch in range(C)]
    y = np.stack([r.y for r in runs], axis=1)
    x = np.stack([slice_(g, y[:, ch]) for ch in range(C)]).reshape(C, g.H, g.W)
    return Solution(g, bs, pyr, A, minv, sc, b, y0, y, x, runs, pre)


def preconditioner(pyr: Pyramid, A: Operator, minv: np.ndarray, p: Params):
    """The Jacobi inverse, or M_hier^-1 with (pre_alpha, pre_beta) (Section 4)."""
    if p.precond == "jacobi":
        return minv
    if p.precond == "hier":
        return HierPrecond(pyr, A.diag(), p.pre_alpha, p.pre_beta)
    raise ValueError("precond must be 'jacobi' or 'hier'")


@dataclass
class Gradients:
    grad_t: np.ndarray            # [C][H][W]
    grad_c: np.ndarray            # [H][W]
    u: np.ndarray                 # [V][C]  S dL/dx
    gb: np.ndarray                # [V][C]  dL/db = A^{-1} u
    runs: list


def unconfident_components(g: Grid, sc: np.ndarray, u: np.ndarray | None = None) -> int:
    """Number of connected components of the grid (vertices joined by blur
    neighbours) whose total confidence S c is zero, where A restricted to the
    component is a singular graph Laplacian (R21); with u [V][C], only those
    on which u does not vanish, where A g = u has no solution.  Labels by
    scipy's connected components."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    rows, cols = [], []
    for j in range(10):
        ok = g.nbr[j] >= 0
        rows.append(np.nonzero(ok)[0])
        cols.append(g.nbr[j][ok])
    r = np.concatenate(rows)
    adj = coo_matrix((np.ones(r.size), (r, np.concatenate(cols))), shape=(g.V, g.V))
    n, lab = connected_components(adj, directed=False)
    bad = np.bincount(lab, weights=np.asarray(sc, np.float64), minlength=n) == 0.0
    if u is not None:
        mass = np.bincount(lab, weights=np.abs(np.asarray(u, np.float64)).reshape(g.V, -1)
                           .sum(axis=1), minlength=n)
        bad &= mass > 0.0
    return int(np.count_nonzero(bad))


def solve_backward(sol: Solution, target: np.ndarray, conf: np.ndarray,
                   grad_x: np.ndarray, p: Params, y_hat: np.ndarray | None = None
                   ) -> Gradients:
    """(dL/dt, dL/dc) from dL/dx (Section 3):
    dL/db = A^{-1} S dL/dx,  dL/ddiag(A) = -dL/db o y_hat,
    dL/dt = c o S^T dL/db,   dL/dc = S^T dL/ddiag(A) + (S^T dL/db) o t.
    A component of the grid without confidence makes A singular (R21): the
    adjoint system is solvable only if dL/dx vanishes on it (a confidence-
    weighted upstream gradient does), and dL/db there is then fixed by the
    initial state; otherwise this raises ValueError."""
    g = sol.grid
    C = target.shape[0]
    gx = np.asarray(grad_x, np.float64).reshape(C, -1)
    t = np.asarray(target, np.float64).reshape(C, -1)
    c = np.asarray(conf, np.float64).reshape(-1)
    yh = sol.y if y_hat is None else np.asarray(y_hat, np.float64)
    u = np.stack([splat(g, gx[ch]) for ch in range(C)], axis=1)
    if unconfident_components(g, sol.sc, u):
        raise ValueError("A g = S dL/dx has no solution: dL/dx does not vanish on a connected "
                         "component of the grid without confidence (R21)")
    u0 = initial_state(sol.pyr, u, sol.sc, p)
    pre = preconditioner(sol.pyr, sol.A, sol.minv, p)
    runs = [pcg(sol.A, u[:, ch], u0[:, ch], pre, p.max_iters, p.rel_tol)
            for ch in range(C)]
    gb = np.stack([r.y for r in runs], axis=1)
    grad_t = np.empty_like(t)
    grad_c = np.zeros_like(c)
    for ch in range(C):
        sgb = slice_(g, gb[:, ch])
        grad_t[ch] = c * sgb
        grad_c += slice_(g, -gb[:, ch] * yh[:, ch]) + sgb * t[ch]
    return Gradients(grad_t.reshape(C, g.H, g.W), grad_c.reshape(g.H, g.W), u, gb, runs)


def true_relative_residual(A: Operator, b: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Per channel ||b - A y|| / ||b|| for a given bilateral-space solution (any size)."""
    b = np.asarray(b, np.float64)
    y = np.asarray(y, np.float64)
    out = []
    for ch in range(b.shape[1]):
        r = b[:, ch] - A(y[:, ch])
        nb = float(np.sqrt(b[:, ch] @ b[:, ch]))
        out.append(float(np.sqrt(r @ r)) / nb if nb > 0 else 0.0)
    return np.array(out)


# ----------------------------------------------------------------------------
# The robust bilateral solver  (supplement Section Robustness, Algorithm RBS;
# R17)
# ----------------------------------------------------------------------------

def gm_weight(e2: np.ndarray, sigma_gm: float) -> np.ndarray:
    """IRLS weight of the Geman-McClure loss for squared errors e2:
    2 sigma^2 / (sigma^2 + e2)^2."""
    s2 = float(sigma_gm) ** 2
    return 2.0 * s2 / (s2 + np.asarray(e2, np.float64)) ** 2


def gm_loss(e2: np.ndarray, sigma_gm: float) -> np.ndarray:
    """Geman-McClure loss of squared errors e2: e2 / (sigma^2 + e2)."""
    e2 = np.asarray(e2, np.float64)
    return e2 / (float(sigma_gm) ** 2 + e2)


@dataclass
class RobustSolution:
    solution: Solution            # the last solve: x_hat and its state
    weights: list                 # the confidence of every solve, [P] each (first: c_init)


def robust_solve(ref: np.ndarray, target: np.ndarray, conf_init: np.ndarray, p: Params,
                 sigma_gm: float, irls_iters: int, prepared=None) -> RobustSolution:
    """Algorithm RBS: solve with the current confidence, then replace the
    confidence by the Geman-McClure weights of the solution's errors; repeat
    irls_iters times (>= 1) and return the last solve."""
    if irls_iters < 1:
        raise ValueError("irls_iters must be >= 1")
    prepared = prepared if prepared is not None else prepare(ref, p)
    C = target.shape[0]
    t = np.asarray(target, np.float64).reshape(C, -1)
    c = np.asarray(conf_init, np.float64).reshape(-1)
    weights = []
    sol = None
    for _ in range(irls_iters):
        weights.append(c)
        sol = solve(ref, target, c.reshape(conf_init.shape), p, prepared=prepared)
        e2 = np.sum((sol.x.reshape(C, -1) - t) ** 2, axis=0)
        c = gm_weight(e2, sigma_gm)
    return RobustSolution(sol, weights)


# ----------------------------------------------------------------------------
# Low-rank reduction of many right-hand sides  (supplement Section Multiple
# Output Channels; R18, R19)
# ----------------------------------------------------------------------------

@dataclass
class LowRank:
    Q: np.ndarray                 # [V][t] Q-tilde, orthonormal columns
    R: np.ndarray                 # [t][C] R-tilde
    rank: int                     # t
    mass: np.ndarray              # row masses of R', non-increasing


def lowrank_reduce(B: np.ndarray, eps: float) -> LowRank:
    """B P = Q R (rank-revealing QR with column pivoting), R' = R P^T with its
    rows sorted by non-increasing squared norm (the columns of Q alike), and
    the smallest t whose rows hold (1 - eps) of the mass."""
    import scipy.linalg
    B = np.asarray(B, np.float64)
    Q, R, piv = scipy.linalg.qr(B, mode="economic", pivoting=True)
    RPt = np.empty_like(R)
    RPt[:, piv] = R
    mass = np.sum(RPt ** 2, axis=1)
    order = np.argsort(-mass, kind="stable")
    mass = mass[order]
    total = float(np.sum(mass))
    if total == 0.0:
        return LowRank(Q[:, :0], RPt[:0], 0, mass)
    t = int(np.searchsorted(np.cumsum(mass), (1.0 - eps) * total) + 1)
    t = min(t, mass.shape[0])
    return LowRank(Q[:, order[:t]], RPt[order[:t]], t, mass)


def solve_lowrank(ref: np.ndarray, target: np.ndarray, conf: np.ndarray, p: Params,
                  eps: float, prepared=None):
    """Y = (A^-1 Q-tilde) R-tilde: the reduced system A Z = Q-tilde solved by
    the same initialisation and PCG as every other right-hand side, then
    expanded.  Returns (Y [V][C], x [C][H][W], LowRank, PCG runs of Z)."""
    g, bs, pyr = prepared if prepared is not None else prepare(ref, p)
    C = target.shape[0]
    c = np.asarray(conf, np.float64).reshape(-1)
    t = np.asarray(target, np.float64).reshape(C, -1)
    sc = splat(g, c)
    B = np.stack([splat(g, c * t[ch]) for ch in range(C)], axis=1)
    lr = lowrank_reduce(B, eps)
    A = Operator(g, bs.n, sc, p.lam)
    pre = preconditioner(pyr, A, A.jacobi_inverse(), p)
    runs = []
    Z = np.zeros((g.V, lr.rank))
    if lr.rank:
        Z0 = initial_state(pyr, lr.Q, sc, p)
        runs = [pcg(A, lr.Q[:, j], Z0[:, j], pre, p.max_iters, p.rel_tol)
                for j in range(lr.rank)]
        Z = np.stack([r.y for r in runs], axis=1)
    Y = Z @ lr.R if lr.rank else np.zeros((g.V, C))
    x = np.stack([slice_(g, Y[:, ch]) for ch in range(C)]).reshape(C, g.H, g.W)
    return Y, x, lr, runs
