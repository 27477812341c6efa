"""FP64 CPU oracle of the domain-transform post-process and of the
variance-based initial confidence of the robust solver.  TEST INFRASTRUCTURE
ONLY: imported by the test-suite, the smoke check and the benchmark's
CPU-baseline leg, never by the product path.  It shares no code with the HIP
library.

The paper smooths the solver's output with the recursive formulation of the
domain transform of Gastal and Oliveira (2011) (Section 4, the paragraph on
post-processing; spatial and range bandwidths sigma'_xy and sigma'_rgb), and
builds the robust solver's initial confidence from an edge-aware variance of
the input depth computed with the same filter (supplement Section Robustness,
Eq. for V and c_init).  The filter itself is the published recursive filter,
written here from its definition:

  * the domain transform of a line of the guide I is
        ct(x) = sum over the samples up to x of  1 + (s_s / s_r) ||I(x) - I(x-1)||_1,
    so two neighbouring samples lie d = 1 + (s_s / s_r) sum_c |I_c(x) - I_c(x-1)|
    apart in the transformed domain;
  * a 1-D pass runs the first-order recursion  J[x] = (1 - a^d[x]) I[x] + a^d[x] J[x-1]
    left to right, then the same recursion right to left on its output, each
    with feedback a = exp(-sqrt(2) / sigma);
  * N iterations each run a horizontal then a vertical pass; iteration i
    (1-based) uses sigma_i = s_s sqrt(3) 2^(N-i) / sqrt(4^N - 1), so that the
    variances of the iterations add up to s_s^2.

Readings (R24-R26 of the design notes):
  R24 the guide is the reference's 8-bit RGB codes (the solver's quantisation,
      clamp(floor(255 v + 1/2), 0, 255)); s_r is in those units, as the
      paper's DT bandwidths (e.g. sigma_r = 64) are.
  R25 N = 3 iterations (the paper gives none; three is the filter's usual
      choice); the first sample of every line passes a recursion unchanged.
  R26 V = DT(Z^2) - DT(Z)^2 is a variance: values below 0 from rounding are
      taken as 0, so c_init = exp(-V / (2 sigma_dt^2)) <= 1; the leftmost
      `zero_cols` columns of c_init are 0 (the paper uses 80 on its stereo
      pairs).

Everything is NumPy float64.  A recursion runs as a Python loop along the line,
with NumPy over all lines at once.
"""
from __future__ import annotations

import math

import numpy as np

from oracle.bilateral import quantise8

DEFAULT_ITERS = 3


def guide_codes(ref: np.ndarray) -> np.ndarray:
    """The guide: 8-bit codes of the reference [3][H][W] (R24), int64."""
    return quantise8(np.asarray(ref, np.float32))


def domain_steps(codes: np.ndarray, sigma_s: float, sigma_r: float):
    """Distances in the transformed domain between neighbouring samples:
    (dh, dv), float64 [H][W].  dh[y, x] lies between (y, x-1) and (y, x),
    dv[y, x] between (y-1, x) and (y, x); dh[:, 0] and dv[0, :] are unused
    (set to 0)."""
    c = np.asarray(codes, np.int64)
    H, W = c.shape[1], c.shape[2]
    dh = np.zeros((H, W))
    dv = np.zeros((H, W))
    k = float(sigma_s) / float(sigma_r)
    dh[:, 1:] = 1.0 + k * np.abs(np.diff(c, axis=2)).sum(axis=0)
    dv[1:, :] = 1.0 + k * np.abs(np.diff(c, axis=1)).sum(axis=0)
    return dh, dv


def iteration_sigmas(sigma_s: float, iters: int) -> list:
    """sigma_i of iterations i = 1..N: s_s sqrt(3) 2^(N-i) / sqrt(4^N - 1)."""
    N = int(iters)
    return [float(sigma_s) * math.sqrt(3.0) * 2.0 ** (N - i) / math.sqrt(4.0 ** N - 1.0)
            for i in range(1, N + 1)]


def recursive_pass(J: np.ndarray, d: np.ndarray, sigma: float, axis: int) -> np.ndarray:
    """One 1-D pass along `axis` (-1: rows, -2: columns) of J [..][H][W]:
    the causal recursion, then the anti-causal one, with feedback
    a^d, a = exp(-sqrt(2) / sigma); d as domain_steps returns it."""
    a = math.exp(-math.sqrt(2.0) / float(sigma))
    J = np.array(J, np.float64, copy=True)
    J = np.moveaxis(J, axis, -1)
    w = np.moveaxis(a ** np.asarray(d, np.float64), axis, -1)   # w[..., x]: edge (x-1, x)
    L = J.shape[-1]
    for x in range(1, L):                     # left to right
        J[..., x] = (1.0 - w[..., x]) * J[..., x] + w[..., x] * J[..., x - 1]
    for x in range(L - 2, -1, -1):            # right to left, edge (x, x+1)
        J[..., x] = (1.0 - w[..., x + 1]) * J[..., x] + w[..., x + 1] * J[..., x + 1]
    return np.moveaxis(J, -1, axis)


def domain_transform(ref: np.ndarray, x: np.ndarray, sigma_s: float, sigma_r: float,
                     iters: int = DEFAULT_ITERS) -> np.ndarray:
    """The recursive-filter domain transform of x [C][H][W] guided by the
    reference [3][H][W]: N iterations of a horizontal then a vertical pass."""
    dh, dv = domain_steps(guide_codes(ref), sigma_s, sigma_r)
    J = np.asarray(x, np.float64)
    for s in iteration_sigmas(sigma_s, iters):
        J = recursive_pass(J, dh, s, axis=-1)
        J = recursive_pass(J, dv, s, axis=-2)
    return J


def dt_confidence(ref: np.ndarray, z: np.ndarray, sigma_s: float, sigma_r: float,
                  sigma_dt: float, zero_cols: int = 0,
                  iters: int = DEFAULT_ITERS) -> np.ndarray:
    """c_init = exp(-V / (2 sigma_dt^2)) with the edge-aware variance
    V = DT(Z^2) - DT(Z)^2 of z [H][W] (R26); the leftmost zero_cols columns 0."""
    z = np.asarray(z, np.float64)
    m1 = domain_transform(ref, z[None], sigma_s, sigma_r, iters)[0]
    m2 = domain_transform(ref, (z * z)[None], sigma_s, sigma_r, iters)[0]
    V = np.maximum(m2 - m1 * m1, 0.0)
    c = np.exp(-V / (2.0 * float(sigma_dt) ** 2))
    c[:, : max(0, int(zero_cols))] = 0.0
    return c
