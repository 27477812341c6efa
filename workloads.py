"""Seeded synthetic workloads for the bilateral solver.

These generators stand in for the paper's stereo, depth-super-resolution,
colorization and segmentation inputs (Section 4; supplement Section 5), whose
datasets are not available.  They produce reference images, targets and
confidences of the paper's shapes and value ranges.  This module holds none of
the solver's arithmetic: it is shared by the FP64 oracle's tests, the GPU
parity tests, the smoke check and the benchmark, so that both sides see the
same bytes.

Every generator is a pure function of its arguments and its seed
(``numpy.random.default_rng(seed)``).  Images are planar float32:
reference ``[3][H][W]`` in [0, 1], target ``[C][H][W]``, confidence ``[H][W]``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial import cKDTree


@dataclass
class Problem:
    """One solver input: reference, target, confidence and parameters."""
    name: str
    ref: np.ndarray            # float32 [3][H][W] in [0,1]
    target: np.ndarray         # float32 [C][H][W]
    conf: np.ndarray           # float32 [H][W], >= 0
    sigma_xy: int
    sigma_l: int
    sigma_uv: int
    lam: float
    max_iters: int
    rel_tol: float             # 0 means: run exactly max_iters iterations
    extra: dict = field(default_factory=dict)

    @property
    def H(self) -> int:
        return self.ref.shape[1]

    @property
    def W(self) -> int:
        return self.ref.shape[2]

    @property
    def C(self) -> int:
        return self.target.shape[0]

    @property
    def pixels(self) -> int:
        return self.H * self.W


def voronoi_labels(rng: np.random.Generator, H: int, W: int, regions: int) -> np.ndarray:
    """Label map of ``regions`` Voronoi cells with uniformly placed seeds.

    Seeds are continuous, so exact distance ties have probability zero.
    """
    seeds = np.stack([rng.uniform(0, W, regions), rng.uniform(0, H, regions)], axis=1)
    yy, xx = np.mgrid[0:H, 0:W]
    pts = np.stack([xx.ravel() + 0.5, yy.ravel() + 0.5], axis=1)
    _, lab = cKDTree(seeds).query(pts, k=1)
    return lab.reshape(H, W).astype(np.int64)


def voronoi_reference(rng: np.random.Generator, H: int, W: int, regions: int,
                      noise: float = 0.02):
    """Reference RGB: per-region uniform colour plus N(0, noise^2), clamped to [0,1]."""
    lab = voronoi_labels(rng, H, W, regions)
    colours = rng.uniform(0.0, 1.0, size=(regions, 3))
    img = colours[lab].transpose(2, 0, 1)
    img = img + rng.normal(0.0, noise, size=img.shape)
    return np.clip(img, 0.0, 1.0).astype(np.float32), lab


def _ramp_target(rng, lab, regions, H, W, span=0.5, noise=0.05):
    """Per-region linear ramp a + gx*x + gy*y with |gx|W + |gy|H <= span, plus noise."""
    a = rng.uniform(0.0, 1.0, regions)
    gx = rng.uniform(-1.0, 1.0, regions) * (0.5 * span / W)
    gy = rng.uniform(-1.0, 1.0, regions) * (0.5 * span / H)
    yy, xx = np.mgrid[0:H, 0:W]
    t = a[lab] + gx[lab] * xx + gy[lab] * yy
    t = t + rng.normal(0.0, noise, size=t.shape)
    return t.astype(np.float32)


def _box_mean(img: np.ndarray, k: int) -> np.ndarray:
    """k x k box mean with replicate padding, per leading channel (input preparation only)."""
    r = k // 2
    pad = np.pad(img, ((0, 0), (r, r), (r, r)), mode="edge")
    cs = np.cumsum(np.cumsum(pad, axis=1), axis=2)
    cs = np.pad(cs, ((0, 0), (1, 0), (1, 0)))
    H, W = img.shape[1:]
    s = cs[:, k:k + H, k:k + W] - cs[:, 0:H, k:k + W] - cs[:, k:k + H, 0:W] + cs[:, 0:H, 0:W]
    return (s / (k * k)).astype(np.float32)


def tiny_ramp(seed: int = 0, H: int = 48, W: int = 64, regions: int = 12,
              sigma=(8, 4, 4), lam: float = 128.0, rel_tol: float = 1e-5,
              max_iters: int = 2000, channels: int = 1) -> Problem:
    """Plain solve on a 64x48 Voronoi reference with a per-region ramp target."""
    rng = np.random.default_rng(seed)
    ref, lab = voronoi_reference(rng, H, W, regions)
    t = np.stack([_ramp_target(rng, lab, regions, H, W) for _ in range(channels)])
    conf = rng.uniform(0.0, 1.0, size=(H, W)).astype(np.float32)
    return Problem("ramp_%dx%d" % (W, H), ref, t, conf, sigma[0], sigma[1], sigma[2],
                   lam, max_iters, rel_tol)


def strip(seed: int = 0, H: int = 3, W: int = 32800, sigma=(1, 8, 8), lam: float = 128.0,
          rel_tol: float = 1e-6, max_iters: int = 20000) -> Problem:
    """A wide strip whose reference is constant down each column (random
    column colours), so at sigma_xy = 1 every pixel is a vertex whose
    neighbour one row down lies W vertex ids away.  Ramp target with noise,
    confidence U[0.2, 1]."""
    rng = np.random.default_rng(seed)
    cols = rng.uniform(0.0, 1.0, size=(3, 1, W)).astype(np.float32)
    ref = np.ascontiguousarray(np.broadcast_to(cols, (3, H, W)))
    x = np.arange(W, dtype=np.float64)[None, :] / W
    y = np.arange(H, dtype=np.float64)[:, None] / max(H, 1)
    t = (0.3 + 0.4 * x + 0.2 * y + rng.normal(0.0, 0.05, size=(H, W)))[None].astype(np.float32)
    conf = rng.uniform(0.2, 1.0, size=(H, W)).astype(np.float32)
    return Problem("strip_%dx%d" % (W, H), ref, t, conf, sigma[0], sigma[1], sigma[2],
                   lam, max_iters, rel_tol)


def stereo_refine(seed: int = 0, H: int = 768, W: int = 1024, regions: int = 300,
                  sigma=(16, 8, 8), lam: float = 128.0, iters: int = 25) -> Problem:
    """Stereo-refinement shape: piecewise-planar disparity in [0,256], 10% outliers."""
    rng = np.random.default_rng(seed)
    ref, lab = voronoi_reference(rng, H, W, regions)
    a = rng.uniform(0.0, 256.0, regions)
    gx = rng.uniform(-1.0, 1.0, regions) * (64.0 / W)
    gy = rng.uniform(-1.0, 1.0, regions) * (64.0 / H)
    yy, xx = np.mgrid[0:H, 0:W]
    t = np.clip(a[lab] + gx[lab] * (xx - W / 2) + gy[lab] * (yy - H / 2), 0.0, 256.0)
    outlier = rng.uniform(0.0, 1.0, size=(H, W)) < 0.10
    t = np.where(outlier, rng.uniform(0.0, 256.0, size=(H, W)), t)
    conf = np.where(outlier, 0.1, rng.uniform(0.5, 1.0, size=(H, W)))
    return Problem("stereo_%dx%d" % (W, H), ref, t[None].astype(np.float32),
                   conf.astype(np.float32), sigma[0], sigma[1], sigma[2], lam,
                   iters, 0.0)


def depth_superres(seed: int = 0, H: int = 1536, W: int = 2048, regions: int = 1000,
                   factor: int = 16, sigma=(8, 4, 4), lam: float = 64.0,
                   rel_tol: float = 1e-5, max_iters: int = 20000) -> Problem:
    """Depth super-resolution shape: smooth low-res depth in [0,10], bilinear x16,
    confidence 1 at the low-res sample centres and 0 elsewhere."""
    rng = np.random.default_rng(seed)
    ref, _ = voronoi_reference(rng, H, W, regions)
    h, w = H // factor, W // factor
    yy, xx = np.mgrid[0:h, 0:w] / np.array([h, w]).reshape(2, 1, 1)
    d = np.zeros((h, w))
    for _ in range(6):
        fy, fx = rng.uniform(0.5, 3.0, 2)
        ph = rng.uniform(0.0, 2 * np.pi, 2)
        amp = rng.uniform(0.5, 1.0)
        d += amp * np.sin(2 * np.pi * fy * yy + ph[0]) * np.cos(2 * np.pi * fx * xx + ph[1])
    d = 10.0 * (d - d.min()) / max(d.max() - d.min(), 1e-12)
    # bilinear upsampling with half-pixel centres, edge-clamped
    sy = (np.arange(H) + 0.5) / factor - 0.5
    sx = (np.arange(W) + 0.5) / factor - 0.5
    y0 = np.clip(np.floor(sy).astype(int), 0, h - 1)
    x0 = np.clip(np.floor(sx).astype(int), 0, w - 1)
    y1 = np.clip(y0 + 1, 0, h - 1)
    x1 = np.clip(x0 + 1, 0, w - 1)
    wy = np.clip(sy - y0, 0.0, 1.0)[:, None]
    wx = np.clip(sx - x0, 0.0, 1.0)[None, :]
    up = ((1 - wy) * ((1 - wx) * d[y0][:, x0] + wx * d[y0][:, x1])
          + wy * ((1 - wx) * d[y1][:, x0] + wx * d[y1][:, x1]))
    conf = np.zeros((H, W), np.float32)
    conf[factor // 2::factor, factor // 2::factor] = 1.0
    return Problem("depthsr_%dx%d" % (W, H), ref, up[None].astype(np.float32), conf,
                   sigma[0], sigma[1], sigma[2], lam, max_iters, rel_tol)


def smoothed_logits(rng, C, H, W, k=9):
    return _box_mean(rng.normal(0.0, 1.0, size=(C, H, W)).astype(np.float32), k)


def segmentation(seed: int = 0, H: int = 512, W: int = 512, regions: int = 100,
                 C: int = 21, sigma=(8, 4, 4), lam: float = 128.0,
                 rel_tol: float = 1e-6, max_iters: int = 20000) -> Problem:
    """Differentiable-solve shape: 21 box-smoothed logits, U[0.2,1] confidence,
    and a random one-hot label (kept in ``extra['label']``) for a squared loss."""
    rng = np.random.default_rng(seed)
    ref, _ = voronoi_reference(rng, H, W, regions)
    t = smoothed_logits(rng, C, H, W)
    conf = rng.uniform(0.2, 1.0, size=(H, W)).astype(np.float32)
    label = rng.integers(0, C, size=(H, W))
    onehot = (np.arange(C)[:, None, None] == label[None]).astype(np.float32)
    return Problem("seg_%dx%d_c%d" % (W, H, C), ref, t, conf, sigma[0], sigma[1],
                   sigma[2], lam, max_iters, rel_tol, extra={"onehot": onehot})


def segmentation_probs(seed: int = 0, H: int = 512, W: int = 512, regions: int = 100,
                       C: int = 21, present: int = 3, sharpness: float = 5.0,
                       sigma=(8, 4, 4), lam: float = 128.0, rel_tol: float = 1e-6,
                       max_iters: int = 20000) -> Problem:
    """Class-probability shape: each region belongs to one of `present` of
    the C classes, and the target is the softmax over classes of
    sharpness * onehot(region class) + box-smoothed N(0,1) logits, the form
    of a segmentation network's output in which few classes carry mass.
    Confidence U[0.2,1]."""
    rng = np.random.default_rng(seed)
    ref, lab = voronoi_reference(rng, H, W, regions)
    classes = rng.choice(C, present, replace=False)
    region_class = classes[rng.integers(0, present, regions)]
    logits = smoothed_logits(rng, C, H, W)
    logits += sharpness * (np.arange(C)[:, None, None] == region_class[lab][None])
    e = np.exp(logits - logits.max(axis=0, keepdims=True))
    t = (e / e.sum(axis=0, keepdims=True)).astype(np.float32)
    conf = rng.uniform(0.2, 1.0, size=(H, W)).astype(np.float32)
    return Problem("segprob_%dx%d_c%d" % (W, H, C), ref, t, conf, sigma[0], sigma[1],
                   sigma[2], lam, max_iters, rel_tol)


def mixed_batch(seed: int = 0, count: int = 64, wmin=320, wmax=1920, hmin=240,
                hmax=1080, lam: float = 128.0, rel_tol: float = 1e-5,
                max_iters: int = 20000) -> list[Problem]:
    """Batch of images of uneven size and channel count (1 depth, 2 chroma, 21 classes)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        W = int(rng.integers(wmin, wmax + 1))
        H = int(rng.integers(hmin, hmax + 1))
        C = int(rng.choice([1, 2, 21]))
        sxy = int(rng.choice([8, 16]))
        regions = int(rng.integers(20, 300))
        ref, lab = voronoi_reference(rng, H, W, regions)
        if C == 21:
            t = smoothed_logits(rng, C, H, W)
        else:
            t = np.stack([_ramp_target(rng, lab, regions, H, W) for _ in range(C)])
        conf = rng.uniform(0.0, 1.0, size=(H, W)).astype(np.float32)
        out.append(Problem("batch%02d_%dx%d_c%d" % (i, W, H, C), ref, t, conf, sxy,
                           sxy // 2, sxy // 2, lam, max_iters, rel_tol))
    return out


def random_case(seed: int) -> Problem:
    """One seeded random configuration for parity sweeps: image 1..160 pixels a
    side, sigma_xy in {1, 2, 4, 8, 16, 32, 64}, colour scales in 1..64, C in
    {1, 2, 3, 4, 5, 7, 21}, lambda log-uniform in [0.1, 1000], Voronoi
    reference (1..30 regions) with colour noise 0..0.1, targets N(0, 1)
    box-smoothed, confidence U[0, 1] with a quarter of the pixels at 0."""
    rng = np.random.default_rng(seed + 104729)
    H, W = (int(v) for v in rng.integers(1, 161, size=2))
    regions = int(rng.integers(1, 31))
    sxy = int(rng.choice([1, 2, 4, 8, 16, 32, 64]))
    sl, suv = (int(v) for v in rng.integers(1, 65, size=2))
    C = int(rng.choice([1, 2, 3, 4, 5, 7, 21]))
    lam = float(10.0 ** rng.uniform(-1.0, 3.0))
    ref, _ = voronoi_reference(rng, H, W, min(regions, H * W), noise=float(rng.uniform(0.0, 0.1)))
    t = smoothed_logits(rng, C, H, W, k=int(rng.choice([1, 3, 5])))
    conf = rng.uniform(0.0, 1.0, size=(H, W)).astype(np.float32)
    conf[rng.uniform(size=(H, W)) < 0.25] = 0.0
    return Problem("random%d_%dx%d_c%d" % (seed, W, H, C), ref, t, conf, sxy, sl, suv, lam,
                   20000, 1e-6)


def random_grad(seed: int, C: int, H: int, W: int) -> np.ndarray:
    """A seeded upstream gradient d(loss)/d(output) of shape [C][H][W]."""
    rng = np.random.default_rng(seed + 7919)
    return rng.normal(0.0, 1.0, size=(C, H, W)).astype(np.float32)


def crop(p: Problem, y0: int, x0: int, h: int, w: int) -> Problem:
    """A crop of a problem (all planes), keeping its parameters."""
    sl = (slice(None), slice(y0, y0 + h), slice(x0, x0 + w))
    extra = {k: v[sl] for k, v in p.extra.items() if isinstance(v, np.ndarray) and v.ndim == 3}
    return Problem(p.name + "_crop", np.ascontiguousarray(p.ref[sl]),
                   np.ascontiguousarray(p.target[sl]),
                   np.ascontiguousarray(p.conf[y0:y0 + h, x0:x0 + w]),
                   p.sigma_xy, p.sigma_l, p.sigma_uv, p.lam, p.max_iters, p.rel_tol, extra)


# The five workload shapes, keyed by name.
WORKLOADS = {
    "ramp64x48": tiny_ramp,
    "stereo1024x768": stereo_refine,
    "depthsr2048x1536": depth_superres,
    "seg16x512x512": segmentation,
}
