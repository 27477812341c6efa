"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the FP64 oracle on the same seeded inputs, and compare."""
from __future__ import annotations

import sys

import numpy as np
import torch

from oracle import bilateral as O


def say(msg: str) -> None:
    """Name the case before a GPU step (flushed, so a fault still shows it)."""
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def gpu_grid(p, **kw):
    from paper_1511_03296_amd import BilateralGrid
    return BilateralGrid(to_dev(p.ref), p.sigma_xy, p.sigma_l, p.sigma_uv, **kw)


def params(p, **kw) -> O.Params:
    base = dict(sigma_xy=p.sigma_xy, sigma_l=p.sigma_l, sigma_uv=p.sigma_uv, lam=p.lam,
                max_iters=p.max_iters, rel_tol=p.rel_tol)
    base.update(kw)
    return O.Params(**base)


def rel_l2(a, b) -> float:
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def grad_c_errors(gc, grad_c, conf):
    """(relative L2 error of dL/dc, relative L2 error of c o dL/dc).

    c o dL/dc is the gradient with respect to log c.  At a pixel of low
    confidence alone on its vertex, the solution equals the target and dL/dc
    is 0, while dL/db there is about (dL/dx) / c: the float32 rounding of the
    solution (an ulp of the target) becomes an error of about ulp / c in
    dL/dc, larger than many exact values when c is near 0.  c o dL/dc
    removes that 1/c; with confidences bounded away from 0 both bars hold."""
    a = np.asarray(gc, np.float64).ravel()
    b = np.asarray(grad_c, np.float64).ravel()
    c = np.asarray(conf, np.float64).ravel()
    return rel_l2(a, b), rel_l2(c * a, c * b)


def check_grad_c(gc, grad_c, conf, tol=1e-4, plain_min_conf=0.1):
    """dL/dc against the oracle: c o dL/dc always, dL/dc itself when every
    confidence is at least plain_min_conf."""
    plain, weighted = grad_c_errors(gc, grad_c, conf)
    assert weighted <= tol, ("c o dL/dc", weighted, "dL/dc", plain)
    if float(np.min(conf)) >= plain_min_conf:
        assert plain <= tol, ("dL/dc", plain)
    return plain, weighted


def grid_arrays(G) -> dict:
    """Host copies of the level-0 grid arrays and the pyramid of a GPU grid."""
    v = G.view()
    cnt = G.counters(40)
    V, P, vcap = int(cnt[0]), G.P, int(v.vcap)
    out = dict(V=V, K=int(cnt[1]), bist_iters=int(cnt[2]), counts=cnt)
    out["key"] = G.array(v.key, V, torch.int64).cpu().numpy()
    out["idx"] = G.array(v.idx, P, torch.int32).cpu().numpy().astype(np.int64)
    out["m"] = G.array(v.m, V, torch.int32).cpu().numpy().astype(np.int64)
    nbr = G.array(v.nbr, 10 * vcap, torch.int32).view(10, vcap)[:, :V]
    out["nbr"] = nbr.cpu().numpy().astype(np.int64)
    # the packed table: word i holds slots 2i, 2i+1 as signed 16-bit u - v
    words = G.array(v.nb16, 5 * vcap, torch.int32).view(5, vcap)[:, :V].cpu().numpy()
    words = words.astype(np.int64) & 0xFFFFFFFF
    halves = np.stack([words & 0xFFFF, words >> 16], axis=1).reshape(10, V)
    off = np.where(halves >= 0x8000, halves - 0x10000, halves)
    out["nb16"] = np.where(off != 0, np.arange(V)[None, :] + off, -1)
    out["nb_wide"] = int(cnt[5])
    out["nb_packed"] = int(v.nb_packed)
    out["pix_ptr"] = G.array(v.pix_ptr, V + 1, torch.int32).cpu().numpy().astype(np.int64)
    out["pix_list"] = G.array(v.pix_list, P, torch.int32).cpu().numpy().astype(np.int64)
    out["n"] = G.array(v.n, V, torch.float64).cpu().numpy()
    out["nf"] = G.array(v.nf, V, torch.float32).cpu().numpy()
    out["nn"] = G.array(v.nn, V, torch.float64).cpu().numpy()
    sizes = [int(cnt[8 + k]) for k in range(v.levels)]
    out["sizes"] = sizes
    out["parents"], out["ones"], out["level_keys"] = [], [], []
    for k in range(v.levels):
        if k >= 1 and sizes[k] > 0:
            out["level_keys"].append(G.array(v.level_key[k], sizes[k], torch.int64).cpu().numpy())
            out["ones"].append(G.array(v.ones[k], sizes[k], torch.int32).cpu().numpy())
        if k + 1 < v.levels and sizes[k] > 1:
            out["parents"].append(
                G.array(v.parent[k], sizes[k], torch.int32).cpu().numpy().astype(np.int64))
    return out


def oracle_level_keys(g: O.Grid, pyr: O.Pyramid) -> list:
    keys, coords = [], g.coords
    for _ in range(pyr.K):
        k, _ = np.unique(O.pack_key(coords >> 1), return_inverse=True)
        keys.append(k)
        coords = O.unpack_key(k)
    return keys
