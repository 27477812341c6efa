#!/usr/bin/env python3
"""Throughput of the bilateral solver's hot path on one MI355X.

One step = the whole path on one batch of synthetic input, inputs resident in
HBM: build the grid and its pyramid, bistochastize, splat, initialise, PCG,
slice (forward), then splat the upstream gradient, adjoint PCG and gradient
scatter (backward).  Prints ONE JSON line with the Mpix/s of forward+backward
steps, the roofline figure of the dominant kernel (timed with HIP events
inside the library, on the launch stream) and the FP64 CPU oracle's rate on a
bounded sample of the same workload.

The default workload is the batch the metric's "solved to rel. residual
1e-5" and "vs plain" refer to: 64 images of uneven size (320x240 to
1920x1080) and channel count (1, 2 or 21), solved forward and backward to a
relative residual of 1e-5 by a batch plan whose forward and backward runs
are captured into one HIP graph and replayed, with the same images solved
one after another by the single-image path as the "plain" reference.  The
21-channel segmentation batch runs through the autograd function instead.

    python bench.py [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s solved to rel. residual 1e-5 (fwd and fwd+bwd), % HBM peak, vs plain"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")

# name -> generator, images, form, forward (max_iters, rel_tol), backward (max_iters, rel_tol)
#   form "single":   the single-image path (grid, bistochastize, solve, slice, backward)
#   form "graph":    a batch plan; its forward and backward runs captured in one graph
#   form "autograd": the batched torch.autograd.Function (eager, with convergence polls)
#   form "lowrank":  the batched low-rank reduction (forward only)
#   form "robust":   the robust solver's IRLS rounds (forward only)
WORKLOADS = {
    "stereo1024x768": dict(gen="stereo_refine", images=1, form="single", fwd=(25, 0.0),
                           bwd=(25, 0.0)),
    # 255 of 256 depth pixels carry no confidence, so A is singular on their
    # grid components; the adjoint system is consistent only for upstream
    # gradients that vanish there, e.g. that of a confidence-weighted loss.
    "depthsr2048x1536": dict(gen="depth_superres", images=1, form="single", fwd=(20000, 1e-5),
                             bwd=(20000, 1e-5), grad="conf_weighted"),
    "ramp64x48": dict(gen="tiny_ramp", images=1, form="single", fwd=(2000, 1e-5),
                      bwd=(2000, 1e-5)),
    # the differentiable 21-channel segmentation batch through the autograd
    # function; the same images solved one after another by the single-image
    # path give the "vs plain" ratio
    "seg16x512x512": dict(gen="segmentation", images=16, form="autograd", fwd=(20000, 1e-6),
                          bwd=(20000, 1e-6)),
    # the mixed batch through a batch plan replayed from a graph
    "mixed64": dict(gen="mixed_batch", images=64, form="graph", fwd=(20000, 1e-5),
                    bwd=(20000, 1e-5)),
    # the robust solver (Geman-McClure IRLS, sigma_gm in disparity units, 8
    # rounds) on the stereo shape, whose targets carry 10 % outlier
    # disparities; forward only (a step is the 8 rounds)
    "robust_stereo1024x768": dict(gen="stereo_refine", images=1, form="robust", fwd=(25, 0.0),
                                  bwd=(0, 0.0), robust=(4.0, 8)),
    # low-rank reduction (eps = 0.01) of 21-channel class-probability maps with
    # three classes present per image, forward only, through the batch engine;
    # the same images solved one after another with all 21 right-hand sides
    # give the "vs plain" ratio
    "segprob16x512x512": dict(gen="segmentation_probs", images=16, form="lowrank",
                              fwd=(20000, 1e-6), bwd=(0, 0.0), lowrank=0.01),
    # the domain transform on the stereo shape: the robust solver's initial
    # confidence from the input disparity (sigma_xy = sigma_rgb = 32,
    # sigma_dt = 2, 80 columns zeroed) and the post-process of a disparity
    # map (sigma'_xy = sigma'_rgb = 4), three iterations each
    "dt_stereo1024x768": dict(gen="stereo_refine", images=1, form="dt", fwd=(0, 0.0),
                              bwd=(0, 0.0), dt=dict(conf=(32.0, 32.0, 2.0, 80),
                                                    post=(4.0, 4.0), iters=3)),
}

# Iteration caps of the graph form: the calibration run's largest count times
# this margin, plus a few (a replayed graph runs a fixed number of launches;
# those after an image has stopped do nothing).
CAP_MARGIN, CAP_EXTRA = 1.2, 8


def pcg_bytes(V: int, iters) -> int:
    """Algorithmic bytes of one solve's PCG iterations: per vertex and
    iteration 48 bytes (neighbour table 40, n 4, diag(A) or its inverse 4)
    plus 24 per channel still iterating (y, r and d read and written once,
    float32), summed over the channels' own iteration counts `iters`."""
    iters = [int(i) for i in iters]
    if not iters:
        return 0
    return int(V) * (48 * max(iters) + 24 * sum(iters))


def _histogram(values) -> dict:
    out = {}
    for v in values:
        out[str(v)] = out.get(str(v), 0) + 1
    return dict(sorted(out.items(), key=lambda kv: float(kv[0])))


def _spread(values) -> dict:
    v = sorted(values)
    return {"min": v[0], "median": v[len(v) // 2], "max": v[-1]}


KERNEL_CODE = os.path.join(ROOT, "paper_1511_03296_amd", "kernel_code.json")


def _measured_traffic(workload: str):
    """HBM bytes per launch of the workload's dominant kernel (pcg_matvec, or
    dt_cols for the domain transform) from the committed counter runs, if
    every kernel of that family they covered still has the machine code it
    had then (digests written by the build), else None."""
    if not (os.path.exists(TRAFFIC_FILE) and os.path.exists(KERNEL_CODE)):
        return None
    with open(TRAFFIC_FILE) as f:
        wl = json.load(f).get("workloads", {}).get(workload)
    with open(KERNEL_CODE) as f:
        code = json.load(f)
    if not wl or not wl.get("kernels"):
        return None
    if any(code.get(k) != d for k, d in wl["kernels"].items()):
        return None
    return wl.get("bytes_per_launch")


def make_problems(name: str):
    import workloads as WL
    spec = WORKLOADS[name]
    gen = getattr(WL, spec["gen"])
    if spec["gen"] == "mixed_batch":
        return gen(seed=0, count=spec["images"])
    return [gen(seed=i) for i in range(spec["images"])]


def gpu_inputs(problems, spec, dev):
    import numpy as np
    import torch
    import workloads as WL
    out = []
    for i, p in enumerate(problems):
        gx = p.extra.get("onehot")
        gx = WL.random_grad(i, p.C, p.H, p.W) if gx is None else (2.0 * (p.target - gx))
        if spec.get("grad") == "conf_weighted":
            gx = gx * p.conf[None]
        out.append(dict(p=p, ref=torch.from_numpy(p.ref).to(dev),
                        t=torch.from_numpy(p.target).to(dev),
                        c=torch.from_numpy(p.conf).to(dev),
                        gx=torch.from_numpy(np.ascontiguousarray(gx, dtype=np.float32)).to(dev)))
    return out


def _sigmas(inputs):
    return [(d["p"].sigma_xy, d["p"].sigma_l, d["p"].sigma_uv) for d in inputs]


def _lam(inputs):
    lam = inputs[0]["p"].lam
    assert all(d["p"].lam == lam for d in inputs), "one lambda per batch"
    return lam


# ---------------------------------------------------------------------------
# One step of each form.  `keep` (a list) receives (V, forward stats,
# backward stats) per image.
# ---------------------------------------------------------------------------
def single_step(inputs, spec, backward=True, keep=None):
    """Image after image through the single-image path (also the "plain"
    reference of the batched forms)."""
    from paper_1511_03296_amd import BilateralGrid
    (fi, ft), (bi, bt) = spec["fwd"], spec["bwd"]
    fce = 0 if ft == 0.0 else 8
    bce = 0 if bt == 0.0 else 8
    pre = spec.get("precond", "jacobi")
    for d in inputs:
        p = d["p"]
        G = BilateralGrid(d["ref"], p.sigma_xy, p.sigma_l, p.sigma_uv)
        if spec.get("robust"):
            sigma_gm, rounds = spec["robust"]
            _, _, st = G.robust_solve(d["t"], d["c"], p.lam, sigma_gm, rounds, max_iters=fi,
                                      rel_tol=ft, check_every=fce)
            if keep is not None:
                keep.append((G.vertex_count(), st, None))
            continue
        ws = G.solve_workspace(p.C)
        y, st = G.solve(d["t"], d["c"], p.lam, max_iters=fi, rel_tol=ft, check_every=fce, ws=ws,
                        precond=pre)
        G.slice(y, p.C)
        bst = None
        if backward and bi > 0:
            _, _, _, bst = G.backward(d["t"], d["c"], y, d["gx"], p.lam, max_iters=bi, rel_tol=bt,
                                      check_every=bce, ws=ws, precond=pre)
        if keep is not None:
            keep.append((G.vertex_count(), st, bst))


class DtStep:
    """One step of the domain-transform workload: the initial confidence of
    the input disparity, then the post-process of the disparity map, with
    the workspace and outputs allocated once."""

    def __init__(self, inputs, spec):
        import torch
        from paper_1511_03296_amd import _lib as L
        d = inputs[0]
        self.ref, self.t = d["ref"], d["t"]
        H, W = d["p"].H, d["p"].W
        self.ws = torch.empty(L.lib.bs_dt_workspace_bytes(H, W), dtype=torch.uint8,
                              device=self.t.device)
        self.out = torch.empty_like(self.t)
        self.dt = spec["dt"]

    def __call__(self, backward=True):
        from paper_1511_03296_amd import domain_transform, dt_confidence
        ss, sr, sdt, zc = self.dt["conf"]
        dt_confidence(self.ref, self.t[0], ss, sr, sdt, zc, self.dt["iters"], ws=self.ws)
        domain_transform(self.ref, self.t, *self.dt["post"], self.dt["iters"], out=self.out,
                         ws=self.ws)


def dt_bytes(P: int, C: int) -> int:
    """Algorithmic bytes of one pass kernel (dt_rows or dt_cols) over C planes
    of P pixels: every sample read and written once (float32) and its domain
    distance word read once, 8 C + 4 bytes per pixel; both directions of the
    pass are one kernel."""
    return int(P) * (8 * int(C) + 4)


def lowrank_step(inputs, spec, backward=False, keep=None, ranks=None):
    from paper_1511_03296_amd import BatchState, SolveOptions
    (fi, ft), _ = spec["fwd"], spec["bwd"]
    state = BatchState([d["ref"] for d in inputs], [d["t"] for d in inputs],
                       [d["c"] for d in inputs], _sigmas(inputs), 1)
    _, fst, rk = state.forward_lowrank(SolveOptions(_lam(inputs), fi, ft, check_every=8),
                                       spec["lowrank"], stats=keep is not None)
    if keep is not None:
        V = state.vertex_counts()
        for i in range(len(inputs)):
            keep.append((V[i], fst[i], None))
        if ranks is not None:
            ranks.extend(rk)


def autograd_step(inputs, spec, backward=True):
    """The batched torch.autograd.Function: forward, then the backward pass
    that autograd drives from the upstream gradient."""
    import torch
    from paper_1511_03296_amd import bilateral_solve_batch
    (fi, ft), (bi, bt) = spec["fwd"], spec["bwd"]
    ts = [d["t"].detach().requires_grad_(backward) for d in inputs]
    cs = [d["c"].detach().requires_grad_(backward) for d in inputs]
    xs = bilateral_solve_batch([d["ref"] for d in inputs], ts, cs, _sigmas(inputs),
                               _lam(inputs), max_iters=fi, rel_tol=ft, bwd_max_iters=bi,
                               bwd_rel_tol=bt)
    if backward:
        torch.autograd.backward(xs, [d["gx"] for d in inputs])


def autograd_stats(inputs, spec, keep):
    """Stats of the same computation as autograd_step (through BatchState,
    the engine behind the autograd function)."""
    from paper_1511_03296_amd import BatchState, SolveOptions
    (fi, ft), (bi, bt) = spec["fwd"], spec["bwd"]
    lam = _lam(inputs)
    state = BatchState([d["ref"] for d in inputs], [d["t"] for d in inputs],
                       [d["c"] for d in inputs], _sigmas(inputs), 1)
    _, fst = state.forward(SolveOptions(lam, fi, ft), stats=True)
    _, _, bst = state.backward([d["gx"] for d in inputs], SolveOptions(lam, bi, bt), stats=True)
    V = state.vertex_counts()
    for i in range(len(inputs)):
        keep.append((V[i], fst[i], bst[i]))


class GraphForm:
    """The batch plan of the graph form: a calibration run that polls the stop
    flags gives every image's PCG and bistochastization iteration counts; the
    plan replayed from the graph runs fixed caps above them (CAP_MARGIN), and
    the stats of every replay say whether each channel stopped on the
    tolerance and each grid's bistochastization before its cap."""

    def __init__(self, inputs, spec):
        self.inputs, self.spec = inputs, spec
        self.plan = None
        self.graphs = {}

    def make(self, fwd_iters, bwd_iters, check_every, bist_iters=200):
        from paper_1511_03296_amd import BatchPlan, SolveOptions
        (_, ft), (_, bt) = self.spec["fwd"], self.spec["bwd"]
        lam = _lam(self.inputs)
        plan = BatchPlan([d["ref"] for d in self.inputs], [d["t"] for d in self.inputs],
                         [d["c"] for d in self.inputs], _sigmas(self.inputs),
                         SolveOptions(lam, fwd_iters, ft, check_every=check_every),
                         SolveOptions(lam, bwd_iters, bt, check_every=check_every),
                         bist_check_every=check_every, bist_max_iters=bist_iters)
        for g, d in zip(plan.grad_xs, self.inputs):
            g.copy_(d["gx"])
        return plan

    def calibrate(self, keep):
        import torch
        (fi, _), (bi, _) = self.spec["fwd"], self.spec["bwd"]
        plan = self.make(fi, bi, 8)
        plan.forward()
        torch.cuda.synchronize()
        fst = [s.clone() for s in plan.stats]
        plan.backward()
        torch.cuda.synchronize()
        bst = [s.clone() for s in plan.stats]
        V = plan.vertex_counts()
        bist = max(plan.bist_iters())
        plan.close()
        for i in range(len(V)):
            keep.append((V[i], fst[i], bst[i]))
        from paper_1511_03296_amd import read_stats
        fmax = max(int(read_stats(s)["iters"].max()) for s in fst)
        bmax = max(int(read_stats(s)["iters"].max()) for s in bst)
        self.caps = (int(math.ceil(fmax * CAP_MARGIN)) + CAP_EXTRA,
                     int(math.ceil(bmax * CAP_MARGIN)) + CAP_EXTRA)
        # the bistochastization's updates are capped the same way
        self.bist_cap = int(math.ceil(bist * CAP_MARGIN)) + CAP_EXTRA
        return self.caps

    def build(self):
        import torch
        if self.plan is not None:
            self.plan.close()
        self.graphs = {}
        self.plan = self.make(self.caps[0], self.caps[1], 0, self.bist_cap)
        self.plan.forward()
        self.plan.backward()
        torch.cuda.synchronize()

    def capture(self):
        self.graphs[True] = self.plan.capture(backward=True)
        self.graphs[False] = self.plan.capture(backward=False)

    def step(self, backward=True):
        self.graphs[backward].replay()

    def eager(self, backward=True):
        self.plan.forward()
        if backward:
            self.plan.backward()

    def converged(self) -> bool:
        """Whether every channel of the last run stopped on the tolerance (or
        had a zero right-hand side)."""
        import torch
        torch.cuda.synchronize()
        bist_ok = all(n < self.bist_cap for n in self.plan.bist_iters())
        return bist_ok and all(set(s["reason"].tolist()) <= {1, 5} for s in self.plan.read_stats())


def timed(step, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


KERNELS = ["level_count", "level_scan", "level_write", "neighbour_table", "bist_step",
           "bist_other", "splat", "init", "pcg_start", "pcg_matvec", "pcg_update", "pcg_reduce",
           "slice", "grad_scatter", "dt_rows", "dt_cols", "dt_other"]


def kernel_times(step, steps):
    """Per-kernel summed launch durations and launch counts per step (the
    start and end events every launch carries, on its own stream)."""
    from paper_1511_03296_amd import _lib as L
    import ctypes as ct
    L.check(L.lib.bs_timing_reset(), "timing_reset")
    L.check(L.lib.bs_timing_enable(1), "timing_enable")
    sec = timed(step, steps)
    L.check(L.lib.bs_timing_enable(0), "timing_enable")
    out = {}
    for n in KERNELS:
        ms, cnt = ct.c_double(), ct.c_int64()
        L.check(L.lib.bs_timing_read(n.encode(), ct.byref(ms), ct.byref(cnt)), "timing_read")
        out[n] = (ms.value / steps, cnt.value / steps)
    return sec, out


# ---------------------------------------------------------------------------
# The oracle on the host's cores.
# ---------------------------------------------------------------------------
def _oracle_sample(args):
    """One forward+backward (or the workload's own pass) of the oracle on one
    image crop; returns its pixel count.  Runs in a worker process."""
    import numpy as np  # noqa: F401
    from oracle import bilateral as O
    import workloads as WL
    p, spec = args
    if spec.get("dt"):
        from oracle import domain_transform as DT
        ss, sr, sdt, zc = spec["dt"]["conf"]
        DT.dt_confidence(p.ref, p.target[0], ss, sr, sdt, zc, spec["dt"]["iters"])
        DT.domain_transform(p.ref, p.target, *spec["dt"]["post"], spec["dt"]["iters"])
        return p.pixels
    (fi, ft), (bi, bt) = spec["fwd"], spec["bwd"]
    prm = O.Params(p.sigma_xy, p.sigma_l, p.sigma_uv, p.lam, max_iters=fi, rel_tol=ft)
    if spec.get("robust"):
        O.robust_solve(p.ref, p.target, p.conf, prm, *spec["robust"])
    elif spec.get("lowrank") is not None:
        O.solve_lowrank(p.ref, p.target, p.conf, prm, spec["lowrank"])
    else:
        gx = p.extra.get("onehot")
        gx = WL.random_grad(0, p.C, p.H, p.W) if gx is None else 2.0 * (p.target - gx)
        if spec.get("grad") == "conf_weighted":
            gx = gx * p.conf[None]
        sol = O.solve(p.ref, p.target, p.conf, prm)
        prmb = O.Params(p.sigma_xy, p.sigma_l, p.sigma_uv, p.lam, max_iters=bi, rel_tol=bt)
        O.solve_backward(sol, p.target, p.conf, gx, prmb)
    return p.pixels


def _worker_init():
    # one thread per worker process: the host's cores are shared by processes
    os.environ["OMP_NUM_THREADS"] = "1"
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)


def cpu_baseline(problems, spec, seconds, cores):
    """The FP64 oracle, as it stands, on a bounded sample of the workload: a
    crop of each image (cycling through the images), one crop per worker
    process, as many processes as cores, for about `seconds`."""
    import multiprocessing as mp
    import workloads as WL
    crops = []
    for p in problems:
        if not spec.get("dt") and (p.pixels > 200_000 or spec["fwd"][1] > 0):
            h, w = (min(p.H, 256), min(p.W, 256)) if p.C < 8 else (min(p.H, 96), min(p.W, 96))
            p = WL.crop(p, (p.H - h) // 2, (p.W - w) // 2, h, w)
        crops.append(p)
    what = {"robust": "robust forward", "lowrank": "low-rank forward",
            "dt": "domain-transform (confidence + post-process)"}
    kind = next((v for k, v in what.items() if spec.get(k) is not None), "forward+backward")
    ctx = mp.get_context("fork")
    done_px, n = 0, 0
    t0 = time.perf_counter()
    with ctx.Pool(cores, initializer=_worker_init) as pool:
        pending = []
        k = 0
        while time.perf_counter() - t0 < seconds or pending:
            while len(pending) < cores and time.perf_counter() - t0 < seconds:
                pending.append(pool.apply_async(_oracle_sample, ((crops[k % len(crops)], spec),)))
                k += 1
            pending[0].wait()
            done_px += pending.pop(0).get()
            n += 1
        el = time.perf_counter() - t0
    shape = f"{crops[0].W}x{crops[0].H}" if len(crops) == 1 else "crops"
    return {"value": round(done_px / el / 1e6, 4), "unit": "Mpix/s", "cores": cores,
            "kind": "oracle",
            "sample": (f"{n} {kind} passes of the full {shape} image" if spec.get("dt") else
                       f"{n} {kind} passes of centre crops (at most 256x256, 96x96 for "
                       f"21 channels; {shape}) cycling through the workload's images")
                      + f", {cores} worker processes of one thread each, {el:.1f} s, "
                        f"NumPy float64"}


def dt_line(args, problems, inputs, spec) -> dict:
    """The JSON line of the domain-transform workload: Mpix/s of steps, and
    the roofline of the slower pass kernel."""
    import torch
    step = DtStep(inputs, spec)
    for _ in range(max(1, args.warmup)):
        step()
    torch.cuda.synchronize()
    print("bench: warm-up done", file=sys.stderr, flush=True)
    sec = timed(step, args.steps)
    sec_inst, kt = kernel_times(step, args.steps)
    p = problems[0]
    it = spec["dt"]["iters"]
    # per step each pass kernel runs `iters` times on the confidence's two
    # signals and `iters` times on the C planes of the post-process
    bytes_step = it * (dt_bytes(p.pixels, 2) + dt_bytes(p.pixels, p.C))
    name = max(("dt_rows", "dt_cols"), key=lambda k: kt[k][0])
    ms, launches = kt[name]
    achieved = bytes_step / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return {
        "metric": METRIC,
        "value": round(p.pixels / sec / 1e6, 3),
        "unit": "Mpix/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "images": 1, "pixels": p.pixels,
                   "channels": p.C, "confidence": dict(zip(
                       ("sigma_xy", "sigma_rgb", "sigma_dt", "zero_cols"), spec["dt"]["conf"])),
                   "post_process": dict(zip(("sigma_xy", "sigma_rgb"), spec["dt"]["post"])),
                   "iterations": it, "parallelism": "single-gpu",
                   "engine": "domain transform (confidence + post-process)"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": _measured_traffic(args.workload), "kernel": name,
                     "bytes_per_launch": int(bytes_step / launches) if launches else 0,
                     "avg_us": round(ms / launches * 1e3, 3) if launches else None,
                     "launches_per_step": launches,
                     "bytes_rule": "8 x channels + 4 per pixel and pass (samples read and "
                                   "written once, the domain distance word read once)"},
        "kernel_ms_per_step": {k: round(kt[k][0], 4) for k in ("dt_rows", "dt_cols", "dt_other")},
        "kernel_launches_per_step": {k: kt[k][1] for k in ("dt_rows", "dt_cols", "dt_other")},
        "instrumented_ms_per_step": round(sec_inst * 1e3, 4),
    }


# ---------------------------------------------------------------------------
def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mixed64", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-cores", type=int, default=0,
                    help="worker processes of the CPU baseline (0: min(16, host cores))")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="graph form: keep the default tiles per block instead of tuning "
                         "them on the batch first")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched forms: skip the single-image comparison (counter runs)")
    ap.add_argument("--precond", default="jacobi", choices=["jacobi", "hier"],
                    help="PCG preconditioner; the hierarchical one runs image after image "
                         "through the single-image path")
    ap.add_argument("--profile", action="store_true",
                    help="the launches of forward+backward steps only, for a profiler's "
                         "kernel trace: no autotuning, single-image comparison, "
                         "forward-only timing or CPU baseline")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="copy a MIB-sized device buffer once (a reference kernel of known "
                         "traffic for hardware counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(a batch would shard by images across GPUs, one large image by slabs of "
              "cell rows with a halo exchange per PCG iteration)", file=sys.stderr)
        return 2

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    from paper_1511_03296_amd import read_stats
    dev = torch.device("cuda:0")
    spec = dict(WORKLOADS[args.workload])
    if args.precond != "jacobi":
        if spec["form"] in ("lowrank", "robust", "dt"):
            print("the low-rank, robust and domain-transform workloads use no other "
                  "preconditioner",
                  file=sys.stderr)
            return 2
        spec["precond"] = args.precond
        if spec["form"] in ("graph", "autograd"):
            spec["form"] = "single"
    form = spec["form"]
    problems = make_problems(args.workload)
    inputs = gpu_inputs(problems, spec, dev)
    pixels = sum(p.pixels for p in problems)
    print(f"bench: {args.workload} images={len(problems)} pixels={pixels} form={form}",
          file=sys.stderr, flush=True)

    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if form == "dt":
        line = dt_line(args, problems, inputs, spec)
        if not (args.no_cpu_baseline or args.profile):
            cores = args.cpu_cores or min(16, os.cpu_count() or 1)
            print(f"bench: cpu baseline (oracle, {cores} processes)", file=sys.stderr, flush=True)
            line["cpu_baseline"] = cpu_baseline(problems, spec, args.cpu_seconds, cores)
        print(json.dumps(line), flush=True)
        return 0

    keep, ranks = [], []
    tuned, caps, converged, graph_form, bist_cap = None, None, None, None, None
    if form == "graph":
        graph_form = GraphForm(inputs, spec)
        caps = graph_form.calibrate(keep)
        bist_cap = graph_form.bist_cap
        print(f"bench: calibration run done, iteration caps {caps}, bistochastization cap "
              f"{bist_cap}", file=sys.stderr, flush=True)
        if not (args.no_autotune or args.profile):
            from paper_1511_03296_amd import autotune

            def trial():
                graph_form.build()
                return lambda: graph_form.eager(True)
            tuned = autotune.tune_plan(trial, [p.C for p in problems], lanes=True)
            print(f"bench: autotuned lane widths and tiles per block {tuned}", file=sys.stderr,
                  flush=True)
        graph_form.build()
        graph_form.capture()
        for _ in range(max(1, args.warmup)):
            graph_form.step(True)
        torch.cuda.synchronize()
        step = graph_form.step
    elif form == "autograd":
        autograd_stats(inputs, spec, keep)
        for _ in range(max(1, args.warmup)):
            autograd_step(inputs, spec, True)
        step = lambda backward=True: autograd_step(inputs, spec, backward)
    elif form == "lowrank":
        lowrank_step(inputs, spec, keep=keep, ranks=ranks)
        for _ in range(max(0, args.warmup - 1)):
            lowrank_step(inputs, spec)
        step = lambda backward=False: lowrank_step(inputs, spec)
    else:
        for _ in range(max(1, args.warmup)):
            keep.clear()
            single_step(inputs, spec, True, keep)
        step = lambda backward=True: single_step(inputs, spec, backward)
    torch.cuda.synchronize()
    print("bench: warm-up done", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    step(True)
    host_ms = (time.perf_counter() - t0) * 1e3
    torch.cuda.synchronize()
    print(f"bench: host time of one step's calls {host_ms:.3f} ms", file=sys.stderr, flush=True)
    sec_fb = timed(lambda: step(True), args.steps)
    if graph_form is not None:
        converged = graph_form.converged()      # the backward runs' stats
    sec_f = None
    if not args.profile:
        sec_f = timed(lambda: step(False), args.steps)
        if graph_form is not None:
            converged = converged and graph_form.converged()
    print(f"bench: fwd+bwd {sec_fb * 1e3:.3f} ms/step, fwd "
          f"{'-' if sec_f is None else round(sec_f * 1e3, 3)} ms/step", file=sys.stderr,
          flush=True)

    plain = None
    if form in ("graph", "autograd", "lowrank") and not (args.no_plain or args.profile):
        full = {k: v for k, v in spec.items() if k != "lowrank"}
        bw = form != "lowrank"
        sec_plain = timed(lambda: single_step(inputs, full, bw), args.steps)
        plain = pixels / sec_plain / 1e6
        print(f"bench: plain single-image path {sec_plain * 1e3:.3f} ms/step",
              file=sys.stderr, flush=True)

    # kernel durations: the same launches, each with its start and end events
    # (the graph form runs its plan eagerly: the graph's launch sequence)
    if graph_form is not None:
        sec_inst, kt = kernel_times(lambda: graph_form.eager(True), args.steps)
    else:
        sec_inst, kt = kernel_times(lambda: step(True), args.steps)
    mv_ms, mv_launches = kt["pcg_matvec"]
    it_ms = kt["pcg_matvec"][0] + kt["pcg_update"][0] + kt["pcg_reduce"][0]

    # algorithmic bytes of one step's PCG iterations (forward and backward),
    # each channel counted for its own iterations
    V = [v for v, _, _ in keep]
    rounds = spec["robust"][1] if spec.get("robust") else 1
    fwd_it = [rounds * read_stats(st)["iters"][: (ranks[i] if ranks else None)]
              for i, (_, st, _) in enumerate(keep)]
    bwd_it = [[] if bst is None else read_stats(bst)["iters"] for _, _, bst in keep]
    step_bytes = sum(pcg_bytes(v, f) + pcg_bytes(v, b) for v, f, b in zip(V, fwd_it, bwd_it))
    achieved = step_bytes / (mv_ms * 1e-3) / 1e9 if mv_ms > 0 else 0.0
    achieved_it = step_bytes / (it_ms * 1e-3) / 1e9 if it_ms > 0 else 0.0
    avg_us = mv_ms / mv_launches * 1e3 if mv_launches else float("nan")
    # per lane width (the PCG launches' groups): images, vertices, bytes
    groups = {}
    from paper_1511_03296_amd import _lib as L
    for i, (v, f, b) in enumerate(zip(V, fwd_it, bwd_it)):
        c = ranks[i] if ranks else problems[i].C
        if c == 0:
            continue
        gK = groups.setdefault(str(int(L.lib.bs_lane_width(int(c)))),
                               {"images": 0, "vertices": 0, "pcg_bytes_per_step": 0})
        gK["images"] += 1
        gK["vertices"] += int(v)
        gK["pcg_bytes_per_step"] += pcg_bytes(v, f) + pcg_bytes(v, b)
    fwd_max = [int(max(f)) if len(f) else 0 for f in fwd_it]
    bwd_max = [int(max(b)) if len(b) else 0 for b in bwd_it]
    traffic = _measured_traffic(args.workload)
    C = problems[0].C
    engine = {"single": "single-image path", "robust": "single-image path",
              "graph": "batch plan, forward+backward graph replay",
              "autograd": "batched autograd function (batch plan per call, convergence polls)",
              "lowrank": "batched low-rank reduction"}[form]

    line = {
        "metric": METRIC,
        "value": round(pixels / sec_fb / 1e6, 3),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec_fb * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "images": len(problems), "pixels": pixels,
                   "channels": C if len(V) == 1 else _histogram(p.C for p in problems),
                   "sigma": [problems[0].sigma_xy, problems[0].sigma_l, problems[0].sigma_uv]
                   if len({p.sigma_xy for p in problems}) == 1
                   else {"sigma_xy": _histogram(p.sigma_xy for p in problems),
                         "sigma_l = sigma_uv": "sigma_xy / 2"},
                   "lambda": problems[0].lam, "vertices": V[0] if len(V) == 1 else sum(V),
                   "fwd_pcg": list(spec["fwd"]), "bwd_pcg": list(spec["bwd"]),
                   "fwd_iters": fwd_max[0] if len(V) == 1 else _spread(fwd_max),
                   "bwd_iters": bwd_max[0] if len(V) == 1 else _spread(bwd_max),
                   **({"robust": {"sigma_gm": spec["robust"][0], "irls_rounds": rounds,
                                  "pass": "forward only"}} if spec.get("robust") else {}),
                   **({"lowrank": {"eps": spec["lowrank"], "ranks": _histogram(ranks),
                                   "pass": "forward only"}}
                      if spec.get("lowrank") is not None else {}),
                   **({"graph": {"iteration_caps": list(caps),
                                 "bistochastization_cap": bist_cap,
                                 "all_channels_stopped_on_tolerance": converged}}
                      if caps else {}),
                   **({"lane_widths": {str(C): v["lane"]
                                       for C, v in tuned.get("lanes", {}).items()},
                       "tiles_per_block": {str(K): v["tiles"] for K, v in tuned.items()
                                           if K != "lanes"}}
                      if tuned else {}),
                   "precond": args.precond,
                   "parallelism": "single-gpu",
                   "engine": engine},
        "fwd_mpix_s": None if sec_f is None else round(pixels / sec_f / 1e6, 3),
        "plain_mpix_s": None if plain is None else round(plain, 3),
        "vs_plain": None if plain is None else round(pixels / sec_fb / 1e6 / plain, 3),
        "host_ms_per_step": round(host_ms, 3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "pcg_matvec",
                     "bytes_per_launch": int(step_bytes / mv_launches) if mv_launches else 0,
                     "avg_us": round(avg_us, 3), "launches_per_step": mv_launches,
                     "bytes_rule": "48 + 24 x (channels still iterating) per vertex and "
                                   "PCG iteration",
                     "lane_width_groups": groups,
                     "pcg_iteration": {"kernels": "pcg_matvec + pcg_update + pcg_reduce",
                                       "ms_per_step": round(it_ms, 4),
                                       "achieved": round(achieved_it, 1),
                                       "frac": round(achieved_it / HBM_PEAK_GBS, 4)}},
        "kernel_ms_per_step": {k: round(v[0], 4) for k, v in kt.items()},
        "kernel_launches_per_step": {k: v[1] for k, v in kt.items()},
        "instrumented_ms_per_step": round(sec_inst * 1e3, 4),
    }
    if not (args.no_cpu_baseline or args.profile):
        cores = args.cpu_cores or min(16, os.cpu_count() or 1)
        print(f"bench: cpu baseline (oracle, {cores} processes)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(problems, spec, args.cpu_seconds, cores)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
