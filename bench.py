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
relative residual of 1e-5 through the batch engine, with the same images
solved one after another by the single-image path as the "plain" reference.

    python bench.py [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpix/s solved to rel. residual 1e-5 (fwd and fwd+bwd), % HBM peak, vs plain"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")

# name -> (generator kwargs, images, forward (max_iters, rel_tol), backward (max_iters, rel_tol))
WORKLOADS = {
    "stereo1024x768": dict(gen="stereo_refine", images=1, fwd=(25, 0.0), bwd=(25, 0.0)),
    # 255 of 256 depth pixels carry no confidence, so A is singular on their
    # grid components; the adjoint system is consistent only for upstream
    # gradients that vanish there, e.g. that of a confidence-weighted loss.
    "depthsr2048x1536": dict(gen="depth_superres", images=1, fwd=(20000, 1e-5),
                             bwd=(20000, 1e-5), grad="conf_weighted"),
    "ramp64x48": dict(gen="tiny_ramp", images=1, fwd=(2000, 1e-5), bwd=(2000, 1e-5)),
    # batched forms: every image of the batch through the batch engine (images
    # on concurrent library streams); the same images solved one after another
    # by the single-image path give the "vs plain" ratio
    "seg16x512x512": dict(gen="segmentation", images=16, batch=True, fwd=(20000, 1e-6),
                          bwd=(20000, 1e-6)),
    "mixed64": dict(gen="mixed_batch", images=64, batch=True, fwd=(20000, 1e-5),
                    bwd=(20000, 1e-5)),
    # the robust solver (Geman-McClure IRLS, sigma_gm in disparity units, 8
    # rounds) on the stereo shape, whose targets carry 10 % outlier
    # disparities; forward only (a step is the 8 rounds)
    "robust_stereo1024x768": dict(gen="stereo_refine", images=1, fwd=(25, 0.0), bwd=(0, 0.0),
                                  robust=(4.0, 8)),
    # low-rank reduction (eps = 0.01) of 21-channel class-probability maps with
    # three classes present per image, forward only, through the batch engine;
    # the same images solved one after another with all 21 right-hand sides
    # give the "vs plain" ratio
    "segprob16x512x512": dict(gen="segmentation_probs", images=16, batch=True,
                              fwd=(20000, 1e-6), bwd=(0, 0.0), lowrank=0.01),
}


def matvec_bytes(C: int, iters: int) -> int:
    """Algorithmic bytes per vertex of `iters` pcg_matvec iterations.

    The exact form (every 4th iteration) reads the neighbour table (40 B),
    n, S c and M^-1 (4 B each), r, the old d and y (4C B each) and writes y,
    d and q (4C B each): 52 + 24C.  The recurrence form (the other three)
    reads the table, n and M^-1, r, d, the old q and y and writes y, d and
    q: 48 + 28C.  (y += alpha d of the previous iteration is applied here.)
    The neighbours' gathered values are cache hits in the count."""
    exact = iters // 4
    return exact * (52 + 24 * C) + (iters - exact) * (48 + 28 * C)


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
    """HBM bytes per pcg_matvec launch from the committed counter runs, if
    every pcg_matvec kernel they covered still has the machine code it had
    then (digests written by the build), else None."""
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


def run_step(inputs, spec, backward=True, keep=None, streams=0):
    """One pass of the hot path over every image of the batch: through the
    batch engine on `streams` library streams, or (streams=0) image after
    image through the single-image path."""
    from paper_1511_03296_amd import BilateralGrid
    (fi, ft), (bi, bt) = spec["fwd"], spec["bwd"]
    fce = 0 if ft == 0.0 else 8
    bce = 0 if bt == 0.0 else 8
    if streams > 0:
        return run_batch_step(inputs, spec, backward, keep, streams)
    if spec.get("lowrank") is not None:
        for d in inputs:
            p = d["p"]
            G = BilateralGrid(d["ref"], p.sigma_xy, p.sigma_l, p.sigma_uv)
            y, st, rank = G.solve_lowrank(d["t"], d["c"], p.lam, spec["lowrank"], max_iters=fi,
                                          rel_tol=ft, check_every=fce)
            G.slice(y, p.C)
            if keep is not None:
                keep.append((G.vertex_count(), st, None))
                RANKS.append(rank)
        return
    if spec.get("robust"):
        sigma_gm, rounds = spec["robust"]
        for d in inputs:
            p = d["p"]
            G = BilateralGrid(d["ref"], p.sigma_xy, p.sigma_l, p.sigma_uv)
            _, _, st = G.robust_solve(d["t"], d["c"], p.lam, sigma_gm, rounds, max_iters=fi,
                                      rel_tol=ft, check_every=fce)
            if keep is not None:
                keep.append((G.vertex_count(), st, None))
        return
    for d in inputs:
        p = d["p"]
        G = BilateralGrid(d["ref"], p.sigma_xy, p.sigma_l, p.sigma_uv)
        ws = G.solve_workspace(p.C)
        y, st = G.solve(d["t"], d["c"], p.lam, max_iters=fi, rel_tol=ft, check_every=fce, ws=ws)
        x = G.slice(y, p.C)
        if backward:
            gt, gc, _, bst = G.backward(d["t"], d["c"], y, d["gx"], p.lam, max_iters=bi,
                                        rel_tol=bt, check_every=bce, ws=ws)
        if keep is not None:
            keep.append((G.vertex_count(), st, bst if backward else None))


RANKS = []   # reduced ranks of the low-rank workload's images (warm-up step)


def run_batch_step(inputs, spec, backward, keep, streams):
    from paper_1511_03296_amd import BatchState, SolveOptions
    (fi, ft), (bi, bt) = spec["fwd"], spec["bwd"]
    lam = inputs[0]["p"].lam
    assert all(d["p"].lam == lam for d in inputs), "one lambda per batch"
    state = BatchState([d["ref"] for d in inputs], [d["t"] for d in inputs],
                       [d["c"] for d in inputs],
                       [(d["p"].sigma_xy, d["p"].sigma_l, d["p"].sigma_uv) for d in inputs],
                       streams)
    want = keep is not None
    fwd = SolveOptions(lam, fi, ft, check_every=0 if ft == 0.0 else 8)
    bwd = SolveOptions(lam, bi, bt, check_every=0 if bt == 0.0 else 8)
    if spec.get("lowrank") is not None:
        _, fst, ranks = state.forward_lowrank(fwd, spec["lowrank"], stats=want)
        if want:
            V = state.vertex_counts()
            for i in range(len(inputs)):
                keep.append((V[i], fst[i], None))
            RANKS.extend(ranks)
        return
    _, fst = state.forward(fwd, stats=want)
    bst = None
    if backward:
        _, _, bst = state.backward([d["gx"] for d in inputs], bwd, stats=want)
    if want:
        V = state.vertex_counts()
        for i in range(len(inputs)):
            keep.append((V[i], fst[i], bst[i] if backward else None))


def timed(inputs, spec, steps, backward=True, streams=0):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run_step(inputs, spec, backward, streams=streams)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def kernel_times(inputs, spec, steps, streams=0):
    """Per-kernel average launch duration (HIP events on the launch stream)."""
    from paper_1511_03296_amd import _lib as L
    import ctypes as ct
    names = ["level_count", "level_scan", "level_write", "neighbour_table", "bist_step",
             "bist_other", "splat", "init", "pcg_start", "pcg_matvec", "pcg_update", "pcg_reduce",
             "slice",
             "grad_scatter"]
    L.check(L.lib.bs_timing_reset(), "timing_reset")
    L.check(L.lib.bs_timing_enable(1), "timing_enable")
    sec = timed(inputs, spec, steps, streams=streams)
    L.check(L.lib.bs_timing_enable(0), "timing_enable")
    out = {}
    for n in names:
        ms, cnt = ct.c_double(), ct.c_int64()
        L.check(L.lib.bs_timing_read(n.encode(), ct.byref(ms), ct.byref(cnt)), "timing_read")
        out[n] = (ms.value / steps, cnt.value / steps)
    return sec, out


def cpu_baseline(problems, spec, seconds):
    """The FP64 oracle, as it stands, on a bounded sample of the workload."""
    import numpy as np
    from oracle import bilateral as O
    import workloads as WL
    (fi, ft), (bi, bt) = spec["fwd"], spec["bwd"]
    p = problems[0]
    sample = f"{p.name}: full forward+backward of image 0"
    if p.pixels > 1_000_000 or ft > 0:
        # tolerance-driven workloads: a centre crop keeps the sample bounded
        h, w = (min(p.H, 384), min(p.W, 512)) if p.C < 8 else (min(p.H, 128), min(p.W, 128))
        p = WL.crop(p, (p.H - h) // 2, (p.W - w) // 2, h, w)
        sample = f"{p.name} ({w}x{h} centre crop), full forward+backward"
    gx = WL.random_grad(0, p.C, p.H, p.W)
    if spec.get("grad") == "conf_weighted":
        gx = gx * p.conf[None]
    if spec.get("robust"):
        sample = sample.replace("forward+backward", "robust forward")
    if spec.get("lowrank") is not None:
        sample = sample.replace("forward+backward", "low-rank forward")
    t0 = time.perf_counter()
    n = 0
    while True:
        prm = O.Params(p.sigma_xy, p.sigma_l, p.sigma_uv, p.lam, max_iters=fi, rel_tol=ft)
        if spec.get("robust"):
            O.robust_solve(p.ref, p.target, p.conf, prm, *spec["robust"])
        elif spec.get("lowrank") is not None:
            O.solve_lowrank(p.ref, p.target, p.conf, prm, spec["lowrank"])
        else:
            sol = O.solve(p.ref, p.target, p.conf, prm)
            prmb = O.Params(p.sigma_xy, p.sigma_l, p.sigma_uv, p.lam, max_iters=bi, rel_tol=bt)
            O.solve_backward(sol, p.target, p.conf, gx, prmb)
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {"value": round(n * p.pixels / el / 1e6, 4), "unit": "Mpix/s", "cores": 1,
            "kind": "oracle", "sample": f"{sample}, {n} step(s) in {el:.1f} s, NumPy float64, "
                                        "one thread"}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mixed64", choices=sorted(WORKLOADS))
    ap.add_argument("--streams", type=int, default=4,
                    help="library streams of the batch engine (batched workloads)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched workloads: keep the default tiles per block instead of "
                         "tuning them on the batch first")
    ap.add_argument("--no-plain", action="store_true",
                    help="batched workloads: skip the single-image comparison (counter runs)")
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
    dev = torch.device("cuda:0")
    spec = WORKLOADS[args.workload]
    problems = make_problems(args.workload)
    inputs = gpu_inputs(problems, spec, dev)
    pixels = sum(p.pixels for p in problems)
    print(f"bench: {args.workload} images={len(problems)} pixels={pixels}", file=sys.stderr,
          flush=True)

    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    streams = args.streams if spec.get("batch") else 0
    keep = []
    for _ in range(max(1, args.warmup)):
        keep.clear()
        RANKS.clear()
        run_step(inputs, spec, True, keep, streams)
        torch.cuda.synchronize()
        print("bench: warmup step done", file=sys.stderr, flush=True)
    tuned = None
    if streams and not args.no_autotune:
        from paper_1511_03296_amd import autotune
        # lane widths of the systems the batched PCG runs: the reduced ranks
        # of a low-rank workload, else the channel counts
        channels = list(RANKS) if RANKS else [p.C for p in problems]
        tuned = autotune.tune_batch(lambda: run_step(inputs, spec, True, streams=streams),
                                    channels)
        print(f"bench: autotuned tiles per block {tuned}", file=sys.stderr, flush=True)
    from paper_1511_03296_amd import read_stats
    V = [v for v, _, _ in keep]
    # PCG iterations per step (the robust solver's rounds each solve anew)
    rounds = spec["robust"][1] if spec.get("robust") else 1
    fwd_iters = [rounds * int(read_stats(st)["iters"].max()) for _, st, _ in keep]
    bwd_iters = [0 if bst is None else int(read_stats(bst)["iters"].max()) for _, _, bst in keep]
    C = problems[0].C

    t0 = time.perf_counter()
    run_step(inputs, spec, True, streams=streams)
    host_ms = (time.perf_counter() - t0) * 1e3
    torch.cuda.synchronize()
    print(f"bench: host time of one step's calls {host_ms:.3f} ms", file=sys.stderr, flush=True)
    sec_fb = timed(inputs, spec, args.steps, backward=True, streams=streams)
    sec_f = timed(inputs, spec, args.steps, backward=False, streams=streams)
    print(f"bench: fwd+bwd {sec_fb * 1e3:.3f} ms/step, fwd {sec_f * 1e3:.3f} ms/step",
          file=sys.stderr, flush=True)
    plain = None
    if spec.get("lowrank") is not None and not args.no_plain:
        full = {k: v for k, v in spec.items() if k != "lowrank"}
        sec_plain = timed(inputs, full, args.steps, backward=False, streams=0)
        plain = pixels / sec_plain / 1e6
        print(f"bench: full-rank single-image path fwd {sec_plain * 1e3:.3f} ms/step",
              file=sys.stderr, flush=True)
    elif streams and not args.no_plain:
        sec_plain = timed(inputs, spec, args.steps, backward=True, streams=0)
        plain = pixels / sec_plain / 1e6
        print(f"bench: plain single-image path fwd+bwd {sec_plain * 1e3:.3f} ms/step",
              file=sys.stderr, flush=True)
    sec_inst, kt = kernel_times(inputs, spec, args.steps, streams)
    mv_ms, mv_launches = kt["pcg_matvec"]
    # Algorithmic bytes of one step's pcg_matvec launches over their summed
    # durations (matvec_bytes).  Launches past convergence (between stop
    # polls) return at once and count as time only.
    solved_c = RANKS if RANKS else [p.C for p in problems]   # right-hand sides solved
    step_bytes = sum(v * matvec_bytes(c, fi + bi) for v, c, fi, bi in
                     zip(V, solved_c, fwd_iters, bwd_iters))
    avg_us = mv_ms / mv_launches * 1e3 if mv_launches else float("nan")
    bytes_per_launch = step_bytes / mv_launches if mv_launches else 0.0
    achieved = step_bytes / (mv_ms * 1e-3) / 1e9 if mv_launches else 0.0

    traffic = _measured_traffic(args.workload)

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
                   "fwd_iters": fwd_iters[0] if len(V) == 1 else _spread(fwd_iters),
                   "bwd_iters": bwd_iters[0] if len(V) == 1 else _spread(bwd_iters),
                   **({"robust": {"sigma_gm": spec["robust"][0], "irls_rounds": rounds,
                                  "pass": "forward only"}} if spec.get("robust") else {}),
                   **({"lowrank": {"eps": spec["lowrank"], "ranks": _histogram(RANKS),
                                   "pass": "forward only"}}
                      if spec.get("lowrank") is not None else {}),
                   **({"tiles_per_block": {str(K): v["tiles"] for K, v in tuned.items()}}
                      if tuned else {}),
                   "parallelism": "single-gpu",
                   "engine": f"batch, {streams} streams" if streams else "single-image"},
        "fwd_mpix_s": round(pixels / sec_f / 1e6, 3),
        "plain_mpix_s": None if plain is None else round(plain, 3),
        "vs_plain": None if plain is None else round(pixels / sec_fb / 1e6 / plain, 3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": "pcg_matvec",
                     "bytes_per_launch": int(bytes_per_launch), "avg_us": round(avg_us, 3),
                     "launches_per_step": mv_launches},
        "kernel_ms_per_step": {k: round(v[0], 4) for k, v in kt.items()},
        "instrumented_ms_per_step": round(sec_inst * 1e3, 4),
    }
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(problems, spec, args.cpu_seconds)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
