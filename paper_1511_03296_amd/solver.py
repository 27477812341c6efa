"""Python API of the MI355X bilateral solver.

PyTorch supplies device memory (the caching allocator) and the stream; every
step of the solver runs in the HIP library behind the C ABI (``_lib``):

    grid = BilateralGrid(ref, sigma_xy=8, sigma_l=4, sigma_uv=4)  # grid + bistochastization
    y, stats = grid.solve(target, conf, lam=128.0, rel_tol=1e-5)  # PCG in bilateral space
    x = grid.slice(y)                                             # back to pixels
    gt, gc, g = grid.backward(target, conf, y, grad_x, lam=128.0)  # Section 3 adjoint

``bilateral_solve`` wraps these in a ``torch.autograd.Function`` that is
differentiable in the target and the confidence.  ``domain_transform``
post-processes an output; ``dt_confidence`` gives the robust solver an initial
confidence from the edge-aware variance of its input.
"""
from __future__ import annotations

import ctypes as ct
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

_STATS_DTYPE = np.dtype([("iters", "<i4"), ("reason", "<i4"), ("rel_residual", "<f8"),
                         ("bnorm", "<f8")])


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dev_f32(t: torch.Tensor, name: str, shape) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.contiguous()


@dataclass
class SolveOptions:
    lam: float
    max_iters: int = 25
    rel_tol: float = 0.0
    init: str = "hier"
    init_alpha: float = 4.0
    init_beta: float = 0.0
    check_every: int = 8
    precond: str = "jacobi"
    pre_alpha: float = 2.0
    pre_beta: float = 5.0

    def struct(self) -> L.SolveParams:
        if self.init not in ("hier", "flat"):
            raise ValueError("init must be 'hier' or 'flat'")
        if self.precond not in ("jacobi", "hier"):
            raise ValueError("precond must be 'jacobi' or 'hier'")
        return L.SolveParams(float(self.lam),
                             L.BS_INIT_HIER if self.init == "hier" else L.BS_INIT_FLAT,
                             int(self.max_iters), int(self.check_every), float(self.rel_tol),
                             float(self.init_alpha), float(self.init_beta),
                             L.BS_PRECOND_HIER if self.precond == "hier" else L.BS_PRECOND_JACOBI,
                             float(self.pre_alpha), float(self.pre_beta))


class BilateralGrid:
    """A simplified bilateral grid of one reference image, bistochastized."""

    def __init__(self, ref: torch.Tensor, sigma_xy: int, sigma_l: int, sigma_uv: int,
                 bist_tol: float = 1e-10, bist_max_iters: int = 200, check_every: int = 8,
                 bistochastize: bool = True):
        if ref.dim() != 3 or ref.shape[0] != 3:
            raise ValueError("reference must be [3][H][W]")
        self.H, self.W = int(ref.shape[1]), int(ref.shape[2])
        ref = _dev_f32(ref, "reference", (3, self.H, self.W))
        self.device = ref.device
        self.params = L.GridParams(int(sigma_xy), int(sigma_l), int(sigma_uv))
        nbytes = L.lib.bs_grid_workspace_bytes(self.H, self.W, ct.byref(self.params))
        if nbytes == 0:
            L.check(L.lib.bs_build_grid(None, self.H, self.W, ct.byref(self.params), None, 0,
                                        None, None), "bs_build_grid")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.handle = L.Grid()
        L.check(L.lib.bs_build_grid(ref.data_ptr(), self.H, self.W, ct.byref(self.params),
                                    self.ws.data_ptr(), nbytes, _stream(),
                                    ct.byref(self.handle)), "bs_build_grid")
        self._ref = ref
        if bistochastize:
            self.bistochastize(bist_tol, bist_max_iters, check_every)

    # -- construction ------------------------------------------------------
    def bistochastize(self, tol: float = 1e-10, max_iters: int = 200, check_every: int = 8):
        p = L.BistochParams(int(max_iters), int(check_every), float(tol))
        L.check(L.lib.bs_bistochastize(ct.byref(self.handle), ct.byref(p), _stream()),
                "bs_bistochastize")

    @property
    def P(self) -> int:
        return self.H * self.W

    def view(self) -> L.GridView:
        v = L.GridView()
        L.check(L.lib.bs_grid_get_view(ct.byref(self.handle), ct.byref(v)), "bs_grid_get_view")
        return v

    def counters(self, n: int = 40) -> np.ndarray:
        out = (ct.c_int32 * n)()
        L.check(L.lib.bs_read_counters(ct.byref(self.handle), out, n, _stream()),
                "bs_read_counters")
        return np.array(out[:], dtype=np.int64)

    def vertex_count(self) -> int:
        v = ct.c_int32()
        L.check(L.lib.bs_grid_vertex_count(ct.byref(self.handle), ct.byref(v), _stream()),
                "bs_grid_vertex_count")
        return int(v.value)

    def array(self, ptr: int, count: int, dtype: torch.dtype) -> torch.Tensor:
        """A device tensor aliasing `count` elements of the grid workspace at `ptr`."""
        off = int(ptr) - self.ws.data_ptr()
        size = torch.tensor([], dtype=dtype).element_size() * count
        if off < 0 or off + size > self.ws.numel():
            raise ValueError("pointer outside the grid workspace")
        return self.ws[off:off + size].view(dtype)

    @property
    def vcap(self) -> int:
        return int(self.view().vcap)

    # -- solve -------------------------------------------------------------
    def solve_workspace(self, C: int) -> torch.Tensor:
        nbytes = L.lib.bs_solve_workspace_bytes(ct.byref(self.handle), int(C))
        if nbytes == 0:
            raise ValueError("invalid channel count")
        return torch.empty(nbytes, dtype=torch.uint8, device=self.device)

    def solve(self, target: torch.Tensor, conf: torch.Tensor, lam: float, max_iters: int = 25,
              rel_tol: float = 0.0, init: str = "hier", init_alpha: float = 4.0,
              init_beta: float = 0.0, check_every: int = 8, ws: torch.Tensor | None = None,
              y: torch.Tensor | None = None, stats: torch.Tensor | None = None,
              precond: str = "jacobi", pre_alpha: float = 2.0, pre_beta: float = 5.0,
              strict: bool = False):
        """Bilateral-space solution y [Vcap][C] and per-channel stats (device bytes).
        strict (with rel_tol > 0): raise NotConverged if a channel missed the
        tolerance (reads the stats, so the call synchronises)."""
        C = int(target.shape[0])
        target = _dev_f32(target, "target", (C, self.H, self.W))
        conf = _dev_f32(conf, "confidence", (self.H, self.W))
        opts = SolveOptions(lam, max_iters, rel_tol, init, init_alpha, init_beta, check_every,
                            precond, pre_alpha, pre_beta)
        if ws is None:
            ws = self.solve_workspace(C)
        if y is None:
            y = torch.empty((self.vcap, C), dtype=torch.float32, device=self.device)
        if stats is None:
            stats = torch.empty(C * _STATS_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        p = opts.struct()
        L.check(L.lib.bs_solve(ct.byref(self.handle), target.data_ptr(), conf.data_ptr(), C,
                               ct.byref(p), y.data_ptr(), ws.data_ptr(), ws.numel(),
                               stats.data_ptr(), _stream()), "bs_solve")
        self._last_ws = ws
        if strict and rel_tol > 0:
            require_converged(stats, "solve")
        return y, stats

    def robust_solve(self, target: torch.Tensor, conf_init: torch.Tensor, lam: float,
                     sigma_gm: float, irls_iters: int, max_iters: int = 25, rel_tol: float = 0.0,
                     init: str = "hier", init_alpha: float = 4.0, init_beta: float = 0.0,
                     check_every: int = 8):
        """Robust bilateral solver (Geman-McClure IRLS): the last round's y
        [Vcap][C], its slice x [C][H][W] and per-channel stats (device bytes)."""
        C = int(target.shape[0])
        target = _dev_f32(target, "target", (C, self.H, self.W))
        conf_init = _dev_f32(conf_init, "confidence", (self.H, self.W))
        opts = SolveOptions(lam, max_iters, rel_tol, init, init_alpha, init_beta, check_every)
        nbytes = L.lib.bs_robust_workspace_bytes(ct.byref(self.handle), C)
        if nbytes == 0:
            raise ValueError("invalid channel count")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        y = torch.empty((self.vcap, C), dtype=torch.float32, device=self.device)
        x = torch.empty((C, self.H, self.W), dtype=torch.float32, device=self.device)
        stats = torch.empty(C * _STATS_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        p = opts.struct()
        L.check(L.lib.bs_robust_solve(ct.byref(self.handle), target.data_ptr(),
                                      conf_init.data_ptr(), C, ct.byref(p), float(sigma_gm),
                                      int(irls_iters), y.data_ptr(), x.data_ptr(), ws.data_ptr(),
                                      ws.numel(), stats.data_ptr(), _stream()),
                "bs_robust_solve")
        return y, x, stats

    def solve_lowrank(self, target: torch.Tensor, conf: torch.Tensor, lam: float,
                      eps: float = 0.01, max_iters: int = 25, rel_tol: float = 0.0,
                      init: str = "hier", init_alpha: float = 4.0, init_beta: float = 0.0,
                      check_every: int = 8, ws: torch.Tensor | None = None):
        """A Y = B through the low-rank reduction of B: y [Vcap][C], the
        reduced systems' stats (device bytes, first `rank` entries) and the
        rank.  Synchronises the current stream."""
        C = int(target.shape[0])
        target = _dev_f32(target, "target", (C, self.H, self.W))
        conf = _dev_f32(conf, "confidence", (self.H, self.W))
        opts = SolveOptions(lam, max_iters, rel_tol, init, init_alpha, init_beta, check_every)
        if ws is None:
            nbytes = L.lib.bs_lowrank_workspace_bytes(ct.byref(self.handle), C)
            if nbytes == 0:
                raise ValueError("invalid channel count")
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        y = torch.empty((self.vcap, C), dtype=torch.float32, device=self.device)
        stats = torch.zeros(C * _STATS_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        rank = ct.c_int32(0)
        p = opts.struct()
        L.check(L.lib.bs_solve_lowrank(ct.byref(self.handle), target.data_ptr(), conf.data_ptr(),
                                       C, ct.byref(p), float(eps), y.data_ptr(), ws.data_ptr(),
                                       ws.numel(), stats.data_ptr(), ct.byref(rank), _stream()),
                "bs_solve_lowrank")
        return y, stats, int(rank.value)

    def slice(self, y: torch.Tensor, C: int | None = None, out: torch.Tensor | None = None):
        C = int(y.shape[1]) if C is None else int(C)
        if out is None:
            out = torch.empty((C, self.H, self.W), dtype=torch.float32, device=self.device)
        L.check(L.lib.bs_slice(ct.byref(self.handle), y.data_ptr(), C, out.data_ptr(), _stream()),
                "bs_slice")
        return out

    def backward(self, target: torch.Tensor, conf: torch.Tensor, y_hat: torch.Tensor,
                 grad_x: torch.Tensor, lam: float, max_iters: int = 25, rel_tol: float = 0.0,
                 init: str = "hier", init_alpha: float = 4.0, init_beta: float = 0.0,
                 check_every: int = 8, ws: torch.Tensor | None = None,
                 stats: torch.Tensor | None = None, want_g: bool = False,
                 precond: str = "jacobi", pre_alpha: float = 2.0, pre_beta: float = 5.0,
                 strict: bool = False):
        """(dL/dt, dL/dc, dL/db or None, stats) from dL/dx (Section 3).  strict
        (with rel_tol > 0): raise NotConverged if the adjoint solve missed the
        tolerance, as when dL/dx does not vanish on a grid component without
        confidence and A g = S dL/dx has no solution (synchronises)."""
        C = int(target.shape[0])
        target = _dev_f32(target, "target", (C, self.H, self.W))
        conf = _dev_f32(conf, "confidence", (self.H, self.W))
        grad_x = _dev_f32(grad_x, "grad_x", (C, self.H, self.W))
        opts = SolveOptions(lam, max_iters, rel_tol, init, init_alpha, init_beta, check_every,
                            precond, pre_alpha, pre_beta)
        if ws is None:
            ws = self.solve_workspace(C)
        gt = torch.empty((C, self.H, self.W), dtype=torch.float32, device=self.device)
        gc = torch.empty((self.H, self.W), dtype=torch.float32, device=self.device)
        g = torch.empty((self.vcap, C), dtype=torch.float32, device=self.device) if want_g else None
        if stats is None:
            stats = torch.empty(C * _STATS_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
        p = opts.struct()
        L.check(L.lib.bs_solve_backward(ct.byref(self.handle), target.data_ptr(),
                                        conf.data_ptr(), y_hat.data_ptr(), grad_x.data_ptr(), C,
                                        ct.byref(p), gt.data_ptr(), gc.data_ptr(),
                                        g.data_ptr() if g is not None else None, ws.data_ptr(),
                                        ws.numel(), stats.data_ptr(), _stream()),
                "bs_solve_backward")
        self._last_ws = ws
        if strict and rel_tol > 0:
            require_converged(stats, "adjoint solve")
        return gt, gc, g, stats

    def solve_ws_arrays(self, ws: torch.Tensor, C: int):
        """Device tensors (b [Vcap][C] (a strided view), S c, diag(A), Jacobi inverse) of a
        solve workspace."""
        ptrs = [ct.c_void_p() for _ in range(4)]
        L.check(L.lib.bs_solve_ws_view(ct.byref(self.handle), int(C), ws.data_ptr(), ws.numel(),
                                       *[ct.byref(p) for p in ptrs]), "bs_solve_ws_view")
        vcap = self.vcap

        def alias(ptr, count):
            off = int(ptr.value) - ws.data_ptr()
            return ws[off:off + 4 * count].view(torch.float32)

        cs = int(L.lib.bs_solve_channel_stride(int(C)))
        return (alias(ptrs[0], vcap * cs).view(vcap, cs)[:, :C], alias(ptrs[1], vcap),
                alias(ptrs[2], vcap), alias(ptrs[3], vcap))


def read_stats(stats: torch.Tensor) -> np.ndarray:
    """Per-channel solve stats (iters, reason, rel_residual, bnorm) as a NumPy record array."""
    return np.frombuffer(stats.cpu().numpy().tobytes(), dtype=_STATS_DTYPE)


class NotConverged(RuntimeError):
    """A solve to a tolerance stopped without meeting it."""


# reasons of bs_chan_stats that end a solve to a tolerance without meeting it
_FAILED = {2: "iteration cap reached", 4: "d^T A d <= 0"}


def require_converged(stats: torch.Tensor, what: str = "solve") -> None:
    """Raises NotConverged when a channel stopped at the iteration cap or on
    d^T A d <= 0 instead of on the tolerance (the symptom of a system with no
    solution, e.g. an adjoint whose dL/dx does not vanish on a grid component
    without confidence, Section 3).  Reads the stats: synchronises."""
    rec = read_stats(stats)
    bad = [(c, int(r["reason"]), float(r["rel_residual"])) for c, r in enumerate(rec)
           if int(r["reason"]) in _FAILED]
    if bad:
        detail = "; ".join(f"channel {c}: {_FAILED[k]}, rel. residual {res:.3g}"
                           for c, k, res in bad[:4])
        raise NotConverged(f"{what} did not meet its tolerance ({len(bad)} of {len(rec)} "
                           f"channels): {detail}")


def _dt_workspace(H: int, W: int, device, ws: torch.Tensor | None) -> torch.Tensor:
    nbytes = L.lib.bs_dt_workspace_bytes(H, W)
    if nbytes == 0:
        raise ValueError(f"unsupported image size {H}x{W}")
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    return ws


def domain_transform(ref: torch.Tensor, x: torch.Tensor, sigma_s: float, sigma_r: float,
                     iters: int = 3, out: torch.Tensor | None = None,
                     ws: torch.Tensor | None = None) -> torch.Tensor:
    """The recursive-filter domain transform of x [C][H][W] guided by the
    reference [3][H][W] (the post-process of the solver's output, Section 4);
    out=x filters in place."""
    H, W = int(ref.shape[1]), int(ref.shape[2])
    ref = _dev_f32(ref, "reference", (3, H, W))
    C = int(x.shape[0])
    x = _dev_f32(x, "x", (C, H, W))
    if out is None:
        out = torch.empty_like(x)
    elif not out.is_contiguous() or tuple(out.shape) != (C, H, W) or out.dtype != torch.float32:
        raise ValueError("out must be a contiguous float32 tensor shaped like x")
    ws = _dt_workspace(H, W, x.device, ws)
    p = L.DtParams(float(sigma_s), float(sigma_r), int(iters))
    L.check(L.lib.bs_domain_transform(ref.data_ptr(), H, W, x.data_ptr(), C, ct.byref(p),
                                      out.data_ptr(), ws.data_ptr(), ws.numel(), _stream()),
            "bs_domain_transform")
    return out


def dt_confidence(ref: torch.Tensor, z: torch.Tensor, sigma_s: float, sigma_r: float,
                  sigma_dt: float, zero_cols: int = 0, iters: int = 3,
                  ws: torch.Tensor | None = None) -> torch.Tensor:
    """The robust solver's initial confidence exp(-V / (2 sigma_dt^2)) from the
    edge-aware variance V = DT(z^2) - DT(z)^2 of z [H][W] (supplement Section
    Robustness), 0 in the leftmost zero_cols columns."""
    H, W = int(ref.shape[1]), int(ref.shape[2])
    ref = _dev_f32(ref, "reference", (3, H, W))
    z = _dev_f32(z, "z", (H, W))
    conf = torch.empty((H, W), dtype=torch.float32, device=z.device)
    ws = _dt_workspace(H, W, z.device, ws)
    p = L.DtParams(float(sigma_s), float(sigma_r), int(iters))
    L.check(L.lib.bs_dt_confidence(ref.data_ptr(), H, W, z.data_ptr(), ct.byref(p),
                                   float(sigma_dt), int(zero_cols), conf.data_ptr(),
                                   ws.data_ptr(), ws.numel(), _stream()),
            "bs_dt_confidence")
    return conf


class _BilateralSolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, target, conf, grid: BilateralGrid, fwd: dict, bwd: dict):
        y, _ = grid.solve(target, conf, **fwd)
        x = grid.slice(y, target.shape[0])
        ctx.grid, ctx.bwd = grid, bwd
        ctx.save_for_backward(target, conf, y)
        return x

    @staticmethod
    def backward(ctx, grad_x):
        target, conf, y = ctx.saved_tensors
        gt, gc, _, _ = ctx.grid.backward(target, conf, y, grad_x.contiguous(), **ctx.bwd)
        return gt, gc, None, None, None


def bilateral_solve(grid: BilateralGrid, target: torch.Tensor, conf: torch.Tensor, lam: float,
                    max_iters: int = 25, rel_tol: float = 0.0, init: str = "hier",
                    bwd_max_iters: int | None = None, bwd_rel_tol: float | None = None,
                    check_every: int = 8) -> torch.Tensor:
    """x_hat = S^T A^{-1} b, differentiable in `target` and `conf` (Section 3)."""
    fwd = dict(lam=lam, max_iters=max_iters, rel_tol=rel_tol, init=init, check_every=check_every)
    bwd = dict(lam=lam, max_iters=max_iters if bwd_max_iters is None else bwd_max_iters,
               rel_tol=rel_tol if bwd_rel_tol is None else bwd_rel_tol, init=init,
               check_every=check_every)
    return _BilateralSolveFn.apply(target, conf, grid, fwd, bwd)


class BatchState:
    """Grids, workspaces and solutions of a batch, kept from forward to backward."""

    def __init__(self, refs, targets, confs, sigmas, n_streams: int):
        n = len(refs)
        if not (len(targets) == len(confs) == len(sigmas) == n) or n == 0:
            raise ValueError("refs, targets, confs and sigmas must have the same non-zero length")
        self.n, self.n_streams = n, int(n_streams)
        self.items = (L.BatchItem * n)()
        self.grids = (L.Grid * n)()
        self.keep = []
        self.ys, self.grid_ws = [], []
        dev = refs[0].device
        for i, (ref, t, c, sg) in enumerate(zip(refs, targets, confs, sigmas)):
            H, W = int(ref.shape[1]), int(ref.shape[2])
            C = int(t.shape[0])
            ref = _dev_f32(ref, f"refs[{i}]", (3, H, W))
            t = _dev_f32(t, f"targets[{i}]", (C, H, W))
            c = _dev_f32(c, f"confs[{i}]", (H, W))
            gp = L.GridParams(*[int(v) for v in sg])
            nb = L.lib.bs_grid_workspace_bytes(H, W, ct.byref(gp))
            if nb == 0:
                raise ValueError(f"image {i}: " + L.lib.bs_last_error().decode())
            gws = torch.empty(nb, dtype=torch.uint8, device=dev)
            vcap = H * W
            y = torch.empty((vcap, C), dtype=torch.float32, device=dev)
            it = self.items[i]
            it.ref, it.target, it.conf = ref.data_ptr(), t.data_ptr(), c.data_ptr()
            it.H, it.W, it.C, it.sigma = H, W, C, gp
            it.grid_ws, it.grid_ws_bytes = gws.data_ptr(), nb
            it.y, it.x, it.grad_x, it.grad_t, it.grad_c, it.stats = y.data_ptr(), None, None, None, None, None
            self.keep += [ref, t, c]
            self.ys.append(y)
            self.grid_ws.append(gws)
        nbytes = L.lib.bs_batch_workspace_bytes(self.items, n, self.n_streams)
        if nbytes == 0:
            raise ValueError("invalid batch")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.shapes = [(int(t.shape[0]), int(r.shape[1]), int(r.shape[2]))
                       for r, t in zip(refs, targets)]
        self.device = dev

    def vertex_counts(self) -> list[int]:
        """V of every image's grid (after forward; synchronises the stream)."""
        out = []
        for i in range(self.n):
            v = ct.c_int32()
            L.check(L.lib.bs_grid_vertex_count(ct.byref(self.grids[i]), ct.byref(v), _stream()),
                    "bs_grid_vertex_count")
            out.append(int(v.value))
        return out

    def forward(self, opts: SolveOptions, bist_tol=1e-10, bist_max_iters=200, stats=False):
        xs = [torch.empty(s, dtype=torch.float32, device=self.device) for s in self.shapes]
        st = [torch.empty(s[0] * _STATS_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
              for s in self.shapes] if stats else None
        for i, x in enumerate(xs):
            self.items[i].x = x.data_ptr()
            self.items[i].stats = st[i].data_ptr() if stats else None
        p = opts.struct()
        b = L.BistochParams(int(bist_max_iters), 8, float(bist_tol))
        L.check(L.lib.bs_batch_forward(self.items, self.n, ct.byref(p), ct.byref(b), self.grids,
                                       self.n_streams, self.ws.data_ptr(), self.ws.numel(),
                                       _stream()), "bs_batch_forward")
        for i in range(self.n):
            self.items[i].x = None
        return xs, st

    def forward_lowrank(self, opts: SolveOptions, eps: float, bist_tol=1e-10,
                        bist_max_iters=200, stats=False):
        """Forward pass through the low-rank reduction of every image's
        right-hand sides: outputs, stats (first rank entries) and ranks."""
        nbytes = L.lib.bs_batch_lowrank_workspace_bytes(self.items, self.n, self.n_streams)
        if nbytes == 0:
            raise ValueError("invalid batch")
        if getattr(self, "ws_lowrank", None) is None or self.ws_lowrank.numel() < nbytes:
            self.ws_lowrank = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        xs = [torch.empty(s, dtype=torch.float32, device=self.device) for s in self.shapes]
        st = [torch.zeros(s[0] * _STATS_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
              for s in self.shapes] if stats else None
        for i, x in enumerate(xs):
            self.items[i].x = x.data_ptr()
            self.items[i].stats = st[i].data_ptr() if stats else None
        ranks = (ct.c_int32 * self.n)()
        p = opts.struct()
        b = L.BistochParams(int(bist_max_iters), 8, float(bist_tol))
        L.check(L.lib.bs_batch_forward_lowrank(self.items, self.n, ct.byref(p), ct.byref(b),
                                               self.grids, self.n_streams, float(eps), ranks,
                                               self.ws_lowrank.data_ptr(),
                                               self.ws_lowrank.numel(), _stream()),
                "bs_batch_forward_lowrank")
        for i in range(self.n):
            self.items[i].x = None
        return xs, st, [int(r) for r in ranks]

    def backward(self, grad_xs, opts: SolveOptions, stats=False):
        gts = [torch.empty(s, dtype=torch.float32, device=self.device) for s in self.shapes]
        gcs = [torch.empty(s[1:], dtype=torch.float32, device=self.device) for s in self.shapes]
        st = [torch.empty(s[0] * _STATS_DTYPE.itemsize, dtype=torch.uint8, device=self.device)
              for s in self.shapes] if stats else None
        gx_keep = []
        for i, (g, gt, gc) in enumerate(zip(grad_xs, gts, gcs)):
            g = _dev_f32(g, f"grad_x[{i}]", self.shapes[i])
            gx_keep.append(g)
            it = self.items[i]
            it.grad_x, it.grad_t, it.grad_c = g.data_ptr(), gt.data_ptr(), gc.data_ptr()
            it.stats = st[i].data_ptr() if stats else None
        p = opts.struct()
        L.check(L.lib.bs_batch_backward(self.items, self.n, self.grids, ct.byref(p),
                                        self.n_streams, self.ws.data_ptr(), self.ws.numel(),
                                        _stream()), "bs_batch_backward")
        return gts, gcs, st


class BatchPlan:
    """A batch laid out once (``bs_batch_plan_create``): many images of uneven
    size and channel count, with their inputs, outputs and workspace bound.

    ``forward()`` and ``backward()`` run the whole path over every image;
    with ``check_every = 0`` in the options (and ``bist_check_every = 0``)
    they only enqueue kernels on the current stream, so ``capture()`` can
    record them into one graph, replayed with fixed iteration counts.  Write
    new inputs into ``targets``, ``confs`` and ``grad_xs`` (in place) between
    runs; ``xs``, ``ys``, ``grad_ts`` and ``grad_cs`` receive the outputs."""

    def __init__(self, refs, targets, confs, sigmas, fwd: SolveOptions,
                 bwd: SolveOptions | None = None, bist_tol: float = 1e-10,
                 bist_max_iters: int = 200, bist_check_every: int = 0, slice_out: bool = True):
        n = len(refs)
        if not (len(targets) == len(confs) == len(sigmas) == n) or n == 0:
            raise ValueError("refs, targets, confs and sigmas must have the same non-zero length")
        self.n = n
        dev = refs[0].device
        self.device = dev
        self.shapes = []
        self.refs, self.targets, self.confs = [], [], []
        self.ys, self.xs, self.stats = [], [], []
        self.grad_xs, self.grad_ts, self.grad_cs = [], [], []
        self.items = (L.BatchItem * n)()
        for i, (ref, t, c, sg) in enumerate(zip(refs, targets, confs, sigmas)):
            H, W, C = int(ref.shape[1]), int(ref.shape[2]), int(t.shape[0])
            self.shapes.append((C, H, W))
            ref = _dev_f32(ref, f"refs[{i}]", (3, H, W))
            t = _dev_f32(t, f"targets[{i}]", (C, H, W))
            c = _dev_f32(c, f"confs[{i}]", (H, W))
            self.refs.append(ref)
            self.targets.append(t)
            self.confs.append(c)
            y = torch.empty((H * W, C), dtype=torch.float32, device=dev)
            x = torch.empty((C, H, W), dtype=torch.float32, device=dev) if slice_out else None
            st = torch.zeros(C * _STATS_DTYPE.itemsize, dtype=torch.uint8, device=dev)
            self.ys.append(y)
            self.xs.append(x)
            self.stats.append(st)
            it = self.items[i]
            it.ref, it.target, it.conf = ref.data_ptr(), t.data_ptr(), c.data_ptr()
            it.H, it.W, it.C = H, W, C
            it.sigma = L.GridParams(*[int(v) for v in sg])
            it.grid_ws, it.grid_ws_bytes = None, 0
            it.y, it.x = y.data_ptr(), (x.data_ptr() if x is not None else None)
            it.stats = st.data_ptr()
            if bwd is not None:
                gx = torch.zeros((C, H, W), dtype=torch.float32, device=dev)
                gt = torch.empty((C, H, W), dtype=torch.float32, device=dev)
                gc = torch.empty((H, W), dtype=torch.float32, device=dev)
                self.grad_xs.append(gx)
                self.grad_ts.append(gt)
                self.grad_cs.append(gc)
                it.grad_x, it.grad_t, it.grad_c = gx.data_ptr(), gt.data_ptr(), gc.data_ptr()
        nbytes = L.lib.bs_batch_plan_workspace_bytes(self.items, n)
        if nbytes == 0:
            raise ValueError("invalid batch")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.fwd, self.bwd = fwd, bwd
        pf = fwd.struct()
        pb = bwd.struct() if bwd is not None else None
        bp = L.BistochParams(int(bist_max_iters), int(bist_check_every), float(bist_tol))
        plan = ct.c_void_p()
        L.check(L.lib.bs_batch_plan_create(self.items, n, ct.byref(pf),
                                           ct.byref(pb) if pb is not None else None, ct.byref(bp),
                                           self.ws.data_ptr(), self.ws.numel(), _stream(),
                                           ct.byref(plan)), "bs_batch_plan_create")
        self._plan = plan

    def forward(self) -> None:
        L.check(L.lib.bs_batch_run_forward(self._plan, _stream()), "bs_batch_run_forward")

    def backward(self) -> None:
        if self.bwd is None:
            raise ValueError("the plan was made without backward options")
        L.check(L.lib.bs_batch_run_backward(self._plan, _stream()), "bs_batch_run_backward")

    def capture(self, backward: bool = True) -> "torch.cuda.CUDAGraph":
        """A graph of one forward (and backward) run, for replay."""
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            self.forward()
            if backward:
                self.backward()
        return graph

    def grid(self, i: int) -> L.Grid:
        g = L.Grid()
        L.check(L.lib.bs_batch_plan_grid(self._plan, int(i), ct.byref(g)), "bs_batch_plan_grid")
        return g

    def bist_iters(self) -> list[int]:
        """Bistochastization updates every image's grid took in the last
        forward run (its cap when it did not converge; synchronises)."""
        out = []
        for i in range(self.n):
            g = self.grid(i)
            c = (ct.c_int32 * 3)()
            L.check(L.lib.bs_read_counters(ct.byref(g), c, 3, _stream()), "bs_read_counters")
            out.append(int(c[2]))   # the counter of updates applied
        return out

    def vertex_counts(self) -> list[int]:
        """V of every image's grid (after a forward run; synchronises the stream)."""
        out = []
        for i in range(self.n):
            g = self.grid(i)
            v = ct.c_int32()
            L.check(L.lib.bs_grid_vertex_count(ct.byref(g), ct.byref(v), _stream()),
                    "bs_grid_vertex_count")
            out.append(int(v.value))
        return out

    def read_stats(self) -> list:
        return [read_stats(st) for st in self.stats]

    def close(self) -> None:
        if getattr(self, "_plan", None) is not None and self._plan.value:
            L.lib.bs_batch_plan_destroy(self._plan)
            self._plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _BatchSolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, meta, *tensors):
        n = meta["n"]
        refs, targets, confs = tensors[:n], tensors[n:2 * n], tensors[2 * n:]
        state = BatchState(refs, targets, confs, meta["sigmas"], meta["n_streams"])
        xs, _ = state.forward(meta["fwd"])
        ctx.state, ctx.meta = state, meta
        return tuple(xs)

    @staticmethod
    def backward(ctx, *grad_xs):
        n = ctx.meta["n"]
        gts, gcs, _ = ctx.state.backward([g.contiguous() for g in grad_xs], ctx.meta["bwd"])
        return (None,) + (None,) * n + tuple(gts) + tuple(gcs)


def bilateral_solve_batch(refs, targets, confs, sigmas, lam: float, max_iters: int = 25,
                          rel_tol: float = 0.0, bwd_max_iters: int | None = None,
                          bwd_rel_tol: float | None = None, init: str = "hier",
                          n_streams: int = 4):
    """x_hat for a batch of images of any sizes and channel counts (lists of
    tensors), differentiable in the targets and confidences."""
    n = len(refs)
    meta = dict(n=n, sigmas=[tuple(s) for s in sigmas], n_streams=n_streams,
                fwd=SolveOptions(lam, max_iters, rel_tol, init),
                bwd=SolveOptions(lam, max_iters if bwd_max_iters is None else bwd_max_iters,
                                 rel_tol if bwd_rel_tol is None else bwd_rel_tol, init))
    return list(_BatchSolveFn.apply(meta, *refs, *targets, *confs))
