"""Learned lookup tables for a parameterised family of reference tiles.

The paper builds one lookup table per reference tile (eq. (52)) in an offline
step.  For a family of tiles described by a few design parameters this module
replaces the per-design build by a POD basis of the family's tables and a small
MLP from the parameters to the POD coefficients; the exact table builder stays
the fallback and the check: a seeded subset of table rows is built exactly and
compared with the learned table, and the exact table replaces it when the
estimated relative error exceeds the tolerance.  The per-design path queues
everything on the stream, the fallback decision included.

Every numerical step runs in libigamt kernels (table builder, POD Gram and
modes, MLP forward/backward/Adam, reconstruction, row error); this module only
prepares inputs (parameter scaling, target scaling, initial weights) and drives
the loop.
"""
from __future__ import annotations

import ctypes as C
import math
import time
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import check, lib


def _torch():
    import torch
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(_torch().cuda.current_stream().cuda_stream)


class MLP:
    """Flat-parameter MLP driven by the library kernels (FP32)."""

    def __init__(self, widths: Sequence[int], batch: int, seed: int = 0):
        torch = _torch()
        self.desc = _lib.MlpDesc()
        self.desc.n_layers = len(widths) - 1
        for i, wd in enumerate(widths):
            self.desc.widths[i] = int(wd)
        self.desc.batch = int(batch)
        self.widths = list(widths)
        n = lib().igamt_mlp_n_params(C.byref(self.desc))
        if n <= 0:
            raise ValueError("invalid MLP shape")
        rng = np.random.default_rng(seed)
        host = []
        for fi, fo in zip(widths[:-1], widths[1:]):
            bound = 1.0 / math.sqrt(fi)
            host.append(rng.uniform(-bound, bound, size=fi * fo))
            host.append(np.zeros(fo))
        self.params = torch.from_numpy(np.concatenate(host).astype(np.float32)).cuda()
        assert self.params.numel() == n
        self.n_params = n
        self._alloc(batch)

    def _alloc(self, batch):
        torch = _torch()
        self.desc.batch = int(batch)
        self.act = torch.empty(batch * sum(self.widths[1:]), dtype=torch.float32, device="cuda")
        self.y = torch.empty((batch, self.widths[-1]), dtype=torch.float32, device="cuda")

    def set_batch(self, batch):
        if batch != self.desc.batch:
            self._alloc(batch)

    def forward(self, x):
        self.set_batch(x.shape[0])
        check(lib().igamt_mlp_forward(C.byref(self.desc), _ptr(self.params), _ptr(x), _ptr(self.act), _ptr(self.y),
                                      _stream()))
        return self.y

    def param_views(self):
        """(W, b) views of the flat parameters, for inspection."""
        out, off = [], 0
        for fi, fo in zip(self.widths[:-1], self.widths[1:]):
            W = self.params[off:off + fi * fo].view(fi, fo)
            off += fi * fo
            b = self.params[off:off + fo]
            off += fo
            out.append((W, b))
        return out


class Trainer:
    """Full-batch Adam on the mean-squared error, all steps in library kernels."""

    def __init__(self, mlp: MLP, x, target, lr=1e-3, lr_min=1e-5, betas=(0.9, 0.999), eps=1e-8):
        torch = _torch()
        self.mlp = mlp
        self.x = x.contiguous()
        self.t = target.contiguous()
        B = x.shape[0]
        mlp.set_batch(B)
        self.dy = torch.empty_like(mlp.y)
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.grads = torch.zeros_like(mlp.params)
        self.m = torch.zeros_like(mlp.params)
        self.v = torch.zeros_like(mlp.params)
        self.scratch = torch.empty(2 * B * max(mlp.widths), dtype=torch.float32, device="cuda")
        self.lr, self.lr_min, self.betas, self.eps = lr, lr_min, betas, eps
        self.step_no = 0

    def step(self, lr):
        L = lib()
        d = C.byref(self.mlp.desc)
        s = _stream()
        check(L.igamt_mlp_forward(d, _ptr(self.mlp.params), _ptr(self.x), _ptr(self.mlp.act), _ptr(self.mlp.y), s))
        check(L.igamt_mse_loss(d, _ptr(self.mlp.y), _ptr(self.t), _ptr(self.dy), _ptr(self.loss), s))
        check(L.igamt_mlp_backward(d, _ptr(self.mlp.params), _ptr(self.x), _ptr(self.mlp.act), _ptr(self.dy),
                                   _ptr(self.grads), _ptr(self.scratch), s))
        self.step_no += 1
        check(L.igamt_adam_step(_ptr(self.mlp.params), _ptr(self.grads), _ptr(self.m), _ptr(self.v),
                                self.mlp.n_params, float(lr), float(self.betas[0]), float(self.betas[1]),
                                float(self.eps), self.step_no, s))

    def run(self, steps, log_every=0):
        """Cosine decay from lr to lr_min over `steps`; returns the loss history at log points."""
        hist = []
        for i in range(1, steps + 1):
            lr = self.lr_min + 0.5 * (self.lr - self.lr_min) * (1 + math.cos(math.pi * i / steps))
            self.step(lr)
            if log_every and (i % log_every == 0 or i == steps):
                hist.append((i, float(self.loss.item())))
        return hist


class TableNet:
    """POD + MLP model of the lookup tables of a tile family, on one plan's topology.

    plan: a Plan whose reference tile belongs to the family (same knots and degree);
    params_lo/hi: the box of design parameters (inputs are mapped to [-1, 1]).
    """

    def __init__(self, plan, rank=64, hidden=(128, 128), params_lo=0.0, params_hi=0.3, seed=0, tol=1e-3,
                 n_check_rows=64):
        self.plan = plan
        self.rank = rank
        self.hidden = tuple(hidden)
        self.lo, self.hi = float(params_lo), float(params_hi)
        self.seed = seed
        self.tol = tol
        self.n_e = plan.n_pairs * plan.n_cols
        rng = np.random.default_rng(seed + 17)
        self.check_rows = np.sort(rng.choice(plan.n_pairs, size=min(n_check_rows, plan.n_pairs), replace=False))
        self.mlp: Optional[MLP] = None

    def scale_inputs(self, p):
        torch = _torch()
        x = (np.asarray(p, dtype=np.float64) - self.lo) / (self.hi - self.lo) * 2.0 - 1.0
        return torch.from_numpy(x.astype(np.float32)).cuda()

    def _buffers(self):
        """Device buffers of the per-design path and pinned host staging (allocated once)."""
        torch = _torch()
        if getattr(self, "_dev", None) is None:
            n_c = 3 * self.plan.n_tile_ctrl
            self._dev = {
                "rows": torch.from_numpy(self.check_rows.astype(np.int32)).cuda(),
                "ctrl": torch.empty(n_c, dtype=torch.float64, device="cuda"),
                "x": torch.empty((1, 4), dtype=torch.float32, device="cuda"),
                "err": torch.empty(1, dtype=torch.float64, device="cuda"),
                "gate": torch.empty(1, dtype=torch.int32, device="cuda"),
                "exact_rows": torch.empty((len(self.check_rows), self.plan.n_cols), dtype=torch.float64,
                                          device="cuda"),
                "h_ctrl": torch.empty(n_c, dtype=torch.float64).pin_memory(),
                "h_x": torch.empty((1, 4), dtype=torch.float32).pin_memory(),
                "copied": torch.cuda.Event(),
            }
        return self._dev

    def _upload(self, p, tile_ctrl):
        """Design parameters (scaled to [-1, 1]) and tile control points to the device, asynchronously."""
        torch = _torch()
        b = self._buffers()
        b["copied"].synchronize()          # the staging buffers of the previous design have been read
        x = (np.asarray(p, dtype=np.float64).reshape(1, -1) - self.lo) / (self.hi - self.lo) * 2.0 - 1.0
        b["h_x"].numpy()[...] = x
        b["h_ctrl"].numpy()[...] = np.ascontiguousarray(tile_ctrl, dtype=np.float64).ravel()
        b["x"].copy_(b["h_x"], non_blocking=True)
        b["ctrl"].copy_(b["h_ctrl"], non_blocking=True)
        b["copied"].record()
        return b

    # ---- offline ----------------------------------------------------------------------
    def exact_tables(self, tile_ctrls):
        """Exact FP64 tables of the given designs (device table builder), shape (n, n_e)."""
        torch = _torch()
        out = torch.empty((len(tile_ctrls), self.n_e), dtype=torch.float64, device="cuda")
        chunk = 64
        for i in range(0, len(tile_ctrls), chunk):
            c = np.stack([np.ascontiguousarray(t, dtype=np.float64) for t in tile_ctrls[i:i + chunk]])
            c = torch.from_numpy(c.reshape(len(c), -1)).cuda()
            self.plan.tables_build_batch(c, out=out[i:i + len(c)])
        self.plan.check()
        return out

    def fit_pod(self, snaps):
        torch = _torch()
        self._graph = None        # a captured graph reads the old mean and basis
        n_s = snaps.shape[0]
        self.mean = torch.empty(self.n_e, dtype=torch.float32, device="cuda")
        self.basis = torch.empty((self.rank, self.n_e), dtype=torch.float32, device="cuda")
        sigma = np.empty(n_s)
        coeffs = np.empty((n_s, self.rank))
        work = torch.empty(17 * n_s * n_s + n_s * self.rank + self.n_e, dtype=torch.float64, device="cuda")
        check(lib().igamt_pod_build(_ptr(snaps.contiguous()), n_s, self.n_e, self.rank, _ptr(self.mean),
                                    _ptr(self.basis), sigma.ctypes.data_as(C.c_void_p),
                                    coeffs.ctypes.data_as(C.c_void_p), _ptr(work), _stream()))
        del work
        self.sigma = sigma
        self.train_coeffs = coeffs
        # targets scaled so that the leading mode has unit root-mean-square over the snapshots
        self.coeff_scale = sigma[0] / math.sqrt(n_s)
        return sigma, coeffs

    def train(self, params, steps=8000, lr=2e-3, lr_min=1e-5, log_every=1000):
        torch = _torch()
        x = self.scale_inputs(params)
        t = torch.from_numpy((self.train_coeffs / self.coeff_scale).astype(np.float32)).cuda()
        self.mlp = MLP([x.shape[1], *self.hidden, self.rank], batch=x.shape[0], seed=self.seed)
        self._graph = None        # a captured graph reads the old network's parameters
        if getattr(self, "_dev", None) is not None:
            self._dev.pop("desc1", None)
        tr = Trainer(self.mlp, x, t, lr=lr, lr_min=lr_min)
        t0 = time.perf_counter()
        hist = tr.run(steps, log_every)
        torch.cuda.synchronize()
        self.train_seconds = time.perf_counter() - t0
        return hist

    # ---- online ------------------------------------------------------------------------
    def predict_coeffs(self, p):
        x = self.scale_inputs(np.atleast_2d(p))
        return self.mlp.forward(x)

    def table_for_async(self, p, tile_ctrl):
        """Queue the table of design p (tile control points tile_ctrl) into the plan: learned
        reconstruction, exact rebuild of the check rows, error estimate, and the exact table in
        place of the learned one when the estimate exceeds the tolerance -- the decision is taken
        on the device, nothing waits on the host.  Returns device tensors (estimated relative
        error [1] float64, fallback flag [1] int32)."""
        self._upload(p, tile_ctrl)
        self._enqueue_learned()
        b = self._buffers()
        return b["err"], b["gate"]

    def table_for_device(self, x, tile_ctrl):
        """table_for_async for a design already on the device: x its parameters scaled by
        scale_inputs (float32 [1, 4]), tile_ctrl its tile control points (float64, n_tile_ctrl x 3
        values).  Returns the same device tensors."""
        torch = _torch()
        if not (x.is_cuda and tile_ctrl.is_cuda and x.dtype == torch.float32 and tile_ctrl.dtype == torch.float64
                and x.numel() == 4 and tile_ctrl.numel() == 3 * self.plan.n_tile_ctrl):
            raise ValueError("x must be float32 [1, 4] and tile_ctrl float64 [n_tile_ctrl x 3], both on the device")
        self._enqueue_learned(x.contiguous(), tile_ctrl.contiguous())
        b = self._buffers()
        return b["err"], b["gate"]

    def tables_for_batch(self, params, tile_ctrls):
        """Tables of a batch of designs (params [B, 4], tile control points as a device float64
        tensor [B, n_tile_ctrl, 3]) into a dense [B, n_pairs, n_cols] tensor: one MLP forward over
        the batch, one reconstruction that reads the POD basis once per group of designs, exact
        check rows of every design, and exact tables for the designs whose estimated error
        exceeds the tolerance, all queued on the stream.  Returns (tables, estimated relative
        errors [B] float64, fallback flags [B] int32), all on the device."""
        torch = _torch()
        B = int(tile_ctrls.shape[0])
        assert tile_ctrls.is_cuda and tile_ctrls.dtype == torch.float64 and tile_ctrls.is_contiguous()
        rows = self._buffers()["rows"]
        x = self.scale_inputs(np.atleast_2d(params))
        assert x.shape[0] == B
        self.mlp.set_batch(B)
        r = self.rank
        work = torch.empty(lib().igamt_pod_batch_work_doubles(r, B), dtype=torch.float64, device="cuda")
        exact_rows = torch.empty((B, rows.numel(), self.plan.n_cols), dtype=torch.float64, device="cuda")
        err = torch.empty(B, dtype=torch.float64, device="cuda")
        gate = torch.empty(B, dtype=torch.int32, device="cuda")
        tables = torch.empty((B, self.plan.n_pairs, self.plan.n_cols), dtype=torch.float64, device="cuda")
        check(lib().igamt_tables_learned_batch(self.plan._h, C.byref(self.mlp.desc), _ptr(self.mlp.params), _ptr(x),
                                               _ptr(self.mlp.act), _ptr(self.mlp.y), _ptr(self.mean),
                                               _ptr(self.basis), float(self.coeff_scale), _ptr(tile_ctrls),
                                               _ptr(rows), int(rows.numel()), _ptr(exact_rows), float(self.tol),
                                               _ptr(err), _ptr(gate), _ptr(work), _ptr(tables), _stream()))
        return tables, err, gate

    def _enqueue_learned(self, x=None, ctrl=None):
        """Queue the per-design learned path on the current stream, reading the design from the
        device buffers x and ctrl, or from the given device tensors (no host work, no allocation):
        the MLP runs with a batch-1 descriptor and activation buffers of its own, which no later
        call reallocates."""
        b = self._buffers()
        x = b["x"] if x is None else x
        ctrl = b["ctrl"] if ctrl is None else ctrl
        if "desc1" not in b:
            torch = _torch()
            b["desc1"] = _lib.MlpDesc()
            b["desc1"].n_layers = self.mlp.desc.n_layers
            for i in range(len(self.mlp.widths)):
                b["desc1"].widths[i] = self.mlp.widths[i]
            b["desc1"].batch = 1
            b["act1"] = torch.empty(sum(self.mlp.widths[1:]), dtype=torch.float32, device="cuda")
            b["y1"] = torch.empty((1, self.mlp.widths[-1]), dtype=torch.float32, device="cuda")
        self.plan.set_tile_ctrl(ctrl)
        check(lib().igamt_table_learned(self.plan._h, C.byref(b["desc1"]), _ptr(self.mlp.params), _ptr(x),
                                        _ptr(b["act1"]), _ptr(b["y1"]), _ptr(self.mean), _ptr(self.basis),
                                        float(self.coeff_scale), _ptr(b["rows"]), int(b["rows"].numel()),
                                        _ptr(b["exact_rows"]), float(self.tol), _ptr(b["err"]), _ptr(b["gate"]),
                                        _stream()))

    def table_for_graph(self, p, tile_ctrl):
        """The per-design path of table_for_async replayed from a HIP graph: the dozen kernel
        launches are captured once (on the first call, after one eager run that allocates the
        scratch buffers) and replayed for every design, so a design costs one graph launch.
        Returns the same device tensors (estimated error [1], fallback flag [1])."""
        torch = _torch()
        b = self._upload(p, tile_ctrl)
        if getattr(self, "_graph", None) is None:
            self._enqueue_learned()                    # eager: allocates the scratch buffers
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()                 # default priority
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                with torch.cuda.graph(g, stream=side):
                    self._enqueue_learned()
            torch.cuda.current_stream().wait_stream(side)
            self._graph = g
        self._graph.replay()
        return b["err"], b["gate"]

    def table_for(self, p, tile_ctrl, force_exact=False):
        """Put the table of design p (tile control points tile_ctrl) into the plan.

        Returns (estimated relative error of the learned table on the check rows,
        True if the exact builder was used)."""
        if force_exact:
            self.plan.set_tile_ctrl(tile_ctrl)
            self.plan.tables_build()
            return float("nan"), True
        err, gate = self.table_for_async(p, tile_ctrl)
        return float(err.item()), bool(gate.item())
