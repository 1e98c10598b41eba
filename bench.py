#!/usr/bin/env python3
"""Benchmark of the lookup-table stiffness assembly on one MI355X.

A step is one pass of the assembly path over the synthetic workload: the FP64
macro-field fit, the MFMA contraction of eq. (58) and the deterministic scatter
into the CSR structure (plan, CSR structure and lookup table are built once,
outside the timed region, as in the paper's timing convention).  Inputs are
resident in HBM before timing starts.

Prints ONE JSON line (rank 0): the tile-block rate of the FP64 step, the
contraction kernel's roofline figures (algorithmic FLOPs per launch over its
average launch time from HIP events on its stream, against the FP64 MFMA peak,
with the HBM bytes of the committed byte-counter summary when its source hash
matches), the split-precision variants, the next rows' kernels, and the oracle
timed on a bounded sample of tiles on the host cores.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tile stiffness blocks/s + % MFMA peak; mixed/learned vs plain FP64 @ rel.err"
PEAK = {"f64": 78.6e12, "f32": 157.3e12, "bf16x3": 2.5e15, "f16x3": 2.5e15}   # dense MFMA, FLOP/s
HBM_PEAK = 8.0e12
WORKLOADS = {
    "cfg3": "torus sector, 32x32x32 tiles, degree-2 macro map, degree-2 3x3x3-element tile, q=2",
    "cfg2": "curved cantilever, 16x4x4 tiles, degree-3 macro map, degree-3 4x4x4-element tile, q=3",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash(path):
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def pmc_traffic(kernel_src, config, prec):
    """HBM bytes per launch of the contraction from a committed rocprofv3 --pmc summary, or None if
    absent or taken on a different version of the kernel source."""
    path = os.path.join(ROOT, "profiles", f"contract_{prec}_{config}_pmc.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"source_sha256_16:\s*([0-9a-f]+)", text)
    b = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m or not b or m.group(1) != source_hash(kernel_src):
        return None
    return float(b.group(1))


def _timed(torch, steps, calls):
    """Run `calls` (callables) `steps` times with HIP events between them on torch's stream;
    returns per-step durations [steps, len(calls)] in ms."""
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(calls) + 1)] for _ in range(steps)]
    for k in range(steps):
        ev[k][0].record()
        for i, c in enumerate(calls):
            c()
            ev[k][i + 1].record()
    torch.cuda.synchronize()
    return np.array([[ev[k][i].elapsed_time(ev[k][i + 1]) for i in range(len(calls))] for k in range(steps)])


def time_stages(torch, plan, w, prec, steps, warmup, ws):
    cb, bb = plan.workspace_bytes(prec)
    coef = ws
    blocks = ws.view(torch.uint8)[cb:].view(torch.float64 if prec == "f64" else torch.float32)
    dt = torch.float64 if prec == "f64" else torch.float32
    vals = torch.empty(plan.nnz, dtype=dt, device="cuda")
    for _ in range(warmup):
        plan.fit(w.E, w.nu, prec, out=coef)
        plan.contract(coef, prec, out=blocks)
        plan.scatter(blocks, prec, out=vals)
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    t0 = time.perf_counter()
    for s in range(steps):
        ev[s][0].record()
        plan.fit(w.E, w.nu, prec, out=coef)
        ev[s][1].record()
        plan.contract(coef, prec, out=blocks)
        ev[s][2].record()
        plan.scatter(blocks, prec, out=vals)
        ev[s][3].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.check()
    st = np.array([[ev[s][i].elapsed_time(ev[s][i + 1]) for i in range(3)] for s in range(steps)])
    # the step proper: igamt_assemble (the three stages in one call)
    for _ in range(warmup):
        plan.assemble(w.E, w.nu, prec, values=vals, workspace=ws)
    torch.cuda.synchronize()
    ea = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in ea:
        a.record()
        plan.assemble(w.E, w.nu, prec, values=vals, workspace=ws)
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.check()
    step = np.array([a.elapsed_time(b) for a, b in ea])
    return {"wall_s": wall, "fit_ms": st[:, 0], "contract_ms": st[:, 1], "scatter_ms": st[:, 2],
            "serial_step_ms": st.sum(axis=1), "step_ms": step}, vals, blocks


def rigid_residuals(torch, P, rp, ci, vals):
    """K times the three rigid translations t_a (1 on every dof of component a): the translations lie
    in the kernel of K exactly (the table's row sums vanish), so the residual measures the rounding of
    the assembled values.  Reported as |K t_a| / (|K|_F |t_a|) and as the worst row's
    |(K t_a)_i| / sum_j |K_ij| (the cancellation left in one row), maxima over a."""
    import math
    n = rp.numel() - 1
    dt = vals.dtype
    kf = torch.linalg.vector_norm(vals, dtype=torch.float64).item()
    rowabs = P.spmv(rp, ci, vals.abs(), torch.ones(n, dtype=dt, device="cuda")).double()
    p6 = row = 0.0
    for a in range(3):
        t = torch.zeros(n, dtype=dt, device="cuda")
        t[a::3] = 1
        y = P.spmv(rp, ci, vals, t)
        p6 = max(p6, torch.linalg.vector_norm(y, dtype=torch.float64).item() / (kf * math.sqrt(n / 3)))
        row = max(row, (y.abs().double() / rowabs.clamp_min(1e-300)).max().item())
        del t, y
    return {"normalized": p6, "worst_row": row}


def oracle_comparisons(w, sample, gpu_sample_blocks, cfg1_gpu):
    """The precision study against the FP64 oracle (part of the CPU-baseline leg): per-tile relative
    Frobenius error of every precision's blocks on the sampled tiles, and on the 2x2x2-tile workload
    E_mat (eq. (62)) and E_vec (eq. (63)) of the GPU's K^pi and f^pi against the oracle's plain
    Gauss-quadrature K and f."""
    from oracle import assembly, load, projection, standard, tables
    pairs = tables.pair_set(w.tile)
    table = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
    ref = assembly.tile_blocks(table, projection.all_coefficients(w, sample))
    rn = np.linalg.norm(ref.reshape(len(sample), -1), axis=1)
    out = {"sample_tiles": int(len(sample))}
    for name, blk in gpu_sample_blocks.items():
        e = np.linalg.norm((blk - ref).reshape(len(sample), -1), axis=1) / rn
        out[name] = {"max_tile_block_rel_err": float(e.max()), "median_tile_block_rel_err": float(np.median(e))}
    # E_mat / E_vec on the small workload, for each projection degree the GPU ran
    w1 = cfg1_gpu["workload"]
    pairs1 = tables.pair_set(w1.tile)
    kb = np.stack([standard.tile_block_standard(w1, t, pairs1) for t in range(w1.n_tiles)])
    rp, ci, kbull = assembly.assemble_csr(w1, pairs1, kb)
    fb = load.standard_load(w1, cfg1_gpu["body"], cfg1_gpu["traction"])
    em = {}
    for q, (vals, blocks, f) in cfg1_gpu["by_q"].items():
        tile_err = np.linalg.norm((blocks - kb).reshape(w1.n_tiles, -1), axis=1) / \
            np.linalg.norm(kb.reshape(w1.n_tiles, -1), axis=1)
        em[f"q{q}"] = {"E_mat": float(np.linalg.norm(vals - kbull) / np.linalg.norm(kbull)),
                       "E_mat_max_tile": float(tile_err.max()),
                       "E_vec": float(np.linalg.norm(f - fb) / np.linalg.norm(fb))}
    out["E_mat_E_vec_2x2x2_tiles"] = em
    return out


def cfg1_gpu_results(torch, W, P):
    """GPU K^pi (FP64 CSR values and tile blocks) and f^pi on the 2x2x2-tile workload at q = 1..4, for
    E_mat and E_vec against the oracle's Gauss-quadrature operators."""
    import dataclasses
    w = W.make("cfg1")
    body = np.array([0.0, 0.0, -1.0])
    traction = np.zeros((6, 3))
    traction[1] = [0.0, 0.0, -1.0]
    by_q = {}
    for q in (1, 2, 3, 4):
        wq = dataclasses.replace(w, q=q, n_fit=q + 1)
        plan = P.Plan.from_workload(wq)
        plan.tables_build()
        plan.load_table_build()
        blocks = plan.contract(plan.fit(wq.E, wq.nu, "f64"), "f64")
        vals = plan.scatter(blocks, "f64")
        f = plan.load_assemble(body, traction)
        plan.check()
        by_q[q] = (vals.cpu().numpy(), blocks.cpu().numpy(), f.cpu().numpy())
    return {"workload": w, "body": body, "traction": traction, "by_q": by_q}


def cpu_baseline(w, n_sample, seed=11, one_thread=False):
    """The CPU oracle on a seeded sample of tiles: fit + table contraction + CSR scatter of the sample
    (with all host threads, or with one BLAS thread)."""
    if one_thread:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            r = cpu_baseline(w, n_sample, seed)
        r["cores"] = 1
        return r
    from oracle import assembly, projection, tables
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count()
    pairs = tables.pair_set(w.tile)
    table = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)     # prebuilt, not timed
    rng = np.random.default_rng(seed)
    sample = np.sort(rng.choice(w.n_tiles, size=n_sample, replace=False))
    t0 = time.perf_counter()
    coefs = projection.all_coefficients(w, sample)
    blocks = assembly.tile_blocks(table, coefs)
    t_nz = time.perf_counter() - t0
    rows, cols, vals = assembly.coo_entries(w, pairs, blocks, sample)
    assembly.csr_from_coo(3 * int(np.prod([w.tiles[k] * (w.tile.n_ctrl[k] - 1) + 1 for k in range(3)])),
                          rows, cols, vals)
    dt = time.perf_counter() - t0
    return {"value": n_sample / dt, "unit": "tile blocks/s", "cores": int(threads), "kind": "oracle",
            "value_nonzeros_only": n_sample / t_nz,
            "cpu_model": _cpu_model(),
            "sample": f"{n_sample} seeded tiles of the same workload (fit + contraction + CSR of the sample), "
                      f"{dt:.1f} s, of which fit + contraction (the nonzeros alone, the paper's timing scope) "
                      f"{t_nz:.1f} s; host has {os.cpu_count()} logical CPUs"}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def bench_load(torch, plan, steps, warmup):
    """Load vector f^pi (body force and face tractions) on the assembly workload: the projection
    coefficients of every tile, then the gather into the global vector (table prebuilt)."""
    body = np.array([0.0, 0.0, -1.0])
    traction = np.zeros((6, 3))
    traction[1] = [0.0, 0.5, 0.0]
    traction[5] = [0.2, 0.0, -0.3]
    plan.load_table_build()
    coef = plan.load_fit(body, traction)
    f = plan.load_gather(coef)
    for _ in range(warmup):
        plan.load_fit(body, traction, out=coef)
        plan.load_gather(coef, out=f)
    st = _timed(torch, steps, [lambda: plan.load_fit(body, traction, out=coef), lambda: plan.load_gather(coef, out=f)])
    plan.check()
    fit_ms, gather_ms = float(np.median(st[:, 0])), float(np.median(st[:, 1]))
    coef_bytes = coef.numel() * 8
    return {"workload": "assembly workload, body force (0, 0, -1), tractions on faces xi_1 = 1 and xi_3 = 1",
            "n_dofs": int(f.numel()), "fit_ms": fit_ms, "gather_ms": gather_ms, "step_ms": fit_ms + gather_ms,
            "tiles_per_s": plan.n_tiles / ((fit_ms + gather_ms) * 1e-3),
            "bytes": {"coef_written": coef_bytes, "f_written": int(f.numel()) * 8}}


def bench_linop(torch, W, P, plan, w, steps, warmup):
    """Matrix-free product K u (eq. (74)) on the assembly workload: from stored tile blocks (FP64
    and FP32 blocks), on the fly per slab of tiles from the table and the coefficients (FP64), and
    the CSR product of the assembled FP64 matrix beside them."""
    u = torch.from_numpy(W.random_displacement(plan.n_dofs, 3)).cuda()
    y = torch.empty_like(u)
    ws0 = plan.linop_workspace("f64", 0)
    coef = plan.fit(w.E, w.nu, "f64")
    blocks = plan.contract(coef, "f64")
    coef32 = plan.fit(w.E, w.nu, "f32")
    blocks32 = plan.contract(coef32, "f32")
    del coef32
    ytile_b = plan.n_tiles * 3 * plan.n_tile_ctrl * 8
    vec_b = 2 * plan.n_dofs * 8
    calls = {"apply_blocks_f64": (lambda: plan.apply_blocks(blocks, u, "f64", out=y, workspace=ws0),
                                  blocks.numel() * 8 + 2 * ytile_b + vec_b),
             "apply_blocks_f32": (lambda: plan.apply_blocks(blocks32, u, "f32", out=y, workspace=ws0),
                                  blocks32.numel() * 4 + 2 * ytile_b + vec_b)}
    for slab in (256, 512, 1024, 2048):
        wsl = plan.linop_workspace("f64", slab)
        calls[f"linop_f64_slab{slab}"] = (
            lambda wsl=wsl, slab=slab: plan.linop(coef, u, "f64", slab_tiles=slab, out=y, workspace=wsl), None)
    out = {"workload": "assembly workload, seeded random u", "n_dofs": plan.n_dofs}
    ys = {}
    for name, (fn, nbytes) in calls.items():
        for _ in range(warmup):
            fn()
        st = _timed(torch, steps, [fn])
        ms = float(np.median(st[:, 0]))
        ys[name] = y.clone()
        out[name] = {"ms": ms, "products_per_s": 1e3 / ms}
        if nbytes:
            out[name]["bytes"] = int(nbytes)
            out[name]["effective_GBps"] = nbytes / (ms * 1e-3) / 1e9
    del blocks32
    torch.cuda.empty_cache()
    vals = plan.scatter(blocks, "f64")
    rp, ci = plan.csr_device()
    del blocks
    torch.cuda.empty_cache()
    fn = lambda: P.spmv(rp, ci, vals, u, out=y)
    for _ in range(warmup):
        fn()
    ms = float(np.median(_timed(torch, steps, [fn])[:, 0]))
    nb = plan.nnz * 12 + (plan.n_dofs + 1) * 8 + 2 * plan.n_dofs * 8
    out["csr_spmv_f64"] = {"ms": ms, "products_per_s": 1e3 / ms, "bytes": int(nb),
                           "effective_GBps": nb / (ms * 1e-3) / 1e9}
    ref = y.clone()
    out["rel_err_vs_csr"] = {k: ((v - ref).norm() / ref.norm()).item() for k, v in ys.items()}
    # the product from stored FP64 blocks is bound by HBM: algorithmic bytes (blocks once, u once,
    # tile products written and read by the gather, y written) per call against 8 TB/s
    a = out["apply_blocks_f64"]
    out["roofline_apply_blocks_f64"] = {"bound": "hbm", "achieved": a["effective_GBps"], "peak": 8000.0,
                                        "unit": "GB/s", "frac": a["effective_GBps"] / 8000.0,
                                        "bytes_per_call": a["bytes"]}
    out["onthefly_equals_stored_bitwise"] = all(torch.equal(ys["apply_blocks_f64"], ys[k])
                                                for k in ys if k.startswith("linop_f64"))
    plan.check()
    return out


def bench_solve(torch, W, P, plan, w):
    """Krylov solve of K u = f (Jacobi CG with the matrix-free product of the FP64 tile blocks),
    clamped on xi_3 = 0, body force and a traction on xi_3 = 1: the cost per iteration on the
    assembly workload, and a solve to 1e-8 on the 16^3-tile uniform-box workload."""
    import time
    body = np.array([0.0, 0.0, -1.0])
    traction = np.zeros((6, 3))
    traction[5] = [0.2, 0.0, 0.5]

    def setup(pl, wl):
        pl.load_table_build()
        f = pl.load_assemble(body, traction)
        blocks = pl.contract(pl.fit(wl.E, wl.nu, "f64"), "f64")
        return f, blocks, pl.face_mask([4])

    def run(pl, f, blocks, fixed, **kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, it, res = pl.pcg(blocks, f, fixed, **kw)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, it, res

    f, blocks, fixed = setup(plan, w)
    run(plan, f, blocks, fixed, rtol=1e-30, max_iter=3)
    t10, _, _ = run(plan, f, blocks, fixed, rtol=1e-30, max_iter=10)
    t40, it40, res40 = run(plan, f, blocks, fixed, rtol=1e-30, max_iter=40)
    out = {"assembly_workload": {"n_dofs": plan.n_dofs, "ms_per_iteration": (t40 - t10) / 30 * 1e3,
                                 "rel_residual_after_40": res40}}
    del blocks
    torch.cuda.empty_cache()
    w4 = W.make("cfg4", n_boxes=16)
    p4 = P.Plan.from_workload(w4)
    p4.tables_build()
    f4, b4, fx4 = setup(p4, w4)
    run(p4, f4, b4, fx4, rtol=1e-8, max_iter=2)
    dt, it, res = run(p4, f4, b4, fx4, rtol=1e-8, max_iter=20000)
    out["uniform_boxes_16^3"] = {"n_dofs": p4.n_dofs, "iterations": it, "rel_residual": res, "solve_s": dt,
                                 "ms_per_iteration": dt / max(it, 1) * 1e3}
    return out


def bench_volume(torch, plan, steps, warmup):
    """Volume of the assembly workload and its gradient with respect to the macro control points
    (table prebuilt): one pass over the tiles' fit samples, the fixed-order sums."""
    plan.volume_table_build()
    ws = plan.volume_workspace()
    v, tv, g = plan.volume(grad=True, workspace=ws)
    for _ in range(warmup):
        plan.volume(grad=True, workspace=ws)
    st = _timed(torch, steps, [lambda: plan.volume(grad=False, workspace=ws),
                               lambda: plan.volume(grad=True, workspace=ws)])
    plan.check()
    return {"workload": "assembly workload", "volume": v.item(), "volume_ms": float(np.median(st[:, 0])),
            "volume_and_gradient_ms": float(np.median(st[:, 1])), "n_macro_ctrl": int(g.shape[0])}


def bench_eproj(torch, plan, w):
    """Sampled projection error (5^3 samples per tile) at degrees 2 and 4 on the assembly workload,
    and the adaptive degree for tolerance 1e-3 (a host loop over the same kernel)."""
    import time
    out = {"workload": "assembly workload, 5^3 uniform samples per tile"}
    for q in (2, 4):
        plan.eproj(w.E, w.nu, q)
        t0 = time.perf_counter()
        e = plan.eproj(w.E, w.nu, q)
        out[f"q{q}"] = {"E_proj": e, "ms": (time.perf_counter() - t0) * 1e3}
    t0 = time.perf_counter()
    q, e = plan.select_q(w.E, w.nu, 1e-3)
    out["select_q_tol_1e-3"] = {"q": q, "E_proj": e, "ms": (time.perf_counter() - t0) * 1e3}
    plan.check()
    return out


def bench_nurbs(torch, W, P, steps, warmup):
    """The FP64 assembly step on the exact NURBS quarter torus under 32^3 uniform boxes (same tile
    count, pair count and table as the assembly workload; the fit evaluates the rational map)."""
    w = W.make("nurbs_torus", n_boxes=32)
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    cb, bb = plan.workspace_bytes("f64")
    ws = plan._empty_bytes(cb + bb)
    vals = torch.empty(plan.nnz, dtype=torch.float64, device="cuda")
    fit = lambda: plan.fit(w.E, w.nu, "f64", out=ws)
    step = lambda: plan.assemble(w.E, w.nu, "f64", values=vals, workspace=ws)
    for _ in range(warmup):
        step()
    st = _timed(torch, steps, [fit, step])
    plan.check()
    out = {"workload": "NURBS quarter torus, 32^3 uniform boxes, q=2", "n_tiles": plan.n_tiles,
           "fit_ms": float(np.median(st[:, 0])), "step_ms": float(np.median(st[:, 1]))}
    del ws, vals, plan
    torch.cuda.empty_cache()
    return out


def bench_adjoint(torch, W, P, steps):
    """Shape gradient of u^T K u on the differentiation workload (16^3 uniform boxes, cubic macro net)."""
    w = W.make("cfg4")
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    u = torch.from_numpy(W.random_displacement(plan.n_dofs, 7)).cuda()
    out = {"workload": "16x16x16 uniform boxes on a degree-3 8x8x8 macro net, degree-2 2x2x2-element tile, q=3",
           "n_tiles": plan.n_tiles}
    for prec in ("f64", "f32"):
        ws = plan.grad_workspace(prec)
        for _ in range(2):
            plan.uKu_grad(w.E, w.nu, u, prec, workspace=ws)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for a, b in ev:
            a.record()
            plan.uKu_grad(w.E, w.nu, u, prec, workspace=ws)
            b.record()
        torch.cuda.synchronize()
        ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
        out[prec] = {"ms_per_gradient": ms, "tile_gradients_per_s": plan.n_tiles / (ms * 1e-3),
                     "contraction_flops": 2.0 * plan.n_pairs * plan.n_cols * 9 * plan.n_tiles}
        del ws
    # the compliance c = f^T K^-1 f as stated: clamp on xi_1 = 0, traction (0, 0, -1) on xi_1 = 1,
    # f = f^pi (moves with the geometry), FP64 blocks, CG to 1e-10, dc/dm = 2 u.df/dm - u^T dK/dm u
    import time
    traction = np.zeros((6, 3))
    traction[1] = [0.0, 0.0, -1.0]
    body = np.zeros(3)
    plan.load_table_build()
    fixed = plan.face_mask([0])
    gws = plan.grad_workspace("f32")

    def chain():
        f = plan.load_assemble(body, traction)
        blocks = plan.contract(plan.fit(w.E, w.nu, "f64"), "f64")
        u, it, res = plan.pcg(blocks, f, fixed, rtol=1e-10, max_iter=20000)
        t1 = time.perf_counter()
        _, gf = plan.uf_grad(body, traction, u)
        _, gk = plan.uKu_grad(w.E, w.nu, u, "f32", workspace=gws)
        g = 2.0 * gf - gk
        torch.cuda.synchronize()
        return u, it, res, time.perf_counter() - t1

    chain()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, it, res, t_grad = chain()
    total = time.perf_counter() - t0
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record()
        plan.uf_grad(body, traction, u)
        b.record()
    torch.cuda.synchronize()
    out["compliance"] = {"load": "traction (0, 0, -1) on xi_1 = 1, clamp xi_1 = 0, f = f^pi(ctrl)",
                         "cg_iterations": it, "rel_residual": res,
                         "ms_total_assemble_solve_gradient": total * 1e3,
                         "ms_gradient_after_solve_f32": t_grad * 1e3,
                         "ms_load_gradient": float(np.median([a.elapsed_time(b) for a, b in ev]))}
    plan.check()
    return out


def bench_learned(torch, W, P, n_designs=32):
    """Per-design table latency on the parameterised tile family: exact table build on the GPU
    versus MLP + POD reconstruction (+ the exact-row error estimate)."""
    from paper_2107_09568_amd import learned as L
    w = W.make("cfg5")
    plan = P.Plan.from_workload(w)
    tn = L.TableNet(plan, rank=w.extra["pod_rank"])
    p_train = W.family_params(w.extra["train_seed"], w.extra["n_train"])
    p_test = W.family_params(w.extra["test_seed"], w.extra["n_test"])[:n_designs]
    t0 = time.perf_counter()
    snaps = tn.exact_tables([W.tile_family(p).ctrl for p in p_train])
    torch.cuda.synchronize()
    t_snap = time.perf_counter() - t0
    t0 = time.perf_counter()
    tn.fit_pod(snaps)
    t_pod = time.perf_counter() - t0
    del snaps
    torch.cuda.empty_cache()
    hist = tn.train(p_train, steps=8000)
    ctrls = [W.tile_family(p).ctrl for p in p_test]
    ctrls_d = [torch.from_numpy(np.ascontiguousarray(c).ravel()).cuda() for c in ctrls]
    t_exact, t_learn, t_est, t_dev, errs, fallbacks = [], [], [], [], [], 0
    for p, c, cd in zip(p_test, ctrls, ctrls_d):
        # exact table build (device-resident design, as the learned path gets it)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.set_tile_ctrl(cd)
        plan.tables_build()
        torch.cuda.synchronize()
        t_exact.append(time.perf_counter() - t0)
        exact = plan.tables_get()
        # learned table alone: MLP + POD reconstruction
        t0 = time.perf_counter()
        plan.set_tile_ctrl(cd)
        plan.table_from_pod(tn.mean, tn.basis, tn.predict_coeffs(p)[0], tn.coeff_scale)
        torch.cuda.synchronize()
        t_learn.append(time.perf_counter() - t0)
        errs.append(((plan.tables_get() - exact).norm() / exact.norm()).item())
        # the full learned path: upload, MLP, reconstruction, exact check rows, estimate, and the
        # exact table in its place when the estimate exceeds the tolerance (decided on the device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        err_t, gate_t = tn.table_for_async(p, c)
        torch.cuda.synchronize()
        t_est.append(time.perf_counter() - t0)
        fallbacks += int(gate_t.item())
        # the same with the design already on the device, as the exact build above gets it
        xd = tn.scale_inputs(np.atleast_2d(p))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tn.table_for_device(xd, cd)
        torch.cuda.synchronize()
        t_dev.append(time.perf_counter() - t0)
    # the same per-design path replayed from a HIP graph (captured on the first call)
    tn.table_for_graph(p_test[0], ctrls[0])
    torch.cuda.synchronize()
    t_graph = []
    for p, c in zip(p_test, ctrls):
        t0 = time.perf_counter()
        tn.table_for_graph(p, c)
        torch.cuda.synchronize()
        t_graph.append(time.perf_counter() - t0)
    med = lambda x: float(np.median(x)) * 1e3
    # a batch of designs: exact tables of all of them, against the batched learned path
    # (one MLP forward, one reconstruction, exact check rows, exact tables where the gate is set)
    p_all = W.family_params(w.extra["test_seed"], w.extra["n_test"])
    c_all = torch.from_numpy(np.stack([np.ascontiguousarray(W.tile_family(p).ctrl).ravel() for p in p_all])).cuda()
    out = plan.tables_build_batch(c_all)
    tn.tables_for_batch(p_all, c_all)
    t_bx, t_bl = [], []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.tables_build_batch(c_all, out=out)
        torch.cuda.synchronize()
        t_bx.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        tabs, err_b, gate_b = tn.tables_for_batch(p_all, c_all)
        torch.cuda.synchronize()
        t_bl.append(time.perf_counter() - t0)
    batch_err = ((tabs - out).flatten(1).norm(dim=1) / out.flatten(1).norm(dim=1)).max().item()
    batch = {"designs": len(p_all), "exact_ms": med(t_bx), "learned_with_estimate_ms": med(t_bl),
             "speedup": med(t_bx) / med(t_bl), "fallbacks": int(gate_b.sum().item()),
             "table_rel_err_max": batch_err}
    del out, tabs
    return {"workload": "degree-2 3x3x3-element tile family (pinch, anisotropy x/y/z) ~ U(0,0.3)^4, "
                        "512 training / held-out designs, POD r=64, MLP 4-128-128-64 GELU",
            "designs_timed": len(p_test), "exact_table_ms": med(t_exact), "learned_table_ms": med(t_learn),
            "learned_with_estimate_ms": med(t_est), "speedup_learned_vs_exact": med(t_exact) / med(t_learn),
            "learned_with_estimate_device_design_ms": med(t_dev),
            "speedup_with_estimate_device_design_vs_exact": med(t_exact) / med(t_dev),
            "speedup_with_estimate_vs_exact": med(t_exact) / med(t_est),
            "learned_with_estimate_graph_ms": med(t_graph),
            "speedup_with_estimate_graph_vs_exact": med(t_exact) / med(t_graph),
            "table_rel_err_max": float(max(errs)), "table_rel_err_median": float(np.median(errs)),
            "fallbacks": fallbacks, "offline_s": {"exact_tables_512": t_snap, "pod": t_pod,
                                                 "train_8000_steps": tn.train_seconds},
            "final_loss": hist[-1][1], "batch": batch}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--config", default="cfg3", choices=sorted(WORKLOADS))
    ap.add_argument("--precisions", default="f64,f32,bf16x3,f16x3")
    ap.add_argument("--cpu-tiles", type=int, default=4096)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the gradient and learned-table sections")
    ap.add_argument("--assembly-only", action="store_true",
                    help="only the assembly step and its precision variants (for profiler passes)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one plain 1 GiB device copy first (reference dispatch for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import workloads as W
    import paper_2107_09568_amd as P

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("bench: calibration copy of 1 GiB done")
    w = W.make(args.config)
    log(f"bench: {args.config} plan")
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    torch.cuda.synchronize()
    M, K, N = plan.n_pairs, plan.n_cols, 9 * plan.n_tiles
    flops = 2.0 * M * K * N

    precs = args.precisions.split(",")
    results = {}
    ref_blocks = None
    rng = np.random.default_rng(5)
    sample = torch.from_numpy(np.sort(rng.choice(plan.n_tiles, size=min(512, plan.n_tiles), replace=False))).cuda()
    host_blocks = {}          # sampled tiles' blocks per precision, for the oracle comparison
    rigid = {}
    ablations = {}
    rp_d = ci_d = None
    if not args.assembly_only:
        rp_d, ci_d = plan.csr_device()
    for prec in precs:
        log(f"bench: {prec}")
        cb, bb = plan.workspace_bytes(prec)
        ws = plan._empty_bytes(cb + bb)
        r, vals, blocks = time_stages(torch, plan, w, prec, args.steps, args.warmup, ws)
        blk = blocks[: plan.n_tiles * M * 9].view(plan.n_tiles, M, 9)[sample].double()
        if prec == "f64":
            ref_blocks = blk
            err = 0.0
        elif ref_blocks is None:
            err = None
        else:
            d = (blk - ref_blocks).reshape(len(sample), -1).norm(dim=1) / ref_blocks.reshape(len(sample), -1).norm(dim=1)
            err = d.max().item()
        host_blocks[prec] = blk.cpu().numpy()
        if rp_d is not None:
            rigid[prec] = rigid_residuals(torch, P, rp_d, ci_d, vals)
        if prec == "bf16x3" and not args.assembly_only:
            # ablations of the split: the table split alone (coefficients rounded once), and four products
            coef = ws
            bview = blocks[: plan.n_tiles * M * 9].view(plan.n_tiles, M, 9)
            for prods in (2, 4):
                plan.contract_products(coef, prods, out=bview)
                st = _timed(torch, args.steps, [lambda: plan.contract_products(coef, prods, out=bview)])
                ab = bview[sample].double()
                dd = (ab - ref_blocks).reshape(len(sample), -1).norm(dim=1) / ref_blocks.reshape(len(sample), -1).norm(dim=1)
                name = {2: "bf16_table_split_only", 4: "bf16x4_products"}[prods]
                ablations[name] = {"contract_ms": float(np.mean(st[:, 0])), "max_block_rel_err_vs_f64": dd.max().item()}
                host_blocks[name] = ab.cpu().numpy()
        results[prec] = (r, err)
        del ws, vals, blocks, blk
        torch.cuda.empty_cache()
    del rp_d, ci_d
    torch.cuda.empty_cache()

    main_prec = precs[0]
    r, _ = results[main_prec]
    step_ms = float(np.median(r["step_ms"]))
    con_ms = float(np.mean(r["contract_ms"]))
    achieved = flops / (con_ms * 1e-3)
    kernel_src = os.path.join(ROOT, "paper_2107_09568_amd", "csrc", "contract.hip")
    traffic = pmc_traffic(kernel_src, args.config, main_prec)
    out = {
        "metric": METRIC,
        "value": plan.n_tiles / (step_ms * 1e-3),
        "unit": "tile blocks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_prec,
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config], "name": args.config, "n_tiles": plan.n_tiles,
                   "n_pairs": M, "table_cols": K, "nnz": plan.nnz, "precision": main_prec},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK[main_prec] / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK[main_prec], "traffic": traffic,
                     "kernel": f"contract_kernel<{main_prec}>", "flops_per_launch": flops,
                     "avg_launch_ms": con_ms},
        "stages_ms": {k[:-3]: float(np.median(v)) for k, v in r.items() if k.endswith("_ms")},
        "blocks_per_s_nonzeros_only": plan.n_tiles / (float(np.median(r["fit_ms"] + r["contract_ms"])) * 1e-3),
    }
    variants = {}
    f64_ms = float(np.median(results["f64"][0]["step_ms"])) if "f64" in results else None
    for prec, (rr, err) in results.items():
        sm = float(np.median(rr["step_ms"]))
        cm = float(np.mean(rr["contract_ms"]))
        variants[prec] = {"ms_per_step": sm, "tile_blocks_per_s": plan.n_tiles / (sm * 1e-3),
                          "speedup_vs_f64": f64_ms / sm if f64_ms else None,
                          "contract_ms": cm, "contract_tflops": flops / (cm * 1e-3) / 1e12,
                          "mfma_frac": flops / (cm * 1e-3) / PEAK[prec],
                          "scatter_ms": float(np.median(rr["scatter_ms"])), "fit_ms": float(np.median(rr["fit_ms"])),
                          "max_block_rel_err_vs_f64": err, "rigid_residual": rigid.get(prec)}
    out["variants"] = variants
    if ablations:
        out["ablations"] = ablations
    out["blocks_3x3_per_s"] = plan.n_pairs * out["value"]
    out["ms_per_step_min"] = float(np.min(r["step_ms"]))
    if args.assembly_only:
        print(json.dumps(out))
        return
    log("bench: load vector")
    out["load_vector"] = bench_load(torch, plan, args.steps, args.warmup)
    log("bench: matrix-free product")
    out["linop"] = bench_linop(torch, W, P, plan, w, args.steps, args.warmup)
    log("bench: Krylov solve")
    out["solve"] = bench_solve(torch, W, P, plan, w)
    log("bench: volume")
    out["volume"] = bench_volume(torch, plan, args.steps, args.warmup)
    log("bench: projection error")
    out["eproj"] = bench_eproj(torch, plan, w)
    if not args.no_extras:
        log("bench: NURBS macro map")
        out["nurbs"] = bench_nurbs(torch, W, P, args.steps, args.warmup)
    if not args.no_extras:
        log("bench: shape gradient")
        out["adjoint"] = bench_adjoint(torch, W, P, args.steps)
        log("bench: learned tables")
        out["learned"] = bench_learned(torch, W, P)
    cfg1 = cfg1_gpu_results(torch, W, P) if not args.no_cpu else None
    if not args.no_cpu:
        log("bench: cpu baseline")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_tiles)
        log("bench: precision study against the oracle")
        study = oracle_comparisons(w, sample.cpu().numpy(), host_blocks, cfg1)
        for name, v in study.items():
            if name in out["variants"]:
                out["variants"][name]["max_block_rel_err_vs_oracle"] = v["max_tile_block_rel_err"]
            elif name in out.get("ablations", {}):
                out["ablations"][name]["max_block_rel_err_vs_oracle"] = v["max_tile_block_rel_err"]
        out["precision_study"] = study
        log("bench: cpu baseline, one thread")
        out["cpu_baseline_1thread"] = cpu_baseline(w, max(256, args.cpu_tiles // 8), one_thread=True)
        out["cpu_baseline"]["note"] = ("cores counts the BLAS threads the oracle's table contraction may use; the "
                                       "one-thread run (cpu_baseline_1thread) reaches about the same rate, so most "
                                       "of the oracle's time is single-threaded numpy")
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
