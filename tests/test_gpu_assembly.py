"""GPU parity of the assembly path (fit, table, contraction, scatter) against the CPU oracle.

Tolerances (relative Frobenius norm per tile block, against the FP64 oracle):
FP64 1e-12, FP32 1e-6, BF16x3 / F16x3 1e-4.  Integer work (pairs, CSR structure)
is compared bit for bit; two runs of the same call must be bitwise identical.
"""
import numpy as np
import pytest

import workloads as W
from oracle import assembly, projection, tables

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6, "bf16x3": 1e-4, "f16x3": 1e-4}


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def P():
    import paper_2107_09568_amd as P
    return P


class OracleCase:
    def __init__(self, w, tile_ids=None):
        self.w = w
        self.pairs = tables.pair_set(w.tile)
        self.table = tables.stiffness_table(w.tile, w.q, w.n_gauss, self.pairs)
        self.tile_ids = list(range(w.n_tiles)) if tile_ids is None else list(tile_ids)
        self.coef = projection.all_coefficients(w, self.tile_ids)
        self.blocks = assembly.tile_blocks(self.table, self.coef)
        self._bt = dict(zip(self.tile_ids, self.blocks))

    def block(self, t):
        if t not in self._bt:
            self._bt[t] = self.table @ projection.tile_coefficients(self.w, t)
        return self._bt[t]


@pytest.fixture(scope="module")
def cfg1(P, torch):
    w = W.make("cfg1")
    _say("cfg1: oracle")
    oc = OracleCase(w)
    plan = P.Plan.from_workload(w)
    _say("cfg1: tables_build")
    plan.tables_build()
    torch.cuda.synchronize()
    return w, oc, plan


def _block_errs(got, ref):
    d = np.linalg.norm((got - ref).reshape(len(ref), -1), axis=1)
    return d / np.linalg.norm(ref.reshape(len(ref), -1), axis=1)


def test_table_cfg1(cfg1, torch):
    w, oc, plan = cfg1
    T = plan.tables_get().cpu().numpy()
    err = np.linalg.norm(T - oc.table) / np.linalg.norm(oc.table)
    _say(f"cfg1 table rel err {err:.2e}")
    assert err < 1e-13
    assert np.abs(T - oc.table).max() < 1e-13 * np.abs(oc.table).max()


def test_fit_cfg1(cfg1, torch):
    w, oc, plan = cfg1
    coef = plan.fit(w.E, w.nu, "f64")
    plan.check()
    got = plan.coef_view(coef).cpu().numpy()
    err = np.abs(got - oc.coef).max() / np.abs(oc.coef).max()
    _say(f"cfg1 coef max rel err {err:.2e}")
    assert err < 1e-13


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fit_coefficients_symmetric(torch, P, prec):
    """A_ij,ab = A_ji,ba (eq. (37)); both fit kernels evaluate each such pair once, so the stored
    coefficients at (9 C + 3 i + j, 3 a + b) and (9 C + 3 j + i, 3 b + a) agree bit for bit: the
    compile-time-shape kernel (q = 2 on 3 nodes) and the general one (least squares on 4 nodes)."""
    import dataclasses
    w0 = W.make("cfg1")
    for w in (w0, dataclasses.replace(w0, n_fit=w0.n_fit + 1)):
        plan = P.Plan.from_workload(w)
        c = plan.coef_view(plan.fit(w.E, w.nu, prec), prec).cpu().numpy()
        plan.check()
        c = c.reshape(w.n_tiles, -1, 3, 3, 3, 3)        # [t][C][i][j][a][b]
        _say(f"fit symmetry {prec}, n_fit = {w.n_fit}: {c.shape[1]} coefficients per component")
        assert np.abs(c).max() > 0
        assert np.array_equal(c, c.transpose(0, 1, 3, 2, 5, 4))


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "f16x3"])
def test_blocks_cfg1(cfg1, torch, prec):
    w, oc, plan = cfg1
    _say(f"cfg1 contract {prec}")
    coef = plan.fit(w.E, w.nu, prec)
    blocks = plan.contract(coef, prec)
    torch.cuda.synchronize()
    e = _block_errs(blocks.double().cpu().numpy(), oc.blocks)
    _say(f"cfg1 {prec} per-block rel err max {e.max():.2e} median {np.median(e):.2e}")
    assert e.max() < TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "f16x3"])
def test_csr_cfg1_full(cfg1, torch, prec):
    w, oc, plan = cfg1
    _say(f"cfg1 assemble {prec}")
    vals = plan.assemble(w.E, w.nu, prec)
    plan.check()
    rp, ci, v = assembly.assemble_csr(w, oc.pairs, oc.blocks)
    got = vals.double().cpu().numpy()
    err = np.linalg.norm(got - v) / np.linalg.norm(v)
    _say(f"cfg1 {prec} CSR rel err {err:.2e}")
    assert err < TOL[prec]
    again = plan.assemble(w.E, w.nu, prec)
    torch.cuda.synchronize()
    assert torch.equal(vals, again), "assembly is not bitwise reproducible"


def test_device_csr_structure_cfg1(cfg1, torch):
    w, oc, plan = cfg1
    rp_d, ci_d = plan.csr_device()
    rp, ci = plan.csr_host()
    np.testing.assert_array_equal(rp_d.cpu().numpy(), rp)
    np.testing.assert_array_equal(ci_d.cpu().numpy(), ci)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "f16x3"])
def test_stage_entry_points_compose(cfg1, torch, prec):
    """fit -> contract -> scatter through the stage entry points equals assemble bit for bit."""
    w, oc, plan = cfg1
    coef = plan.fit(w.E, w.nu, prec)
    blocks = plan.contract(coef, prec)
    vals = plan.scatter(blocks, prec)
    ref = plan.assemble(w.E, w.nu, prec)
    torch.cuda.synchronize()
    assert torch.equal(vals, ref)


def test_rigid_translations_gpu(cfg1, torch, P):
    w, oc, plan = cfg1
    vals = plan.assemble(w.E, w.nu, "f64")
    rp, ci = plan.csr_device()
    scale = vals.abs().max().item()
    for a in range(3):
        t = torch.zeros(plan.n_dofs, dtype=torch.float64, device="cuda")
        t[a::3] = 1.0
        r = P.spmv(rp, ci, vals, t)
        assert r.abs().max().item() < 1e-12 * scale


def test_tables_missing_is_an_error(P, torch):
    w = W.make("cfg1")
    plan = P.Plan.from_workload(w)
    with pytest.raises(P.IgamtError) as e:
        plan.assemble(w.E, w.nu, "f64")
    assert e.value.code == -7


def test_degenerate_macro_reported(P, torch):
    w = W.make("cfg1")
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    folded = w.macro.ctrl.copy()
    folded[1, 1, 1, 0] = -0.6   # interior point mirrored past the boundary: det J < 0 at fit points of tile 0 only
    plan.set_macro_ctrl(folded)
    plan.assemble(w.E, w.nu, "f64")
    with pytest.raises(P.IgamtError) as e:
        plan.check()
    assert e.value.code == -3
    assert "tile 0" in str(e.value)
    plan.set_macro_ctrl(w.macro.ctrl)
    plan.assemble(w.E, w.nu, "f64")
    plan.check()


def test_ragged_tile_count_uniform_boxes(P, torch):
    """27 tiles (not a multiple of 16), uniform boxes straddling macro knots, cubic macro map."""
    w = W.make("cfg4", n_boxes=3)
    _say("cfg4(3^3) oracle")
    oc = OracleCase(w)
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    for prec in ("f64", "f32", "bf16x3"):
        vals = plan.assemble(w.E, w.nu, prec)
        plan.check()
        rp, ci, v = assembly.assemble_csr(w, oc.pairs, oc.blocks)
        err = np.linalg.norm(vals.double().cpu().numpy() - v) / np.linalg.norm(v)
        _say(f"cfg4(3^3) {prec} CSR rel err {err:.2e}")
        assert err < TOL[prec]


def test_tables_set_roundtrip(P, torch, cfg1):
    w, oc, plan = cfg1
    plan2 = P.Plan.from_workload(w)
    plan2.tables_set(torch.from_numpy(oc.table).cuda())
    a = plan2.assemble(w.E, w.nu, "f64")
    b = plan.assemble(w.E, w.nu, "f64")
    torch.cuda.synchronize()
    assert (a - b).abs().max().item() <= 1e-13 * b.abs().max().item()
    np.testing.assert_array_equal(plan2.tables_get().cpu().numpy(), oc.table)


@pytest.fixture(scope="module")
def cfg2(P, torch):
    w = W.make("cfg2")
    rng = np.random.default_rng(2)
    sample = sorted(rng.choice(w.n_tiles, size=12, replace=False).tolist())
    _say("cfg2: oracle (table + 12 tiles)")
    oc = OracleCase(w, sample)
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    torch.cuda.synchronize()
    return w, oc, plan


def test_table_cfg2(cfg2, torch):
    w, oc, plan = cfg2
    T = plan.tables_get().cpu().numpy()
    err = np.linalg.norm(T - oc.table) / np.linalg.norm(oc.table)
    _say(f"cfg2 table rel err {err:.2e}")
    assert err < 1e-13


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "f16x3"])
def test_blocks_cfg2(cfg2, torch, prec):
    w, oc, plan = cfg2
    coef = plan.fit(w.E, w.nu, prec)
    blocks = plan.contract(coef, prec)
    plan.check()
    got = blocks[oc.tile_ids].double().cpu().numpy()
    e = _block_errs(got, oc.blocks)
    _say(f"cfg2 {prec} per-block rel err max {e.max():.2e}")
    assert e.max() < TOL[prec]


def test_csr_rows_cfg2(cfg2, torch):
    w, oc, plan = cfg2
    vals = plan.assemble(w.E, w.nu, "f64")
    rp, ci = plan.csr_host()
    rng = np.random.default_rng(5)
    rows = rng.choice(plan.n_dofs, size=6, replace=False)
    ref = assembly.csr_rows(w, oc.pairs, oc.block, rows)
    v = vals.cpu().numpy()
    for r in rows:
        cols, rv = ref[int(r)]
        np.testing.assert_array_equal(ci[rp[r]:rp[r + 1]], cols)
        got = v[rp[r]:rp[r + 1]]
        assert np.linalg.norm(got - rv) <= 1e-12 * np.linalg.norm(rv)


@pytest.mark.parametrize("grid", [(1, 1, 1), (1, 2, 3), (5, 1, 1)])
def test_small_and_flat_tile_grids(P, torch, grid):
    """A single tile (nothing shared, 15 padding tiles in the contraction), a 1x2x3 grid and a
    5x1x1 row of tiles (sharing along one direction only), against the oracle's CSR."""
    import dataclasses
    w = dataclasses.replace(W.make("cfg4", n_boxes=1), tiles=grid)
    oc = OracleCase(w)
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    rp, ci, v = assembly.assemble_csr(w, oc.pairs, oc.blocks)
    for prec in ("f64", "f32", "bf16x3"):
        vals = plan.assemble(w.E, w.nu, prec)
        plan.check()
        err = np.linalg.norm(vals.double().cpu().numpy() - v) / np.linalg.norm(v)
        _say(f"grid {grid} {prec} CSR rel err {err:.2e}")
        assert err < TOL[prec]
        assert torch.equal(vals, plan.assemble(w.E, w.nu, prec))
        assert torch.equal(vals, plan.scatter(plan.contract(plan.fit(w.E, w.nu, prec), prec), prec))


@pytest.mark.parametrize("tiles", [(16, 16, 20), (7, 5, 3)])
def test_assembly_equals_stages(P, torch, tiles):
    """16x16x20 tiles and 7x5x3 (a partial last tile group): assemble equals the three stages run
    one after the other, bit for bit."""
    import dataclasses
    w = dataclasses.replace(W.make("cfg4", n_boxes=16), tiles=tiles)
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    for prec in ("f64", "f32", "bf16x3", "f16x3"):
        cb, bb = plan.workspace_bytes(prec)
        ws = plan.workspace(prec)
        v_pipe = plan.assemble(w.E, w.nu, prec, workspace=ws)
        dt = torch.float64 if prec == "f64" else torch.float32
        blocks = ws.view(torch.uint8)[cb:cb + bb].view(dt)
        plan.fit(w.E, w.nu, prec, out=ws)
        plan.contract(ws, prec, out=blocks)
        v_serial = plan.scatter(blocks, prec)
        plan.check()
        torch.cuda.synchronize()
        assert torch.equal(v_pipe, v_serial)
