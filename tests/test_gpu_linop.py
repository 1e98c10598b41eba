"""GPU parity of the matrix-free product K u (Section 4.2, eq. (74)) against the FP64 oracle: the
product from stored tile blocks and the on-the-fly product from the table and the coefficients,
in every precision, on knot-span tiles, uniform boxes, a ragged grid and, sampled, the full-size
torus sector."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import assembly, projection, tables

pytestmark = pytest.mark.gpu

# relative norm error of y against the FP64 oracle: the block tolerances of the contraction
TOL = {"f64": 1e-12, "f32": 1e-6, "bf16x3": 1e-4, "f16x3": 1e-4}


def _say(m):
    print(m, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2107_09568_amd as P
    return torch, P


_BLOCKS = {}


def _oracle_blocks(key, w):
    if key not in _BLOCKS:
        pairs = tables.pair_set(w.tile)
        T = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
        _BLOCKS[key] = (pairs, assembly.tile_blocks(T, projection.all_coefficients(w)))
    return _BLOCKS[key]


# knot-span tiles; a ragged grid of uniform boxes; the cubic tile (343 control points, 25498
# pairs: a hundred record chunks) on uniform boxes
CASES = [("cfg1", {}, None), ("cfg4", {"n_boxes": 4}, (3, 2, 5)), ("cfg2", {}, (2, 1, 2))]


@pytest.mark.parametrize("name,kw,tiles", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "f16x3"])
def test_apply_and_linop_vs_oracle(env, name, kw, tiles, prec):
    torch, P = env
    w = W.make(name, **kw)
    if tiles is not None:
        w = dataclasses.replace(w, tiles=tiles, box_mode=1)
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    u = torch.from_numpy(W.random_displacement(plan.n_dofs, 11)).cuda()
    _say(f"{name} {w.tiles} {prec}: fit, contract, apply")
    coef = plan.fit(w.E, w.nu, prec)
    blocks = plan.contract(coef, prec)
    y = plan.apply_blocks(blocks, u, prec)
    plan.check()
    pairs, ob = _oracle_blocks((name, tiles), w)
    ref = assembly.linop_apply(w, pairs, ob, u.cpu().numpy())
    e = np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref)
    _say(f"{name} {w.tiles} {prec}: y rel err {e:.2e}")
    assert e < TOL[prec]
    assert torch.equal(y, plan.apply_blocks(blocks, u, prec)), "not bitwise reproducible"
    # on the fly: the same tile products, whatever the slab
    for slab in (16, 32, 4096):
        assert torch.equal(plan.linop(coef, u, prec, slab_tiles=slab), y), slab


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_apply_equals_csr_product(env, prec):
    """The product from the tile blocks equals the assembled CSR matrix times u (4096 tiles,
    uniform boxes), and K is symmetric: v.(K u) = u.(K v)."""
    torch, P = env
    w = W.make("cfg4", n_boxes=4)
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    coef = plan.fit(w.E, w.nu, prec)
    blocks = plan.contract(coef, prec)
    vals = plan.scatter(blocks, prec)
    rp, ci = plan.csr_device()
    u = torch.from_numpy(W.random_displacement(plan.n_dofs, 5)).cuda()
    v = torch.from_numpy(W.random_displacement(plan.n_dofs, 6)).cuda()
    y = plan.apply_blocks(blocks, u, prec)
    ref = P.spmv(rp, ci, vals.double() if prec != "f64" else vals, u)
    e = ((y - ref).norm() / ref.norm()).item()
    _say(f"cfg4 {prec}: |y - K_csr u| / |K_csr u| = {e:.2e}")
    assert e < (1e-13 if prec == "f64" else 1e-6)   # FP32 CSR values are sums rounded to FP32
    Kv = plan.apply_blocks(blocks, v, prec)
    a, b = torch.dot(v, y).item(), torch.dot(u, Kv).item()
    # FP32 blocks: the two off-diagonal entries of a diagonal 3x3 block agree to FP32 rounding only
    assert abs(a - b) <= (1e-12 if prec == "f64" else 1e-8) * (v.norm() * y.norm()).item()
    # slabs that do not divide the tile count; a slab beyond the tile count
    for slab in (48, 1008, 8192):
        assert torch.equal(plan.linop(coef, u, prec, slab_tiles=slab), y), slab


def test_cfg3_sampled_linop(env):
    """Full-size torus sector (32^3 tiles, q = 2), the on-the-fly product with the slab size the
    benchmark times: sampled entries of y against the oracle's CSR rows dotted with u."""
    torch, P = env
    w = W.make("cfg3")
    plan = P.Plan.from_workload(w)
    _say("cfg3: tables, fit, on-the-fly product")
    plan.tables_build()
    coef = plan.fit(w.E, w.nu, "f64")
    u_np = W.random_displacement(plan.n_dofs, 3)
    u = torch.from_numpy(u_np).cuda()
    y = plan.linop(coef, u, "f64", slab_tiles=512).cpu().numpy()
    plan.check()
    pairs = tables.pair_set(w.tile)
    T = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
    P_ = projection.projection_operator(w.q, w.n_fit)
    cache = {}

    def blk(t):
        if t not in cache:
            cache[t] = T @ projection.tile_coefficients(w, t, P_)
        return cache[t]

    rng = np.random.default_rng(19)
    rows = [0, plan.n_dofs - 1] + rng.choice(plan.n_dofs, 4, replace=False).tolist()
    ref = assembly.csr_rows(w, pairs, blk, rows)
    for r in rows:
        cols, rv = ref[int(r)]
        yr = float(rv @ u_np[cols])
        scale = float(np.abs(rv) @ np.abs(u_np[cols]))
        _say(f"cfg3 row {r}: y {y[r]:.6e} ref {yr:.6e}")
        assert abs(y[r] - yr) <= 1e-12 * scale


def test_linop_arguments(env):
    torch, P = env
    w = W.make("cfg1")
    plan = P.Plan.from_workload(w)
    u = torch.zeros(plan.n_dofs, dtype=torch.float64, device="cuda")
    coef = plan.fit(w.E, w.nu, "f64")
    with pytest.raises(P.IgamtError) as e:
        plan.linop(coef, u, "f64", slab_tiles=16)
    assert e.value.code == -7                      # no tables yet
    plan.tables_build()
    for slab in (0, 8, -16):
        with pytest.raises(P.IgamtError) as e:
            plan.linop(coef, u, "f64", slab_tiles=slab, workspace=plan.linop_workspace("f64", 16))
        assert e.value.code == -1
    assert plan.linop(coef, u, "f64", slab_tiles=16).abs().max().item() == 0.0
