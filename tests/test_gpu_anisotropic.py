"""GPU parity of anisotropic projection degrees (q_x, q_y, q_z) (Section 3.3.4) against the oracle:
the table, the tile blocks in every precision, affine exactness, E_proj and the anisotropic
degree selection; the isotropic-only entry points refuse such plans."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import adaptive, assembly, projection, standard, tables

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-6, "bf16x3": 1e-4, "f16x3": 1e-4}


def _say(m):
    print(m, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2107_09568_amd as P
    return torch, P


def _aniso(q, name="cfg1", **kw):
    w = W.make(name, **kw)
    return dataclasses.replace(w, q=q, n_fit=max(q) + 1)


# (1, 1, 1) and (1, 1, 2): 72 and 108 table columns, padded to 128 (the register-table contraction's
# 128-column shape in FP32, BF16x3 and FP16x3); (1, 2, 3), (3, 1, 2): 256; (0, 2, 1): 64
@pytest.mark.parametrize("q", [(1, 2, 3), (3, 1, 2), (0, 2, 1), (1, 1, 1), (1, 1, 2)])
def test_table_and_blocks_vs_oracle(env, q):
    torch, P = env
    w = _aniso(q)
    plan = P.Plan.from_workload(w)
    assert plan.n_cols == 9 * projection.n_pi(q)
    plan.tables_build()
    pairs = tables.pair_set(w.tile)
    T = tables.stiffness_table(w.tile, q, w.n_gauss, pairs)
    got = plan.tables_get().cpu().numpy()
    assert np.linalg.norm(got - T) <= 1e-13 * np.linalg.norm(T)
    ref = assembly.tile_blocks(T, projection.all_coefficients(w))
    for prec in ("f64", "f32", "bf16x3", "f16x3"):
        blocks = plan.contract(plan.fit(w.E, w.nu, prec), prec).double().cpu().numpy()
        plan.check()
        e = np.linalg.norm(blocks - ref) / np.linalg.norm(ref)
        _say(f"q={q} {prec}: block rel err {e:.2e}")
        assert e < TOL[prec]


def test_anisotropic_assembly_composes_and_affine_is_exact(env):
    torch, P = env
    w = _aniso((1, 3, 2), "cfg4", n_boxes=3)
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    vals = plan.assemble(w.E, w.nu, "f64")
    assert torch.equal(vals, plan.scatter(plan.contract(plan.fit(w.E, w.nu, "f64"))))
    A = np.array([[1.3, 0.2, -0.1], [0.1, 0.8, 0.15], [-0.05, 0.1, 1.1]])
    macro = W.affine_macro((2, 2, 2), (2, 2, 2), A, np.array([0.5, -1.0, 2.0]))
    wa = W.Workload("affine", macro, W.make("cfg1").tile, (2, 2, 2), 0, (0, 1, 2), 3, 3)
    pa = P.Plan.from_workload(wa)
    pa.tables_build()
    blocks = pa.contract(pa.fit(wa.E, wa.nu, "f64")).cpu().numpy()
    pairs = tables.pair_set(wa.tile)
    for t in (0, 7):
        ref = standard.tile_block_standard(wa, t, pairs)
        assert np.linalg.norm(blocks[t] - ref) <= 1e-13 * np.linalg.norm(ref)


def test_twisted_square_eproj_and_selection(env):
    torch, P = env
    w = W.make("twisted_square")
    plan = P.Plan.from_workload(w)
    for q in [(2, 2, 2), (2, 2, 3), (3, 3, 2), (2, 3, 4)]:
        e = plan.eproj(w.E, w.nu, q)
        ref = adaptive.eproj(w, q)
        _say(f"twisted square q={q}: E_proj {e:.6e} oracle {ref:.6e}")
        assert abs(e - ref) <= 1e-8 * ref
    q, e = plan.select_q_aniso(w.E, w.nu, 1e-3)
    rq, re = adaptive.select_q_aniso(w, 1e-3)
    _say(f"twisted square: selected {q} (oracle {rq}), E_proj {e:.3e}")
    assert q == rq == (2, 2, 3)
    assert e == pytest.approx(re, rel=1e-8)
    q, _ = plan.select_q_aniso(w.E, w.nu, 1e-30, q_max=3)
    assert q is None


def test_anisotropic_compliance_gradient_vs_oracle(env):
    torch, P = env
    from oracle import adjoint
    w = _aniso((1, 3, 2), "cfg4", n_boxes=3)
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    u = W.random_displacement(plan.n_dofs, 7)
    val, grad = plan.uKu_grad(w.E, w.nu, torch.from_numpy(u).cuda(), "f64")
    plan.check()
    pairs = tables.pair_set(w.tile)
    T = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
    g_ref = adjoint.grad_uKu(w, T, pairs, u).reshape(-1, 3)
    err = np.abs(grad.cpu().numpy().reshape(-1, 3) - g_ref).max() / np.abs(g_ref).max()
    _say(f"anisotropic compliance gradient vs oracle: {err:.2e}")
    assert err < 1e-10
    assert val.item() == pytest.approx(adjoint.uKu(w, T, pairs, u), rel=1e-12)


def test_anisotropic_volume_vs_oracle(env):
    torch, P = env
    from oracle import volume
    w = _aniso((1, 2, 3))
    plan = P.Plan.from_workload(w)
    plan.volume_table_build()
    t, tp = plan.volume_table_get()
    assert t.numel() == projection.n_pi(w.q)
    ref_th = volume.volume_table(w.tile, w.q, w.n_gauss)
    ref_tpi = volume.folded_table(w.q, ref_th)
    assert np.abs(t.cpu().numpy() - ref_th).max() <= 1e-13 * np.abs(ref_th).max()
    assert np.abs(tp.cpu().numpy() - ref_tpi).max() <= 1e-11 * np.abs(ref_tpi).max()
    v, tv, g = plan.volume(grad=True)
    ref_tv = volume.tile_volumes(w, ref_th)
    assert np.abs(tv.cpu().numpy() - ref_tv).max() <= 1e-13 * np.abs(ref_tv).max()
    ref_g = volume.volume_grad(w, ref_tpi).reshape(-1, 3)
    assert np.abs(g.cpu().numpy() - ref_g).max() <= 1e-11 * np.abs(ref_g).max()


def test_anisotropic_load_vector_vs_oracle(env):
    torch, P = env
    from oracle import load
    for q, name, kw, tiles in [((1, 2, 3), "cfg1", {}, None), ((2, 0, 1), "cfg4", {"n_boxes": 4}, (3, 2, 5))]:
        w = _aniso(q, name, **kw)
        if tiles is not None:
            w = dataclasses.replace(w, tiles=tiles)
        plan = P.Plan.from_workload(w)
        plan.load_table_build()
        got_t = plan.load_table_get().cpu().numpy()
        ref_t = load.load_table(w.tile, w.q, w.n_gauss)
        assert np.abs(got_t - ref_t).max() <= 1e-13 * np.abs(ref_t).max()
        body = np.array([0.3, -1.2, 0.7])
        tr = np.zeros((6, 3))
        tr[1] = [1.0, 0.0, 0.5]
        tr[4] = [0.0, -2.0, 1.0]
        f = plan.load_assemble(body, tr).cpu().numpy()
        ref = load.assemble_load(w, ref_t, body, tr)
        e = np.linalg.norm(f - ref) / np.linalg.norm(ref)
        _say(f"q={q} {name} {w.tiles}: load vector rel err {e:.2e}")
        assert e < 1e-13
