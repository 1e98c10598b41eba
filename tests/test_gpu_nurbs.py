"""GPU parity on the exact NURBS quarter torus (rational macro map) against the oracle: tile
blocks, load vector, volume (and its closed form), projection error, and the volume and compliance
gradients with respect to the control points (weights fixed)."""
import numpy as np
import pytest

import workloads as W
from oracle import adaptive, assembly, load, projection, tables, volume

pytestmark = pytest.mark.gpu

BODY = np.array([0.0, 0.0, -1.0])
TRACTION = np.zeros((6, 3))
TRACTION[3] = [0.2, 0.5, 0.0]


def _say(m):
    print(m, flush=True)


@pytest.fixture(scope="module")
def case():
    import torch
    import paper_2107_09568_amd as P
    w = W.make("nurbs_torus", n_boxes=2)
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    return torch, P, w, plan


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-6)])
def test_blocks_vs_oracle(case, prec, tol):
    torch, P, w, plan = case
    blocks = plan.contract(plan.fit(w.E, w.nu, prec), prec).double().cpu().numpy()
    plan.check()
    pairs = tables.pair_set(w.tile)
    T = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
    ref = assembly.tile_blocks(T, projection.all_coefficients(w))
    e = np.linalg.norm(blocks - ref) / np.linalg.norm(ref)
    _say(f"nurbs torus {prec}: block rel err {e:.2e}")
    assert e < tol


def test_load_vector_vs_oracle(case):
    torch, P, w, plan = case
    plan.load_table_build()
    f = plan.load_assemble(BODY, TRACTION).cpu().numpy()
    ref = load.assemble_load(w, load.load_table(w.tile, w.q, w.n_gauss), BODY, TRACTION)
    e = np.linalg.norm(f - ref) / np.linalg.norm(ref)
    _say(f"nurbs torus: load vector rel err {e:.2e}")
    assert e < 1e-13


def test_volume_vs_oracle_and_closed_form(case):
    torch, P, w, plan = case
    plan.volume_table_build()
    v, tv, _ = plan.volume()
    ref = volume.tile_volumes(w, volume.volume_table(w.tile, w.q, w.n_gauss))
    assert np.abs(tv.cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
    # at a higher projection degree the volume approaches the exact torus volume
    R, r1, r2 = 2.0, 0.5, 1.0
    exact = 0.5 * np.pi * (R * (r2 ** 2 - r1 ** 2) * np.pi / 4 + (r2 ** 3 - r1 ** 3) / 3)
    p5 = P.Plan(w.macro, w.tile, w.tiles, w.box_mode, 5, 6, 8)
    p5.volume_table_build()
    v5 = p5.volume()[0].item()
    _say(f"nurbs torus: V(q=2) {v.item():.12f}, V(q=5) {v5:.12f}, exact {exact:.12f}")
    assert abs(v5 - exact) < 1e-8 * exact
    assert abs(v5 - exact) < abs(v.item() - exact)


def test_eproj_vs_oracle(case):
    torch, P, w, plan = case
    for q in (1, 2, 3):
        e = plan.eproj(w.E, w.nu, q)
        ref = adaptive.eproj(w, q)
        _say(f"nurbs torus q={q}: E_proj {e:.6e} oracle {ref:.6e}")
        assert abs(e - ref) <= 1e-9 * ref


def test_nurbs_gradients_vs_oracle(case):
    """Volume and compliance gradients of the rational map (weights fixed) against the oracle."""
    torch, P, w, plan = case
    from oracle import adjoint
    plan.volume_table_build()
    _, _, g = plan.volume(grad=True)
    plan.check()
    t_h = volume.volume_table(w.tile, w.q, w.n_gauss)
    ref = volume.volume_grad(w, volume.folded_table(w.q, t_h)).reshape(-1, 3)
    e = np.abs(g.cpu().numpy() - ref).max() / np.abs(ref).max()
    _say(f"nurbs torus: volume gradient rel err {e:.2e}")
    assert e < 1e-12
    u = W.random_displacement(plan.n_dofs, 5) * 0.1
    val, grad = plan.uKu_grad(w.E, w.nu, torch.from_numpy(u).cuda(), "f64")
    pairs = tables.pair_set(w.tile)
    T = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
    refc = adjoint.grad_uKu(w, T, pairs, u).reshape(-1, 3)
    e = np.abs(grad.cpu().numpy().reshape(-1, 3) - refc).max() / np.abs(refc).max()
    _say(f"nurbs torus: compliance gradient rel err {e:.2e}")
    assert e < 1e-10
    assert val.item() == pytest.approx(adjoint.uKu(w, T, pairs, u), rel=1e-12)
