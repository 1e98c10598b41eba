"""GPU parity of the volume V^pi (eq. (14)-(19), (25)-(26)) and its shape sensitivity
(eq. (66)-(67)) against the FP64 oracle; at the full-size torus sector, sampled tile volumes and
two exact properties of the discrete V^pi (translation invariance, cubic homogeneity)."""
import dataclasses
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import volume

pytestmark = pytest.mark.gpu
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_oracle_volume import _curved_trilinear, _workload  # noqa: E402


def _say(m):
    print(m, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2107_09568_amd as P
    return torch, P


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


CASES = {
    "cfg1": lambda: W.make("cfg1"),
    "cfg2": lambda: W.make("cfg2"),
    "trilinear_spans": lambda: _workload(_curved_trilinear(), 2, tiles=(3, 3, 3), box_mode=0),
    "cfg4_ragged": lambda: dataclasses.replace(W.make("cfg4", n_boxes=4), tiles=(3, 2, 5)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_volume_and_gradient_vs_oracle(env, name):
    torch, P = env
    w = CASES[name]()
    plan = P.Plan.from_workload(w)
    _say(f"{name}: volume table")
    plan.volume_table_build()
    t_h, t_pi = (x.cpu().numpy() for x in plan.volume_table_get())
    ref_th = volume.volume_table(w.tile, w.q, w.n_gauss)
    ref_tpi = volume.folded_table(w.q, ref_th)
    assert _rel(t_h, ref_th) < 1e-13
    # t_pi = M_pi^-1 t^h: the two sides invert M_pi by different routes (closed-form 1-D inverse
    # against a solve of the assembled 3-D matrix), so they agree to cond(M_pi) times the
    # rounding unit (cond = 1e3 at q = 2, 4.3e4 at q = 3); the oracle's gradient goes through t_pi
    tol_fold = max(1e-13, 4e-16 * np.linalg.cond(volume.mass_matrix(w.q)))
    assert _rel(t_pi, ref_tpi) < tol_fold
    v, tv, g = plan.volume(grad=True)
    plan.check()
    ref_tv = volume.tile_volumes(w, ref_th)
    ref_g = volume.volume_grad(w, ref_tpi).reshape(-1, 3)
    e_v = abs(v.item() - ref_tv.sum()) / ref_tv.sum()
    e_g = _rel(g.cpu().numpy(), ref_g)
    _say(f"{name}: V {v.item():.15f}, rel err {e_v:.2e}; tile volumes {_rel(tv.cpu().numpy(), ref_tv):.2e}; "
         f"gradient {e_g:.2e}")
    assert e_v < 1e-13
    assert _rel(tv.cpu().numpy(), ref_tv) < 1e-13
    assert e_g < max(1e-12, tol_fold)
    v2, tv2, g2 = plan.volume(grad=True)
    assert torch.equal(v, v2) and torch.equal(g, g2), "not bitwise reproducible"


def test_cfg3_volume_properties(env):
    """Full-size torus sector (32^3 tiles): sampled tile volumes against the oracle; the gradient
    sums to zero over the control points per component (translations keep V) and satisfies
    sum_i m_i . dV/dm_i = 3 V (det J is cubic in the control points)."""
    torch, P = env
    w = W.make("cfg3")
    plan = P.Plan.from_workload(w)
    plan.volume_table_build()
    v, tv, g = plan.volume(grad=True)
    plan.check()
    t_h = volume.volume_table(w.tile, w.q, w.n_gauss)
    rng = np.random.default_rng(21)
    sample = sorted(set([0, w.n_tiles - 1] + rng.choice(w.n_tiles, 12, replace=False).tolist()))
    P_ = __import__("oracle.projection", fromlist=["projection_operator"]).projection_operator(w.q, w.n_fit)
    tvn = tv.cpu().numpy()
    for t in sample:
        ref = t_h @ (P_ @ volume.tile_detJ(w, t))
        assert abs(tvn[t] - ref) <= 1e-13 * abs(ref), t
    gn = g.cpu().numpy()
    m = w.macro.ctrl.reshape(-1, 3)
    V = v.item()
    scale = np.abs(gn).sum(axis=0)
    _say(f"cfg3: V = {V:.12f}; sum grad = {gn.sum(axis=0)}; sum m.grad / 3V = {(m * gn).sum() / (3 * V):.15f}")
    assert np.all(np.abs(gn.sum(axis=0)) <= 1e-12 * scale)
    assert (m * gn).sum() == pytest.approx(3 * V, rel=1e-12)
    assert V == pytest.approx(float(np.sum(tvn)), rel=1e-13)


def test_volume_needs_its_table(env):
    torch, P = env
    w = W.make("cfg1")
    plan = P.Plan.from_workload(w)
    with pytest.raises(P.IgamtError) as e:
        plan.volume()
    assert e.value.code == -7
    plan.volume_table_build()
    plan.volume()
    plan.set_tile_ctrl(np.ascontiguousarray(w.tile.ctrl))
    with pytest.raises(P.IgamtError):
        plan.volume()
