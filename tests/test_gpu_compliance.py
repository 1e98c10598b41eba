"""GPU parity of the compliance sensitivity with a load that moves with the geometry
(Section 4.1.2, eq. (68)-(73); the external work of eq. (69) differentiated through the load
projections of eq. (40)-(41), (44)-(45)).

* d(u . f^pi)/dm (igamt_uf_grad) against the oracle's chain (complex-step d|det J|/dJ and
  d area/dJ) on small B-spline and NURBS instances;
* the differentiation workload as stated: 16^3 uniform boxes on the cubic 8^3 macro net, clamp on
  xi_1 = 0, uniform traction (0, 0, -1) on xi_1 = 1, f = f^pi assembled on the GPU, u from the
  GPU's CG to 1e-10, dc/dm = 2 u . df/dm - u^T (dK/dm) u with the contraction of the stiffness
  adjoint in FP64 and in FP32, against central differences (h = 1e-6) of c = f^T K^-1 f with the
  load and the tile blocks re-assembled and the system re-solved for every perturbation, on 20
  seeded control points x 3 coordinates.
"""
import numpy as np
import pytest

import workloads as W
from oracle import geometry, load

pytestmark = pytest.mark.gpu

BODY = np.array([0.0, 0.0, -0.5])


def _traction(extra=False):
    t = np.zeros((6, 3))
    t[1] = [0.0, 0.0, -1.0]            # uniform traction on xi_1 = 1
    if extra:
        t[4] = [0.3, -0.2, 0.1]        # and one on xi_3 = 0
        t[3] = [0.05, 0.2, 0.0]        # and one on xi_2 = 1
    return t


def _say(m):
    print(m, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2107_09568_amd as P
    return torch, P


@pytest.mark.parametrize("name,kw", [("cfg4", {"n_boxes": 3}), ("nurbs_torus", {"n_boxes": 2}),
                                     ("cfg1", {})])
def test_uf_grad_vs_oracle(env, name, kw):
    torch, P = env
    w = W.make(name, **kw)
    trac = _traction(extra=True)
    plan = P.Plan.from_workload(w)
    plan.load_table_build()
    u = W.random_displacement(plan.n_dofs, 31)
    ud = torch.from_numpy(u).cuda()
    _say(f"{name} {w.tiles}: uf_grad")
    val, grad = plan.uf_grad(BODY, trac, ud)
    plan.check()
    F = load.load_table(w.tile, w.q, w.n_gauss)
    g_ref = load.grad_uf(w, F, BODY, trac, u)
    v_ref = load.uf(w, F, BODY, trac, u)
    g = grad.cpu().numpy()
    err = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    _say(f"{name}: d(u.f)/dm vs oracle {err:.2e}; u.f {val.item():.12e} vs {v_ref:.12e}")
    assert err < 1e-10
    assert val.item() == pytest.approx(v_ref, rel=1e-12)
    # u . f from the assembled load vector
    f = plan.load_assemble(BODY, trac)
    assert val.item() == pytest.approx(float(torch.dot(f, ud)), rel=1e-12)
    _, grad2 = plan.uf_grad(BODY, trac, ud)
    assert torch.equal(grad, grad2), "not bitwise reproducible"


def test_uf_grad_zero_load_and_translation(env):
    torch, P = env
    w = W.make("cfg4", n_boxes=2)
    plan = P.Plan.from_workload(w)
    plan.load_table_build()
    ud = torch.from_numpy(W.random_displacement(plan.n_dofs, 5)).cuda()
    _, g0 = plan.uf_grad(np.zeros(3), np.zeros((6, 3)), ud)
    assert torch.count_nonzero(g0).item() == 0
    _, g = plan.uf_grad(BODY, _traction(extra=True), ud)
    g = g.cpu().numpy().reshape(-1, 3)
    # a rigid translation of the net changes no |det J| and no area element
    assert np.abs(g.sum(axis=0)).max() < 1e-12 * np.abs(g).max() * g.size


def _solve(plan, w, torch, f, fixed, u0=None, rtol=1e-10):
    blocks = plan.contract(plan.fit(w.E, w.nu, "f64"), "f64")
    u, it, res = plan.pcg(blocks, f, fixed, rtol=rtol, max_iter=20000, u0=u0)
    return u, blocks, it, res


@pytest.mark.timeout(600)
def test_compliance_cfg4_vs_central_fd(env):
    torch, P = env
    w = W.make("cfg4")
    trac = _traction()
    body = np.zeros(3)
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    plan.load_table_build()
    fixed = plan.face_mask([0])
    f = plan.load_assemble(body, trac)
    _say("cfg4 16^3: solve at the initial geometry")
    u, blocks, it, res = _solve(plan, w, torch, f, fixed)
    _say(f"cfg4: {it} CG iterations, relative residual {res:.2e}")
    assert res <= 1e-10
    c0 = float(torch.dot(f, u))
    _, gf = plan.uf_grad(body, trac, u)
    uKu64, gk64 = plan.uKu_grad(w.E, w.nu, u, "f64")
    assert uKu64.item() == pytest.approx(c0, rel=1e-9)   # u^T K u = f . u at the solution
    _, gk32 = plan.uKu_grad(w.E, w.nu, u, "f32")
    plan.check()
    g64 = (2.0 * gf - gk64).cpu().numpy()
    g32 = (2.0 * gf - gk32).cpu().numpy()
    g_frozen = (-gk64).cpu().numpy()
    gscale = np.abs(g64).max()
    # through the autograd bridge
    from paper_2107_09568_amd.autograd import Compliance
    ctrl = torch.from_numpy(w.macro.ctrl.copy()).cuda().requires_grad_(True)
    c = Compliance.apply(ctrl, u, plan, w.E, w.nu, "f32", (body, trac))
    c.backward()
    assert torch.equal(ctrl.grad, 2.0 * gf - gk32)
    assert c.item() == pytest.approx(c0, rel=1e-5)       # FP32 contraction of u^T K u

    def compliance(cp):
        """c = f^T K^-1 f at control points cp, as 2 f.u - u.K u (equal at the solution, and its
        error is quadratic in the solver's error), warm-started from the unperturbed solution."""
        plan.set_macro_ctrl(cp)
        fp = plan.load_assemble(body, trac)
        up, bp, itp, resp = _solve(plan, w, torch, fp, fixed, u0=u, rtol=1e-12)
        Ku = plan.apply_blocks(bp, up)
        return 2.0 * float(torch.dot(fp, up)) - float(torch.dot(up, Ku))

    rng = np.random.default_rng(20)
    ctrl0 = w.macro.ctrl.copy()
    h = 1e-6
    worst64 = worst32 = 0.0
    frozen_gap = 0.0
    for n in range(20):
        k = tuple(int(v) for v in rng.integers(0, 8, size=3))
        for cc in range(3):
            idx = (k[2], k[1], k[0], cc)
            vals = []
            for sgn in (1, -1):
                cp = ctrl0.copy()
                cp[idx] += sgn * h
                vals.append(compliance(cp))
            fd = (vals[0] - vals[1]) / (2 * h)
            worst64 = max(worst64, abs(g64[idx] - fd) / gscale)
            worst32 = max(worst32, abs(g32[idx] - fd) / gscale)
            frozen_gap = max(frozen_gap, abs(g_frozen[idx] - fd) / gscale)
        if n % 5 == 4:
            _say(f"cfg4: {n + 1} of 20 control points")
    plan.set_macro_ctrl(ctrl0)
    _say(f"cfg4 compliance c = {c0:.6e}: FD err / max|dc/dm| f64 {worst64:.2e}, f32 {worst32:.2e}; "
         f"without the load term {frozen_gap:.2e}; FD rounding floor {2.2e-16 * abs(c0) / h / gscale:.1e}")
    assert worst64 < 1e-7
    assert worst32 < 1e-4
    # the load moves with the geometry: the frozen-load formula misses the derivative
    assert frozen_gap > 1e-3
