"""GPU checks of the learned-table path: MLP kernels against the FP64 oracle (forward, loss,
backward, Adam), the POD build against the oracle's eigen-decomposition, and the full
parameterised-tile workflow (exact tables -> POD -> training -> prediction with the
exact-rows error estimate and the fallback)."""
import time

import numpy as np
import pytest

import workloads as W
from oracle import learned as OL

pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2107_09568_amd as P
    from paper_2107_09568_amd import learned as L
    return torch, P, L


def _flat(params):
    return np.concatenate([p.ravel() for p in params])


@pytest.mark.parametrize("widths,batch", [([4, 16, 12, 8], 10), ([4, 128, 128, 64], 512)],
                         ids=["small", "trained_shape"])
def test_mlp_kernels_vs_oracle(env, widths, batch):
    """Forward, loss, backward and one Adam step against the FP64 oracle, at a small shape and at the
    trained network's shape (4-128-128-64, the full training batch of 512 designs)."""
    torch, P, L = env
    mlp = L.MLP(widths, batch=batch, seed=3)
    params64 = OL.init_mlp(widths, seed=3)        # same recipe and seed: identical values
    assert np.allclose(mlp.params.cpu().numpy(), _flat(params64).astype(np.float32))
    params64 = [p.astype(np.float32).astype(np.float64) for p in params64]
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, size=(batch, widths[0]))
    t = rng.standard_normal((batch, widths[-1]))
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    td = torch.from_numpy(t.astype(np.float32)).cuda()
    tr = L.Trainer(mlp, xd, td)
    y = mlp.forward(xd).cpu().numpy()
    y_ref, _ = OL.mlp_forward(params64, x.astype(np.float32).astype(np.float64))
    assert np.abs(y - y_ref).max() < 1e-5 * np.abs(y_ref).max()
    # one training step: loss, gradients and the Adam update
    loss_ref, g_ref = OL.loss_and_grads(params64, x.astype(np.float32).astype(np.float64), t.astype(np.float32))
    tr.step(1e-3)
    torch.cuda.synchronize()
    assert tr.loss.item() == pytest.approx(loss_ref, rel=1e-5)
    g = tr.grads.cpu().numpy()
    gr = _flat(g_ref)
    err = np.abs(g - gr).max() / np.abs(gr).max()
    _say(f"MLP {widths} batch {batch}: grads vs FP64 oracle: {err:.2e}")
    assert err < 1e-5
    p_ref = [p.copy() for p in params64]
    m = [np.zeros_like(p) for p in p_ref]
    v = [np.zeros_like(p) for p in p_ref]
    for p, gg, mm, vv in zip(p_ref, g_ref, m, v):
        OL.adam_update(p, gg, mm, vv, step=1, lr=1e-3)
    err = np.abs(mlp.params.cpu().numpy() - _flat(p_ref)).max()
    assert err < 2e-6


def test_pod_vs_oracle(env):
    torch, P, L = env
    rng = np.random.default_rng(8)
    n_s, n_e, r = 48, 5000, 6
    X = rng.standard_normal((n_s, 9)) @ rng.standard_normal((9, n_e)) + 1e-3 * rng.standard_normal((n_s, n_e))
    X += 3.0
    mean, basis, sigma = OL.pod(X, r)
    Xd = torch.from_numpy(X).cuda()
    plan_like = type("PlanLike", (), {"n_pairs": 1, "n_cols": n_e})()
    tn = L.TableNet.__new__(L.TableNet)
    tn.n_e, tn.rank = n_e, r
    s, c = tn.fit_pod(Xd)
    np.testing.assert_allclose(s[: n_s - 1], sigma[: n_s - 1], rtol=1e-9, atol=1e-9 * sigma[0])
    B = tn.basis.double().cpu().numpy()
    np.testing.assert_allclose(B @ B.T, np.eye(r), atol=1e-6)
    overlap = np.abs(B @ basis)          # same subspace, modes equal up to sign
    np.testing.assert_allclose(overlap, np.eye(r), atol=1e-5)
    np.testing.assert_allclose(tn.mean.double().cpu().numpy(), mean, rtol=1e-6)
    ref_c = (X - mean) @ basis
    np.testing.assert_allclose(np.abs(c), np.abs(ref_c), rtol=1e-6, atol=1e-9 * np.abs(ref_c).max())


@pytest.fixture(scope="module")
def family(env):
    torch, P, L = env
    w = W.make("cfg5")
    plan = P.Plan.from_workload(w)
    n_train, n_test = w.extra["n_train"], w.extra["n_test"]
    p_train = W.family_params(w.extra["train_seed"], n_train)
    p_test = W.family_params(w.extra["test_seed"], n_test)
    tn = L.TableNet(plan, rank=w.extra["pod_rank"])
    _say("cfg5: exact tables of the training designs")
    t0 = time.perf_counter()
    snaps = tn.exact_tables([W.tile_family(p).ctrl for p in p_train])
    torch.cuda.synchronize()
    t_snap = time.perf_counter() - t0
    _say(f"cfg5: {n_train} exact tables in {t_snap:.2f} s; POD")
    sigma, _ = tn.fit_pod(snaps)
    del snaps
    _say(f"cfg5: sigma[0] {sigma[0]:.3e}, sigma[63] {sigma[63]:.3e}, sigma[64] {sigma[64]:.3e}; training")
    hist = tn.train(p_train, steps=8000)
    _say(f"cfg5: training {tn.train_seconds:.2f} s, loss {hist[0][1]:.3e} -> {hist[-1][1]:.3e}")
    return torch, P, L, w, plan, tn, p_test


def test_learned_tables_heldout(family):
    torch, P, L, w, plan, tn, p_test = family
    true_errs, est_errs, fallbacks = [], [], 0
    for p in p_test:
        ctrl = W.tile_family(p).ctrl
        plan.set_tile_ctrl(ctrl)
        plan.tables_build()
        exact = plan.tables_get()
        est, fb = tn.table_for(p, ctrl)
        got = plan.tables_get()
        true = ((got - exact).norm() / exact.norm()).item()
        fallbacks += int(fb)
        if fb:
            assert torch.equal(got, exact)
        else:
            true_errs.append(true)
            est_errs.append(est)
            assert true < 3 * tn.tol
    _say(f"held-out designs: {len(p_test) - fallbacks} learned, {fallbacks} fallbacks; "
         f"true table err max {max(true_errs, default=0):.2e}, estimator max {max(est_errs, default=0):.2e}")
    if est_errs:
        ratio = np.array(est_errs) / np.array(true_errs)
        assert ratio.min() > 0.2 and ratio.max() < 5.0


def test_fallback_out_of_range(family):
    torch, P, L, w, plan, tn, p_test = family
    p = np.array([0.6, 0.6, 0.1, 0.55])          # outside the training box
    ctrl = W.tile_family(p).ctrl
    est, fb = tn.table_for(p, ctrl)
    got = plan.tables_get().clone()
    plan.tables_build()                        # exact table of the same design
    assert fb and est > tn.tol
    assert torch.equal(got, plan.tables_get())


def test_learned_table_in_assembly(family):
    """Assembling with a learned table differs from the exact-table assembly by about the table error."""
    torch, P, L, w, plan, tn, p_test = family
    p = p_test[0]
    ctrl = W.tile_family(p).ctrl
    plan.set_tile_ctrl(ctrl)
    plan.tables_build()
    ref = plan.assemble(w.E, w.nu, "f64")
    est, fb = tn.table_for(p, ctrl)
    got = plan.assemble(w.E, w.nu, "f64")
    plan.check()
    err = ((got - ref).norm() / ref.norm()).item()
    _say(f"assembly with learned table: CSR rel err {err:.2e} (estimated table err {est:.2e}, fallback {fb})")
    assert err < 3 * tn.tol


def test_device_tile_ctrl_and_gated_build(env):
    """Tile control points from device memory, the device boundary check, and the gated exact
    build: gate 0 keeps the plan's table, gate 1 replaces it by the exact one."""
    torch, P, L = env
    w = W.make("cfg1")
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    exact_host = plan.tables_get().clone()
    ctrl_d = torch.from_numpy(np.ascontiguousarray(w.tile.ctrl).ravel()).cuda()
    plan.set_tile_ctrl(ctrl_d)
    plan.tables_build()
    assert torch.equal(plan.tables_get(), exact_host)
    plan.check()
    # a learned-looking table, then the gate decides
    fake = exact_host * (1.0 + 1e-3)
    plan.tables_set(fake)
    gate = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.tables_build(gate=gate)
    assert torch.equal(plan.tables_get(), fake)
    rows = torch.arange(0, plan.n_pairs, 7, dtype=torch.int32, device="cuda")
    exact_rows = plan.tables_build_rows(rows)
    err, gate = plan.table_rows_check(rows, exact_rows, 5e-4)
    assert gate.item() == 1 and err.item() == pytest.approx(1e-3, rel=1e-6)
    err2, gate2 = plan.table_rows_check(rows, exact_rows, 2e-3)
    assert gate2.item() == 0
    plan.tables_build(gate=gate)
    assert torch.equal(plan.tables_get(), exact_host)
    # a moved boundary point is reported by the next check
    bad = ctrl_d.clone()
    bad[0] += 0.01
    plan.set_tile_ctrl(bad)
    with pytest.raises(P.IgamtError, match="Greville"):
        plan.check()
    plan.set_tile_ctrl(ctrl_d)
    plan.check()


# ---- batches of designs -------------------------------------------------------------------
def _family_ctrls(torch, params):
    c = np.stack([np.ascontiguousarray(W.tile_family(p).ctrl, dtype=np.float64) for p in params])
    return torch.from_numpy(c.reshape(len(c), -1)).cuda()


def test_batch_exact_tables_bit_identical(env):
    """Exact tables of a batch of designs equal, bit for bit, the one-design builds; the gate
    leaves the designs it switches off untouched; batch check rows are rows of the batch tables."""
    torch, P, L = env
    w = W.make("cfg5")
    plan = P.Plan.from_workload(w)
    params = W.family_params(77, 5)
    ctrls = _family_ctrls(torch, params)
    _say(f"batch exact tables: {len(params)} designs of the degree-2 tile family")
    got = plan.tables_build_batch(ctrls)
    for b in range(len(params)):
        plan.set_tile_ctrl(ctrls[b])
        plan.tables_build()
        assert torch.equal(got[b], plan.tables_get()), b
    plan.check()
    gate = torch.tensor([1, 0, 1, 0, 0], dtype=torch.int32, device="cuda")
    out = torch.full_like(got, 7.0)
    plan.tables_build_batch(ctrls, gate=gate, out=out)
    for b in range(len(params)):
        assert torch.equal(out[b], got[b] if b in (0, 2) else torch.full_like(got[b], 7.0)), b
    rows = torch.tensor([0, 5, 17, plan.n_pairs - 1, 5], dtype=torch.int32, device="cuda")
    er = plan.tables_build_rows_batch(ctrls, rows)
    assert torch.equal(er, got[:, rows.long()])
    # a design whose boundary point moved is reported
    bad = ctrls.clone()
    bad[3, 0] += 0.01
    plan.tables_build_batch(bad)
    with pytest.raises(P.IgamtError, match="Greville"):
        plan.check()


def test_batch_pod_and_check_bit_identical(env):
    """Batched reconstruction (ragged over the 16-design groups) and per-design row checks equal
    the one-design kernels bit for bit."""
    torch, P, L = env
    w = W.make("cfg1")
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    n_e = plan.n_pairs * plan.n_cols
    g = torch.Generator().manual_seed(5)
    r, B = 24, 37
    mean = torch.randn(n_e, generator=g).float().cuda()
    basis = torch.randn((r, n_e), generator=g).float().cuda()
    coeffs = torch.randn((B, r), generator=g).float().cuda()
    _say(f"batch POD reconstruction: {B} designs, r={r}, {n_e} entries")
    tabs = plan.tables_from_pod_batch(mean, basis, coeffs, 0.37)
    rows = torch.arange(0, plan.n_pairs, 3, dtype=torch.int32, device="cuda")
    exact = plan.tables_build_rows(rows)
    exact_b = exact.unsqueeze(0).expand(B, -1, -1).contiguous()
    err_b, gate_b = plan.tables_rows_check_batch(tabs, rows, exact_b, 1.5)
    for b in range(B):
        plan.table_from_pod(mean, basis, coeffs[b], 0.37)
        assert torch.equal(tabs[b], plan.tables_get()), b
        err, gate = plan.table_rows_check(rows, exact, 1.5)
        assert torch.equal(err, err_b[b:b + 1]) and torch.equal(gate, gate_b[b:b + 1]), b


def test_learned_batch_matches_per_design(family):
    """The batched learned path gives every design the table, error estimate and fallback
    decision of the one-design path, bit for bit."""
    torch, P, L, w, plan, tn, p_test = family
    params = np.concatenate([p_test[:20], np.array([[0.6, 0.6, 0.1, 0.55]])])   # the last one falls back
    ctrls = _family_ctrls(torch, params)
    tabs, err_b, gate_b = tn.tables_for_batch(params, ctrls)
    assert int(gate_b[-1].item()) == 1
    for b, p in enumerate(params):
        err, gate = tn.table_for_async(p, W.tile_family(p).ctrl)
        assert torch.equal(tabs[b], plan.tables_get()), b
        assert torch.equal(err, err_b[b:b + 1]) and torch.equal(gate, gate_b[b:b + 1]), b
    plan.check()
    _say(f"learned batch: {len(params)} designs, {int(gate_b.sum())} fallbacks, "
         f"estimated err max over learned {err_b[gate_b == 0].max().item():.2e}")


def test_learned_device_resident_design(family):
    """table_for_device (design already on the device) gives table_for_async's table, error
    estimate and fallback flag bit for bit, a design that falls back included; malformed device
    inputs are refused."""
    torch, P, L, w, plan, tn, p_test = family
    for i, p in enumerate(list(p_test[:3]) + [np.array([0.6, 0.6, 0.1, 0.55])]):
        ctrl = W.tile_family(p).ctrl
        err_a, gate_a = tn.table_for_async(p, ctrl)
        ref, ref_err, ref_gate = plan.tables_get().clone(), err_a.clone(), gate_a.clone()
        x = tn.scale_inputs(np.atleast_2d(p))
        cd = torch.from_numpy(np.ascontiguousarray(ctrl, dtype=np.float64).ravel()).cuda()
        err_d, gate_d = tn.table_for_device(x, cd)
        torch.cuda.synchronize()
        assert torch.equal(plan.tables_get(), ref), i
        assert torch.equal(err_d, ref_err) and torch.equal(gate_d, ref_gate), i
    assert int(ref_gate.item()) == 1
    with pytest.raises(ValueError):
        tn.table_for_device(x.double(), cd)
    with pytest.raises(ValueError):
        tn.table_for_device(x, cd[:-3])
    plan.check()


def test_learned_graph_replay_matches_eager(family):
    """The per-design learned path replayed from a HIP graph gives, design after design, the
    eager path's table, error estimate and fallback flag bit for bit, with eager work and
    synchronisations between the replays (a design that falls back included)."""
    torch, P, L, w, plan, tn, p_test = family
    designs = list(p_test[:4]) + [np.array([0.6, 0.6, 0.1, 0.55]), p_test[0]]
    for i, p in enumerate(designs):
        ctrl = W.tile_family(p).ctrl
        err_e, gate_e = tn.table_for_async(p, ctrl)
        ref = plan.tables_get().clone()
        ref_err, ref_gate = err_e.clone(), gate_e.clone()
        scratch = torch.randn(1 << 20, device="cuda").sum()      # eager work between replays
        torch.cuda.synchronize()
        err_g, gate_g = tn.table_for_graph(p, ctrl)
        got = plan.tables_get()
        torch.cuda.synchronize()
        assert torch.equal(got, ref), i
        assert torch.equal(err_g, ref_err) and torch.equal(gate_g, ref_gate), i
        assert bool(torch.isfinite(scratch))
    assert int(gate_g.item()) == 0 and int(ref_gate.item()) == 0
    plan.check()


def test_pod_reconstruction_vs_host(family):
    """The reconstruction T = mean + Phi^T (s c) of the trained tables (r = 64 modes of 848 556
    entries), one design at a time and in a batch, entry by entry against the same sum on the host
    in FP64 from the same FP32 mean, basis and network outputs."""
    torch, P, L, w, plan, tn, p_test = family
    coeffs = tn.predict_coeffs(p_test).clone()                  # [64, r] FP32 network outputs
    mean = tn.mean.double().cpu().numpy()
    basis = tn.basis.double().cpu().numpy()                      # [r, n_e]
    c = coeffs.double().cpu().numpy() * float(tn.coeff_scale)
    ref = mean[None, :] + c @ basis                              # [64, n_e]
    scale = np.abs(ref).max()
    tabs = plan.tables_from_pod_batch(tn.mean, tn.basis, coeffs, float(tn.coeff_scale))
    got = tabs.reshape(len(p_test), -1).cpu().numpy()
    err_b = np.abs(got - ref).max() / scale
    plan.table_from_pod(tn.mean, tn.basis, coeffs[3], float(tn.coeff_scale))
    one = plan.tables_get().reshape(-1).cpu().numpy()
    err_1 = np.abs(one - ref[3]).max() / scale
    _say(f"POD reconstruction vs host FP64: batch {err_b:.2e}, one design {err_1:.2e} (of max |T|)")
    assert err_b < 1e-6 and err_1 < 1e-6


def test_learned_batch_gain_preconditions(family):
    """What the batched learned path's gain rests on, over all 64 held-out designs: no design falls
    back, every learned table is within 1e-3 of its exact table, and assembling the 24^3-tile mesh
    with a learned table stays within 3e-3 of the exact-table assembly (the time ratio itself is a
    benchmark figure)."""
    torch, P, L, w, plan, tn, p_test = family
    ctrls = _family_ctrls(torch, p_test)
    tabs, err_b, gate_b = tn.tables_for_batch(p_test, ctrls)
    exact = plan.tables_build_batch(ctrls)
    plan.check()
    assert int(gate_b.sum().item()) == 0, "a held-out design fell back to the exact table"
    true = ((tabs - exact).flatten(1).norm(dim=1) / exact.flatten(1).norm(dim=1)).cpu().numpy()
    assert true.max() < 1e-3, true.max()
    ws = plan.workspace("f64")
    worst = 0.0
    for b in range(len(p_test)):
        plan.set_tile_ctrl(ctrls[b])
        plan.tables_set(exact[b])
        ref = plan.assemble(w.E, w.nu, "f64", workspace=ws).clone()
        plan.tables_set(tabs[b])
        got = plan.assemble(w.E, w.nu, "f64", workspace=ws)
        worst = max(worst, ((got - ref).norm() / ref.norm()).item())
        del ref, got
    plan.check()
    _say(f"64 held-out designs: no fallback, table err max {true.max():.2e}; "
         f"24^3 assembly with the learned table vs exact: max CSR rel err {worst:.2e}")
    assert worst < 3e-3
