"""GPU parity of the sampled projection error E_proj (eq. (59)) and the adaptive degree (eq. (65))
against the oracle."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import adaptive, projection

pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2107_09568_amd as P
    return torch, P


@pytest.mark.parametrize("name,tiles", [("cfg1", None), ("cfg1", (4, 3, 5)), ("cfg4", None)])
def test_eproj_vs_oracle(env, name, tiles):
    torch, P = env
    w = W.make(name) if name != "cfg4" else W.make("cfg4", n_boxes=3)
    if tiles is not None:
        w = dataclasses.replace(w, tiles=tiles, box_mode=1)
    plan = P.Plan.from_workload(w)
    for q in (0, 1, 2, 4):
        for n_s in (2, 5):
            e, te = plan.eproj(w.E, w.nu, q, n_s, per_tile=True)
            ref = [adaptive.tile_eproj(dataclasses.replace(w, q=q, n_fit=q + 1), t, n_s) for t in range(w.n_tiles)]
            _say(f"{name} {w.tiles} q={q} n_s={n_s}: E_proj {e:.9e} oracle {max(ref):.9e}")
            # E_proj is the norm of a small difference of nearly equal fields: rounding in the fitted
            # coefficients, about n_pi |P|_inf eps |A| (|P|_inf grows with q), is amplified by
            # |A| / |A - Pi A| = 1 / E_proj
            Pinf = np.abs(projection.projection_operator(q, q + 1)).sum(axis=1).max()
            ref = np.array(ref)
            bound = 1e-10 * ref + (q + 1) ** 3 * Pinf * 1e-16 + 1e-15      # absolute, per tile
            got = te.cpu().numpy()
            assert np.all(np.abs(got - ref) <= bound), np.abs(got - ref) / bound
            assert e == got.max()
    plan.check()


def test_select_q_vs_oracle(env):
    torch, P = env
    w = W.make("cfg1")
    plan = P.Plan.from_workload(w)
    for tol in (1e-1, 1e-2, 1e-3, 1e-4):
        q, e = plan.select_q(w.E, w.nu, tol)
        rq, re = adaptive.select_q(w, tol)
        _say(f"tol {tol:.0e}: q {q} (oracle {rq}), E_proj {e:.3e}")
        assert q == rq
        assert e == pytest.approx(re, rel=1e-9)
    q, e = plan.select_q(w.E, w.nu, 1e-30, q_max=3)
    assert q is None and e == pytest.approx(adaptive.eproj(w, 3), rel=1e-9)
    with pytest.raises(P.IgamtError):
        plan.eproj(w.E, w.nu, 2, n_sample=9)
