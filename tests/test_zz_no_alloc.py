"""The allocation-free volume entry point (igamt_volume_noalloc) against igamt_volume: the same
kernels with the library's static device scratch in place of the caller's workspace, so the tile
volumes, the volume and its shape gradient (eq. (14)-(19), (66)-(67)) must agree bit for bit.
Two calls in a row share the scratch, the second on a smaller plan; a plan whose gradient needs
more than the scratch holds is refused without touching the outputs."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2107_09568_amd as P
    return torch, P


def _plan(P, w):
    plan = P.Plan.from_workload(w)
    plan.volume_table_build()
    return plan


def _compare(torch, plan, name):
    v0, tv0, g0 = plan.volume(grad=True)
    v1, tv1, g1 = plan.volume_noalloc(grad=True)
    v2, tv2, _ = plan.volume_noalloc(grad=False)
    plan.check()
    torch.cuda.synchronize()
    _say(f"{name}: {plan.n_tiles} tiles, V = {v1.item():.15f}")
    assert torch.equal(v0, v1) and torch.equal(tv0, tv1) and torch.equal(g0, g1)
    assert torch.equal(v0, v2) and torch.equal(tv0, tv2)
    return v1, g1


def test_noalloc_matches_workspace_entry_point_twice(env):
    torch, P = env
    big = _plan(P, W.make("cfg3"))                        # 32^3 tiles: 21.5 MB of the 32 MiB scratch
    _compare(torch, big, "torus sector 32^3")
    small = _plan(P, W.make("cfg4", n_boxes=5))           # then a smaller plan in the same scratch
    v, g = _compare(torch, small, "unit box 5^3 boxes")
    # and the first plan again after the second overwrote the scratch
    _compare(torch, big, "torus sector 32^3 again")


def test_noalloc_refuses_what_does_not_fit(env):
    torch, P = env
    import paper_2107_09568_amd as PK
    w = W.make("cfg4", n_boxes=24)                        # 13824 tiles x 125 x 24 B of local gradients > 32 MiB
    plan = _plan(P, w)
    v = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    tv = torch.full((plan.n_tiles,), -1.0, dtype=torch.float64, device="cuda")
    g = torch.full((plan.n_macro_ctrl, 3), -1.0, dtype=torch.float64, device="cuda")
    with pytest.raises(PK.IgamtError) as e:
        plan.volume_noalloc(grad=True, v=v, tv=tv, g=g)
    assert e.value.code == -5 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert (v == -1.0).all() and (tv == -1.0).all() and (g == -1.0).all()
    # without the gradient it fits and agrees with the workspace entry point
    v1, tv1, _ = plan.volume_noalloc(grad=False)
    v0, tv0, _ = plan.volume(grad=False)
    assert torch.equal(v0, v1) and torch.equal(tv0, tv1)


def test_noalloc_needs_the_table(env):
    torch, P = env
    import paper_2107_09568_amd as PK
    plan = P.Plan.from_workload(W.make("cfg1"))
    with pytest.raises(PK.IgamtError) as e:
        plan.volume_noalloc()
    assert e.value.code == -7
