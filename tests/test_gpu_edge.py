"""Degenerate grids through every entry point of the path: a single tile (one workgroup, one
tile group padded to 16, a single contraction item) and a one-tile-wide ragged strip, each checked
against the oracle or an exact property."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import assembly, load, projection, solve, tables, volume

pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2107_09568_amd as P
    return torch, P


@pytest.mark.parametrize("tiles", [(1, 1, 1), (1, 1, 7)])
def test_degenerate_grids_every_entry_point(env, tiles):
    torch, P = env
    w = dataclasses.replace(W.make("cfg1"), tiles=tiles, box_mode=1)
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    _say(f"{tiles}: assembly, product, solve, load, volume, E_proj")
    pairs = tables.pair_set(w.tile)
    T = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
    ob = assembly.tile_blocks(T, projection.all_coefficients(w))
    rp_ref, ci_ref, v_ref = assembly.assemble_csr(w, pairs, ob)
    vals = plan.assemble(w.E, w.nu, "f64")
    rp, ci = plan.csr_device()
    np.testing.assert_array_equal(rp.cpu().numpy(), rp_ref)
    np.testing.assert_array_equal(ci.cpu().numpy(), ci_ref)
    assert np.abs(vals.cpu().numpy() - v_ref).max() <= 1e-12 * np.abs(v_ref).max()
    # products: stored blocks, on the fly, against the CSR product
    coef = plan.fit(w.E, w.nu, "f64")
    blocks = plan.contract(coef)
    u = torch.from_numpy(W.random_displacement(plan.n_dofs, 2)).cuda()
    y = plan.apply_blocks(blocks, u)
    assert torch.equal(plan.linop(coef, u, slab_tiles=16), y)
    ref = P.spmv(rp, ci, vals, u)
    assert ((y - ref).norm() / ref.norm()).item() < 1e-13
    # load vector and the clamped solve
    plan.load_table_build()
    tr = np.zeros((6, 3))
    tr[5] = [0.1, 0.0, 0.4]
    f = plan.load_assemble(np.array([0.0, 0.0, -1.0]), tr)
    f_ref = load.assemble_load(w, load.load_table(w.tile, w.q, w.n_gauss), np.array([0.0, 0.0, -1.0]), tr)
    assert np.linalg.norm(f.cpu().numpy() - f_ref) <= 1e-13 * np.linalg.norm(f_ref)
    uu, it, res = plan.pcg(blocks, f, plan.face_mask([4]), rtol=1e-12)
    u_ref = solve.dirichlet_solve(rp_ref, ci_ref, v_ref, f_ref, solve.face_dofs(w, 4))
    assert res < 1e-11
    assert np.linalg.norm(uu.cpu().numpy() - u_ref) <= 1e-9 * np.linalg.norm(u_ref)
    # volume and E_proj
    plan.volume_table_build()
    v, tv, g = plan.volume(grad=True)
    ref_tv = volume.tile_volumes(w, volume.volume_table(w.tile, w.q, w.n_gauss))
    assert np.abs(tv.cpu().numpy() - ref_tv).max() <= 1e-13 * np.abs(ref_tv).max()
    e = plan.eproj(w.E, w.nu, 2)
    assert np.isfinite(e) and e >= 0.0
    plan.check()
