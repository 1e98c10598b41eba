"""Full-size checks at the benchmark's workload (torus sector, 32^3 tiles, q = 2) for the rows
built on the assembly: the load vector at sampled dofs and E_proj at sampled tiles against the
oracle, which computes them one by one; the Krylov solve's reported residual against the CSR
product of the assembled matrix (an independent operator)."""
import numpy as np
import pytest

import workloads as W
from oracle import adaptive, assembly, load

pytestmark = pytest.mark.gpu


def _say(m):
    print(m, flush=True)


@pytest.fixture(scope="module")
def case():
    import torch
    import paper_2107_09568_amd as P
    w = W.make("cfg3")
    _say("cfg3: plan")
    plan = P.Plan.from_workload(w)
    return torch, P, w, plan


BODY = np.array([0.0, 0.0, -1.0])
TRACTION = np.zeros((6, 3))
TRACTION[5] = [0.2, 0.0, 0.5]
TRACTION[1] = [0.0, 0.3, 0.0]


def test_cfg3_sampled_load_vector(case):
    torch, P, w, plan = case
    plan.load_table_build()
    f = plan.load_assemble(BODY, TRACTION).cpu().numpy()
    plan.check()
    F = load.load_table(w.tile, w.q, w.n_gauss)
    rng = np.random.default_rng(4)
    # corners and faces of the macro domain (traction terms) and interior points
    G = [0, plan.n_dofs // 3 - 1] + rng.choice(plan.n_dofs // 3, 6, replace=False).tolist()
    cache = {}
    for g in G:
        ref = np.zeros(3)
        for t in assembly.tiles_of_dof(w, int(g)):
            if t not in cache:
                cache[t] = load.tile_load(F, load.load_coefficients(w, t, BODY, TRACTION))
            Gt = load.tile_global_indices(w, t)
            A = int(np.nonzero(Gt == g)[0][0])
            ref += cache[t][A]
        got = f[3 * g:3 * g + 3]
        _say(f"cfg3 load vector at G={g}: {got} vs {ref}")
        assert np.abs(got - ref).max() <= 1e-13 * max(np.abs(ref).max(), 1e-300) + 1e-18


def test_cfg3_sampled_eproj(case):
    torch, P, w, plan = case
    e, te = plan.eproj(w.E, w.nu, 2, per_tile=True)
    te = te.cpu().numpy()
    assert e == te.max()
    rng = np.random.default_rng(9)
    for t in sorted(set([0, w.n_tiles - 1] + rng.choice(w.n_tiles, 6, replace=False).tolist())):
        ref = adaptive.tile_eproj(w, int(t), 5)
        assert abs(te[t] - ref) <= 1e-9 * ref + 1e-14, t


def test_cfg3_solve_residual_against_the_csr_product(case):
    torch, P, w, plan = case
    plan.tables_build()
    plan.load_table_build()
    f = plan.load_assemble(BODY, TRACTION)
    blocks = plan.contract(plan.fit(w.E, w.nu, "f64"))
    fixed = plan.face_mask([4])
    u, it, res = plan.pcg(blocks, f, fixed, rtol=1e-30, max_iter=25)
    assert it == 25
    vals = plan.scatter(blocks)
    rp, ci = plan.csr_device()
    r = f - P.spmv(rp, ci, vals, u)
    free = fixed == 0
    rel = (r[free].norm() / f[free].norm()).item()
    _say(f"cfg3 CG: 25 iterations, reported residual {res:.6e}, CSR residual {rel:.6e}")
    assert abs(rel - res) <= 1e-10 * res
    assert u[fixed.bool()].abs().max().item() == 0.0
    assert res < 1.0
