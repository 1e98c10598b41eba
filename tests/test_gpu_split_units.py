"""Split-mode contraction on the persistent grid at intermediate sizes of the torus-sector workload
(8^3 and 11^3 tiles of the degree-2, 3-element tile, q = 2).  At these column counts each XCD's
workgroups take 2 and 4 column splits of 14 row blocks, so workgroups run one or several units and
some take none; every tile block is compared with the oracle's eq. (58) product.  A degree-3,
2-element tile (6146 pairs, not a multiple of 4) takes the epilogue's 4-byte stores throughout."""
import numpy as np
import pytest

import workloads as W
from oracle import projection, tables

pytestmark = pytest.mark.gpu

TOL = 1e-4   # per-block relative Frobenius error of the three-product split modes


@pytest.mark.parametrize("n_el", [8, 11, "p3"])
def test_split_every_block(n_el):
    import dataclasses
    import torch
    import paper_2107_09568_amd as P
    if n_el == "p3":
        rng = np.random.default_rng(41)
        tile = W.identity_spline((3, 3, 3), (2, 2, 2))
        W._pull_interior(tile, rng, 0.2)
        w = dataclasses.replace(W.make("cfg3", n_el=5), tile=tile)
    else:
        w = W.make("cfg3", n_el=n_el)
    print(f"split units: {w.n_tiles} tiles", flush=True)
    plan = P.Plan.from_workload(w)
    plan.tables_build()
    pairs = tables.pair_set(w.tile)
    ref_table = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
    P_ = projection.projection_operator(w.q, w.n_fit)
    ref = np.stack([ref_table @ projection.tile_coefficients(w, t, P_) for t in range(w.n_tiles)])
    for prec in ("bf16x3", "f16x3"):
        blocks = plan.contract(plan.fit(w.E, w.nu, prec), prec)
        torch.cuda.synchronize()
        got = blocks.view(w.n_tiles, plan.n_pairs, 9).double().cpu().numpy()
        err = np.linalg.norm(got - ref, axis=(1, 2)) / np.linalg.norm(ref, axis=(1, 2))
        print(f"split units {prec}: max per-block rel err {err.max():.2e}", flush=True)
        assert err.max() < TOL
