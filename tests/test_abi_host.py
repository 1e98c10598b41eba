"""Host-side checks of the C ABI: the library loads, exports every declared symbol, and the
integer plan (pair set, CSR structure) is bit-identical to the oracle's brute force.
No GPU work is done here."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import assembly, geometry, tables

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "igamt.h")
LIB = os.path.join(ROOT, "paper_2107_09568_amd", "libigamt.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libigamt.so not built")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(igamt_[a-z0-9_]+)\s*\(", text)))


def test_all_declared_symbols_exported():
    L = ctypes.CDLL(LIB)
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(L, n), n


@pytest.fixture(scope="module")
def P():
    import paper_2107_09568_amd as P
    return P


@pytest.mark.parametrize("name,kw", [("cfg1", {}), ("cfg4", {"n_boxes": 3}), ("cfg3", {"n_el": 2}),
                                     ("cfg2", {})])
def test_pairs_bit_exact(P, name, kw):
    w = W.make(name, **kw)
    plan = P.Plan.from_workload(w)
    np.testing.assert_array_equal(plan.pairs(), tables.pair_set(w.tile).astype(np.int32))


@pytest.mark.parametrize("name,kw", [("cfg1", {}), ("cfg4", {"n_boxes": 3}), ("cfg3", {"n_el": 3})])
def test_csr_structure_bit_exact(P, name, kw):
    w = W.make(name, **kw)
    plan = P.Plan.from_workload(w)
    rp, ci = plan.csr_host()
    orp, oci = assembly.csr_pattern(w, tables.pair_set(w.tile))
    assert plan.nnz == len(oci)
    np.testing.assert_array_equal(rp, orp)
    np.testing.assert_array_equal(ci, oci)


def test_sizes_cfg3_full(P):
    w = W.make("cfg3")
    plan = P.Plan.from_workload(w)
    assert plan.n_tiles == 32768
    assert plan.n_pairs == 3492
    assert plan.n_cols == 243
    assert plan.n_dofs == 3 * 129 ** 3
    assert plan.nnz == 9 * 577 ** 3   # 1-D neighbour count 577 = 31*5 + 2*3 + 64*4 + 32*5


def test_sampled_rows_cfg2(P):
    """cfg2 CSR structure on sampled rows against the oracle's one-by-one enumeration."""
    w = W.make("cfg2")
    plan = P.Plan.from_workload(w)
    rp, ci = plan.csr_host()
    pairs = tables.pair_set(w.tile)
    zero = np.zeros((len(pairs), 9))
    rows = [0, 1, 2, 3 * 777 + 1, plan.n_dofs // 2, plan.n_dofs - 1]
    got = assembly.csr_rows(w, pairs, lambda t: zero, rows)
    for r in rows:
        np.testing.assert_array_equal(ci[rp[r]:rp[r + 1]], got[r][0])


def _with(w, **changes):
    import dataclasses
    return dataclasses.replace(w, **changes)


def test_error_codes(P):
    w = W.make("cfg1")
    # box_mode 0 with the wrong tile count
    with pytest.raises(P.IgamtError) as e:
        P.Plan(w.macro, w.tile, (3, 2, 2), 0, 2, 3, 3)
    assert e.value.code == -1
    # tile boundary moved away from the identity
    bad = w.tile.copy()
    bad.ctrl[0, 0, 0, 0] += 0.01
    with pytest.raises(P.IgamtError) as e:
        P.Plan(w.macro, bad, w.tiles, 0, 2, 3, 3)
    assert e.value.code == -1
    # decreasing knots
    badm = w.macro.copy()
    k = badm.knots[0].copy()
    k[3], k[4] = 0.9, 0.2
    badm.knots = (k, badm.knots[1], badm.knots[2])
    with pytest.raises(P.IgamtError):
        P.Plan(badm, w.tile, w.tiles, 0, 2, 3, 3)
    # NaN control point
    badm = w.macro.copy()
    badm.ctrl[1, 1, 1, 0] = np.nan
    with pytest.raises(P.IgamtError):
        P.Plan(badm, w.tile, w.tiles, 0, 2, 3, 3)
    # n_fit < q + 1
    with pytest.raises(P.IgamtError):
        P.Plan(w.macro, w.tile, w.tiles, 0, 2, 2, 3)
    # repeated interior tile knot
    t2 = W.identity_spline((2, 2, 2), (2, 2, 2))
    t2.knots = (np.array([0, 0, 0, .5, .5, 1, 1, 1.]), t2.knots[1], t2.knots[2])
    t2.ctrl = np.concatenate([t2.ctrl, t2.ctrl[:, :, -1:]], axis=2)
    with pytest.raises(P.IgamtError) as e:
        P.Plan(w.macro, t2, w.tiles, 0, 2, 3, 3)
    assert e.value.code in (-1, -6)


def test_argument_checks_before_device_work(P):
    """Entry points reject invalid arguments with IGAMT_EINVAL before any device work (these
    calls return on a host without a GPU)."""
    from paper_2107_09568_amd import _lib
    L = _lib.lib()
    w = W.make("cfg1")
    plan = P.Plan.from_workload(w)
    h, vp, EINVAL = plan._h, ctypes.c_void_p, -1
    null = vp(0)
    fake = vp(16)   # never dereferenced: the checks below fail first
    # NULL pointers and bad sizes
    assert L.igamt_fit(None, 1.0, 0.3, 0, fake, null) == EINVAL
    assert L.igamt_contract(h, 0, null, fake, null) == EINVAL
    assert L.igamt_contract(h, 7, fake, fake, null) == EINVAL            # unknown precision
    assert L.igamt_scatter(h, 0, fake, null, null) == EINVAL
    assert L.igamt_assemble(h, 1.0, 0.3, 0, null, fake, null) == EINVAL
    assert L.igamt_tables_build_rows(h, fake, 0, fake, null) == EINVAL   # no rows
    assert L.igamt_tables_build_batch(h, fake, 0, null, fake, null) == EINVAL        # no designs
    assert L.igamt_tables_build_batch(h, fake, 65536, null, fake, null) == EINVAL    # grid y limit
    assert L.igamt_tables_build_rows_batch(h, fake, 2, fake, 0, fake, null) == EINVAL
    assert L.igamt_tables_from_pod_batch(h, fake, fake, 0, fake, 4, 1.0, fake, fake, null) == EINVAL   # r = 0
    assert L.igamt_tables_from_pod_batch(h, fake, fake, 257, fake, 4, 1.0, fake, fake, null) == EINVAL
    assert L.igamt_tables_rows_check_batch(h, fake, 3, fake, 2, fake, -1.0, fake, fake, null) == EINVAL  # tol < 0
    assert L.igamt_apply_blocks(h, 0, null, fake, fake, fake, null) == EINVAL
    assert L.igamt_apply_blocks(h, 9, fake, fake, fake, fake, null) == EINVAL          # unknown precision
    assert L.igamt_linop(h, 0, 0, fake, fake, fake, fake, null) == EINVAL              # slab of 0 tiles
    assert L.igamt_linop(h, 0, 24, fake, fake, fake, fake, null) == EINVAL             # not a multiple of 16
    nb = ctypes.c_int64()
    assert L.igamt_linop_workspace_bytes(h, 0, 8, ctypes.byref(nb)) == EINVAL
    assert L.igamt_linop_workspace_bytes(h, 0, 0, ctypes.byref(nb)) == 0
    assert nb.value == 8 * 3 * 64 * 8                                                 # tile products only
    assert L.igamt_linop_workspace_bytes(h, 1, 32, ctypes.byref(nb)) == 0
    assert nb.value == 8 * 3 * 64 * 8 + 16 * plan.n_pairs * 9 * 4                     # slab clamped to 16 tiles
    assert L.igamt_pod_batch_work_doubles(0, 4) == -1
    assert L.igamt_pod_batch_work_doubles(64, 17) == 64 * 32      # designs padded to groups of 16
    assert L.igamt_adam_step(fake, fake, fake, fake, 10, 1e-3, 0.9, 0.999, 1e-8, 0, null) == EINVAL  # step 0
    bad = _lib.MlpDesc()
    bad.n_layers = 0
    assert L.igamt_mlp_n_params(ctypes.byref(bad)) == -1
    good = _lib.MlpDesc()
    good.n_layers, good.batch = 2, 3
    good.widths[0], good.widths[1], good.widths[2] = 4, 8, 5
    assert L.igamt_mlp_n_params(ctypes.byref(good)) == 4 * 8 + 8 + 8 * 5 + 5
    assert b"invalid" in L.igamt_last_error().lower() or len(L.igamt_last_error()) > 0
    plan.close()


def test_plan_limits(P):
    """Empty tile grids and tiles beyond the supported size are rejected when the plan is made."""
    w = W.make("cfg1")
    with pytest.raises(P.IgamtError) as e:
        P.Plan(w.macro, w.tile, (0, 2, 2), 1, 2, 3, 3)
    assert e.value.code == -1
    big = W.identity_spline((2, 2, 2), (15, 2, 2))        # 17 control points along x
    with pytest.raises(P.IgamtError) as e:
        P.Plan(w.macro, big, w.tiles, 0, 2, 3, 3)
    assert e.value.code == -6
    ok = W.identity_spline((2, 2, 2), (14, 2, 2))         # 16: the largest supported
    P.Plan(w.macro, ok, w.tiles, 0, 2, 3, 3).close()
    # anisotropic degrees: 0..6 per direction, n_fit at least the largest degree + 1
    pa = P.Plan(w.macro, w.tile, w.tiles, 0, (1, 2, 3), 4, 3)
    assert pa.n_cols == 9 * 2 * 3 * 4 and pa.q_dir == (1, 2, 3)
    pa.close()
    with pytest.raises(P.IgamtError) as e:
        P.Plan(w.macro, w.tile, w.tiles, 0, (1, 2, 7), 8, 3)
    assert e.value.code == -6
    with pytest.raises(P.IgamtError) as e:
        P.Plan(w.macro, w.tile, w.tiles, 0, (1, 2, 3), 3, 3)
    assert e.value.code == -1
    # NURBS: positive weights on the macro map only
    import dataclasses
    torus = W.nurbs_quarter_torus()
    P.Plan(torus, w.tile, (2, 2, 2), 1, 2, 3, 3).close()
    bad = dataclasses.replace(torus, weights=-torus.weights)
    with pytest.raises(P.IgamtError) as e:
        P.Plan(bad, w.tile, (2, 2, 2), 1, 2, 3, 3)
    assert e.value.code == -1
    rational_tile = dataclasses.replace(w.tile, weights=np.ones(w.tile.ctrl.shape[:3]))
    with pytest.raises(P.IgamtError) as e:
        P.Plan(w.macro, rational_tile, w.tiles, 0, 2, 3, 3)
    assert e.value.code == -6
    # a tile whose displacements do not fit the matrix-free product's LDS (1024 control points)
    from paper_2107_09568_amd import _lib
    wide = P.Plan(w.macro, W.identity_spline((2, 2, 2), (14, 14, 2)), w.tiles, 0, 2, 3, 3)
    fake = ctypes.c_void_p(16)
    assert _lib.lib().igamt_apply_blocks(wide._h, 0, fake, fake, fake, fake, None) == -6
    wide.close()
