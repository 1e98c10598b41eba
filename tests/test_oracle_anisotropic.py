"""Pins for anisotropic projection degrees (q_x, q_y, q_z) (Section 3.3.4, the twisted square's
(3, 3, 4); eq. (21), (23)-(24), (57), (59), (65)) in the oracle."""
import numpy as np
import pytest

import workloads as W
from oracle import adaptive, assembly, projection, standard, tables


def test_isotropic_triple_is_the_scalar_degree():
    rng = np.random.default_rng(2)
    pts = rng.random((20, 3))
    np.testing.assert_array_equal(projection.bernstein3((2, 2, 2), pts), projection.bernstein3(2, pts))
    assert projection.n_pi((1, 2, 3)) == 24
    tile = W.make("cfg1").tile
    pairs = tables.pair_set(tile)
    np.testing.assert_array_equal(tables.stiffness_table(tile, (1, 1, 1), 3, pairs),
                                  tables.stiffness_table(tile, 1, 3, pairs))


def test_projection_reproduces_per_direction_degrees():
    """The tensor L2 projection with degrees (q_x, q_y, q_z) reproduces x^a y^b z^c exactly when
    a <= q_x, b <= q_y, c <= q_z, and not when one exponent exceeds its degree."""
    q = (1, 3, 2)
    P = projection.projection_operator(q, 4)
    pts, _ = projection.fit_points(4)
    rng = np.random.default_rng(5)
    chk = rng.random((30, 3))
    Bc = projection.bernstein3(q, chk)
    for (a, b, c), ok in [((1, 3, 2), True), ((0, 2, 1), True), ((2, 0, 0), False), ((0, 0, 3), False)]:
        f = pts[:, 0] ** a * pts[:, 1] ** b * pts[:, 2] ** c
        g = Bc @ (P @ f)
        exact = chk[:, 0] ** a * chk[:, 1] ** b * chk[:, 2] ** c
        err = np.abs(g - exact).max()
        assert (err < 1e-13) == ok, ((a, b, c), err)


def test_degree_elevation_across_anisotropic_tables():
    """For a field g in Q_(1,2,1), the anisotropic table times g's (1,2,1) coefficients equals the
    isotropic q = 2 table times g's q = 2 coefficients: both sum the same integrals of g, which
    checks the per-direction Bernstein indexing of the table."""
    tile = W.make("cfg1").tile
    pairs = tables.pair_set(tile)
    Ta = tables.stiffness_table(tile, (1, 2, 1), 3, pairs)
    Ti = tables.stiffness_table(tile, 2, 3, pairs)
    pts, _ = projection.fit_points(3)
    g = 1.0 + 0.3 * pts[:, 0] - 0.7 * pts[:, 1] ** 2 * pts[:, 2] + 0.2 * pts[:, 0] * pts[:, 1] * pts[:, 2]
    da = projection.projection_operator((1, 2, 1), 3) @ g
    di = projection.projection_operator(2, 3) @ g
    for ij in range(9):
        ya = Ta[:, ij::9] @ da
        yi = Ti[:, ij::9] @ di
        assert np.abs(ya - yi).max() <= 1e-13 * np.abs(yi).max()


def test_affine_map_exact_with_anisotropic_degrees():
    A = np.array([[1.3, 0.2, -0.1], [0.1, 0.8, 0.15], [-0.05, 0.1, 1.1]])
    macro = W.affine_macro((2, 2, 2), (2, 2, 2), A, np.array([0.5, -1.0, 2.0]))
    w = W.Workload("affine", macro, W.make("cfg1").tile, (2, 2, 2), 0, (0, 1, 2), 3, 3)
    pairs = tables.pair_set(w.tile)
    T = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
    blocks = assembly.tile_blocks(T, projection.all_coefficients(w))
    for t in (0, 5):
        ref = standard.tile_block_standard(w, t, pairs)
        assert np.linalg.norm(blocks[t] - ref) <= 1e-13 * np.linalg.norm(ref)


def test_anisotropic_volume_and_gradient():
    """Volume with degrees (1, 2, 3): the mass matrix is the Kronecker product of the 1-D ones of
    each degree; affine maps give |det A|; the gradient matches central differences."""
    from math import comb
    from oracle import volume
    def m1(q):
        return np.array([[comb(q, a) * comb(q, b) / ((2 * q + 1) * comb(2 * q, a + b)) for b in range(q + 1)]
                         for a in range(q + 1)])
    np.testing.assert_allclose(volume.mass_matrix((1, 2, 3)), np.kron(np.kron(m1(3), m1(2)), m1(1)), rtol=1e-13)
    A = np.array([[1.3, 0.2, -0.1], [0.1, 0.8, 0.15], [-0.05, 0.1, 1.1]])
    wa = W.Workload("affine", W.affine_macro((2, 2, 2), (2, 2, 2), A, np.zeros(3)), W.make("cfg1").tile,
                    (2, 2, 2), 0, (1, 2, 3), 4, 3)
    assert volume.volume(wa, volume.volume_table(wa.tile, wa.q, 8)) == pytest.approx(abs(np.linalg.det(A)), rel=1e-12)
    import dataclasses
    w = dataclasses.replace(W.make("cfg1"), q=(1, 2, 3), n_fit=4)
    t_h = volume.volume_table(w.tile, w.q, w.n_gauss)
    g = volume.volume_grad(w, volume.folded_table(w.q, t_h))
    eps = 1e-6
    for (k, j, i, c) in [(1, 1, 1, 0), (2, 0, 3, 2)]:
        vals = []
        for sgn in (1, -1):
            ctrl = w.macro.ctrl.copy()
            ctrl[k, j, i, c] += sgn * eps
            ws = dataclasses.replace(w, macro=dataclasses.replace(w.macro, ctrl=ctrl))
            vals.append(volume.volume(ws, t_h))
        assert g[k, j, i, c] == pytest.approx((vals[0] - vals[1]) / (2 * eps), rel=1e-6, abs=1e-9)


def test_twisted_square_selects_an_anisotropic_degree():
    """The twist varies along the axis only: raising the section degrees leaves E_proj unchanged,
    raising the axial degree lowers it; the anisotropic selection stops at (2, 2, 3) for 1e-3 with
    36 Bernstein functions where the isotropic rule needs q = 3 (64)."""
    w = W.make("twisted_square")
    e222 = adaptive.eproj(w, (2, 2, 2))
    assert adaptive.eproj(w, (3, 3, 2)) == pytest.approx(e222, rel=0.05)
    assert adaptive.eproj(w, (2, 2, 3)) < 0.2 * e222
    q, e = adaptive.select_q_aniso(w, 1e-3)
    assert q == (2, 2, 3) and e <= 1e-3
    qi, _ = adaptive.select_q(w, 1e-3)
    assert qi == 3 and projection.n_pi(q) < projection.n_pi(qi)


def test_anisotropic_load_table_and_affine_vector():
    """Load table with degrees (1, 2, 3): sum_A F[A, C, 0] = int N_C = prod_k 1/(q_k+1) (identity
    tile, exact rule); sum_A F[A, C, 1+f] = prod_{k != d} 1/(q_k+1) on I_f and 0 off it; an affine map
    gives f^pi = f^bullet."""
    from oracle import load
    q = (1, 2, 3)
    F = load.load_table(W.identity_spline((2, 2, 2), (2, 2, 2)), q, 4)
    np.testing.assert_allclose(F[:, :, 0].sum(axis=0), 1.0 / (2 * 3 * 4), rtol=1e-13)
    for f in range(6):
        d = f // 2
        I = load.face_index_set(q, f)
        s = F[:, :, 1 + f].sum(axis=0)
        expect = np.prod([1.0 / (q[k] + 1) for k in range(3) if k != d])
        np.testing.assert_allclose(s[I], expect, rtol=1e-13)
        mask = np.ones(len(s), bool)
        mask[I] = False
        assert np.abs(s[mask]).max() < 1e-15
    A = np.array([[1.3, 0.2, -0.1], [0.1, 0.8, 0.15], [-0.05, 0.1, 1.1]])
    macro = W.affine_macro((2, 2, 2), (2, 2, 2), A, np.array([0.5, -1.0, 2.0]))
    w = W.Workload("affine", macro, W.make("cfg1").tile, (2, 3, 2), 1, (0, 1, 2), 3, 3)
    body = np.array([0.3, -1.2, 0.7])
    tr = np.zeros((6, 3))
    tr[1] = [1.0, 0.0, 0.5]
    tr[4] = [0.0, -2.0, 1.0]
    fpi = load.assemble_load(w, load.load_table(w.tile, w.q, 3), body, tr)
    fstd = load.standard_load(w, body, tr)
    assert np.linalg.norm(fpi - fstd) <= 1e-13 * np.linalg.norm(fstd)


def test_anisotropic_compliance_gradient_against_differences():
    import dataclasses
    from oracle import adjoint
    w = dataclasses.replace(W.make("cfg4", n_boxes=2), q=(1, 3, 2), n_fit=4)
    pairs = tables.pair_set(w.tile)
    T = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
    n = 3 * int(np.prod([w.tiles[k] * (w.tile.n_ctrl[k] - 1) + 1 for k in range(3)]))
    u = W.random_displacement(n, 7)
    g = adjoint.grad_uKu(w, T, pairs, u)
    eps = 1e-6
    for idx in [(1, 1, 1, 0), (2, 3, 1, 2)]:
        vals = []
        for sgn in (1, -1):
            c = w.macro.ctrl.copy()
            c[idx] += sgn * eps
            vals.append(adjoint.uKu(dataclasses.replace(w, macro=dataclasses.replace(w.macro, ctrl=c)), T, pairs, u))
        assert g[idx] == pytest.approx((vals[0] - vals[1]) / (2 * eps), rel=1e-6)


# ---- macro maps with a different degree per direction (the twisted square of Section 3.3: a NURBS
#      of degrees (1, 1, 2)) -------------------------------------------------------------------------
def test_affine_macro_map_with_per_direction_degrees_is_exact():
    """An affine map written as a B-spline of degrees (1, 2, 3): the macro field is constant on every
    tile, so K^pi equals the Gauss-quadrature matrix of the composed map (eq. (62) = 0)."""
    A = np.array([[1.1, 0.15, -0.2], [0.05, 0.9, 0.1], [0.1, -0.05, 1.3]])
    macro = W.affine_macro((1, 2, 3), (2, 1, 2), A, np.array([0.2, 0.1, -0.3]))
    w = W.Workload("affine123", macro, W.make("cfg1").tile, (2, 1, 2), 0, 1, 2, 3)
    pairs = tables.pair_set(w.tile)
    T = tables.stiffness_table(w.tile, w.q, w.n_gauss, pairs)
    blocks = assembly.tile_blocks(T, projection.all_coefficients(w))
    for t in range(w.n_tiles):
        ref = standard.tile_block_standard(w, t, pairs)
        assert np.linalg.norm(blocks[t] - ref) <= 1e-13 * np.linalg.norm(ref)


def test_nurbs_twisted_square_is_an_exact_twist():
    """Every section point keeps its distance to the axis, the section turns by 45 degrees half way
    and by 90 degrees at the end, and the volume (eq. (14) by full quadrature) is the length."""
    from oracle import geometry, volume
    w = W.make("twisted_square_nurbs")
    m = w.macro
    assert tuple(m.degree) == (1, 1, 2)
    t = np.linspace(0.0, 1.0, 9)
    X, J = geometry.eval_volume_grid(m.degree, m.knots, m.ctrl, np.array([0.0, 1.0]), np.array([0.0, 1.0]), t,
                                     weights=m.weights)
    r = np.linalg.norm(X[..., :2], axis=-1)
    np.testing.assert_allclose(r, np.sqrt(0.5), rtol=0, atol=1e-15)
    ang = np.unwrap(np.arctan2(X[:, 0, 0, 1], X[:, 0, 0, 0]) - np.arctan2(-0.5, -0.5))
    assert ang[0] == pytest.approx(0.0, abs=1e-15)
    assert ang[4] == pytest.approx(np.pi / 4, abs=1e-14)
    assert ang[-1] == pytest.approx(np.pi / 2, abs=1e-14)
    assert np.all(np.diff(ang) > 0)
    assert np.linalg.det(J).min() > 0
    assert volume.volume_standard(w, 6) == pytest.approx(3.0, rel=1e-13)


def test_twisted_square_nurbs_degrees_start_at_the_macro_degrees():
    """Eq. (65) on the (1, 1, 2) NURBS twist: the search starts at the macro map's own degrees and
    raises the axis direction most, the section directions stay lower."""
    w = W.make("twisted_square_nurbs")
    q, e = adaptive.select_q_aniso(w, 1e-3)
    assert e <= 1e-3
    assert q[2] > max(q[0], q[1]) >= 1
    assert adaptive.eproj(w, (1, 1, 2)) > 1e-3
