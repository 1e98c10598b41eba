"""Pins for the sampled projection error E_proj (eq. (59)) and the adaptive degree (eq. (65))."""
import dataclasses
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import adaptive, projection

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_oracle_volume import A, _curved_trilinear, _workload  # noqa: E402


def test_affine_map_has_no_projection_error():
    """Affine M: A is constant, reproduced by every Q_q (q = 0 included)."""
    w = _workload(W.affine_macro((2, 2, 2), (2, 2, 2), A, np.zeros(3)), 1)
    for q in (0, 1, 2):
        assert adaptive.eproj(w, q) < 1e-13


def test_samples_at_the_fit_nodes_reproduce():
    """Pi A interpolates A at the q + 1 Gauss-Legendre nodes: the error there vanishes, and the
    uniform grid sees a nonzero error of the curved map."""
    w = dataclasses.replace(W.make("cfg1"), q=2, n_fit=3)
    x, _ = __import__("oracle.basis", fromlist=["gauss01"]).gauss01(3)
    Afit = adaptive.tile_field_at(w, 3, x)
    coef = projection.tile_coefficients(w, 3)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    B = projection.bernstein3(2, np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1))
    PA = np.einsum("sC,Cijab->sijab", B, coef.reshape(-1, 3, 3, 3, 3)).reshape(len(B), 81)
    assert np.abs(Afit - PA).max() <= 1e-13 * np.abs(Afit).max()
    assert adaptive.tile_eproj(w, 3, 5) > 1e-6


def test_eproj_decreases_and_select_q():
    """E_proj falls with q for the curved map; eq. (65) returns the first degree from p_M on that
    meets the tolerance, consistent with the errors of the degrees below it."""
    w = W.make("cfg1")
    errs = [adaptive.eproj(w, q) for q in range(0, 6)]
    assert all(b < a for a, b in zip(errs[:-1], errs[1:])), errs
    q0 = max(w.macro.degree)
    tol = errs[4] * 1.01
    q, e = adaptive.select_q(w, tol)
    assert q == 4 and e == pytest.approx(errs[4], rel=1e-14)
    assert all(errs[k] > tol for k in range(q0, 4))
    q, e = adaptive.select_q(w, 1e-30, q_max=5)
    assert q is None and e == pytest.approx(errs[5], rel=1e-14)
    # a looser tolerance met at the macro degree itself
    q, _ = adaptive.select_q(w, errs[q0] * 1.5)
    assert q == q0


def test_finer_tiling_lowers_the_error():
    """More tiles on the same macro map: smaller boxes, smoother A per box, lower E_proj, by about
    2^(q+1) per halving of the box (the trend of the paper's tile-count study)."""
    w = W.make("cfg1")
    for q in (1, 2):
        e = [adaptive.eproj(dataclasses.replace(w, tiles=(n, n, n), box_mode=1), q) for n in (2, 4, 8)]
        assert e[0] > e[1] > e[2], e
        assert e[1] / e[2] > 2.0 ** (q + 1) * 0.9, e
