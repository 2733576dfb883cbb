"""Pins of the oracle's crystallography against closed forms and the paper.

Sec. 1 (twin shear 0.129, ~86 degree misorientation), Sec. 2.1 (c/a = 1.633,
six {10-12}<-1011> variants, the twin-stiffness rotation formula), Table 2
(elastic constants), Table 6 (global Schmid factors).
"""

import numpy as np
import pytest

from oracle import crystal as cr
from oracle import mech


def rodrigues(axis, angle):
    k = np.asarray(axis, float) / np.linalg.norm(axis)
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * K @ K


def test_variant1_closed_form():
    # (10-12): normal from the reciprocal basis is (2/sqrt3, 0, 2/c);
    # [-1011] = -2 a1 - a2 + c = (-sqrt3, 0, c) with a = 1.
    c = cr.C_OVER_A
    m_ref = np.array([2 / np.sqrt(3), 0.0, 2 / c])
    s_ref = np.array([-np.sqrt(3), 0.0, c])
    m, s = cr.twin_systems()[0]
    np.testing.assert_allclose(m, m_ref / np.linalg.norm(m_ref), atol=1e-14)
    np.testing.assert_allclose(s, s_ref / np.linalg.norm(s_ref), atol=1e-14)


def test_variants_are_tension_twins_related_by_hex_symmetry():
    systems = cr.twin_systems()
    zc = np.array([0, 0, 1.0])
    rot60 = rodrigues(zc, np.pi / 3)
    ms = [(np.round(m, 12), np.round(s, 12)) for m, s in systems]
    for m, s in systems:
        assert abs(m @ s) < 1e-14                 # direction lies in the plane
        assert (m @ zc) * (s @ zc) > 0            # tension twin: extends along c
        # all six variants are images of each other under the 6-fold axis
        m6, s6 = rot60 @ m, rot60 @ s
        assert any(np.allclose(m6, a, atol=1e-12) and np.allclose(s6, b, atol=1e-12) for a, b in ms)
    # six distinct planes
    assert len({tuple(np.round(m, 8)) for m, _ in systems}) == 6


def test_misorientation_about_86_degrees():
    # Sec. 1: lattice rotation of 86 degrees; Q = 2mm - I turns c by
    # arccos(2 (m.c)^2 - 1), ~86.6 degrees for c/a = 1.633.
    m, _ = cr.twin_systems()[0]
    Q = cr.twin_rotation(m)
    zc = np.array([0, 0, 1.0])
    ang = np.degrees(np.arccos(np.clip((Q @ zc) @ zc, -1, 1)))
    assert abs(ang - 86.0) < 1.0
    np.testing.assert_allclose(Q @ Q.T, np.eye(3), atol=1e-14)
    assert abs(np.linalg.det(Q) - 1) < 1e-14


def test_twin_stiffness_equals_rotation_about_11_20_axis():
    # The 180-degree rotation about m and the ~86.6-degree rotation about the
    # variant's <11-20> axis (m x s) give the same stiffness for a
    # transversely isotropic crystal.
    C = cr.voigt_to_tensor4(cr.hex_stiffness_voigt(*cr.MG_HEX_PA))
    zc = np.array([0, 0, 1.0])
    for m, s in cr.twin_systems():
        Q = cr.twin_rotation(m)
        axis = np.cross(m, s)
        ang = np.arccos(np.clip((Q @ zc) @ zc, -1, 1))
        candidates = [rodrigues(axis, ang), rodrigues(axis, -ang)]
        C_q = cr.rotate4(C, Q)
        err = min(np.abs(cr.rotate4(C, Rr) - C_q).max() for Rr in candidates)
        assert err < 1e-6 * np.abs(C).max()


def test_rotate4_index_map():
    C = cr.voigt_to_tensor4(cr.hex_stiffness_voigt(*cr.MG_HEX_PA))
    # any rotation about c leaves a hexagonal stiffness unchanged
    np.testing.assert_allclose(cr.rotate4(C, rodrigues([0, 0, 1], 0.37)), C, atol=1e-3)
    # a 90-degree rotation about y sends z to x: C'_1111 = C_3333, C'_3333 = C_1111
    R = rodrigues([0, 1, 0], np.pi / 2)
    C2 = cr.rotate4(C, R)
    assert abs(C2[0, 0, 0, 0] - cr.MG_HEX_PA[3]) < 1e-3
    assert abs(C2[2, 2, 2, 2] - cr.MG_HEX_PA[0]) < 1e-3
    assert abs(C2[0, 0, 2, 2] - cr.MG_HEX_PA[2]) < 1e-3
    # rank-2 rotation of a dyad
    v = np.array([0.3, -0.2, 0.9])
    np.testing.assert_allclose(cr.rotate2(np.outer(v, v), R), np.outer(R @ v, R @ v), atol=1e-15)


def test_twin_stiffness_spd_same_spectrum():
    C = cr.voigt_to_tensor4(cr.hex_stiffness_voigt(*cr.MG_HEX_PA))
    W = np.diag([1, 1, 1, np.sqrt(2), np.sqrt(2), np.sqrt(2)])   # Mandel weights
    ev0 = np.linalg.eigvalsh(W @ cr.tensor4_to_voigt(C) @ W)
    for m, _ in cr.twin_systems():
        Ct = cr.rotate4(C, cr.twin_rotation(m))
        Mt = W @ cr.tensor4_to_voigt(Ct) @ W
        np.testing.assert_allclose(Mt, Mt.T, atol=1e-3)
        np.testing.assert_allclose(np.linalg.eigvalsh(Mt), ev0, rtol=1e-12)
        assert ev0.min() > 0


def test_schmid_factors_table6():
    # Table 6: twin 0.49 in the matrix under compression along [10-10] (x);
    # basal slip 0 in the matrix.
    d = np.array([1.0, 0, 0])
    sf = [cr.schmid_factor_compression(d, m, s) for m, s in cr.twin_systems()]
    assert abs(max(sf) - 0.49) < 0.01
    assert int(np.argmax(sf)) == 0
    basal_n = cr.mb_plane_normal((0, 0, 0, 1))
    for dirn in [(2, -1, -1, 0), (-1, 2, -1, 0), (-1, -1, 2, 0)]:
        b = cr.mb_direction(dirn)
        assert abs(basal_n @ b) < 1e-14
        assert abs(cr.schmid_factor_compression(d, basal_n, b)) < 1e-14


def test_eigenstrain_properties():
    for m, s in cr.twin_systems():
        e0 = cr.twin_eigenstrain(m, s)
        assert abs(np.trace(e0)) < 1e-15                      # isochoric shear
        np.testing.assert_allclose((e0 * e0).sum(), cr.GAMMA_TW ** 2 / 2, rtol=1e-14)
        # resolved shear of uniaxial compression sigma0 along d: sigma0*gamma*SF
        d = np.array([1.0, 0.0, 0.0])
        sig = -1.0 * np.outer(d, d)
        np.testing.assert_allclose((sig * e0).sum(),
                                   cr.GAMMA_TW * cr.schmid_factor_compression(d, m, s), atol=1e-15)


def test_voigt_strain_to_stress_map_engineering_identity():
    Cv = cr.hex_stiffness_voigt(*cr.MG_HEX_PA)
    M = mech.strain_to_stress_voigt(cr.voigt_to_tensor4(Cv))
    np.testing.assert_allclose(M, Cv @ np.diag([1, 1, 1, 2, 2, 2]), rtol=1e-15)


@pytest.mark.parametrize("g", [0, 3])
def test_mg_tables_frames(g):
    rng = np.random.default_rng(g)
    R = np.linalg.qr(rng.standard_normal((3, 3)))[0]
    if np.linalg.det(R) < 0:
        R[:, 0] *= -1
    Cg, Cvar, e0 = cr.mg_tables(R[None], [0, 2])
    m, s = cr.twin_systems()[2]
    np.testing.assert_allclose(e0[0, 1], cr.GAMMA_TW * 0.5 * (np.outer(R @ s, R @ m) + np.outer(R @ m, R @ s)), atol=1e-15)
    # stress-free rotation check: C_g : (R a R^T) = R (C : a) R^T
    C = cr.voigt_to_tensor4(cr.hex_stiffness_voigt(*cr.MG_HEX_PA))
    a = rng.standard_normal((3, 3)); a = a + a.T
    lhs = np.einsum("ijkl,kl->ij", Cg[0], R @ a @ R.T)
    rhs = R @ np.einsum("ijkl,kl->ij", C, a) @ R.T
    np.testing.assert_allclose(lhs, rhs, atol=1e-3)
