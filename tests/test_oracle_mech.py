"""Pins of the oracle's equilibrium solve (Moulinec-Suquet + mixed BC).

The paper takes its elastic strain from the finite-element solution (Sec. 2.2)
and has no Green's-operator solver; the solve is pinned against exact
solutions that hold for any correct equilibrium solver:
* the periodic laminate, solved plane by plane in closed form;
* independence of the converged solution from the reference medium C0;
* the uniaxial state of a homogeneous body under the mixed condition;
* the stress-free invariant-plane-strain twin lamella (twin plane on a grid
  plane), with and without the parent/twin stiffness contrast of eq. (5).
"""

import numpy as np
import pytest

from oracle import crystal as cr
from oracle import mech
from oracle import phasefield as pf
from tests import oracle_cases as oc

BASIS_Z = [((2, 2),), ((1, 2), (2, 1)), ((0, 2), (2, 0))]   # zz, yz, xz unit tensors


def unit(pairs):
    B = np.zeros((3, 3))
    for i, j in pairs:
        B[i, j] = 1.0
    return B


def laminate_exact(tabs, eta_z, epsp_z, ebar):
    """Exact strain/stress of a z-laminate (fields depending on z only) under
    full strain control: in-plane strains equal ebar, sigma_iz uniform."""
    Cg, Cv, e0 = tabs
    V = eta_z.shape[0]
    nz = eta_z.shape[1]
    Bs = [unit(p) for p in BASIS_Z]
    known = ebar.copy()
    for pairs in BASIS_Z:
        for i, j in pairs:
            known[i, j] = 0.0
    ubar = np.array([ebar[2, 2], ebar[1, 2], ebar[0, 2]])
    Ainv, t = [], []
    Cz, estar = [], []
    for z in range(nz):
        C = Cg[0] + sum(eta_z[a, z] * (Cv[0, a] - Cg[0]) for a in range(V))
        es = epsp_z[z] + sum(eta_z[a, z] * e0[0, a] for a in range(V))
        A = np.array([[np.einsum("ijkl,kl->ij", C, B)[r] for B in Bs]
                      for r in [(2, 2), (1, 2), (0, 2)]])
        tt = np.einsum("ijkl,kl->ij", C, known - es)
        t.append(np.array([tt[2, 2], tt[1, 2], tt[0, 2]]))
        Ainv.append(np.linalg.inv(A))
        Cz.append(C)
        estar.append(es)
    Am = np.mean(Ainv, axis=0)
    S = np.linalg.solve(Am, ubar + np.mean([Ai @ ti for Ai, ti in zip(Ainv, t)], axis=0))
    eps, sig = [], []
    for z in range(nz):
        u = Ainv[z] @ (S - t[z])
        e = known + sum(u[c] * Bs[c] for c in range(3))
        eps.append(e)
        sig.append(np.einsum("ijkl,kl->ij", Cz[z], e - estar[z]))
    return np.array(eps), np.array(sig)


@pytest.mark.parametrize("homogeneous,variants", [(True, [0]), (False, [0]), (False, [0, 3])])
def test_laminate_exact(homogeneous, variants):
    rng = np.random.default_rng(11)
    R = np.linalg.qr(rng.standard_normal((3, 3)))[0]
    R *= np.sign(np.linalg.det(R))
    tabs = oc.tables(R[None], variants, homogeneous=homogeneous)
    shape = (16, 4, 4)
    V = len(variants)
    eta_z = rng.random((V, shape[0])) / V
    epsp_z = rng.standard_normal((shape[0], 3, 3)) * 1e-3
    epsp_z = epsp_z + np.swapaxes(epsp_z, -1, -2)
    ebar = rng.standard_normal((3, 3)) * 2e-3
    ebar = ebar + ebar.T
    eta = np.broadcast_to(eta_z[:, :, None, None], (V,) + shape).copy()
    epsp6 = mech.tensor_to_voigt6(np.broadcast_to(epsp_z[:, None, None], shape + (3, 3)))
    prob = oc.problem(shape, tabs)
    eps, _, sigma, _, _, iters, res = oc.solve(prob, eta, epsp6, oc.load(eps_bar=mech.tensor_to_voigt6(ebar)))
    assert res <= 1e-12
    eps_ex, sig_ex = laminate_exact(tabs, eta_z, epsp_z, ebar)
    scale = np.abs(sig_ex).max()
    np.testing.assert_allclose(sigma[:, 1, 2], sig_ex, atol=1e-9 * scale)
    np.testing.assert_allclose(eps[:, 0, 3], eps_ex, atol=1e-11)
    # every voxel of a plane has the plane's value
    np.testing.assert_allclose(sigma, np.broadcast_to(sig_ex[:, None, None], sigma.shape), atol=1e-9 * scale)


def random_3d_case(seed, shape=(8, 8, 8)):
    rng = np.random.default_rng(seed)
    rots = np.stack([oc.frame_from(*cr.twin_systems()[1]),
                     np.linalg.qr(rng.standard_normal((3, 3)))[0]])
    for r in rots:
        if np.linalg.det(r) < 0:
            r[:, 0] *= -1
    tabs = oc.tables(rots, [0, 4])
    gid = (rng.random(shape) < 0.5).astype(np.int64)
    eta = rng.random((2,) + shape) * 0.5
    epsp = rng.standard_normal((6,) + shape) * 1e-3
    return tabs, gid, eta, epsp


def test_solution_independent_of_reference_medium():
    tabs, gid, eta, epsp = random_3d_case(3)
    shape = eta.shape[1:]
    C0 = pf.reference_stiffness_average(tabs[0], tabs[1])
    ld = oc.load(eps_bar=[-2e-3, 0, 0, 0, 0, 0], stress_mask=[0, 1, 1, 1, 1, 1])
    sols = []
    for scale in (1.0, 1.4):
        prob = oc.problem(shape, tabs, gid=gid, C0=C0 * scale, tol=1e-13, max_iter=2000)
        sols.append(oc.solve(prob, eta, epsp, ld))
    (e1, b1, s1, *_), (e2, b2, s2, *_) = sols
    np.testing.assert_allclose(e1, e2, atol=1e-10 * np.abs(e1).max())
    np.testing.assert_allclose(s1, s2, atol=1e-9 * np.abs(s1).max())
    # mixed condition met: stress-controlled mean components vanish
    sbar = mech.tensor_to_voigt6(s1.mean(axis=(0, 1, 2)))
    assert np.abs(sbar[1:]).max() < 1e-8 * np.abs(sbar[0])
    assert b1[0, 0] == pytest.approx(-2e-3, abs=1e-18)


def test_uniaxial_homogeneous_closed_form():
    tabs = oc.tables(np.eye(3)[None], [0], homogeneous=True)
    shape = (4, 4, 4)
    eta = np.full((1,) + shape, 0.3)
    epsp6 = np.zeros((6,) + shape)
    epsp6[3] = 4e-4
    e = -2e-3
    ld = oc.load(eps_bar=[e, 0, 0, 0, 0, 0], stress_mask=[0, 1, 1, 1, 1, 1])
    prob = oc.problem(shape, tabs)
    eps, _, sigma, *_ = oc.solve(prob, eta, epsp6, ld)
    # closed form through the compliance: eps = eps* + M^-1 sigma, sigma = s e_x e_x
    M = mech.strain_to_stress_voigt(tabs[0][0])
    Sc = np.linalg.inv(M)
    estar6 = 0.3 * mech.tensor_to_voigt6(tabs[2][0, 0]) + epsp6[:, 0, 0, 0]
    s = (e - estar6[0]) / Sc[0, 0]
    eps6 = estar6 + Sc[:, 0] * s
    np.testing.assert_allclose(mech.tensor_to_voigt6(eps[0, 0, 0]), eps6, atol=1e-15)
    np.testing.assert_allclose(sigma[..., 0, 0], s, rtol=1e-11)
    assert np.abs(sigma[..., 1:, :]).max() < 1e-9 * abs(s)


@pytest.mark.parametrize("homogeneous", [True, False])
def test_ips_lamella_is_stress_free(homogeneous):
    # A twin lamella bounded by the twin plane (normal m along z) is an
    # invariant-plane-strain state: with free mean stress it carries none,
    # whatever the stiffness contrast, for any profile across the plane.
    m, s = cr.twin_systems()[0]
    R = oc.frame_from(m, s)
    tabs = oc.tables(R[None], [0], homogeneous=homogeneous)
    shape = (32, 4, 6)
    z = np.arange(shape[0])
    prof = 0.5 * (np.tanh((z - 8.3) / 2.0) - np.tanh((z - 20.6) / 1.5))
    eta = np.broadcast_to(prof[None, :, None, None], (1,) + shape).copy()
    ld = oc.load(stress_mask=[1] * 6)
    prob = oc.problem(shape, tabs)
    eps, _, sigma, *_ = oc.solve(prob, eta, None, ld)
    e0 = tabs[2][0, 0]
    scale = np.abs(np.einsum("ijkl,kl->ij", tabs[0][0], e0)).max()
    assert np.abs(sigma).max() < 1e-10 * scale
    # the total strain is the eigenstrain itself
    np.testing.assert_allclose(eps, np.broadcast_to(prof[:, None, None, None, None] * e0, eps.shape),
                               atol=1e-14)


def test_homogeneous_fixed_point_exact_in_one_iteration():
    # With C0 = C everywhere the fixed point is reached in one iteration on
    # any eigenstrain field (sharp nucleus, random plastic strain, mixed
    # condition): the second iteration changes nothing.
    rng = np.random.default_rng(12)
    R = np.linalg.qr(rng.standard_normal((3, 3)))[0]
    R *= np.sign(np.linalg.det(R))
    tabs = oc.tables(R[None], [0], homogeneous=True)
    shape = (8, 10, 12)
    eta = np.zeros((1,) + shape)
    eta[0, 2:6, 3:8, 4:9] = 1.0
    epsp = rng.standard_normal((6,) + shape) * 1e-3
    ld = oc.load(eps_bar=[-2e-3, 0, 0, 0, 0, 0], stress_mask=[0, 1, 1, 1, 1, 1])
    prob = oc.problem(shape, tabs, tol=0.0, max_iter=2)
    *_, iters, res = oc.solve(prob, eta, epsp, ld)
    assert iters == 2 and res < 1e-14
