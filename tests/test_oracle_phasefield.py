"""Pins of the oracle's phase-field step (eqs. (12)-(20), Table 1).

Closed forms and invariants that any correct implementation of the readings
(A = c1, kappa = c2, single-variant Allen-Cahn -L dF/d(eta), semi-implicit
Laplacian) must satisfy:
* the double-well force is the derivative of eq. (13) (pairwise exchange form
  of eq. (17) for several variants);
* the mechanical force is minus the derivative of eq. (15) at fixed strain;
* single Fourier modes decay by exactly 1/(1 + 2 L dt kappa |xi|^2), with the
  linearised double-well factor around eta = 0;
* the flat interface keeps the tanh profile of width sqrt(kappa/A) and carries
  sqrt(A kappa)/3 per unit area;
* a driven flat twin front on the twin plane (stress-free lamella, constant
  driving force) moves at the exact Nagumo speed, with O(dt) error;
* the free energy decreases every step for a small enough step;
* several variants with one non-zero reduce to the single-variant step;
  relabelling variants and translating the grid commute with the step.
"""

import numpy as np
import pytest

from oracle import crystal as cr
from oracle import mech
from oracle import phasefield as pf
from tests import oracle_cases as oc


def test_chemical_force_single_variant_is_derivative():
    A = 1e7
    eta = np.linspace(-0.2, 1.2, 29)[None]
    h = 1e-6
    fd = (pf.double_well_density(eta + h, A) - pf.double_well_density(eta - h, A)) / (2 * h)
    np.testing.assert_allclose(pf.chemical_force(eta, A)[0], fd, rtol=1e-7, atol=1e-2)
    np.testing.assert_allclose(pf.chemical_force(eta, A)[0],
                               2 * A * eta[0] * (1 - eta[0]) * (1 - 2 * eta[0]), rtol=1e-13, atol=1e-8)


def test_chemical_force_pairwise_exchange_form():
    # eq. (17) first term: sum over the other phases b of the exchange
    # derivative (d/df_a - d/df_b) of A f_a^2 f_b^2 (matrix included).
    A = 1.0
    rng = np.random.default_rng(3)
    eta = rng.random((3, 5)) * 0.4
    phases = list(eta) + [1 - eta.sum(0)]
    expect = np.zeros_like(eta)
    for a in range(3):
        for b in range(4):
            if b == a:
                continue
            fa, fb = phases[a], phases[b]
            expect[a] += A * (2 * fa * fb ** 2 - 2 * fa ** 2 * fb)
    np.testing.assert_allclose(pf.chemical_force(eta, A), expect, rtol=1e-13, atol=1e-15)


def elastic_density(eps, eta, epsp, tabs, h_kind):
    gid = np.zeros(eps.shape[:3], dtype=np.int64)
    _, el, sig = mech.eigenstrain_and_stress(eps, eta, epsp, gid, *tabs, h_kind)
    return 0.5 * np.einsum("...ij,...ij->...", el, sig)


@pytest.mark.parametrize("h_kind", ["linear", "quintic"])
def test_mechanical_force_is_minus_energy_derivative(h_kind):
    rng = np.random.default_rng(4)
    R = np.linalg.qr(rng.standard_normal((3, 3)))[0]
    R *= np.sign(np.linalg.det(R))
    tabs = oc.tables(R[None], [1, 5])
    shape = (2, 2, 3)
    eps = rng.standard_normal(shape + (3, 3)) * 3e-3
    eps = eps + np.swapaxes(eps, -1, -2)
    epsp = rng.standard_normal(shape + (3, 3)) * 1e-3
    epsp = epsp + np.swapaxes(epsp, -1, -2)
    eta = rng.random((2,) + shape) * 0.8
    gid = np.zeros(shape, dtype=np.int64)
    _, el, sig = mech.eigenstrain_and_stress(eps, eta, epsp, gid, *tabs, h_kind)
    mechf = pf.mechanical_force(eta, sig, el, None, *tabs, h_kind)
    d = 1e-5
    for a in range(2):
        ep, em = eta.copy(), eta.copy()
        ep[a] += d
        em[a] -= d
        fd = (elastic_density(eps, ep, epsp, tabs, h_kind) - elastic_density(eps, em, epsp, tabs, h_kind)) / (2 * d)
        np.testing.assert_allclose(mechf[a], -fd, rtol=1e-6, atol=1e-6 * np.abs(fd).max())


def no_mech_problem(shape, dx, A, kappa, L, dt):
    tabs = oc.tables(np.eye(3)[None], [0], homogeneous=True, no_eigenstrain=True)
    return oc.problem(shape, tabs, dx=dx, A=A, kappa=kappa, L=L, dt=dt)


def one_step(prob, eta, ld=None, epsp6=None):
    st = pf.State.initial(eta, np.zeros(6))
    new, stats, _ = pf.step(prob, st, epsp6, ld or oc.load())
    return new.eta, stats


def test_single_mode_amplification():
    shape, dx = (4, 6, 32), 1e-8
    kappa, L, dt = 1e-9, 1.0, 3e-10
    prob = no_mech_problem(shape, dx, A=0.0, kappa=kappa, L=L, dt=dt)
    x = np.arange(shape[2]) * dx
    k = 2 * np.pi * 5 / (shape[2] * dx)
    eta = np.broadcast_to(0.5 + 0.1 * np.cos(k * x), shape)[None].copy()
    new, _ = one_step(prob, eta)
    g = 1.0 / (1.0 + 2 * L * dt * kappa * k * k)
    np.testing.assert_allclose(new[0], np.broadcast_to(0.5 + 0.1 * g * np.cos(k * x), shape), atol=1e-14)


def test_small_mode_around_zero_linearised_double_well():
    shape, dx = (4, 4, 32), 1e-8
    A, kappa, L, dt = 1e7, 1e-9, 1.0, 2e-9
    prob = no_mech_problem(shape, dx, A=A, kappa=kappa, L=L, dt=dt)
    x = np.arange(shape[2]) * dx
    k = 2 * np.pi * 3 / (shape[2] * dx)
    amp = 1e-7
    eta = np.broadcast_to(amp * np.cos(k * x), shape)[None].copy()
    new, _ = one_step(prob, eta)
    g = (1 - 2 * A * L * dt) / (1 + 2 * L * dt * kappa * k * k)
    np.testing.assert_allclose(new[0], g * eta[0], rtol=1e-5, atol=amp * 1e-6)


def tanh_profile(n, dx, ell, x1, x2):
    x = (np.arange(n) + 0.5) * dx
    return 0.5 * (np.tanh((x - x1) / (2 * ell)) - np.tanh((x - x2) / (2 * ell)))


def test_flat_interface_tanh_profile_and_energy():
    A, kappa = 1e7, 1e-9
    ell = np.sqrt(kappa / A)
    dx = ell / 4
    n = 256
    shape = (1, 2, n)
    L = 1.0
    dt = 0.02 / (2 * A * L)
    prob = no_mech_problem(shape, dx, A, kappa, L, dt)
    prof = tanh_profile(n, dx, ell, 64 * dx, 192 * dx)
    eta = np.broadcast_to(prof, shape)[None].copy()
    st = pf.State.initial(eta, np.zeros(6))
    for _ in range(100):
        st, stats, _ = pf.step(prob, st, None, oc.load())
    assert np.abs(st.eta[0] - eta[0]).max() < 2e-4
    area = shape[0] * shape[1] * dx * dx
    sigma_int = np.sqrt(A * kappa) / 3
    np.testing.assert_allclose(stats["G_dw"] + stats["G_gd"], 2 * sigma_int * area, rtol=1e-3)
    # equipartition on the exact profile: bulk and gradient parts are equal
    np.testing.assert_allclose(stats["G_dw"], stats["G_gd"], rtol=2e-3)


def nagumo_run(dt_factor, steps_scale=1.0):
    A, kappa, L = 1e7, 1e-9, 1.0
    ell = np.sqrt(kappa / A)
    dx = ell / 4
    n = 512
    shape = (1, 1, n)
    m, s = cr.twin_systems()[0]
    R = oc.frame_m_along_x(m, s)      # twin plane normal along x, shear along z
    tabs = oc.tables(R[None], [0], homogeneous=True)
    gamma = cr.GAMMA_TW
    Delta = 0.1 * A                    # constant driving force sigma : eps0
    tau = Delta / gamma                # sigma_xz with eps0_xz = gamma / 2
    ld = oc.load(sig_bar=[0, 0, 0, 0, tau, 0], stress_mask=[1] * 6)
    dt = dt_factor / (2 * A * L)
    prob = oc.problem(shape, tabs, dx=dx, A=A, kappa=kappa, L=L, dt=dt)
    r1, r2, r3 = np.sort(np.roots([4 * A, -6 * A, 2 * A, -Delta]).real)
    c = 2 * L * np.sqrt(A * kappa) * (r1 + r3 - 2 * r2)
    w = 1.0 / ((r3 - r1) * np.sqrt(A / kappa))
    x = (np.arange(n) + 0.5) * dx
    x1, x2 = 160 * dx, 352 * dx
    prof = r1 + (r3 - r1) * 0.5 * (np.tanh((x - x1) / (2 * w)) - np.tanh((x - x2) / (2 * w)))
    st = pf.State.initial(prof[None, None, None], np.zeros(6))
    t_total = 40 * dx / c * steps_scale
    steps = int(round(t_total / dt))
    masses, times = [], []
    for i in range(steps):
        st, stats, sig = pf.step(prob, st, None, ld)
        if i == 0:
            np.testing.assert_allclose(sig[..., 0, 2], tau, rtol=1e-10)
        masses.append(st.eta.sum() * dx)
        times.append((i + 1) * dt)
    half = len(masses) // 2
    rate = np.polyfit(times[half:], masses[half:], 1)[0]
    return rate / (2 * (r3 - r1)), c


def test_nagumo_front_speed_first_order_in_dt():
    v1, c = nagumo_run(0.04)
    v2, _ = nagumo_run(0.02)
    e1, e2 = abs(v1 - c) / c, abs(v2 - c) / c
    assert e2 < 0.03
    assert e2 < 0.75 * e1           # error shrinks with the step (first order)


def test_energy_decreases():
    rng = np.random.default_rng(8)
    shape = (8, 8, 8)
    R = np.linalg.qr(rng.standard_normal((3, 3)))[0]
    R *= np.sign(np.linalg.det(R))
    tabs = oc.tables(R[None], [0])
    prob = oc.problem(shape, tabs, dt=2e-5)
    eta = rng.random((1,) + shape)
    st = pf.State.initial(eta, np.zeros(6))
    epsp = rng.standard_normal((6,) + shape) * 1e-3
    ld = oc.load(eps_bar=[-2e-3, 0, 0, 0, 0, 0], stress_mask=[0, 1, 1, 1, 1, 1])
    G = []
    for _ in range(25):
        st, stats, _ = pf.step(prob, st, epsp, ld)
        G.append(stats["G"])
    assert np.all(np.diff(G) < 0)


def test_multi_variant_reduces_to_single():
    rng = np.random.default_rng(5)
    shape = (6, 8, 10)
    R = np.linalg.qr(rng.standard_normal((3, 3)))[0]
    R *= np.sign(np.linalg.det(R))
    tabs1 = oc.tables(R[None], [2])
    tabs3 = oc.tables(R[None], [2, 0, 5])
    eta1 = rng.random((1,) + shape)
    eta3 = np.concatenate([eta1, np.zeros((2,) + shape)])
    epsp = rng.standard_normal((6,) + shape) * 1e-3
    ld = oc.load(eps_bar=[-2e-3, 0, 0, 0, 0, 0], stress_mask=[0, 1, 1, 1, 1, 1])
    C0 = pf.reference_stiffness_average(*tabs1[:2])
    p1 = oc.problem(shape, tabs1, h_kind="quintic", C0=C0)
    p3 = oc.problem(shape, tabs3, h_kind="quintic", C0=C0)
    n1, s1 = one_step(p1, eta1, ld, epsp)
    n3, s3 = one_step(p3, eta3, ld, epsp)
    np.testing.assert_allclose(n3[0], n1[0], atol=1e-13)
    assert np.abs(n3[1:]).max() == 0.0


def test_variant_relabelling_and_translation_commute_with_step():
    rng = np.random.default_rng(6)
    shape = (6, 8, 10)
    rots = np.stack([np.linalg.qr(rng.standard_normal((3, 3)))[0] for _ in range(2)])
    for r in rots:
        r *= np.sign(np.linalg.det(r))
    ids = [0, 3, 4]
    perm = [2, 0, 1]
    gid = (rng.random(shape) < 0.4).astype(np.int64)
    eta = rng.random((3,) + shape) * 0.3
    epsp = rng.standard_normal((6,) + shape) * 1e-3
    ld = oc.load(eps_bar=[0, 0, -3e-3, 0, 0, 0], stress_mask=[1, 1, 0, 1, 1, 1])
    tabs = oc.tables(rots, ids)
    C0 = pf.reference_stiffness_average(*tabs[:2])
    base, _ = one_step(oc.problem(shape, tabs, gid=gid, C0=C0), eta, ld, epsp)
    tabs_p = oc.tables(rots, [ids[p] for p in perm])
    perm_out, _ = one_step(oc.problem(shape, tabs_p, gid=gid, C0=C0), eta[perm], ld, epsp)
    np.testing.assert_allclose(perm_out, base[perm], atol=1e-12)
    sh = (1, 3, -2)
    roll = lambda f: np.roll(f, sh, axis=(-3, -2, -1))
    tr_out, _ = one_step(oc.problem(shape, tabs, gid=roll(gid), C0=C0), roll(eta), ld, roll(epsp))
    np.testing.assert_allclose(tr_out, roll(base), atol=1e-12)


def test_gradient_energy_of_a_sine():
    shape, dx = (4, 6, 16), 2e-8
    kappa = 1e-9
    x = np.arange(shape[2]) * dx
    k = 2 * np.pi * 3 / (shape[2] * dx)
    a = 0.2
    eta = np.broadcast_to(0.5 + a * np.sin(k * x), shape)[None].copy()
    vol = np.prod(shape) * dx ** 3
    np.testing.assert_allclose(pf.gradient_energy(eta, kappa, dx), kappa * a * a * k * k * vol / 2, rtol=1e-12)


# ---------------------------------------------------------------- several variants
# Eq. (13) sums c1 f_a^2 f_b^2 over every pair of phases, the matrix
# f_M = 1 - sum f (eq. (18)) included. The pins below do not restate the
# oracle's loops: a value summed by hand, an algebraic identity of the pair
# sum, the symmetry of the energy under exchanging any two phases, and the
# exchange derivatives of single pair terms taken by finite differences.

def test_double_well_three_variants_hand_sum():
    # f = (0.1, 0.2, 0.3), f_M = 0.4: the six pair products f_a^2 f_b^2 are
    # 0.0004, 0.0009, 0.0016, 0.0036, 0.0064, 0.0144, total 0.0273
    A = 1e7
    eta = np.array([0.1, 0.2, 0.3]).reshape(3, 1)
    np.testing.assert_allclose(pf.double_well_density(eta, A), [0.0273 * A], rtol=1e-13)


def test_double_well_pair_sum_identity():
    # sum_{a<b} x_a^2 x_b^2 = ((sum x^2)^2 - sum x^4) / 2 over all phases
    A = 3.0
    rng = np.random.default_rng(11)
    for V in (2, 3, 6):
        eta = rng.random((V, 7)) * (1.2 / V) - 0.05
        x = np.concatenate([eta, 1.0 - eta.sum(0, keepdims=True)])
        expect = A * 0.5 * ((x ** 2).sum(0) ** 2 - (x ** 4).sum(0))
        np.testing.assert_allclose(pf.double_well_density(eta, A), expect, rtol=1e-12)


def test_double_well_symmetric_in_all_phases():
    # swapping a variant with the matrix (or with another variant) leaves the
    # energy unchanged: the matrix enters the pair sum like any variant
    A = 1.0
    rng = np.random.default_rng(12)
    eta = rng.random((3, 9)) * 0.3
    fm = 1.0 - eta.sum(0)
    base = pf.double_well_density(eta, A)
    for a in range(3):
        sw = eta.copy()
        sw[a] = fm                      # the old matrix becomes variant a
        np.testing.assert_allclose(pf.double_well_density(sw, A), base, rtol=1e-12)
    np.testing.assert_allclose(pf.double_well_density(eta[[2, 0, 1]], A), base, rtol=1e-13)


def test_chemical_force_several_variants_exchange_derivatives():
    # eq. (17), first term: chem_a = sum_{b != a} (d/df_a - d/df_b) of the pair
    # term A f_a^2 f_b^2, b over the other variants and the matrix; each
    # exchange derivative is taken here by central differences of the pair
    # term in the direction e_a - e_b with every phase held independent.
    A = 2.5e7
    rng = np.random.default_rng(13)
    V = 3
    eta = rng.random((V, 11)) * 0.3
    phases = np.concatenate([eta, 1.0 - eta.sum(0, keepdims=True)])
    h = 1e-5

    def pair(x, a, b):
        return A * x[a] ** 2 * x[b] ** 2

    expect = np.zeros_like(eta)
    for a in range(V):
        for b in range(V + 1):
            if b == a:
                continue
            up, dn = phases.copy(), phases.copy()
            up[a] += h
            up[b] -= h
            dn[a] -= h
            dn[b] += h
            expect[a] += (pair(up, a, b) - pair(dn, a, b)) / (2 * h)
    np.testing.assert_allclose(pf.chemical_force(eta, A), expect, rtol=1e-8, atol=1e-8 * A)


def test_chemical_force_exchange_forces_cancel_over_all_phases():
    # the pairwise exchange forces are antisymmetric, so the forces of all
    # V + 1 phases add up to zero; the matrix's own force is the force of
    # variant 0 after the matrix and variant 0 trade places
    A = 1e7
    rng = np.random.default_rng(14)
    eta = rng.random((3, 13)) * 0.3
    fm = 1.0 - eta.sum(0)
    chem = pf.chemical_force(eta, A)
    sw = eta.copy()
    sw[0] = fm
    chem_m = pf.chemical_force(sw, A)[0]
    total = chem.sum(0) + chem_m
    np.testing.assert_allclose(total, 0.0, atol=1e-9 * A)
    assert np.abs(chem).max() > 1e-3 * A
