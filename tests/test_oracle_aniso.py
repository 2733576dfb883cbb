"""Pins of the oracle's anisotropic gradient energy (Table 5: c2 along the
twin-plane normal and along the shear direction; K_a = c2n m m + c2s s s +
c2t t t per variant).

* K_a has the eigenvalues c2n, c2s, c2t on m, s, t = m x s in the frame the
  variant is turned to.
* A single Fourier mode exp(i xi.x) on a non-cubic grid (negative wave
  numbers included) decays in one step by exactly 1/(1 + 2 L dt xi.K.xi),
  with xi.K.xi written out here from the mode's integer wave numbers: a
  swapped axis, a transposed K or a dropped off-diagonal term fails it.
* A flat interface normal to a grid axis n keeps the tanh profile of width
  sqrt(K_nn / A) and carries sqrt(A K_nn)/3 per unit area, whatever the
  other entries of K (the profile varies along n only).
* K = kappa I reproduces the isotropic step exactly.
* Permuting the grid axes together with the indices of K permutes the step
  (on an even grid this holds only with the Nyquist reading of the cross
  terms: a Nyquist component enters the diagonal term only).
* The macro-step residual's gradient force of a single mode is 2 xi.K.xi
  times the mode.
"""

import numpy as np

from oracle import crystal as cr
from oracle import fno
from oracle import phasefield as pf
from tests import oracle_cases as oc


def random_rotation(seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    q = q * np.sign(np.diag(r))
    return q if np.linalg.det(q) > 0 else -q


def spd(seed, scale=1e-9):
    a = np.random.default_rng(seed).normal(size=(3, 3))
    return scale * (a @ a.T / 3.0 + 0.3 * np.eye(3))


def no_mech_problem(shape, dx, A, kappa, L, dt, K):
    tabs = oc.tables(np.eye(3)[None], [0] * K.shape[0], homogeneous=True, no_eigenstrain=True)
    return oc.problem(shape, tabs, dx=dx, A=A, kappa=kappa, L=L, dt=dt, kappa_var=K)


def one_step(prob, eta):
    st = pf.State.initial(eta, np.zeros(6))
    new, stats, _ = pf.step(prob, st, None, oc.load())
    return new.eta, stats


def test_gradient_tensor_eigenstructure():
    R = random_rotation(1)
    K = cr.twin_gradient_tensors(R[None], list(range(6)), c2n=1.0, c2s=5.0, c2t=2.5)[0]
    for a, (m, s) in enumerate(cr.twin_systems()):
        t = np.cross(m, s)
        for v, c in ((m, 1.0), (s, 5.0), (t, 2.5)):
            np.testing.assert_allclose(K[a] @ (R @ v), c * (R @ v), atol=1e-12)
        np.testing.assert_allclose(K[a], K[a].T, atol=1e-15)
    # the paper's values, crystal frame, variant 1: normal and shear directions
    K0 = cr.twin_gradient_tensors(np.eye(3)[None], [0])[0, 0]
    m, s = cr.twin_systems()[0]
    np.testing.assert_allclose([m @ K0 @ m, s @ K0 @ s], [2.81e-7, 2.81e-6], rtol=1e-12)


def test_single_mode_decay_anisotropic():
    shape, dx = (8, 6, 10), 1e-8          # (nz, ny, nx)
    L, dt = 1.0, 2e-10
    K = spd(2)
    prob = no_mech_problem(shape, dx, 0.0, 1e-9, L, dt, K[None])
    kx, ky, kz = 3, -2, 1
    z, y, x = np.meshgrid(*(np.arange(n) for n in shape), indexing="ij")
    phase = 2 * np.pi * (kx * x / shape[2] + ky * y / shape[1] + kz * z / shape[0])
    eta = (0.5 + 0.1 * np.cos(phase))[None]
    new, _ = one_step(prob, eta)
    xi = 2 * np.pi / dx * np.array([kx / shape[2], ky / shape[1], kz / shape[0]])
    q = sum(K[i, j] * xi[i] * xi[j] for i in range(3) for j in range(3))
    g = 1.0 / (1.0 + 2 * L * dt * q)
    np.testing.assert_allclose(new[0], 0.5 + 0.1 * g * np.cos(phase), rtol=0, atol=1e-13)
    # and the decay differs from the one of the isotropic mean coefficient
    assert abs(g - 1.0 / (1.0 + 2 * L * dt * np.trace(K) / 3 * xi @ xi)) > 1e-3


def tanh_profile(n, dx, ell, x1, x2):
    x = (np.arange(n) + 0.5) * dx
    return 0.5 * (np.tanh((x - x1) / (2 * ell)) - np.tanh((x - x2) / (2 * ell)))


def interface_case(axis, K, A=1e7):
    """Flat interfaces normal to grid axis `axis` (0 = x, 2 = z)."""
    kn = K[axis, axis]
    ell = np.sqrt(kn / A)
    dx = ell / 4
    n = 256
    shape = (1, 2, n) if axis == 0 else (n, 2, 1)
    L = 1.0
    dt = 0.02 / (2 * A * L)
    prob = no_mech_problem(shape, dx, A, 1e-9, L, dt, K[None])
    prof = tanh_profile(n, dx, ell, 64 * dx, 192 * dx)
    eta = (np.broadcast_to(prof, shape) if axis == 0 else np.broadcast_to(prof[:, None, None], shape))[None].copy()
    st = pf.State.initial(eta, np.zeros(6))
    for _ in range(100):
        st, stats, _ = pf.step(prob, st, None, oc.load())
    assert np.abs(st.eta[0] - eta[0]).max() < 2e-4
    area = np.prod(shape) / n * dx * dx
    np.testing.assert_allclose(stats["G_dw"] + stats["G_gd"], 2 * np.sqrt(A * kn) / 3 * area, rtol=1e-3)
    np.testing.assert_allclose(stats["G_dw"], stats["G_gd"], rtol=2e-3)


def test_flat_interface_along_x_and_z():
    K = np.array([[1.0e-9, 0.4e-9, -0.3e-9],
                  [0.4e-9, 2.0e-9, 0.5e-9],
                  [-0.3e-9, 0.5e-9, 4.0e-9]])
    assert np.all(np.linalg.eigvalsh(K) > 0)
    interface_case(0, K)
    interface_case(2, K)


def test_isotropic_tensor_reduces_exactly():
    shape, dx = (6, 8, 10), 5e-8
    rng = np.random.default_rng(3)
    eta = rng.random((2,) + shape) * 0.4
    tabs = oc.tables(np.eye(3)[None], [0, 1], homogeneous=True)
    iso = oc.problem(shape, tabs)
    ani = oc.problem(shape, tabs, kappa_var=np.stack([1e-9 * np.eye(3)] * 2))
    a, sa = one_step(iso, eta)
    b, sb = one_step(ani, eta)
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-14)
    np.testing.assert_allclose(sb["G_gd"], sa["G_gd"], rtol=1e-13)


def test_axis_permutation_equivariance():
    n, dx = 8, 2e-8
    K = spd(4)
    rng = np.random.default_rng(5)
    eta = 0.3 + 0.2 * rng.random((1, n, n, n))
    p1 = no_mech_problem((n, n, n), dx, 1e7, 1e-9, 1.0, 1e-9, K[None])
    P = [2, 1, 0]                              # swap x and z
    Kp = K[np.ix_(P, P)]
    p2 = no_mech_problem((n, n, n), dx, 1e7, 1e-9, 1.0, 1e-9, Kp[None])
    a, sa = one_step(p1, eta)
    b, sb = one_step(p2, np.transpose(eta, (0, 3, 2, 1)).copy())
    np.testing.assert_allclose(np.transpose(b, (0, 3, 2, 1)), a, rtol=0, atol=1e-13)
    np.testing.assert_allclose(sb["G_gd"], sa["G_gd"], rtol=1e-12)


def test_residual_gradient_force_of_a_mode():
    shape, dx = (4, 8, 6), 3e-8
    K = spd(6)
    prob = no_mech_problem(shape, dx, 0.0, 1e-9, 1.0, 1e-9, K[None])
    kx, ky, kz = 1, 3, -1
    z, y, x = np.meshgrid(*(np.arange(n) for n in shape), indexing="ij")
    phase = 2 * np.pi * (kx * x / shape[2] + ky * y / shape[1] + kz * z / shape[0])
    eta = (0.05 * np.sin(phase))[None]
    g = fno.variational_derivative(prob, eta, oc.load())
    xi = 2 * np.pi / dx * np.array([kx / shape[2], ky / shape[1], kz / shape[0]])
    q = sum(K[i, j] * xi[i] * xi[j] for i in range(3) for j in range(3))
    np.testing.assert_allclose(g[0], 2 * q * eta[0], rtol=0, atol=1e-9 * 2 * q * 0.05)
