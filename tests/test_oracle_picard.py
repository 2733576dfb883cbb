"""Pins of the oracle's fixed point i over the phase-field update (Table 1,
eqs. (19)-(20)): each solve re-evaluates the nonlinear (chemical) force at the
previous iterate, the gradient term stays implicit, the mechanical force is
held at f^n; the iteration stops when max |f^i - f^{i-1}| <= ERR_f.

* A uniform single variant without mechanical force: the converged step is
  the root of the scalar backward-Euler equation
  f - f^n + L dt m 2A f (1 - f)(1 - 2f) = 0, found by a bracketing root finder
  (m = 1, and a constant relative mobility m).
* A non-uniform field: the converged step satisfies the backward-Euler
  equation f - f^n + L dt (chem(f) - mech) - 2 L dt kappa lap f = 0 with the
  Laplacian taken by a full complex FFT and wave numbers built here.
* The first solve is the plain semi-implicit step; the L2 change contracts by
  at least 2 A L dt per solve (the implicit gradient factor has norm <= 1 and
  the chemical force is 2A-Lipschitz on [0, 1] for one variant).
* One step of the converged scheme has a local error O(dt^2) against the
  exact ODE solution of a uniform state (ratio near 4 when dt halves).
* m = 0 still freezes f under the iteration; an unconverged run is flagged.
"""

import numpy as np
from scipy import integrate, optimize

from oracle import phasefield as pf
from tests import oracle_cases as oc

A, L = 1e7, 1.2e-5


def problem(shape, dt, pf_max_iter, pf_tol=1e-14, mobility=None, kappa=1e-9, dx=5e-8):
    tabs = oc.tables(np.eye(3)[None], [0], homogeneous=True, no_eigenstrain=True)
    return oc.problem(shape, tabs, dx=dx, A=A, kappa=kappa, L=L, dt=dt, mobility=mobility,
                      pf_tol=pf_tol, pf_max_iter=pf_max_iter)


def one_step(prob, eta):
    st = pf.State.initial(eta, np.zeros(6))
    new, stats, _ = pf.step(prob, st, None, oc.load())
    return new.eta, stats


def dwell(f):
    # single variant: d/df of A f^2 (1 - f)^2
    return 2.0 * A * f * (1.0 - f) * (1.0 - 2.0 * f)


def test_uniform_state_is_the_scalar_backward_euler_root():
    shape, dt, f0 = (4, 4, 4), 2e-3, 0.3
    eta = np.full((1,) + shape, f0)
    for m in (None, 0.4):
        mob = None if m is None else np.full(shape, m)
        mm = 1.0 if m is None else m
        root = optimize.brentq(lambda f: f - f0 + L * dt * mm * dwell(f), 0.0, 0.6, xtol=1e-15, rtol=1e-15)
        new, st = one_step(problem(shape, dt, 80, mobility=mob), eta)
        assert st["pf_converged"] and st["pf_iters"] > 3
        np.testing.assert_allclose(new, root, rtol=0, atol=1e-12)
        plain, _ = one_step(problem(shape, dt, 1, mobility=mob), eta)
        assert abs(plain.ravel()[0] - root) > 1e-4      # the iteration matters here


def smooth_field(shape, seed):
    rng = np.random.default_rng(seed)
    F = np.fft.fftn(rng.standard_normal(shape))
    k2 = sum(np.meshgrid(*[np.fft.fftfreq(n) ** 2 for n in shape], indexing="ij"))
    f = np.real(np.fft.ifftn(F * np.exp(-60.0 * k2)))
    return 0.5 + 0.35 * f / np.abs(f).max()


def laplacian(f, dx):
    ks = [2 * np.pi * np.fft.fftfreq(n, d=dx) for n in f.shape]
    k2 = sum(np.meshgrid(*[k ** 2 for k in ks], indexing="ij"))
    return np.real(np.fft.ifftn(-k2 * np.fft.fftn(f)))


def test_converged_step_solves_backward_euler():
    shape, dt, dx, kappa = (8, 12, 16), 2e-3, 5e-8, 1e-9
    f0 = smooth_field(shape, 3)
    new, st = one_step(problem(shape, dt, 100, kappa=kappa, dx=dx), f0[None])
    assert st["pf_converged"]
    f = new[0]
    r = f - f0 + L * dt * dwell(f) - 2.0 * L * dt * kappa * laplacian(f, dx)
    assert np.abs(r).max() < 1e-11
    plain, _ = one_step(problem(shape, dt, 1, kappa=kappa, dx=dx), f0[None])
    rp = plain[0] - f0 + L * dt * dwell(plain[0]) - 2.0 * L * dt * kappa * laplacian(plain[0], dx)
    assert np.abs(rp).max() > 1e-5


def test_two_variants_converge_to_the_coupled_backward_euler():
    shape, dt, dx, kappa = (6, 8, 10), 2e-3, 5e-8, 1e-9
    f0 = np.stack([0.5 * smooth_field(shape, 5), 0.4 * smooth_field(shape, 6)])
    tabs = oc.tables(np.eye(3)[None], [0, 1], homogeneous=True, no_eigenstrain=True)
    prob = oc.problem(shape, tabs, dx=dx, A=A, kappa=kappa, L=L, dt=dt, pf_tol=1e-14, pf_max_iter=100)
    new, st = one_step(prob, f0)
    assert st["pf_converged"]
    chem = pf.chemical_force(new, A)
    for a in range(2):
        r = new[a] - f0[a] + L * dt * chem[a] - 2.0 * L * dt * kappa * laplacian(new[a], dx)
        assert np.abs(r).max() < 1e-11


def test_first_solve_is_the_plain_step_and_changes_contract():
    shape, dt = (8, 8, 8), 2e-3
    f0 = smooth_field(shape, 7)[None]
    plain, _ = one_step(problem(shape, dt, 1), f0)
    first, st = one_step(problem(shape, dt, 6, pf_tol=1.0), f0)
    assert st["pf_iters"] == 1
    np.testing.assert_array_equal(first, plain)
    prob = problem(shape, dt, 1)
    mech = np.zeros_like(f0)
    prev, changes = f0, []
    for _ in range(6):
        nxt = pf.picard_iterate(f0, prev, mech, prob)
        changes.append(np.sqrt(((nxt - prev) ** 2).sum()))
        prev = nxt
    np.testing.assert_array_equal(pf.picard_iterate(f0, f0, mech, prob), plain)
    for a, b in zip(changes[1:], changes[:-1]):
        assert a <= 2.0 * A * L * dt * b * (1 + 1e-9)


def test_local_error_is_second_order():
    shape, f0 = (4, 4, 4), 0.3
    exact = lambda t: integrate.solve_ivp(lambda _, y: -L * dwell(y), (0, t), [f0], rtol=1e-13,
                                          atol=1e-15).y[0, -1]
    errs = []
    for dt in (1e-3, 5e-4):
        new, st = one_step(problem(shape, dt, 100), np.full((1,) + shape, f0))
        assert st["pf_converged"]
        errs.append(abs(new.ravel()[0] - exact(dt)))
    assert 3.6 < errs[0] / errs[1] < 4.4


def test_zero_mobility_freezes_and_nonconvergence_is_flagged():
    shape, dt = (6, 6, 8), 2e-3
    f0 = smooth_field(shape, 9)[None]
    new, st = one_step(problem(shape, dt, 20, mobility=np.zeros(shape)), f0)
    np.testing.assert_allclose(new, f0, rtol=0, atol=1e-13)
    assert st["pf_converged"]
    _, st = one_step(problem(shape, dt, 2, pf_tol=0.0), f0)
    assert st["pf_iters"] == 2 and not st["pf_converged"]
