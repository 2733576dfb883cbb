"""Pins of the oracle's variable mobility (the pad layer of Sec. 4: very low
mobility outside the specimen; relative mobility m(x) in [0, 1], gradient
term split with the largest mobility implicit).

* m = 1 everywhere is the plain step, exactly.
* m = 0 everywhere leaves f unchanged (to rounding), whatever the forces.
* A single Fourier mode under a constant m decays by exactly
  (1 + 2 L dt (1 - m) q) / (1 + 2 L dt q), q = kappa |xi|^2 written out here
  from the mode's wave numbers; the factor lies in [0, 1] for m in [0, 1].
* A twin nucleus inside a pillar with a pad of m = 0 grows inside while the
  pad stays put (its change is bounded by the implicit smoothing of the
  interface, and much smaller than inside).
"""

import numpy as np

from oracle import phasefield as pf
from tests import oracle_cases as oc


def problem(shape, mobility, A=1e7, dt=2e-4, homogeneous=True, eigen=True):
    tabs = oc.tables(np.eye(3)[None], [0], homogeneous=homogeneous, no_eigenstrain=not eigen)
    return oc.problem(shape, tabs, A=A, dt=dt, mobility=mobility)


def one_step(prob, eta, ld=None):
    st = pf.State.initial(eta, np.zeros(6))
    new, stats, _ = pf.step(prob, st, None, ld or oc.load())
    return new.eta, stats


def test_unit_mobility_is_the_plain_step():
    shape = (8, 10, 12)
    rng = np.random.default_rng(1)
    eta = (rng.random((1,) + shape) * 0.6)
    ld = oc.load(eps_bar=[-2e-3, 0, 0, 0, 0, 0], stress_mask=[False] + [True] * 5)
    a, _ = one_step(problem(shape, None), eta, ld)
    b, _ = one_step(problem(shape, np.ones(shape)), eta, ld)
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-14)


def test_zero_mobility_freezes():
    shape = (8, 10, 12)
    rng = np.random.default_rng(2)
    eta = (rng.random((1,) + shape) * 0.6)
    ld = oc.load(eps_bar=[-2e-3, 0, 0, 0, 0, 0], stress_mask=[False] + [True] * 5)
    b, _ = one_step(problem(shape, np.zeros(shape)), eta, ld)
    np.testing.assert_allclose(b, eta, rtol=0, atol=1e-13)


def test_single_mode_under_constant_mobility():
    shape, dx = (4, 6, 32), 5e-8
    L, dt, kappa = 1.2e-5, 2e-4, 1e-9
    tabs = oc.tables(np.eye(3)[None], [0], homogeneous=True, no_eigenstrain=True)
    for m in (0.0, 0.3, 1.0):
        prob = oc.problem(shape, tabs, dx=dx, A=0.0, kappa=kappa, L=L, dt=dt, mobility=np.full(shape, m))
        x = np.arange(shape[2])
        k = 2 * np.pi * 5 / (shape[2] * dx)
        eta = np.broadcast_to(0.5 + 0.1 * np.cos(2 * np.pi * 5 * x / shape[2]), shape)[None].copy()
        new, _ = one_step(prob, eta)
        q = kappa * k * k
        g = (1 + 2 * L * dt * (1 - m) * q) / (1 + 2 * L * dt * q)
        assert 0.0 <= g <= 1.0
        np.testing.assert_allclose(new[0], 0.5 + 0.1 * g * np.cos(2 * np.pi * 5 * x / shape[2]) * np.ones(shape),
                                   rtol=0, atol=1e-13)


def test_pad_layer_holds_while_the_inside_evolves():
    n = 24
    shape = (n, n, n)
    pad = 4
    m = np.zeros(shape)
    m[pad:-pad, pad:-pad, pad:-pad] = 1.0
    z, y, x = np.meshgrid(*(np.arange(n),) * 3, indexing="ij")
    eta = ((x - 12) ** 2 + (y - 12) ** 2 + (z - 12) ** 2 <= 16).astype(float)[None]
    ld = oc.load(eps_bar=[-2e-3, 0, 0, 0, 0, 0], stress_mask=[False] + [True] * 5)
    prob = problem(shape, m)
    st = pf.State.initial(eta, np.zeros(6))
    for _ in range(10):
        st, _, _ = pf.step(prob, st, None, ld)
    d = np.abs(st.eta[0] - eta[0])
    inside = m > 0
    assert d[inside].max() > 0.05              # the nucleus evolves
    assert d[~inside].max() < 0.2 * d[inside].max()
