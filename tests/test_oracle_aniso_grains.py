"""Pins of the oracle's anisotropic gradient energy on a polycrystal (per-grain
tensors K_a^g, implicit kbar_a I, explicit remainder through spectral first
derivatives).

* First derivatives against the analytic derivatives of band-limited fields;
  a Nyquist mode has zero derivative.
* With a constant tensor the remainder operator equals the Fourier symbol
  -2 xi.K.xi (d_i d_j <-> -xi_i xi_j) on fields without Nyquist content.
* The remainder is a divergence: zero mean; it is symmetric, and
  <f, 2 div(K grad f)> = -2 int grad f . K . grad f (integration by parts).
* The split: kbar_a is the largest eigenvalue over the grains (for the
  Table 5 tensors, c2s in every grain and variant), the remainder is negative
  semidefinite; all grains at kappa I give the isotropic step; one grain of
  constant K gives the per-mode closed form of the split scheme.
* The reported energy's directional derivative is the step's operator.
* A pure gradient flow with the Table 5 tensors stays bounded and loses
  energy monotonically at a time step a thousand times the default.
"""

import numpy as np

from oracle import crystal as cr
from oracle import phasefield as pf
from oracle import spectral
from paper_2302_13612_amd import inputs

DX = 5e-8


def band_limited(shape, rng, kmax=3):
    """Random real field with modes |k_i| <= kmax only (no Nyquist content)."""
    F = np.zeros((shape[0], shape[1], shape[2] // 2 + 1), dtype=complex)
    for kz in range(-kmax, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            for kx in range(0, kmax + 1):
                F[kz % shape[0], ky % shape[1], kx] = rng.normal() + 1j * rng.normal()
    return spectral.irfft3(F, shape)


def random_spd(rng, n):
    M = rng.normal(size=(n, 3, 3))
    return np.einsum("nij,nkj->nik", M, M) * 1e-7 + 1e-8 * np.eye(3)


def test_first_derivatives_closed_form():
    shape = (8, 12, 16)
    z, y, x = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    Lx, Ly, Lz = shape[2] * DX, shape[1] * DX, shape[0] * DX
    f = np.sin(2 * np.pi * 3 * x / shape[2] + 0.3) * np.cos(2 * np.pi * 2 * y / shape[1]) + \
        np.cos(2 * np.pi * z / shape[0] - 0.7)
    g = pf.spectral_gradient(f, DX)
    gx = (2 * np.pi * 3 / Lx) * np.cos(2 * np.pi * 3 * x / shape[2] + 0.3) * np.cos(2 * np.pi * 2 * y / shape[1])
    gy = -(2 * np.pi * 2 / Ly) * np.sin(2 * np.pi * 3 * x / shape[2] + 0.3) * np.sin(2 * np.pi * 2 * y / shape[1])
    gz = -(2 * np.pi / Lz) * np.sin(2 * np.pi * z / shape[0] - 0.7)
    scale = 2 * np.pi * 3 / Lx
    for a, b in zip(g, (gx, gy, gz)):
        np.testing.assert_allclose(a, b, atol=1e-12 * scale)
    # divergence of (gx, gy, gz) is the Laplacian
    lap = -((2 * np.pi * 3 / Lx) ** 2 + (2 * np.pi * 2 / Ly) ** 2) * \
        np.sin(2 * np.pi * 3 * x / shape[2] + 0.3) * np.cos(2 * np.pi * 2 * y / shape[1]) - \
        (2 * np.pi / Lz) ** 2 * np.cos(2 * np.pi * z / shape[0] - 0.7)
    np.testing.assert_allclose(pf.spectral_divergence(g, DX), lap, atol=1e-11 * np.abs(lap).max())
    # a Nyquist mode along x: derivative zero
    nyq = np.cos(np.pi * x)
    assert np.abs(pf.spectral_gradient(nyq, DX)).max() < 1e-9 * np.pi / DX


def test_constant_tensor_is_the_symbol():
    rng = np.random.default_rng(1)
    shape = (12, 16, 10)
    K = random_spd(rng, 1)[0]
    f = band_limited(shape, rng)
    out = pf.remainder_divergence(f, np.broadcast_to(K, shape + (3, 3)), DX)
    sym = pf.gradient_symbol(shape, DX, None, K)
    ref = spectral.irfft3(-2.0 * sym * spectral.rfft3(f), shape)
    np.testing.assert_allclose(out, ref, atol=1e-10 * np.abs(ref).max())


def voronoi_case(rng, shape=(16, 16, 16), G=4):
    gid = inputs.voronoi_grains(shape, G, rng)
    K = random_spd(rng, G)
    return gid, K


def test_remainder_divergence_properties():
    rng = np.random.default_rng(2)
    shape = (16, 16, 16)
    gid, K = voronoi_case(rng, shape)
    Kf = K[gid]
    f, g = rng.normal(size=shape), rng.normal(size=shape)
    Rf, Rg = pf.remainder_divergence(f, Kf, DX), pf.remainder_divergence(g, Kf, DX)
    s = np.abs(Rf).max()
    assert abs(Rf.mean()) <= 1e-12 * s
    np.testing.assert_allclose((g * Rf).sum(), (f * Rg).sum(), rtol=1e-10)
    gf = pf.spectral_gradient(f, DX)
    energy = np.einsum("izyx,zyxij,jzyx->", gf, Kf, gf)
    assert energy > 0
    np.testing.assert_allclose((f * Rf).sum(), -2.0 * energy, rtol=1e-10)


def test_split_of_the_twin_tensors():
    rng = inputs.rng_for(5)
    R = inputs.random_rotations(5, rng)
    kv = cr.twin_gradient_tensors(R, [0, 2, 4], c2n=2.81e-7, c2s=2.81e-6, c2t=2.81e-7)
    kbar, rem = pf.grain_split(kv)
    np.testing.assert_allclose(kbar, 2.81e-6, rtol=1e-12)
    ev = np.linalg.eigvalsh(rem)
    assert ev.max() <= 1e-12 * 2.81e-6
    # per grain and variant: eigenvalues c2n - c2s (twice) and 0
    np.testing.assert_allclose(np.sort(ev, axis=-1)[..., 1], 2.81e-7 - 2.81e-6, rtol=1e-9)


def small_grain_problem(kappa_grain, gid, mobility=None):
    shape = gid.shape
    tabs = cr.mg_tables(np.eye(3)[None].repeat(kappa_grain.shape[0], 0), [0])
    C0 = pf.reference_stiffness_average(tabs[0], tabs[1])
    return pf.Problem(shape, DX, tabs, 1e7, 1e-9, 1.2e-5, 2e-4, C0, gid=gid, kappa_grain=kappa_grain)


def test_isotropic_grains_give_the_isotropic_update():
    rng = np.random.default_rng(3)
    shape = (16, 16, 16)
    gid = inputs.voronoi_grains(shape, 3, rng)
    kap = 2.5e-9
    kg = np.broadcast_to(kap * np.eye(3), (3, 2, 3, 3)).copy()
    prob = small_grain_problem(kg, gid)
    eta = rng.random((2,) + shape) * 0.5
    chem, mech = rng.normal(size=eta.shape) * 1e6, rng.normal(size=eta.shape) * 1e6
    a = pf.allen_cahn_update(eta, chem, mech, prob.L, prob.dt, prob.kappa, DX, grains=prob.grains)
    b = pf.allen_cahn_update(eta, chem, mech, prob.L, prob.dt, kap, DX)
    np.testing.assert_allclose(a, b, atol=1e-13)
    np.testing.assert_allclose(pf.gradient_energy(eta, kap, DX),
                               pf.gradient_energy(eta, None, DX, grains=prob.grains), rtol=1e-12)


def test_one_grain_split_closed_form():
    rng = np.random.default_rng(4)
    shape = (16, 12, 16)
    K = random_spd(rng, 1)[0] * 20
    gid = np.zeros(shape, dtype=np.int64)
    prob = small_grain_problem(K[None, None], gid)
    kbar = np.linalg.eigvalsh(K).max()
    f = band_limited(shape, rng)[None]
    L, dt = prob.L, prob.dt * 50
    zero = np.zeros_like(f)
    out = pf.allen_cahn_update(f, zero, zero, L, dt, prob.kappa, DX, grains=prob.grains)
    xi = spectral.wavevectors(shape, DX)
    sk = np.einsum("...i,ij,...j->...", xi, K, xi)
    x2 = (xi ** 2).sum(-1)
    amp = (1.0 - 2 * L * dt * (sk - kbar * x2)) / (1.0 + 2 * L * dt * kbar * x2)
    ref = spectral.irfft3(amp * spectral.rfft3(f[0]), shape)
    np.testing.assert_allclose(out[0], ref, atol=1e-12 * np.abs(ref).max())
    assert np.all(amp > 0) and np.all(amp <= 1 + 1e-15)


def test_energy_derivative_is_the_operator():
    rng = np.random.default_rng(6)
    shape = (16, 16, 16)
    gid, K = voronoi_case(rng, shape, G=3)
    prob = small_grain_problem(K[:, None], gid)
    kbar, rem, gidf = prob.grains
    f = rng.random((1,) + shape)
    d = rng.normal(size=f.shape)
    eps = 1e-4
    e_p = pf.gradient_energy(f + eps * d, None, DX, grains=prob.grains)
    e_m = pf.gradient_energy(f - eps * d, None, DX, grains=prob.grains)
    fd = (e_p - e_m) / (2 * eps)
    # G f = -2 kbar lap f (symbol form) - 2 div((K - kbar) grad f)
    sym = pf.gradient_symbol(shape, DX, kbar[0])
    Gf = spectral.irfft3(2.0 * sym * spectral.rfft3(f[0]), shape) - \
        pf.grain_remainder_divergence(f[0], rem[:, 0], gidf, DX)
    np.testing.assert_allclose(fd, (d[0] * Gf).sum() * DX ** 3, rtol=1e-7)


def test_gradient_flow_stable_at_large_dt():
    rng = inputs.rng_for(7)
    shape = (16, 16, 16)
    gid = inputs.voronoi_grains(shape, 4, rng)
    R = inputs.random_rotations(4, rng)
    kv = cr.twin_gradient_tensors(R, [0, 3], c2n=2.81e-7, c2s=2.81e-6, c2t=2.81e-7)
    prob = small_grain_problem(kv, gid)
    f = rng.random((2,) + shape)
    zero = np.zeros_like(f)
    e = [pf.gradient_energy(f, None, DX, grains=prob.grains)]
    dt = prob.dt * 1000
    for _ in range(10):
        f = pf.allen_cahn_update(f, zero, zero, prob.L, dt, prob.kappa, DX, grains=prob.grains)
        e.append(pf.gradient_energy(f, None, DX, grains=prob.grains))
        assert np.abs(f).max() <= 2.0       # no growth (no maximum principle for a spectral scheme)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(e, e[1:])), e
    assert e[-1] < 0.5 * e[0]
