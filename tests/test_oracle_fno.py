"""Pins of the oracle's Fourier-neural-operator stepper and its acceptance
residual.

* GELU at points where the normal CDF is known.
* The spectral convolution against an explicit double sum (naive DFT of the
  input, explicit inverse with the half-spectrum weights) on a tiny grid.
* With R = identity the spectral convolution returns a field band-limited
  to the kept modes unchanged (low-pass projection).
* With R = 0 the network is a pointwise perceptron: compared voxel by voxel
  with a scalar loop.
* Translating the input translates the output (no coordinate channels).
* The acceptance residual of one exact plain step is zero (to round-off):
  for S = 1 the corrected trapezoid weights reduce it to the semi-implicit
  step itself, which the oracle computes by a separate route (spectral
  division by the implicit symbol).
* Over S exact plain steps it equals the quadrature defect of the two summed
  forces, built here from the states of the trajectory one by one.
* A perturbation of the prediction raises the residual by at least its size;
  late in a relaxation (16 steps per call) the exact prediction is accepted
  at 1e-3 and the same prediction with a 2e-3 bump, local or smooth, is not.
"""

import math

import numpy as np

from oracle import fno
from oracle import phasefield as pf
from paper_2302_13612_amd import inputs
from tests import cases


def test_gelu_values():
    x = np.array([0.0, 1.0, -1.0, 2.0, 10.0, -10.0])
    expect = np.array([0.0, 0.8413447460685429, -0.15865525393145707, 1.9544997361036416, 10.0, 0.0])
    np.testing.assert_allclose(fno.gelu(x), expect, rtol=1e-14, atol=1e-15)


def naive_spectral_conv(v, R):
    C, nz, ny, nx = v.shape
    m = R.shape[-1]
    iz, iy = fno.kept_index(nz, m), fno.kept_index(ny, m)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ntot = nz * ny * nx
    out = np.zeros((R.shape[0], nz, ny, nx))
    for a, kz in enumerate(iz):
        for b, ky in enumerate(iy):
            for kx in range(m):
                ph = 2 * math.pi * (kz * z / nz + ky * y / ny + kx * x / nx)
                vk = np.array([(v[i] * np.exp(-1j * ph)).sum() for i in range(C)])
                sk = R[:, :, a, b, kx] @ vk
                w = 1.0 if kx == 0 else 2.0
                for o in range(R.shape[0]):
                    out[o] += w * np.real(sk[o] * np.exp(1j * ph)) / ntot
    return out


def test_spectral_conv_matches_explicit_sums():
    rng = np.random.default_rng(1)
    v = rng.normal(size=(3, 6, 8, 10))
    R = rng.normal(size=(2, 3, 4, 4, 2)) + 1j * rng.normal(size=(2, 3, 4, 4, 2))
    np.testing.assert_allclose(fno.spectral_conv(v, R), naive_spectral_conv(v, R), rtol=1e-10, atol=1e-12)


def test_identity_weights_keep_band_limited_fields():
    rng = np.random.default_rng(2)
    C, n, m = 2, 16, 4
    spec = np.zeros((C, n, n, n // 2 + 1), dtype=complex)
    sym = np.concatenate([np.arange(m), np.arange(n - m + 1, n)])   # closed under k -> -k
    for c in range(C):
        for kz in sym:
            for ky in sym:
                spec[c, kz, ky, :m] = rng.normal(size=m) + 1j * rng.normal(size=m)
    v = np.fft.irfftn(spec, s=(n, n, n), axes=(1, 2, 3))
    R = np.zeros((C, C, 2 * m, 2 * m, m), dtype=complex)
    for c in range(C):
        R[c, c] = 1.0
    np.testing.assert_allclose(fno.spectral_conv(v, R), v, atol=1e-12)
    # a field with power outside the kept band loses exactly that part
    w = rng.normal(size=(C, n, n, n))
    out = fno.spectral_conv(w, R)
    assert np.linalg.norm(out) < np.linalg.norm(w)


def test_pointwise_network_when_spectral_weights_vanish():
    p = fno.init_params(width=4, modes=1, hidden=5, n_layers=2, seed=3)
    p["R"][:] = 0.0
    rng = np.random.default_rng(4)
    eta = rng.random((2, 2, 2))
    cond = rng.normal(size=fno.N_COND)
    out = fno.forward(p, eta, cond)

    def g(x):
        return 0.5 * x * (1.0 + math.erf(x / math.sqrt(2.0)))

    for idx in np.ndindex(eta.shape):
        a = [eta[idx]] + list(cond)
        v = [sum(p["P"][o][j] * a[j] for j in range(len(a))) + p["p"][o] for o in range(4)]
        for l in range(2):
            v = [g(sum(p["W"][l][o][i] * v[i] for i in range(4)) + p["b"][l][o]) for o in range(4)]
        h = [g(sum(p["Q1"][k][i] * v[i] for i in range(4)) + p["q1"][k]) for k in range(5)]
        d = sum(p["Q2"][0][k] * h[k] for k in range(5)) + p["q2"][0]
        assert abs(out[idx] - (eta[idx] + d)) < 1e-12


def test_translation_equivariance():
    p = fno.init_params(width=4, modes=3, hidden=6, n_layers=2, seed=5, scale_spec=0.05)
    rng = np.random.default_rng(6)
    eta = rng.random((8, 10, 12))
    cond = rng.normal(size=fno.N_COND)
    a = fno.forward(p, eta, cond)
    b = fno.forward(p, np.roll(eta, (3, -2, 5), axis=(0, 1, 2)), cond)
    np.testing.assert_allclose(np.roll(a, (3, -2, 5), axis=(0, 1, 2)), b, atol=1e-12)


def small_problem():
    cfg = inputs.single_crystal_sphere(n=16, radius=4)
    cfg = dict(cfg, eta0=inputs.sphere((16, 16, 16), (8, 8, 8), 4.0)[None].astype(np.float32))
    prob = cases.oracle_problem(cfg, tol=1e-12)
    load = dict(eps_bar=cfg["eps_bar"], sig_bar=cfg["sig_bar"], stress_mask=cfg["stress_mask"])
    return cfg, prob, load


def trajectory(prob, cfg, load, n):
    st = pf.State.initial(cfg["eta0"].astype(np.float64), np.zeros(6))
    out = [st.eta.copy()]
    for _ in range(n):
        st, _, _ = pf.step(prob, st, None, load)
        out.append(st.eta.copy())
    return out


def test_one_plain_step_has_zero_residual():
    cfg, prob, load = small_problem()
    f = trajectory(prob, cfg, load, 3)
    for k in range(3):
        r, rho = fno.macro_residual(prob, f[k], f[k + 1], 1, load)
        assert np.abs(f[k + 1] - f[k]).max() > 1e-3      # the step moves the field
        assert rho <= 1e-12, (k, rho)
        assert rho == np.abs(r).max()


def test_residual_is_the_quadrature_defect():
    cfg, prob, load = small_problem()
    S = 5
    f = trajectory(prob, cfg, load, 2 + S)[2:]
    r, _ = fno.macro_residual(prob, f[0], f[S], S, load)
    G = [fno.gradient_force(prob, x) for x in f]
    E = [fno.variational_derivative(prob, x, load) - g for x, g in zip(f, G)]   # chem - mech
    a, b = (S + 1) / 2, (S - 1) / 2
    defect = prob.L * prob.dt * (a * E[0] + b * E[S] - sum(E[:S]) + a * G[S] + b * G[0] - sum(G[1:S + 1]))
    scale = np.abs(defect).max()
    assert scale > 1e-6
    np.testing.assert_allclose(r, defect, rtol=0, atol=1e-9 * scale + 1e-13)
    # weights swapped between the two ends: no longer the defect
    bad = f[S] - f[0] + prob.L * prob.dt * (b * (E[0] + G[0]) + a * (E[S] + G[S]) + G[S] - G[0])
    assert np.abs(bad - defect).max() > 1e3 * 1e-9 * scale


def test_accepts_exact_rejects_perturbed_late():
    cfg, prob, load = small_problem()
    f = trajectory(prob, cfg, load, 80)
    tol = 1e-3
    _, rho = fno.macro_residual(prob, f[64], f[80], 16, load)
    assert rho <= 0.5 * tol, rho
    bump = f[80].copy()
    bump[0, 3, 3, 3] += 2e-3
    _, rho_b = fno.macro_residual(prob, f[64], bump, 16, load)
    wave = f[80] + 2e-3 * np.sin(2 * np.pi * np.arange(16) / 16)[None, None, None, :]
    _, rho_w = fno.macro_residual(prob, f[64], wave, 16, load)
    assert rho_b > 2 * tol and rho_w > 2 * tol, (rho_b, rho_w)
    # the backward-Euler residual of the same exact window is first order
    g1 = fno.variational_derivative(prob, f[80], load)
    be = np.abs(f[80] - f[64] + 16 * prob.L * prob.dt * g1).max()
    assert be > 2 * rho


def test_residual_grows_with_perturbation():
    # a window after the initial relaxation: the bump, not the exact
    # trajectory's own defect, sets the maximum
    cfg, prob, load = small_problem()
    f = trajectory(prob, cfg, load, 44)
    r, rho = fno.macro_residual(prob, f[40], f[44], 4, load)
    bumped = f[44].copy()
    bumped[0, 3, 3, 3] += 0.2
    r_b, rho_b = fno.macro_residual(prob, f[40], bumped, 4, load)
    assert r_b[0, 3, 3, 3] - r[0, 3, 3, 3] >= 0.1
    assert rho_b >= 0.1 > rho
