"""Pins of the oracle's FFT conventions and Green's operator.

FFT conventions (the paper solves in Fourier space, Table 1, and is
silent on normalisation) are pinned against a naive DFT written out; the
Green's operator (textbook Moulinec-Suquet / Mura; the paper has none) is
pinned by the projection identity, the isotropic closed form and the
equilibrium of the corrected stress.
"""

import numpy as np
import pytest

from oracle import crystal as cr
from oracle import spectral as sp


def naive_rdft3(f):
    nz, ny, nx = f.shape
    out = np.zeros((nz, ny, nx // 2 + 1), dtype=complex)
    z = np.arange(nz)[:, None, None]
    y = np.arange(ny)[None, :, None]
    x = np.arange(nx)[None, None, :]
    for kz in range(nz):
        for ky in range(ny):
            for kx in range(nx // 2 + 1):
                ph = np.exp(-2j * np.pi * (kz * z / nz + ky * y / ny + kx * x / nx))
                out[kz, ky, kx] = (f * ph).sum()
    return out


@pytest.mark.parametrize("shape", [(4, 6, 8), (6, 12, 16), (3, 4, 6)])
def test_rfft3_matches_naive_dft(shape):
    f = np.random.default_rng(1).standard_normal(shape)
    F = sp.rfft3(f)
    np.testing.assert_allclose(F, naive_rdft3(f), atol=1e-12 * np.abs(F).max())
    np.testing.assert_allclose(sp.irfft3(F, shape), f, atol=1e-13)


@pytest.mark.parametrize("shape", [(8, 6, 10), (4, 4, 9)])
def test_parseval_half_spectrum(shape):
    f = np.random.default_rng(2).standard_normal(shape)
    F = sp.rfft3(f)
    w = sp.half_spectrum_weights(shape)
    lhs = (f * f).sum()
    rhs = (w * np.abs(F) ** 2).sum() / f.size
    if shape[2] % 2:
        # odd nx: there is no Nyquist plane, every kx > 0 counts twice
        w2 = np.full(shape[2] // 2 + 1, 2.0); w2[0] = 1.0
        rhs = (w2 * np.abs(F) ** 2).sum() / f.size
    np.testing.assert_allclose(rhs, lhs, rtol=1e-13)


def test_wavevector_laplacian_symbol_on_a_sine():
    # -|xi|^2 is the symbol of the Laplacian: d^2/dx^2 of sin(2 pi m x / (N dx))
    shape, dx = (8, 12, 16), 0.37
    nz, ny, nx = shape
    xi = sp.wavevectors(shape, dx)
    xi2 = (xi ** 2).sum(-1)
    for axis, n, m in [(2, nx, 3), (1, ny, 5), (0, nz, 2)]:
        coord = np.arange(n) * dx
        k = 2 * np.pi * m / (n * dx)
        prof = np.sin(k * coord)
        sh = [1, 1, 1]; sh[axis] = n
        f = np.broadcast_to(prof.reshape(sh), shape)
        lap = sp.irfft3(-xi2 * sp.rfft3(f), shape)
        np.testing.assert_allclose(lap, -k * k * f, atol=1e-10 * k * k)
    # Nyquist index on the full axes is -N/2
    assert xi[nz // 2, 0, 0, 2] == pytest.approx(-np.pi / dx)
    assert xi[0, 0, nx // 2, 0] == pytest.approx(np.pi / dx)


def random_stiffness(seed):
    rng = np.random.default_rng(seed)
    R = np.linalg.qr(rng.standard_normal((3, 3)))[0]
    C = cr.voigt_to_tensor4(cr.hex_stiffness_voigt(*cr.MG_HEX_PA))
    return cr.rotate4(C, R)


def random_unit(rng):
    v = rng.standard_normal(3)
    return v / np.linalg.norm(v)


@pytest.mark.parametrize("seed", range(4))
def test_gamma_projection_identity(seed):
    C0 = random_stiffness(seed)
    rng = np.random.default_rng(10 + seed)
    n = random_unit(rng)
    G = sp.green_tensor4(C0, n)
    GCG = np.einsum("ijab,abcd,cdkl->ijkl", G, C0, G)
    np.testing.assert_allclose(GCG, G, atol=1e-12 * np.abs(G).max())
    # minor symmetries
    np.testing.assert_allclose(G, G.transpose(1, 0, 2, 3), atol=1e-25)
    np.testing.assert_allclose(G, G.transpose(0, 1, 3, 2), atol=1e-25)


def test_gamma_isotropic_closed_form():
    lam, mu = 40e9, 17e9
    d = np.eye(3)
    C0 = (lam * np.einsum("ij,kl->ijkl", d, d)
          + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))
    n = random_unit(np.random.default_rng(5))
    ref = (np.einsum("ik,j,l->ijkl", d, n, n) + np.einsum("il,j,k->ijkl", d, n, n)
           + np.einsum("jk,i,l->ijkl", d, n, n) + np.einsum("jl,i,k->ijkl", d, n, n)) / (4 * mu)
    ref -= (lam + mu) / (mu * (lam + 2 * mu)) * np.einsum("i,j,k,l->ijkl", n, n, n, n)
    np.testing.assert_allclose(sp.green_tensor4(C0, n), ref, atol=1e-12 * np.abs(ref).max())


def test_green_apply_equilibrium_and_full_form():
    rng = np.random.default_rng(7)
    C0 = random_stiffness(3)
    shape, dx = (4, 6, 8), 1e-7
    xi = sp.wavevectors(shape, dx)
    n, nz = sp.unit_wavevectors(xi)
    N = sp.acoustic_tensor_inverse(C0, n, nz)
    tau = rng.standard_normal(xi.shape[:-1] + (3, 3)) + 1j * rng.standard_normal(xi.shape[:-1] + (3, 3))
    tau = tau + np.swapaxes(tau, -1, -2)
    g = sp.green_apply(N, n, nz, tau)
    # eps = -Gamma:tau makes C0:eps + tau divergence free (sigma.xi = 0)
    sig = np.einsum("ijkl,...kl->...ij", C0, -g) + tau
    div = np.einsum("...ij,...j->...i", sig, xi)
    assert np.abs(div[nz]).max() < 1e-10 * np.abs(np.einsum("...ij,...j->...i", tau, xi)).max()
    assert np.all(g[~nz] == 0)
    # agrees with the 4th-order form
    idx = (1, 2, 3)
    G = sp.green_tensor4(C0, n[idx])
    np.testing.assert_allclose(g[idx], np.einsum("ijkl,kl->ij", G, tau[idx]), rtol=1e-12)


def test_ambiguous_nyquist_mask_small_grid():
    # 4 x 4 x 4: kz, ky in {0, 1, -2, -1}; kx in {0, 1, 2}. Ambiguous = some
    # component on Nyquist (|k| = 2) and another component in {1, -1}.
    mask = sp.ambiguous_nyquist_mask((4, 4, 4))
    k = np.array([0, 1, -2, -1])
    for iz in range(4):
        for iy in range(4):
            for ix in range(3):
                comps = [ix, k[iy], k[iz]]
                nyq = [abs(c) == 2 for c in comps]
                other = [c != 0 and abs(c) != 2 for c in comps]
                assert mask[iz, iy, ix] == (any(nyq) and any(other))
    # odd axes have no Nyquist index
    assert not sp.ambiguous_nyquist_mask((3, 5, 7)).any()


def test_green_operator_maps_real_fields_to_real_fields():
    # The discrete operator applied to the spectrum of a real stress must be
    # the spectrum of a real strain: a round trip through the real field
    # loses nothing (it would at the ambiguous Nyquist wavevectors with the
    # continuous operator).
    from oracle import mech
    C0 = random_stiffness(2)
    shape = (8, 6, 10)
    green = mech.GreenOperator(C0, shape, 1e-7)
    rng = np.random.default_rng(9)
    sig = rng.standard_normal(shape + (3, 3))
    sig = sig + np.swapaxes(sig, -1, -2)
    g = green.apply(mech.fft_tensor(sig))
    back = mech.fft_tensor(mech.ifft_tensor(g, shape))
    np.testing.assert_allclose(back, g, atol=1e-12 * np.abs(g).max())
    # at ambiguous wavevectors it is the reference compliance
    amb = sp.ambiguous_nyquist_mask(shape)
    S = np.linalg.inv(mech.strain_to_stress_voigt(C0))
    sh = mech.fft_tensor(sig)
    np.testing.assert_allclose(mech.tensor_to_voigt6(g[amb]), S @ mech.tensor_to_voigt6(sh[amb]), rtol=1e-12)
