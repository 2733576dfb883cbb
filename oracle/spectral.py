"""Fourier-space conventions and the Green's operator (oracle, test only).

Table 1 and Sec. 3 solve the linearised phase-field equation in Fourier space
on a periodic regular grid (Sec. 4.2). The paper states no
normalisation or wavevector convention; the readings used here:

* fields are stored [z][y][x]; the real-to-complex transform halves x, so a
  spectrum is [z][y][x/2+1];
* the forward transform is unnormalised and the inverse carries 1/N
  (NumPy's convention, used as a library primitive);
* xi = 2*pi*k/(N*dx) with k = 0..N/2-1, -N/2..-1 on the full axes (the
  Nyquist index takes k = -N/2) and k = 0..N/2 on the halved x axis;
* the Laplacian symbol is the continuous -|xi|^2, invariant under the sign
  taken at a Nyquist index;
* the continuous Green's operator is even in xi but not invariant when only
  some components change sign. On an even axis the Nyquist index is its own
  mirror image, so at a wavevector that has a Nyquist component together with
  a non-zero, non-Nyquist component the operator would differ from its value
  at the mirror coefficient and would not map real fields to real fields.
  At exactly those "ambiguous" wavevectors the operator is replaced by the
  reference compliance C0^{-1} (the stress of that mode vanishes at the fixed
  point, as in Moulinec & Suquet's treatment of the highest frequencies);
  everywhere else the continuous operator is used.

The Green's operator is the textbook one of Moulinec & Suquet (1998) and
Mura; the paper takes its elastic strain from the finite-element solution
(Sec. 2.2) and has none.
"""

import numpy as np
import scipy.fft


def rfft3(f, workers=None):
    """Forward real-to-complex 3D transform over the last three axes."""
    return scipy.fft.rfftn(f, axes=(-3, -2, -1), workers=workers)


def irfft3(F, shape, workers=None):
    """Inverse of rfft3 (carries the 1/N factor)."""
    return scipy.fft.irfftn(F, s=shape, axes=(-3, -2, -1), workers=workers)


def wavevectors(shape, dx):
    """xi[..., (x, y, z)] on the half spectrum, shape (nz, ny, nx//2+1, 3)."""
    nz, ny, nx = shape
    kz = np.fft.fftfreq(nz) * nz
    ky = np.fft.fftfreq(ny) * ny
    kx = np.arange(nx // 2 + 1, dtype=float)
    xz = 2.0 * np.pi * kz / (nz * dx)
    xy = 2.0 * np.pi * ky / (ny * dx)
    xx = 2.0 * np.pi * kx / (nx * dx)
    xi = np.empty((nz, ny, nx // 2 + 1, 3))
    xi[..., 0] = xx[None, None, :]
    xi[..., 1] = xy[None, :, None]
    xi[..., 2] = xz[:, None, None]
    return xi


def half_spectrum_weights(shape):
    """Multiplicity of each stored coefficient of a real field's half spectrum
    (1 on the kx = 0 and kx = nx/2 planes, 2 elsewhere) for Parseval sums."""
    nz, ny, nx = shape
    w = np.full(nx // 2 + 1, 2.0)
    w[0] = 1.0
    if nx % 2 == 0:
        w[-1] = 1.0
    return np.broadcast_to(w, (nz, ny, nx // 2 + 1))


def ambiguous_nyquist_mask(shape):
    """True where a wavevector has a component on the Nyquist index of an even
    axis and another component that is neither zero nor Nyquist."""
    nz, ny, nx = shape
    kz = np.fft.fftfreq(nz) * nz
    ky = np.fft.fftfreq(ny) * ny
    kx = np.arange(nx // 2 + 1, dtype=float)
    comps = []
    for k, n, sh in ((kx, nx, (1, 1, -1)), (ky, ny, (1, -1, 1)), (kz, nz, (-1, 1, 1))):
        nyq = (n % 2 == 0) & (np.abs(k) == n // 2)
        other = (k != 0) & ~nyq
        comps.append((np.broadcast_to(nyq.reshape(sh), (nz, ny, nx // 2 + 1)),
                      np.broadcast_to(other.reshape(sh), (nz, ny, nx // 2 + 1))))
    any_nyq = comps[0][0] | comps[1][0] | comps[2][0]
    any_other = comps[0][1] | comps[1][1] | comps[2][1]
    return any_nyq & any_other


def unit_wavevectors(xi):
    """n = xi/|xi| and a mask of xi != 0."""
    norm = np.linalg.norm(xi, axis=-1)
    nonzero = norm > 0
    n = np.zeros_like(xi)
    n[nonzero] = xi[nonzero] / norm[nonzero][:, None]
    return n, nonzero


def acoustic_tensor_inverse(C0, n, nonzero):
    """N = K^{-1} with K_ik = C0_ijkl n_j n_l, zero where xi = 0."""
    K = np.einsum("ijkl,...j,...l->...ik", C0, n, n)
    N = np.zeros_like(K)
    N[nonzero] = np.linalg.inv(K[nonzero])
    return N


def green_apply(N, n, nonzero, tau_hat):
    """Gamma0 : tau_hat, for a symmetric (..., 3, 3) complex tau_hat.

    Gamma0_ijkl = 1/4 (N_ik n_j n_l + N_jk n_i n_l + N_il n_j n_k + N_jl n_i n_k),
    which on a symmetric tau reduces to sym(n (x) N (tau n)). Zero at xi = 0.
    """
    t = np.einsum("...kl,...l->...k", tau_hat, n)
    u = np.einsum("...jk,...k->...j", N, t)
    out = 0.5 * (n[..., :, None] * u[..., None, :] + n[..., None, :] * u[..., :, None])
    out[~nonzero] = 0.0
    return out


def green_tensor4(C0, nvec):
    """Full 4th-order Gamma0 at one unit wavevector (used by the pins)."""
    K = np.einsum("ijkl,j,l->ik", C0, nvec, nvec)
    N = np.linalg.inv(K)
    G = 0.25 * (np.einsum("ik,j,l->ijkl", N, nvec, nvec)
                + np.einsum("jk,i,l->ijkl", N, nvec, nvec)
                + np.einsum("il,j,k->ijkl", N, nvec, nvec)
                + np.einsum("jl,i,k->ijkl", N, nvec, nvec))
    return G
