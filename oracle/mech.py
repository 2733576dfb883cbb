"""Micro-elastic equilibrium for the phase-field step (oracle, test only).

Small-strain analogue of the second Piola-Kirchhoff stress of eq. (4):
sigma = C(x) : (eps - eps*), with the mixture stiffness of eq. (5),
C(x) = C_g + sum_a h(f_a) (C_twin^a - C_g) (using f_M = 1 - sum_a f_a), and the
eigenstrain eps* = eps_p + sum_a h(f_a) eps0_a. eps_p is the plastic strain
the crystal-plasticity side hands over (a given input here).

Readings (the paper takes its strain from the finite-element solution and is
silent on all of this):
* h(f) = f (linear) by default, as eq. (5) mixes stiffness linearly in f and
  eq. (6) accumulates the twin eigenstrain linearly in f; the quintic
  h = f^3 (6 f^2 - 15 f + 10) is available as an option.
* Equilibrium is the Moulinec-Suquet basic fixed point
  eps^{k+1}(xi) = eps^k(xi) - Gamma0(xi) : sigma^k(xi) for xi != 0.
* Mixed boundary condition: strain-controlled mean components are set from
  the load; stress-controlled ones are corrected each iteration by
  dE_S = -(M0_SS)^{-1} (<sigma>_S - sigma_bar_S), M0 = the map from
  tensor-Voigt strain to Voigt stress of the reference medium.
* Convergence: ||eps^{k+1} - eps^k|| <= tol ||eps^{k+1}|| (Frobenius norm over
  all voxels, full tensors).
"""

import numpy as np

from . import spectral
from .crystal import VOIGT_PAIRS


# ---------------------------------------------------------------- helpers
def voigt6_to_tensor(f6):
    """(6, ...) tensor-Voigt component-major field -> (..., 3, 3)."""
    f6 = np.asarray(f6)
    out = np.empty(f6.shape[1:] + (3, 3), dtype=np.result_type(f6.dtype, np.float64))
    for I, (i, j) in enumerate(VOIGT_PAIRS):
        out[..., i, j] = f6[I]
        out[..., j, i] = f6[I]
    return out


def tensor_to_voigt6(t):
    """(..., 3, 3) -> (6, ...) tensor-Voigt (the symmetric part is assumed)."""
    return np.stack([t[..., i, j] for (i, j) in VOIGT_PAIRS])


def contract(C, e):
    """(C : e)_ij = C_ijkl e_kl for a field e of shape (..., 3, 3)."""
    return np.tensordot(e, C, axes=([-2, -1], [2, 3]))


def h_interp(f, kind="linear"):
    if kind == "linear":
        return f
    if kind == "quintic":
        return f ** 3 * (6.0 * f * f - 15.0 * f + 10.0)
    raise ValueError(kind)


def dh_interp(f, kind="linear"):
    if kind == "linear":
        return np.ones_like(f)
    if kind == "quintic":
        return 30.0 * f * f * (f - 1.0) ** 2
    raise ValueError(kind)


def strain_to_stress_voigt(C):
    """M[I, J] = (C : E_J)_I: tensor-Voigt strain -> Voigt stress."""
    M = np.empty((6, 6))
    for J, (k, l) in enumerate(VOIGT_PAIRS):
        E = np.zeros((3, 3))
        E[k, l] = E[l, k] = 1.0
        S = np.einsum("ijkl,kl->ij", C, E)
        for I, (i, j) in enumerate(VOIGT_PAIRS):
            M[I, J] = S[i, j]
    return M


def fft_tensor(t):
    """rfft over the three grid axes of a (nz, ny, nx, 3, 3) field."""
    comp_major = np.ascontiguousarray(np.moveaxis(t, (-2, -1), (0, 1)))
    F = spectral.rfft3(comp_major, workers=-1)
    return np.moveaxis(F, (0, 1), (-2, -1))


def ifft_tensor(T, grid_shape):
    comp_major = np.ascontiguousarray(np.moveaxis(T, (-2, -1), (0, 1)))
    f = spectral.irfft3(comp_major, grid_shape, workers=-1)
    return np.moveaxis(f, (0, 1), (-2, -1))


# ------------------------------------------------------- constitutive law
def eigenstrain_and_stress(eps, eta, eps_p, gid, C_grain, C_var, eps0, h_kind="linear"):
    """eps*, eps_el = eps - eps* and sigma = C(x) : eps_el.

    eps, eps_p: (nz, ny, nx, 3, 3); eta: (V, nz, ny, nx); gid: (nz, ny, nx)
    ints or None for a single grain; C_grain (G,3,3,3,3); C_var (G,V,3,3,3,3)
    twin stiffness; eps0 (G,V,3,3).
    """
    h = h_interp(eta, h_kind)
    if gid is None:
        return _grain_stress(eps, h, eps_p, C_grain[0], C_var[0], eps0[0])
    eps_star = np.empty_like(eps)
    sigma = np.empty_like(eps)
    eps_el = np.empty_like(eps)
    for g in np.unique(gid):
        mask = gid == g
        es, el, s = _grain_stress(eps[mask], h[:, mask], eps_p[mask], C_grain[g], C_var[g], eps0[g])
        eps_star[mask], eps_el[mask], sigma[mask] = es, el, s
    return eps_star, eps_el, sigma


def _grain_stress(eps, h, eps_p, Cg, Cv, e0):
    """One grain: eps* = eps_p + sum_a h_a eps0_a; sigma = (Cg + sum_a h_a (Cv_a - Cg)) : eps_el."""
    eps_star = np.array(eps_p, dtype=np.float64, copy=True)
    for a in range(h.shape[0]):
        eps_star += h[a][..., None, None] * e0[a]
    eps_el = eps - eps_star
    sigma = contract(Cg, eps_el)
    for a in range(h.shape[0]):
        sigma += h[a][..., None, None] * contract(Cv[a] - Cg, eps_el)
    return eps_star, eps_el, sigma


# ------------------------------------------------------ Moulinec-Suquet
class GreenOperator:
    """Precomputed N(xi) = K(n)^{-1} of a reference medium on one grid, with
    the reference compliance at the ambiguous Nyquist wavevectors."""

    def __init__(self, C0, shape, dx):
        self.C0 = C0
        self.shape = tuple(shape)
        xi = spectral.wavevectors(shape, dx)
        self.n, self.nonzero = spectral.unit_wavevectors(xi)
        self.N = spectral.acoustic_tensor_inverse(C0, self.n, self.nonzero)
        self.ambiguous = spectral.ambiguous_nyquist_mask(self.shape)
        self.compliance = np.linalg.inv(strain_to_stress_voigt(C0))

    def apply(self, tau_hat):
        out = spectral.green_apply(self.N, self.n, self.nonzero, tau_hat)
        amb = tau_hat[self.ambiguous]                       # (m, 3, 3)
        out[self.ambiguous] = voigt6_to_tensor(self.compliance @ tensor_to_voigt6(amb))
        return out


def mean_update(ebar, sbar, target_eps, target_sig, stress_mask, M0):
    """New mean strain (3x3) from the mixed boundary condition."""
    e6 = tensor_to_voigt6(ebar)
    s6 = tensor_to_voigt6(sbar)
    S = [i for i in range(6) if stress_mask[i]]
    E = [i for i in range(6) if not stress_mask[i]]
    new = e6.copy()
    new[E] = np.asarray(target_eps)[E]
    if S:
        rhs = s6[S] - np.asarray(target_sig)[S]
        new[S] = e6[S] - np.linalg.solve(M0[np.ix_(S, S)], rhs)
    return voigt6_to_tensor(new)


def ms_solve(eps_start, ebar_start, eta, eps_p, gid, tables, green, load,
             tol, max_iter, h_kind="linear"):
    """Moulinec-Suquet fixed point with a mixed boundary condition.

    eps_start: warm-start strain field (nz,ny,nx,3,3) whose mean is ebar_start.
    load: dict with 'eps_bar' (6), 'sig_bar' (6), 'stress_mask' (6 bools).
    Returns (eps, ebar, sigma, eps_el, eps_star, iters, residual).
    """
    C_grain, C_var, eps0 = tables
    M0 = strain_to_stress_voigt(green.C0)
    mask = load["stress_mask"]
    # Initial guess: the warm start shifted so its strain-controlled mean
    # components already hold this step's target.
    e6 = tensor_to_voigt6(ebar_start)
    for i in range(6):
        if not mask[i]:
            e6[i] = load["eps_bar"][i]
    ebar = voigt6_to_tensor(e6)
    eps = eps_start + (ebar - ebar_start)
    residual = np.inf
    it = 0
    for it in range(1, max_iter + 1):
        _, _, sigma = eigenstrain_and_stress(eps, eta, eps_p, gid, C_grain, C_var, eps0, h_kind)
        sbar = sigma.mean(axis=(0, 1, 2))
        ebar_new = mean_update(ebar, sbar, load["eps_bar"], load["sig_bar"], mask, M0)
        deps = -ifft_tensor(green.apply(fft_tensor(sigma)), green.shape)
        eps_new = eps + deps + (ebar_new - ebar)
        change, size = np.linalg.norm(eps_new - eps), np.linalg.norm(eps_new)
        residual = change / size if size > 0 else (0.0 if change == 0 else np.inf)
        eps, ebar = eps_new, ebar_new
        if residual <= tol:
            break
    eps_star, eps_el, sigma = eigenstrain_and_stress(eps, eta, eps_p, gid, C_grain, C_var, eps0, h_kind)
    return eps, ebar, sigma, eps_el, eps_star, it, residual
