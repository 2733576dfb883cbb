"""Fourier neural operator (FNO) macro stepper and its acceptance residual
(oracle, test infrastructure only: imported by the tests, the smoke check and
the CPU baseline of the benchmark, never by the library path).

The learned stepper replaces S plain steps of the phase-field update by one
evaluation of an FNO (Li et al., Fourier neural operator, ICLR 2021):

    a(x)   = [f(x), c_1 .. c_7]            (order parameter + a constant
                                             conditioning vector: the six
                                             sample-frame eigenstrain
                                             components / gamma_tw and the
                                             applied strain / 5e-3)
    v_0    = P a + p
    v_l    = GELU(W_l v_{l-1} + b_l + K_l v_{l-1}),   l = 1..4
    K v    = irfftn( R(k) rfftn(v)(k) on the kept modes, 0 elsewhere )
    f~     = f + Q_2 GELU(Q_1 v_4 + q_1) + q_2

with kept modes kx in [0, m), ky and kz in [0, m) u [n - m, n) (ordered
positive then negative), R(k) a complex width x width matrix per kept mode,
and GELU(x) = x Phi(x) with the exact normal CDF.

The prediction is accepted when the backward-Euler residual of the macro
step of S plain steps (the Allen-Cahn equation integrated implicitly over
S dt),
    rho = max_x | f~ - f^n + S L dt dF/df (f~) |,
    dF/df = chem - 2 kappa lap f - mech (at the equilibrium of f~),
is below a tolerance (surrogate acceptance test; the reading is stated in the
design notes: the paper has no surrogate).
"""

import numpy as np
from scipy.special import erf

from . import spectral
from .mech import ms_solve, voigt6_to_tensor
from .phasefield import chemical_force, gradient_symbol, mechanical_force

N_COND = 7


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def kept_index(n, m):
    """Indices of the kept modes along a complex axis of length n."""
    return np.concatenate([np.arange(m), np.arange(n - m, n)])


def init_params(width=32, modes=12, hidden=128, n_layers=4, seed=0, scale_spec=None):
    """Random parameters (float64; R complex128 of shape
    (layers, width_out, width_in, 2m, 2m, m) indexed [l, o, i, kz', ky', kx])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cin = 1 + N_COND
    s_spec = scale_spec if scale_spec is not None else 1.0 / (width * width)
    p = {
        "P": rng.normal(0, 1 / np.sqrt(cin), (width, cin)),
        "p": rng.normal(0, 0.1, width),
        "W": rng.normal(0, 1 / np.sqrt(width), (n_layers, width, width)),
        "b": rng.normal(0, 0.1, (n_layers, width)),
        "R": s_spec * (rng.random((n_layers, width, width, 2 * modes, 2 * modes, modes)) +
                       1j * rng.random((n_layers, width, width, 2 * modes, 2 * modes, modes))),
        "Q1": rng.normal(0, 1 / np.sqrt(width), (hidden, width)),
        "q1": rng.normal(0, 0.1, hidden),
        "Q2": rng.normal(0, 1 / np.sqrt(hidden), (1, hidden)),
        "q2": rng.normal(0, 0.01, 1),
    }
    return p


def spectral_conv(v, R):
    """K v for v (C, nz, ny, nx) real and R (C_out, C_in, 2m, 2m, m)."""
    C, nz, ny, nx = v.shape
    m = R.shape[-1]
    V = np.fft.rfftn(v, axes=(1, 2, 3))
    iz, iy = kept_index(nz, m), kept_index(ny, m)
    sub = V[:, iz][:, :, iy][..., :m]                      # (C_in, 2m, 2m, m)
    out_sub = np.einsum("oizyx,izyx->ozyx", R, sub)
    out = np.zeros((R.shape[0], nz, ny, nx // 2 + 1), dtype=complex)
    out[np.ix_(np.arange(R.shape[0]), iz, iy, np.arange(m))] = out_sub
    return np.fft.irfftn(out, s=(nz, ny, nx), axes=(1, 2, 3))


def lift(params, eta, cond):
    """v_0 = P [f, c] + p for eta (nz, ny, nx) and cond (7,)."""
    P, p = params["P"], params["p"]
    const = P[:, 1:] @ np.asarray(cond, dtype=np.float64) + p
    return P[:, 0][:, None, None, None] * eta[None] + const[:, None, None, None]


def fourier_layer(params, l, v):
    W, b, R = params["W"][l], params["b"][l], params["R"][l]
    local = np.einsum("oi,izyx->ozyx", W, v) + b[:, None, None, None]
    return gelu(local + spectral_conv(v, R))


def project(params, v):
    h = gelu(np.einsum("hi,izyx->hzyx", params["Q1"], v) + params["q1"][:, None, None, None])
    return np.einsum("oh,hzyx->ozyx", params["Q2"], h)[0] + params["q2"][0]


def forward(params, eta, cond):
    """Predicted order parameter after one macro step, for eta (nz, ny, nx)."""
    eta = np.asarray(eta, dtype=np.float64)
    v = lift(params, eta, cond)
    for l in range(params["W"].shape[0]):
        v = fourier_layer(params, l, v)
    return eta + project(params, v)


def conditioning(eps0_sample6, eps_bar_xx, gamma_tw=0.129, strain_scale=5e-3):
    """The constant input channels: eps0 (tensor-Voigt, sample frame) / gamma_tw
    and the applied strain / strain_scale."""
    return np.concatenate([np.asarray(eps0_sample6, dtype=np.float64) / gamma_tw,
                           [float(eps_bar_xx) / strain_scale]])


def variational_derivative(prob, eta, load, eps_p6=None):
    """dF/df = chem - 2 kappa lap f - mech for eta (V, nz, ny, nx), with the
    equilibrium of eta solved from a uniform start (with gradient tensors
    K_a, -2 div(K_a grad f_a) in place of -2 kappa lap f_a)."""
    shape = prob.shape
    C_grain, C_var, eps0 = prob.tables
    eps_p = np.zeros(shape + (3, 3)) if eps_p6 is None else voigt6_to_tensor(eps_p6)
    ebar = voigt6_to_tensor(np.asarray(load["eps_bar"], dtype=np.float64))
    eps0_field = np.broadcast_to(ebar, shape + (3, 3)).copy()
    _, _, sigma, eps_el, _, _, _ = ms_solve(eps0_field, ebar, eta, eps_p, prob.gid, prob.tables, prob.green,
                                            load, prob.ms_tol, prob.ms_max_iter, prob.h_kind)
    chem = chemical_force(eta, prob.A)
    mech = mechanical_force(eta, sigma, eps_el, prob.gid, C_grain, C_var, eps0, prob.h_kind)
    kv = getattr(prob, "kappa_var", None)
    grad_force = np.stack([
        spectral.irfft3(2.0 * gradient_symbol(shape, prob.dx, prob.kappa, None if kv is None else kv[a]) *
                        spectral.rfft3(eta[a]), shape)
        for a in range(eta.shape[0])])
    return chem + grad_force - mech


def macro_residual(prob, eta_prev, eta_pred, n_steps, load, eps_p6=None):
    """Field and max-norm of f~ - f^n + S L dt dF/df(f~) over V variants."""
    g = variational_derivative(prob, np.asarray(eta_pred, dtype=np.float64), load, eps_p6)
    r = np.asarray(eta_pred, dtype=np.float64) - np.asarray(eta_prev, dtype=np.float64) + \
        n_steps * prob.L * prob.dt * g
    return r, float(np.abs(r).max())
