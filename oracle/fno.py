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

The prediction is accepted when the residual of the macro step of S plain
steps is below a tolerance (surrogate acceptance test; the paper has no
surrogate, so this is a reading). The plain step (Sec. 3, eqs. (19)-(20))
takes the local force E = chem - mech at the old state and the gradient force
G f = -2 kappa lap f at the new one; summed over S steps it gives exactly
    f^{n+S} - f^n + L dt [ sum_{s=0}^{S-1} E(f^{n+s}) + G sum_{s=1}^{S} f^{n+s} ] = 0.
Both sums are replaced by the trapezoid rule with the end correction of a
left (right) Riemann sum, exact when the summand is linear in s:
    sum_{s=0}^{S-1} x_s ~ (S+1)/2 x_0 + (S-1)/2 x_S,
    sum_{s=1}^{S}   x_s ~ (S-1)/2 x_0 + (S+1)/2 x_S,
so with dF/df = E + G f (mech at the equilibrium of each state)
    r   = f~ - f^n + L dt [ (S+1)/2 dF/df(f^n) + (S-1)/2 dF/df(f~) + G (f~ - f^n) ],
    rho = max_x |r|.
For S = 1 it is the plain step itself (zero on an exact step); on an exact
trajectory of S steps it is the quadrature defect, second order in the step
count times dt, where the backward-Euler residual f~ - f^n + S L dt dF/df(f~)
is first order.
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


def gelu_grad(x):
    """d GELU / dx = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def spectral_conv_adjoint(dy, R, v):
    """Gradients through K v = irfftn(embed(R sub(rfftn(v)))) for the output
    gradient dy (C_out, nz, ny, nx): returns (dv, dR) with dR holding
    dL/dRe R + i dL/dIm R. Written out from the real-pair derivatives of the
    transforms: an output mode's gradient is c(kx)/N rfftn(dy) (c = 1 on the
    kx = 0 plane, 2 elsewhere among the kept kx), dR = that times conj of the
    input's kept modes, and dv is the same convolution with R^H."""
    C, nz, ny, nx = v.shape
    m = R.shape[-1]
    ntot = nz * ny * nx
    iz, iy = kept_index(nz, m), kept_index(ny, m)
    cx = np.where(np.arange(m) == 0, 1.0, 2.0)
    G = np.fft.rfftn(dy, axes=(1, 2, 3))[:, iz][:, :, iy][..., :m] * (cx / ntot)   # (C_out, 2m, 2m, m)
    S = np.fft.rfftn(v, axes=(1, 2, 3))[:, iz][:, :, iy][..., :m]                  # (C_in, 2m, 2m, m)
    dR = G[:, None] * np.conj(S)[None, :]
    GS = np.einsum("oizyx,ozyx->izyx", np.conj(R), G)
    emb = np.zeros((C, nz, ny, nx // 2 + 1), dtype=complex)
    emb[np.ix_(np.arange(C), iz, iy, np.arange(m))] = GS
    # dv(x) = sum over kept modes Re[GS e^{+i theta}] = N irfftn(GS / c)
    dv = np.fft.irfftn(emb / np.concatenate([cx, np.full(nx // 2 + 1 - m, 1.0)]), s=(nz, ny, nx),
                       axes=(1, 2, 3)) * ntot
    return dv, dR


def backward(params, eta, cond, g_out):
    """Gradients of L = sum_x g_out(x) f~(x) with respect to every parameter,
    by the chain rule through the forward pass above (hand-written, FP64).
    Returns a dict shaped like params; R's entry is dL/dRe R + i dL/dIm R."""
    eta = np.asarray(eta, dtype=np.float64)
    g_out = np.asarray(g_out, dtype=np.float64)
    n_layers = params["W"].shape[0]
    vs = [lift(params, eta, cond)]
    us = []
    for l in range(n_layers):
        W, b, R = params["W"][l], params["b"][l], params["R"][l]
        u = np.einsum("oi,izyx->ozyx", W, vs[-1]) + b[:, None, None, None] + spectral_conv(vs[-1], R)
        us.append(u)
        vs.append(gelu(u))
    zh = np.einsum("hi,izyx->hzyx", params["Q1"], vs[-1]) + params["q1"][:, None, None, None]
    h = gelu(zh)
    gr = {}
    gr["q2"] = np.array([g_out.sum()])
    gr["Q2"] = np.einsum("zyx,hzyx->h", g_out, h)[None, :]
    dzh = params["Q2"][0][:, None, None, None] * g_out[None] * gelu_grad(zh)
    gr["Q1"] = np.einsum("hzyx,izyx->hi", dzh, vs[-1])
    gr["q1"] = dzh.sum(axis=(1, 2, 3))
    dv = np.einsum("hi,hzyx->izyx", params["Q1"], dzh)
    gW, gb, gR = [], [], []
    for l in reversed(range(n_layers)):
        du = dv * gelu_grad(us[l])
        gW.append(np.einsum("ozyx,izyx->oi", du, vs[l]))
        gb.append(du.sum(axis=(1, 2, 3)))
        dv_spec, dR = spectral_conv_adjoint(du, params["R"][l], vs[l])
        gR.append(dR)
        dv = np.einsum("oi,ozyx->izyx", params["W"][l], du) + dv_spec
    gr["W"] = np.stack(gW[::-1])
    gr["b"] = np.stack(gb[::-1])
    gr["R"] = np.stack(gR[::-1])
    c = np.asarray(cond, dtype=np.float64)
    dsum = dv.sum(axis=(1, 2, 3))
    gr["P"] = np.concatenate([np.einsum("czyx,zyx->c", dv, eta)[:, None], dsum[:, None] * c[None, :]], axis=1)
    gr["p"] = dsum
    return gr


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
    return chem + gradient_force(prob, eta) - mech


def gradient_force(prob, eta):
    """G f = -2 div(K grad f) per variant (-2 kappa lap f when isotropic),
    through the spectral symbol of the plain step."""
    kv = getattr(prob, "kappa_var", None)
    return np.stack([
        spectral.irfft3(2.0 * gradient_symbol(prob.shape, prob.dx, prob.kappa, None if kv is None else kv[a]) *
                        spectral.rfft3(eta[a]), prob.shape)
        for a in range(eta.shape[0])])


def macro_residual(prob, eta_prev, eta_pred, n_steps, load, eps_p6=None):
    """Field and max-norm of the macro-step residual
    f~ - f^n + L dt [ (S+1)/2 dF/df(f^n) + (S-1)/2 dF/df(f~) + G (f~ - f^n) ]
    over V variants (S = n_steps; the module docstring derives it)."""
    f0 = np.asarray(eta_prev, dtype=np.float64)
    f1 = np.asarray(eta_pred, dtype=np.float64)
    S = float(n_steps)
    g0 = variational_derivative(prob, f0, load, eps_p6)
    g1 = variational_derivative(prob, f1, load, eps_p6)
    r = f1 - f0 + prob.L * prob.dt * (0.5 * (S + 1.0) * g0 + 0.5 * (S - 1.0) * g1 +
                                      gradient_force(prob, f1 - f0))
    return r, float(np.abs(r).max())
