"""Phase-field twin evolution and energies (oracle, test only).

Free energy, eq. (12): G = G_dw + G_gd + G_me, with
* the multiphase double well of eq. (13), c1 sum_{a<b} f_a^2 f_b^2 over the
  N_tw twin variants and the matrix (f_M = 1 - sum_a f_a, eq. (18));
* the gradient energy of eq. (14); with eq. (18) its two gradient sums in the
  rate equation collapse to c2 * laplacian(f_a);
* the stored elastic energy of eq. (15), 1/2 eps_el : C(x) : eps_el.

Evolution: eq. (16)/(17), linearised per eqs. (19)-(20) with the Laplacian
implicit and the rest explicit, solved in Fourier space (Table 1).

Readings (stated once here, used below):
* Symbols: A = c1, kappa = c2, and the mobility maps as c3 -> 2L on the
  chemical and gradient terms and c3 -> L on the mechanical ones, so that a
  single variant follows d(eta)/dt = -L dF/d(eta) for
  F = int [A eta^2 (1-eta)^2 + kappa |grad eta|^2 + 1/2 eps_el:C:eps_el].
* Chemical force: chem_a = 2A f_a sum_{b != a} f_b (f_b - f_a), b running
  over the other variants and the matrix; for one variant this is
  2A eta (1-eta)(1-2eta).
* Mechanical force: mech_a = h'(f_a) [sigma : eps0_a
  - 1/2 eps_el : (C_twin^a - C_g) : eps_el]; eq. (17) prints C_twin^a, the
  derivative of eq. (5) gives the difference (C_twin^a - C_matrix).
* One solve per step by default: with f_M = 1 - sum f the implicit
  coefficient of the converged equation is constant, and the step takes the
  nonlinear force at f^n (the fixed point i of Table 1 is the option below);
  eq. (18) holds by construction, so the loop j is empty.
* Mechanics solved at f^n (the paper also holds the strain fixed during the
  phase-field solve, Sec. 2.2).
* No clipping of f.
* Gradient energy reported as kappa sum_a |grad f_a|^2 through Parseval with
  the -|xi|^2 Laplacian symbol (equal to eq. (14) for one variant).
* Anisotropic gradient energy (Table 5 lists c2 along the twin-plane normal
  and along the shear direction): optionally each variant carries a
  symmetric tensor K_a (sample frame, J/m) and the gradient term becomes
  grad f_a . K_a . grad f_a, so its force is -2 div(K_a grad f_a) and its
  Fourier symbol xi . K_a . xi replaces kappa |xi|^2. K_a = kappa I is the
  isotropic case. With one grain K_a is constant and the implicit step is
  exact in Fourier space.
* Anisotropic gradient energy on a polycrystal: K_a(x) = K_a^g of the voxel's
  grain g (each grain's tensors turned by its rotation). The spectral
  implicit step needs a constant coefficient, so the gradient force is split
  as G = Gbar + (G - Gbar): Gbar f = -2 kbar_a lap f implicit, with kbar_a the
  largest eigenvalue of K_a^g over the grains, and the remainder
  -2 div((K_a(x) - kbar_a I) grad f) explicit at f^n, through spectral first
  derivatives (zero at a Nyquist index). Since kbar_a I - K_a(x) is positive
  semidefinite the amplification of a mode in a region of constant K,
  (1 + 2 L dt (kbar |xi|^2 - xi.K.xi)) / (1 + 2 L dt kbar |xi|^2), lies in
  (0, 1] at any dt. The gradient energy is reported for the same operator:
  the Parseval sum of kbar_a |xi|^2 plus int grad f . (K - kbar I) . grad f.
* Variable mobility (Sec. 4: a pad layer of very low mobility around the
  specimen suppresses the flux into it, a Neumann-like condition): optionally
  a relative mobility m(x) in [0, 1] with L(x) = L m(x). The gradient term is
  split with a constant implicit mobility L (the largest):
  (f^{n+1} - f^n)/dt = L G(f^{n+1}) + L (m - 1) G(f^n) - L m (chem - mech)(f^n),
  G(f) = 2 div(K grad f); for a constant m the amplification of a mode,
  (1 + 2 L dt (1 - m) q) / (1 + 2 L dt q), lies in [0, 1] for every m in
  [0, 1]. m = 1 is the plain step, m = 0 leaves f unchanged.
* The paper's iterated scheme (Table 1 with eqs. (19)-(20)): the fixed point
  i solves f^i/dt - c3 c2 [sum_{b != a} f_b^{i-1}] lap f^i + r^i = 0 with the
  nonlinear terms of r at f^{i-1} and the mechanical ones held at f^n (the
  elastic strain is constant during the phase-field solve, Sec. 2.3). With
  f_M = 1 - sum f the coefficient is 2 L kappa (1 - f_a^{i-1}); splitting it
  as the constant 2 L kappa implicit plus the rest explicit, the explicit
  rest cancels the cross-gradient term of r exactly, so an iterate is
  f^i = [f^n - L dt (chem(f^{i-1}) - mech(f^n))] / (1 + 2 L dt q): the plain
  step re-evaluated with the latest chemical force (a Picard iteration
  converging to backward Euler). The guess f^0 is f^n, so the first iterate
  is the plain step, and the change max |f^i - f^{i-1}| is tested after every
  solve, the first included. All variants are iterated together (Jacobi);
  a per-variant sweep has the same fixed point. The conservation loop j
  holds by construction; the subdomains k are a memory device of the
  paper's CPU code and are one domain here.
"""

import numpy as np

from . import spectral
from .mech import (GreenOperator, contract, dh_interp, h_interp, ms_solve,
                   tensor_to_voigt6, voigt6_to_tensor)


def chemical_force(eta, A):
    """chem_a = 2A f_a sum_{b != a} f_b (f_b - f_a), b over variants + matrix."""
    V = eta.shape[0]
    f_m = 1.0 - eta.sum(axis=0)
    chem = np.empty_like(eta)
    for a in range(V):
        s = f_m * (f_m - eta[a])
        for b in range(V):
            if b != a:
                s = s + eta[b] * (eta[b] - eta[a])
        chem[a] = 2.0 * A * eta[a] * s
    return chem


def mechanical_force(eta, sigma, eps_el, gid, C_grain, C_var, eps0, h_kind="linear"):
    """mech_a = h'(f_a) [sigma : eps0_a - 1/2 eps_el : dC_a : eps_el]."""
    dh = dh_interp(eta, h_kind)
    if gid is None:
        return _grain_mech(dh, sigma, eps_el, C_grain[0], C_var[0], eps0[0])
    mech = np.empty_like(eta)
    for g in np.unique(gid):
        mask = gid == g
        mech[:, mask] = _grain_mech(dh[:, mask], sigma[mask], eps_el[mask], C_grain[g], C_var[g], eps0[g])
    return mech


def _grain_mech(dh, sigma, eps_el, Cg, Cv, e0):
    mech = np.empty_like(dh)
    for a in range(dh.shape[0]):
        work = np.einsum("...ij,ij->...", sigma, e0[a])
        stiff = 0.5 * np.einsum("...ij,...ij->...", eps_el, contract(Cv[a] - Cg, eps_el))
        mech[a] = dh[a] * (work - stiff)
    return mech


def double_well_density(eta, A):
    """A sum_{a<b} f_a^2 f_b^2 over the variants and the matrix."""
    phases = list(eta) + [1.0 - eta.sum(axis=0)]
    g = np.zeros_like(eta[0])
    for a in range(len(phases)):
        for b in range(a + 1, len(phases)):
            g = g + phases[a] ** 2 * phases[b] ** 2
    return A * g


def gradient_symbol(shape, dx, kappa, K=None):
    """Fourier symbol of the gradient energy density on the half spectrum:
    kappa |xi|^2, or xi . K . xi for a tensor K (3, 3) indexed (x, y, z).

    Reading: the cross terms K_ij xi_i xi_j (i != j) are odd in xi_i, and on an
    even axis the Nyquist index stands for both +N/2 and -N/2; a component at
    its Nyquist index therefore enters the diagonal term K_ii xi_i^2 only (the
    mean over the two signs), which keeps the symbol even and the step real."""
    xi = spectral.wavevectors(shape, dx)
    if K is None:
        return kappa * (xi ** 2).sum(axis=-1)
    K = np.asarray(K, dtype=np.float64)
    nz, ny, nx = shape
    xc = xi.copy()
    if nx % 2 == 0:
        xc[:, :, nx // 2, 0] = 0.0
    if ny % 2 == 0:
        xc[:, ny // 2, :, 1] = 0.0
    if nz % 2 == 0:
        xc[nz // 2, :, :, 2] = 0.0
    diag = sum(K[i, i] * xi[..., i] ** 2 for i in range(3))
    cross = sum(K[i, j] * xc[..., i] * xc[..., j] for i in range(3) for j in range(3) if i != j)
    return diag + cross


def gradient_energy(eta, kappa, dx, kappa_var=None, grains=None):
    """sum_a int grad f_a . K_a . grad f_a dV (K_a = kappa I unless kappa_var
    gives the (V, 3, 3) tensors) by Parseval. grains = (kbar, rem, gid): per
    grain tensors split as in grain_split; the energy is then the Parseval
    sum of kbar_a |xi|^2 plus the remainder's int grad f . (K - kbar I) . grad f
    with spectral first derivatives (the operator the step uses)."""
    shape = eta.shape[1:]
    w = spectral.half_spectrum_weights(shape)
    ntot = np.prod(shape)
    dV = dx ** 3
    total = 0.0
    for a in range(eta.shape[0]):
        if grains is not None:
            q = gradient_symbol(shape, dx, grains[0][a])
        else:
            q = gradient_symbol(shape, dx, kappa, None if kappa_var is None else kappa_var[a])
        F = spectral.rfft3(eta[a], workers=-1)
        total += (w * q * np.abs(F) ** 2).sum() * dV / ntot
        if grains is not None:
            g = spectral_gradient(eta[a], dx)
            total += np.einsum("izyx,zyxij,jzyx->", g, grains[1][:, a][grains[2]], g) * dV
    return total


def derivative_wavevectors(shape, dx):
    """xi[..., (x, y, z)] for first derivatives on the half spectrum: a
    component at the Nyquist index of its (even) axis is zero, since the
    derivative is odd in it and that index stands for both signs."""
    xi = spectral.wavevectors(shape, dx).copy()
    nz, ny, nx = shape
    if nx % 2 == 0:
        xi[:, :, nx // 2, 0] = 0.0
    if ny % 2 == 0:
        xi[:, ny // 2, :, 1] = 0.0
    if nz % 2 == 0:
        xi[nz // 2, :, :, 2] = 0.0
    return xi


def spectral_gradient(f, dx):
    """grad f as (3, nz, ny, nx) [(x, y, z) components] by spectral first
    derivatives."""
    shape = f.shape
    F = spectral.rfft3(f, workers=-1)
    xi = derivative_wavevectors(shape, dx)
    return np.stack([spectral.irfft3(1j * xi[..., j] * F, shape, workers=-1) for j in range(3)])


def spectral_divergence(q, dx):
    """div q of a (3, nz, ny, nx) field by spectral first derivatives."""
    shape = q.shape[1:]
    xi = derivative_wavevectors(shape, dx)
    D = sum(1j * xi[..., j] * spectral.rfft3(q[j], workers=-1) for j in range(3))
    return spectral.irfft3(D, shape, workers=-1)


def remainder_divergence(f, K_field, dx):
    """2 div(K(x) grad f) for a field of symmetric tensors K_field
    (nz, ny, nx, 3, 3), through spectral first derivatives."""
    g = spectral_gradient(f, dx)
    flux = np.einsum("zyxij,jzyx->izyx", K_field, g)
    return 2.0 * spectral_divergence(flux, dx)


def grain_split(kappa_grain):
    """Constant-coefficient split of per-grain gradient tensors K_a^g
    (G, V, 3, 3): the implicit part kbar_a I with kbar_a the largest
    eigenvalue of K_a^g over the grains (then kbar_a I - K_a^g is positive
    semidefinite everywhere, which keeps the step stable at any dt), and the
    explicit remainder K_a^g - kbar_a I. Returns (kbar (V,), rem (G, V, 3, 3))."""
    K = np.asarray(kappa_grain, dtype=np.float64)
    kbar = np.linalg.eigvalsh(K).max(axis=(0, 2))
    rem = K - kbar[None, :, None, None] * np.eye(3)
    return kbar, rem


def grain_remainder_divergence(f_a, rem_a, gid, dx):
    """2 div((K_a(x) - kbar_a I) grad f_a) with K_a(x) the tensor of the
    voxel's grain (rem_a: (G, 3, 3))."""
    return remainder_divergence(f_a, rem_a[gid], dx)


def gradient_force(f, q, shape):
    """G(f) = 2 div(K grad f) of one field through its symbol q: -2 q f_hat."""
    return spectral.irfft3(-2.0 * q * spectral.rfft3(f, workers=-1), shape, workers=-1)


def allen_cahn_update(eta, chem, mech, L, dt, kappa, dx, kappa_var=None, mobility=None, grains=None):
    """f_a^{n+1} = IFFT[ FFT(f_a^n - L dt (chem_a - mech_a)) / (1 + 2 L dt q_a(xi)) ]
    with q_a the gradient symbol (kappa |xi|^2, or xi . K_a . xi); with a
    relative mobility m the right-hand side is f_a^n - L dt m (chem_a - mech_a)
    + L dt (m - 1) G(f_a^n). With per-grain tensors (grains = (kbar, rem,
    gid), see grain_split) q_a = kbar_a |xi|^2 and the right-hand side gains
    the explicit remainder L dt 2 div((K_a(x) - kbar_a I) grad f_a^n)."""
    shape = eta.shape[1:]
    out = np.empty_like(eta)
    for a in range(eta.shape[0]):
        if grains is not None:
            q = gradient_symbol(shape, dx, grains[0][a])
        else:
            q = gradient_symbol(shape, dx, kappa, None if kappa_var is None else kappa_var[a])
        denom = 1.0 + 2.0 * L * dt * q
        if grains is not None:
            rhs = eta[a] - L * dt * (chem[a] - mech[a]) + \
                L * dt * grain_remainder_divergence(eta[a], grains[1][:, a], grains[2], dx)
        elif mobility is None:
            rhs = eta[a] - L * dt * (chem[a] - mech[a])
        else:
            rhs = eta[a] - L * dt * mobility * (chem[a] - mech[a]) + \
                L * dt * (mobility - 1.0) * gradient_force(eta[a], q, shape)
        out[a] = spectral.irfft3(spectral.rfft3(rhs, workers=-1) / denom, shape, workers=-1)
    return out


def picard_iterate(eta0, prev, mech, prob, mobility=None):
    """One iterate of the paper's fixed point: the update from f^n (eta0)
    with the chemical force of the previous iterate (see the module notes).
    With a mobility field the explicit gradient remainder is the one of the
    previous iterate."""
    shape = eta0.shape[1:]
    chem = chemical_force(prev, prob.A)
    out = np.empty_like(eta0)
    for a in range(eta0.shape[0]):
        q = gradient_symbol(shape, prob.dx, prob.kappa, None if prob.kappa_var is None else prob.kappa_var[a])
        denom = 1.0 + 2.0 * prob.L * prob.dt * q
        if mobility is None:
            rhs = eta0[a] - prob.L * prob.dt * (chem[a] - mech[a])
        else:
            rhs = eta0[a] - prob.L * prob.dt * mobility * (chem[a] - mech[a]) + \
                prob.L * prob.dt * (mobility - 1.0) * gradient_force(prev[a], q, shape)
        out[a] = spectral.irfft3(spectral.rfft3(rhs, workers=-1) / denom, shape, workers=-1)
    return out


class Problem:
    """Everything fixed over a run (the analogue of the library's problem).

    tables = (C_grain, C_var, eps0) as returned by crystal.mg_tables.
    C0: reference stiffness (3,3,3,3) for the fixed point.
    kappa_var: optional (V, 3, 3) gradient tensors (one grain only).
    kappa_grain: optional (G, V, 3, 3) gradient tensors per grain (with gid):
    the step takes kbar_a I implicitly and the rest explicitly (grain_split);
    not with kappa_var, a mobility field or the fixed point over the update.
    mobility: optional (nz, ny, nx) relative mobility in [0, 1].
    pf_tol, pf_max_iter: the paper's fixed point i over the phase-field update
    (pf_max_iter = 1: the plain semi-implicit step).
    """

    def __init__(self, shape, dx, tables, A, kappa, L, dt, C0, gid=None,
                 h_kind="linear", ms_tol=1e-12, ms_max_iter=200, kappa_var=None, mobility=None,
                 pf_tol=1e-12, pf_max_iter=1, kappa_grain=None):
        self.shape = tuple(shape)
        self.dx = float(dx)
        self.tables = tables
        self.A, self.kappa, self.L, self.dt = float(A), float(kappa), float(L), float(dt)
        if kappa_var is not None:
            if gid is not None and len(np.unique(gid)) > 1:
                raise ValueError("an anisotropic gradient energy needs one grain")
            kappa_var = np.asarray(kappa_var, dtype=np.float64)
        self.kappa_var = kappa_var
        if mobility is not None:
            mobility = np.asarray(mobility, dtype=np.float64)
            if mobility.shape != self.shape or mobility.min() < 0 or mobility.max() > 1:
                raise ValueError("mobility must be (nz, ny, nx) with values in [0, 1]")
        self.mobility = mobility
        self.pf_tol, self.pf_max_iter = float(pf_tol), int(pf_max_iter)
        self.gid = None if gid is None else np.asarray(gid, dtype=np.int64)
        self.grains = None
        if kappa_grain is not None:
            if kappa_var is not None or mobility is not None or self.pf_max_iter > 1:
                raise ValueError("per-grain gradient tensors go without kappa_var, mobility and the update's "
                                 "fixed point")
            kg = np.asarray(kappa_grain, dtype=np.float64)
            gidf = np.zeros(self.shape, dtype=np.int64) if self.gid is None else self.gid
            if kg.ndim != 4 or kg.shape[2:] != (3, 3) or gidf.max() >= kg.shape[0]:
                raise ValueError("kappa_grain must be (G, V, 3, 3) covering every grain id")
            kbar, rem = grain_split(kg)
            self.grains = (kbar, rem, gidf)
        self.h_kind = h_kind
        self.ms_tol, self.ms_max_iter = ms_tol, ms_max_iter
        self.green = GreenOperator(C0, self.shape, self.dx)


class State:
    """eta (V, nz, ny, nx); eps (nz, ny, nx, 3, 3) warm start; ebar (3, 3)."""

    def __init__(self, eta, eps, ebar):
        self.eta = np.asarray(eta, dtype=np.float64)
        self.eps = eps
        self.ebar = ebar

    @classmethod
    def initial(cls, eta0, eps_bar6):
        eta0 = np.asarray(eta0, dtype=np.float64)
        ebar = voigt6_to_tensor(np.asarray(eps_bar6, dtype=np.float64))
        eps = np.broadcast_to(ebar, eta0.shape[1:] + (3, 3)).copy()
        return cls(eta0, eps, ebar)


def step(prob, state, eps_p6, load):
    """One time step: equilibrium at f^n, then the Allen-Cahn update.

    eps_p6: (6, nz, ny, nx) plastic strain (tensor-Voigt) or None.
    load: dict with eps_bar (6), sig_bar (6), stress_mask (6 bools).
    Returns (new_state, stats) where stats describe the state at f^n.
    """
    C_grain, C_var, eps0 = prob.tables
    shape = prob.shape
    if eps_p6 is None:
        eps_p = np.zeros(shape + (3, 3))
    else:
        eps_p = voigt6_to_tensor(eps_p6)
    eps, ebar, sigma, eps_el, _, iters, res = ms_solve(
        state.eps, state.ebar, state.eta, eps_p, prob.gid, prob.tables, prob.green,
        load, prob.ms_tol, prob.ms_max_iter, prob.h_kind)
    chem = chemical_force(state.eta, prob.A)
    mech = mechanical_force(state.eta, sigma, eps_el, prob.gid, C_grain, C_var, eps0, prob.h_kind)
    mob = getattr(prob, "mobility", None)
    grains = getattr(prob, "grains", None)
    eta_new = allen_cahn_update(state.eta, chem, mech, prob.L, prob.dt, prob.kappa, prob.dx, prob.kappa_var, mob,
                                grains)
    # the paper's fixed point i: the guess is f^n, each solve re-evaluates the
    # chemical force at the latest iterate, stop when max |f^i - f^{i-1}| <= tol
    pf_max = max(1, getattr(prob, "pf_max_iter", 1))
    pf_iters = 1
    pf_change = float(np.abs(eta_new - state.eta).max()) if eta_new.size else 0.0
    while pf_iters < pf_max and pf_change > prob.pf_tol:
        prev = eta_new
        eta_new = picard_iterate(state.eta, prev, mech, prob, mob)
        pf_iters += 1
        pf_change = float(np.abs(eta_new - prev).max())
    dV = prob.dx ** 3
    stats = {
        "G_dw": float(double_well_density(state.eta, prob.A).sum() * dV),
        "G_gd": float(gradient_energy(state.eta, prob.kappa, prob.dx, prob.kappa_var, grains)),
        "G_me": float(0.5 * np.einsum("...ij,...ij->...", eps_el, sigma).sum() * dV),
        "sig_mean": tensor_to_voigt6(sigma.mean(axis=(0, 1, 2))),
        "eps_mean": tensor_to_voigt6(eps.mean(axis=(0, 1, 2))),
        "eta_mean": state.eta.mean(axis=(1, 2, 3)),
        "ms_iters": iters,
        "ms_residual": res,
        "pf_iters": pf_iters,
        "pf_change": pf_change,
        "pf_converged": pf_max == 1 or pf_change <= prob.pf_tol,
    }
    stats["G"] = stats["G_dw"] + stats["G_gd"] + stats["G_me"]
    return State(eta_new, eps, ebar), stats, sigma


def stress_voigt6(sigma):
    return tensor_to_voigt6(sigma)


def reference_stiffness_average(C_grain, C_var):
    """Arithmetic mean of every grain and twin-variant stiffness: the default
    reference medium for the fixed point (reading; the paper has no solver of
    this kind)."""
    mats = [C_grain[g] for g in range(C_grain.shape[0])]
    mats += [C_var[g, a] for g in range(C_var.shape[0]) for a in range(C_var.shape[1])]
    return np.mean(mats, axis=0)


__all__ = ["chemical_force", "mechanical_force", "double_well_density",
           "gradient_symbol", "gradient_energy", "allen_cahn_update", "Problem", "State", "step",
           "h_interp", "reference_stiffness_average", "stress_voigt6"]
