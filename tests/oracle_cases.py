"""Small helpers that assemble oracle problems for the pins (tests only)."""

import numpy as np

from oracle import crystal as cr
from oracle import mech
from oracle import phasefield as pf


def frame_from(m, s):
    """Rotation R (crystal -> sample) with R m = e_z and R s = e_x."""
    return np.stack([s, np.cross(m, s), m])


def frame_m_along_x(m, s):
    """Rotation with R m = e_x and R s = e_z."""
    return np.stack([m, -np.cross(m, s), s])


def tables(rotations, variant_ids, homogeneous=False, no_eigenstrain=False):
    Cg, Cv, e0 = cr.mg_tables(rotations, variant_ids)
    if homogeneous:
        Cv = np.broadcast_to(Cg[:, None], Cv.shape).copy()
    if no_eigenstrain:
        e0 = np.zeros_like(e0)
    return Cg, Cv, e0


def problem(shape, tabs, dx=5e-8, A=1e7, kappa=1e-9, L=1.2e-5, dt=2e-4, gid=None,
            C0=None, h_kind="linear", tol=1e-12, max_iter=500, kappa_var=None, mobility=None,
            pf_tol=1e-12, pf_max_iter=1):
    if C0 is None:
        C0 = pf.reference_stiffness_average(tabs[0], tabs[1])
    return pf.Problem(shape, dx, tabs, A, kappa, L, dt, C0, gid=gid, h_kind=h_kind,
                      ms_tol=tol, ms_max_iter=max_iter, kappa_var=kappa_var, mobility=mobility,
                      pf_tol=pf_tol, pf_max_iter=pf_max_iter)


def load(eps_bar=None, sig_bar=None, stress_mask=None):
    return dict(eps_bar=np.zeros(6) if eps_bar is None else np.asarray(eps_bar, float),
                sig_bar=np.zeros(6) if sig_bar is None else np.asarray(sig_bar, float),
                stress_mask=np.zeros(6, bool) if stress_mask is None else np.asarray(stress_mask, bool))


def solve(prob, eta, eps_p6=None, ld=None, eps_bar0=None):
    shape = prob.shape
    eps_p = np.zeros(shape + (3, 3)) if eps_p6 is None else mech.voigt6_to_tensor(eps_p6)
    ld = ld or load()
    e0 = mech.voigt6_to_tensor(np.zeros(6) if eps_bar0 is None else eps_bar0)
    eps_start = np.broadcast_to(e0, shape + (3, 3)).copy()
    return mech.ms_solve(eps_start, e0, np.asarray(eta, float), eps_p, prob.gid, prob.tables,
                         prob.green, ld, prob.ms_tol, prob.ms_max_iter, prob.h_kind)
