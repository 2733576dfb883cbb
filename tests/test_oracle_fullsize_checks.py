"""CPU: the full-size property checks of the 256^3 GPU test, run on a small
polycrystal whose fields come from the oracle's own converged step. The
exact fields pass; fields carrying a plausible mistake (a perturbed strain,
a stress without the twin eigenstrain, an update without the elastic
driving force) fail the check that is meant to catch it."""

import numpy as np

from oracle import mech
from oracle import phasefield as opf
from tests import cases
from tests.test_gpu_fullsize import ETA_TOL, SIG_TOL, oracle_checks


def _oracle_fields(cfg):
    prob = cases.oracle_problem(cfg, tol=1e-12)
    st0 = opf.State.initial(cfg["eta0"].astype(np.float64), np.zeros(6))
    ld = dict(eps_bar=cfg["eps_bar"], sig_bar=cfg["sig_bar"], stress_mask=cfg["stress_mask"])
    st1, _, sigma = opf.step(prob, st0, cfg["eps_p"].astype(np.float64), ld)
    return prob, mech.tensor_to_voigt6(st1.eps), mech.tensor_to_voigt6(sigma), st1.eta


def test_fullsize_checks_accept_the_oracle_and_reject_planted_mistakes():
    cfg = cases.small_polycrystal(shape=(32, 32, 32), n_grains=6, n_var=6)
    prob, eps6, sig6, eta1 = _oracle_fields(cfg)
    r = oracle_checks(cfg, eps6, sig6, eta1)
    assert r["sig_rel_l2"] <= 1e-12
    assert r["ms_change"] <= 1e-10
    assert r["mean_strain_err"] <= 1e-15
    assert r["mean_stress_rel"] <= 1e-10
    assert r["eta_max_abs"] <= 1e-12
    assert r["eta_change"] > 10 * ETA_TOL

    # a strain off the fixed point by a local shear of 1e-3 of the load
    bad = eps6.copy()
    bad[5, 3:6, 4:9, 7:11] += 1e-3 * abs(cfg["eps_bar"][0])
    assert oracle_checks(cfg, bad, sig6, eta1)["ms_change"] > cfg["ms_tol"]

    # a stress that leaves out the twin eigenstrain
    C_grain, C_var, eps0 = prob.tables
    eps = mech.voigt6_to_tensor(eps6)
    eps_p = mech.voigt6_to_tensor(cfg["eps_p"].astype(np.float64))
    _, _, sig_no_twin = mech.eigenstrain_and_stress(eps, np.zeros_like(eta1), eps_p, prob.gid,
                                                    C_grain, C_var, eps0, prob.h_kind)
    r_bad = oracle_checks(cfg, eps6, mech.tensor_to_voigt6(sig_no_twin), eta1)
    assert r_bad["sig_rel_l2"] > SIG_TOL

    # an update that drops the elastic driving force
    eta0 = cfg["eta0"].astype(np.float64)
    chem = opf.chemical_force(eta0, prob.A)
    eta_no_mech = opf.allen_cahn_update(eta0, chem, np.zeros_like(chem), prob.L, prob.dt, prob.kappa, prob.dx)
    assert oracle_checks(cfg, eps6, sig6, eta_no_mech)["eta_max_abs"] > ETA_TOL
