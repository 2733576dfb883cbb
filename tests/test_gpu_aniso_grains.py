"""GPU: the anisotropic gradient energy on a polycrystal (per-grain tensors of
Table 5 turned by each grain's rotation; kbar I implicit, the remainder
2 div((K(x) - kbar I) grad f) explicit through spectral first derivatives)
through the C ABI against the FP64 oracle. Each side builds its own tensors
(library: C++ helper, oracle: NumPy) and its own split. Tolerances as for
the isotropic fixed point: order parameter max-abs <= 1e-4, stress rel-L2
<= 1e-5, energies (the gradient energy of the split operator included)
<= 1e-4 of their scale.
"""

import numpy as np
import pytest

from paper_2302_13612_amd import binding, inputs
from tests import cases
from tests.test_gpu_batch import check_stats

pytestmark = pytest.mark.gpu

ETA_TOL = 1e-4
SIG_TOL = 1e-5
PAPER = dict(c2n=2.81e-7, c2s=2.81e-6)


def log(msg):
    print(msg, flush=True)


def grain_case(cfg, steps, label):
    log(f"\n[aniso grains] {label} shape={cfg['shape']} n_var={cfg['n_var']} grains={cfg['rotations'].shape[0]} "
        f"steps={steps}")
    solver, eta_g, sig_g = cases.gpu_run(cfg, steps)
    st_g = solver.stats()
    eta_o, sig_o, stats_o = cases.oracle_run(cfg, steps)
    d = np.abs(eta_g - eta_o).max()
    r = cases.stress_rel_l2(sig_g, sig_o)
    log(f"  eta max-abs {d:.2e}  stress rel-L2 {r:.2e}  G_gd gpu {st_g['G_gd']:.6e} oracle "
        f"{stats_o[-1]['G_gd']:.6e}  ms_iters {st_g['ms_iters']}")
    assert np.isfinite(eta_g).all()
    assert d <= ETA_TOL
    assert r <= SIG_TOL
    check_stats(st_g, stats_o[-1], np.abs(sig_o).max())
    solver.close()
    return eta_g


def test_aniso_polycrystal_vs_oracle():
    cfg = dict(cases.small_polycrystal(), aniso_grains=PAPER)
    eta = grain_case(cfg, 4, "6 grains, 6 variants, paper's c2")
    # the anisotropy shows: the isotropic run ends elsewhere
    _, eta_iso, _ = cases.gpu_run(cases.small_polycrystal(), 4, save_stress_last=False)
    assert np.abs(eta - eta_iso).max() > 1e-3


def test_aniso_polycrystal_ragged_two_variants():
    # x = 48 (a ragged last column tile and the Nyquist plane), y = 32, z = 64
    cfg = dict(cases.small_polycrystal(shape=(64, 32, 48), n_grains=5, seed=9, n_var=2),
               aniso_grains=dict(c2n=2.81e-7, c2s=2.81e-6, c2t=1.0e-6))
    grain_case(cfg, 6, "5 grains, 2 variants, c2t != c2n")


def test_isotropic_grain_tensors_equal_the_isotropic_step():
    # every grain at kappa I: no remainder, the implicit part is kappa I
    base = cases.small_polycrystal(n_var=2)
    k = base["kappa"]
    cfg = dict(base, aniso_grains=dict(c2n=k, c2s=k, c2t=k))
    s1, eta_a, _ = cases.gpu_run(cfg, 3, save_stress_last=False)
    s2, eta_b, _ = cases.gpu_run(base, 3, save_stress_last=False)
    d = np.abs(eta_a - eta_b).max()
    log(f"\n[aniso grains] kappa I in every grain vs isotropic: eta max-abs {d:.2e}")
    assert d <= 1e-6
    ga, gb = s1.stats()["G_gd"], s2.stats()["G_gd"]
    assert abs(ga - gb) <= 1e-5 * abs(gb)
    s1.close()
    s2.close()


def test_aniso_polycrystal_radix3_axes():
    # 96 along y and 48 along z: the radix-3 plans in the gradient and divergence z passes and
    # the y passes of 3V components
    cfg = dict(cases.small_polycrystal(shape=(48, 96, 32), n_grains=4, seed=17, n_var=2), aniso_grains=PAPER)
    grain_case(cfg, 3, "4 grains, 2 variants, 48 x 96 x 32")
