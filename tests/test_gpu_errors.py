"""GPU: error paths and restart through the C ABI.

* A non-finite order parameter written through pf_fields makes the next
  step fail with PF_ENONFINITE, on the homogeneous spectral path and on the
  fixed-point path (where the non-finite strain stops the iteration instead
  of running it to its limit).
* A fixed point limited to one iteration on a problem with stiffness
  contrast fails with PF_ENOCONV.
* A checkpoint (order parameters and strain read through pf_fields) restored
  into a fresh context continues the run: bit for bit on the spectral path
  (its state is f alone) and, on the fixed-point path, bit for bit against
  the same checkpoint set back into the running context (both restart the
  strain extrapolation), and within the fixed point's tolerance against the
  uninterrupted run.
* A grain id at or above n_grains is rejected by pf_init (PF_EINVAL).
"""

import math

import numpy as np
import pytest

from paper_2302_13612_amd import binding
from tests import cases
from paper_2302_13612_amd import inputs

pytestmark = pytest.mark.gpu


def _step(solver, cfg, n, epsp=None):
    e, s = cases.loads(cfg, n)
    solver.step(1, e, s, eps_p=epsp)


def _poison(solver):
    eta = solver.field(binding.PF_FIELD_ETA)
    nz, ny, nx = solver.shape
    eta[0, nz // 2, ny // 3, nx // 4] = math.nan
    solver.set_field(binding.PF_FIELD_ETA, eta)


def test_nonfinite_order_parameter_spectral_path():
    cfg = inputs.single_crystal_sphere()
    print("\n[errors] NaN in eta, sphere 32^3 (spectral path)", flush=True)
    solver, _ = cases.gpu_solver(cfg)
    _step(solver, cfg, 0)
    _poison(solver)
    with pytest.raises(binding.PfError) as ei:
        _step(solver, cfg, 1)
    assert ei.value.code == binding.PF_ENONFINITE
    solver.close()


def test_nonfinite_order_parameter_fixed_point_path():
    cfg = cases.small_polycrystal()
    print("\n[errors] NaN in eta, polycrystal 32^3 (fixed point)", flush=True)
    solver, epsp = cases.gpu_solver(cfg)
    _step(solver, cfg, 0, epsp)
    _poison(solver)
    with pytest.raises(binding.PfError) as ei:
        _step(solver, cfg, 1)
    assert ei.value.code == binding.PF_ENONFINITE
    assert "fixed point" in str(ei.value)
    solver.close()


def test_fixed_point_iteration_limit():
    cfg = cases.small_lamellae()
    cfg["ms_max_iter"] = 1
    print("\n[errors] ms_max_iter = 1, lamellae 64x32x32 (contrast)", flush=True)
    solver, epsp = cases.gpu_solver(cfg)
    with pytest.raises(binding.PfError) as ei:
        _step(solver, cfg, 0, epsp)
    assert ei.value.code == binding.PF_ENOCONV
    solver.close()


def test_restart_spectral_path_bitwise():
    cfg = inputs.single_crystal_sphere()
    N = 12
    print(f"\n[restart] sphere 32^3 spectral path, {N} + {N} steps", flush=True)
    ref, _ = cases.gpu_solver(cfg)
    for n in range(2 * N):
        _step(ref, cfg, n)
    eta_ref = ref.field(binding.PF_FIELD_ETA).cpu().numpy()
    st_ref = ref.stats()
    ref.close()
    a, _ = cases.gpu_solver(cfg)
    for n in range(N):
        _step(a, cfg, n)
    ck = a.field(binding.PF_FIELD_ETA).clone()
    a.close()
    b, _ = cases.gpu_solver(cfg)
    b.set_field(binding.PF_FIELD_ETA, ck)
    for n in range(N, 2 * N):
        _step(b, cfg, n)
    eta_b = b.field(binding.PF_FIELD_ETA).cpu().numpy()
    st_b = b.stats()
    b.close()
    assert np.array_equal(eta_b, eta_ref)
    for k in ("G_dw", "G_gd", "G_me"):
        assert st_b[k] == st_ref[k], k


def test_restart_fixed_point_path():
    cfg = cases.small_lamellae()
    N = 6
    print(f"\n[restart] lamellae 64x32x32 fixed point, {N} + {N} steps", flush=True)
    epsp_host = cfg["eps_p"]
    # uninterrupted run
    ref, epsp = cases.gpu_solver(cfg)
    for n in range(2 * N):
        _step(ref, cfg, n, epsp if n == 0 else None)
    eta_ref = ref.field(binding.PF_FIELD_ETA).cpu().numpy()
    ref.close()
    # run with the checkpoint set back into the same context at step N
    a, epsp = cases.gpu_solver(cfg)
    for n in range(N):
        _step(a, cfg, n, epsp if n == 0 else None)
    ck_eta = a.field(binding.PF_FIELD_ETA).clone()
    ck_eps = a.field(binding.PF_FIELD_STRAIN).clone()
    a.set_field(binding.PF_FIELD_ETA, ck_eta)
    a.set_field(binding.PF_FIELD_STRAIN, ck_eps)
    for n in range(N, 2 * N):
        _step(a, cfg, n)
    eta_a = a.field(binding.PF_FIELD_ETA).cpu().numpy()
    a.close()
    # restore into a fresh context
    b, epsp = cases.gpu_solver(cfg)
    b.set_field(binding.PF_FIELD_ETA, ck_eta)
    b.set_field(binding.PF_FIELD_STRAIN, ck_eps)
    for n in range(N, 2 * N):
        _step(b, cfg, n, epsp if n == N else None)
    eta_b = b.field(binding.PF_FIELD_ETA).cpu().numpy()
    b.close()
    d = np.abs(eta_b - eta_ref).max()
    print(f"  restored vs continued in place: bitwise {np.array_equal(eta_b, eta_a)}; "
          f"vs uninterrupted: max-abs {d:.2e}", flush=True)
    assert epsp_host is not None
    assert np.array_equal(eta_b, eta_a)
    # the extrapolated first iterates differ; each step's fixed point stops at
    # a relative strain change of 1e-6, an order below what reaches f
    assert d <= 1e-6


def test_grain_id_out_of_range_rejected():
    # a grain id at or above n_grains would index past the per-grain tables
    cfg = cases.small_polycrystal(n_var=2)
    G = cfg["rotations"].shape[0]      # n_grains handed to the library
    bad = cfg["gid"].copy()
    bad[3, 4, 5] = G
    print(f"\n[errors] grain id {G} with n_grains = {G}, polycrystal 32^3", flush=True)
    with pytest.raises(binding.PfError) as ei:
        cases.gpu_solver(dict(cfg, gid=bad))
    assert ei.value.code == binding.PF_EINVAL
    # the same field with every id in range is accepted
    ok = bad.copy()
    ok[3, 4, 5] = G - 1
    solver, _ = cases.gpu_solver(dict(cfg, gid=ok))
    solver.close()
