"""GPU: the learned macro stepper (FNO forward, acceptance residual,
accept/fallback loop) through the C ABI, against the FP64 oracle.

Tolerance of the forward pass: both sides get the same weights, rounded to
BF16 where the library stores them in BF16 (W, R, Q1), so the difference
comes from the BF16 activations (relative rounding 2^-9 at the lift and after
each of the four layers) and FP32 sums: about sqrt(5) 2^-9 = 0.4% of the
activations, i.e. of the predicted increment; the test allows 2% (rel-L2)."""

import numpy as np
import pytest

from oracle import fno as ofno
from paper_2302_13612_amd import binding, inputs
from tests import cases

pytestmark = pytest.mark.gpu


def bf16_round(a):
    a = np.asarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gpu_params(seed=0, modes=12):
    p = ofno.init_params(width=32, modes=modes, hidden=128, n_layers=4, seed=seed, scale_spec=2e-3)
    p["W"] = bf16_round(p["W"])
    p["Q1"] = bf16_round(p["Q1"])
    p["R"] = bf16_round(p["R"].real) + 1j * bf16_round(p["R"].imag)
    for k in ("P", "p", "b", "q1", "Q2", "q2"):
        p[k] = np.asarray(p[k], dtype=np.float32).astype(np.float64)
    return p


def smooth_field(shape, seed):
    rng = inputs.rng_for(seed)
    g = inputs.gaussian_random_field(shape, 4.0, rng)
    return (0.5 + 0.3 * g / np.abs(g).max()).astype(np.float32)


def homog_solver(shape, eta, seed=31):
    batch = inputs.rve_batch(n_inst=1, seed=seed, sizes=(shape[0],))
    cfg = cases.batch_instance_cfg(batch, 0)
    cfg = dict(cfg, shape=shape, eta0=eta[None])
    solver, _ = cases.gpu_solver(cfg)
    return cfg, solver


# (nz, ny, nx), kept modes: every x length the x sums take (32 to 128), and
# 16 modes, whose 2m = 32 rows fill the whole matrix-core tile
@pytest.mark.parametrize("shape,modes", [((32, 32, 32), 12), ((32, 32, 64), 12), ((48, 64, 96), 12),
                                         ((32, 48, 32), 16), ((128, 128, 128), 12)])
def test_fno_forward_vs_oracle(shape, modes):
    import torch
    print(f"\n[fno forward] {shape} modes {modes}", flush=True)
    eta = smooth_field(shape, 3)
    cfg, solver = homog_solver(shape, eta)
    p = gpu_params(seed=1, modes=modes)
    cond = np.random.default_rng(2).normal(size=7)
    net = binding.Fno(solver, p)
    out = net.forward(cond, torch.from_numpy(eta).cuda()).cpu().numpy()
    ref = ofno.forward(p, eta.astype(np.float64), cond)
    d_gpu, d_ref = out - eta, ref - eta
    rel = np.linalg.norm(d_gpu - d_ref) / np.linalg.norm(d_ref)
    print(f"  increment rel-L2 {rel:.2e}, max-abs {np.abs(d_gpu - d_ref).max():.2e} "
          f"(increment max {np.abs(d_ref).max():.2e})", flush=True)
    assert np.isfinite(out).all()
    assert rel <= 2e-2
    # element by element: fourteen quantities are rounded to BF16 (unit
    # roundoff 2^-8): the activations v_0..v_4, the spectral weights R and the
    # channel-mixing weights W of the four layers, and Q_1 (the matrix-core
    # operands; the twiddles and transformed rows enter as BF16 hi and lo
    # parts, FP32-accurate). Each rounding reaches the output increment at
    # most at the increment's own scale, so no voxel may be off by more than
    # 14 * 2^-8 of the largest increment (measured: about 5 * 2^-8)
    assert np.abs(d_gpu - d_ref).max() <= 14 * 2.0 ** -8 * np.abs(d_ref).max()
    net.close()
    solver.close()


def test_macro_residual_vs_oracle():
    import torch
    shape = (32, 32, 32)
    batch = inputs.rve_batch(n_inst=2, seed=33, sizes=(32,))
    cfg = cases.batch_instance_cfg(batch, 1)
    solver, _ = cases.gpu_solver(cfg)
    solver.step(20, cfg["eps_bar"], cfg["sig_bar"])
    prev = solver.field(binding.PF_FIELD_ETA)
    solver.step(16, cfg["eps_bar"], cfg["sig_bar"])
    cur = solver.field(binding.PF_FIELD_ETA)
    rho = binding.macro_residual(solver, prev, 16, cfg["eps_bar"], cfg["sig_bar"])
    prob = cases.oracle_problem(cfg, tol=1e-12)
    load = dict(eps_bar=cfg["eps_bar"], sig_bar=cfg["sig_bar"], stress_mask=cfg["stress_mask"])
    _, rho_o = ofno.macro_residual(prob, prev.cpu().numpy().astype(np.float64),
                                   cur.cpu().numpy().astype(np.float64), 16, load)
    print(f"\n[residual] gpu {rho:.6e} oracle {rho_o:.6e}", flush=True)
    assert abs(rho - rho_o) <= 1e-5 + 1e-3 * rho_o
    # perturbed prediction
    bumped = cur.clone()
    bumped[0, 5, 6, 7] += 0.25
    solver.set_field(binding.PF_FIELD_ETA, bumped)
    rho_b = binding.macro_residual(solver, prev, 16, cfg["eps_bar"], cfg["sig_bar"])
    _, rho_bo = ofno.macro_residual(prob, prev.cpu().numpy().astype(np.float64),
                                    bumped.cpu().numpy().astype(np.float64), 16, load)
    assert abs(rho_b - rho_bo) <= 1e-5 + 1e-3 * rho_bo
    assert rho_b > rho + 0.2
    # one exact plain step satisfies the residual of one step up to FP32 rounding
    solver.set_field(binding.PF_FIELD_ETA, cur)
    solver.step(1, cfg["eps_bar"], cfg["sig_bar"])
    rho_1 = binding.macro_residual(solver, cur, 1, cfg["eps_bar"], cfg["sig_bar"])
    print(f"[residual] one exact step: {rho_1:.3e}", flush=True)
    assert rho_1 <= 1e-5
    solver.close()
    del torch


def test_macro_residual_accepts_exact_rejects_perturbed():
    # late in the relaxation of a 32^3 instance: the exact 16-step window is
    # accepted at 1e-3, the same state with a 2e-3 bump is not; both as the
    # oracle computes them on the library's fields
    batch = inputs.rve_batch(n_inst=2, seed=99, sizes=(32,))
    cfg = cases.batch_instance_cfg(batch, 0)
    solver, _ = cases.gpu_solver(cfg)
    solver.step(64, cfg["eps_bar"], cfg["sig_bar"])
    prev = solver.field(binding.PF_FIELD_ETA)
    solver.step(16, cfg["eps_bar"], cfg["sig_bar"])
    cur = solver.field(binding.PF_FIELD_ETA)
    rho = binding.macro_residual(solver, prev, 16, cfg["eps_bar"], cfg["sig_bar"])
    bumped = cur.clone()
    bumped[0, 16, 16, 16] += 2e-3
    solver.set_field(binding.PF_FIELD_ETA, bumped)
    rho_b = binding.macro_residual(solver, prev, 16, cfg["eps_bar"], cfg["sig_bar"])
    prob = cases.oracle_problem(cfg, tol=1e-12)
    load = dict(eps_bar=cfg["eps_bar"], sig_bar=cfg["sig_bar"], stress_mask=cfg["stress_mask"])
    p64 = prev.cpu().numpy().astype(np.float64)
    _, rho_o = ofno.macro_residual(prob, p64, cur.cpu().numpy().astype(np.float64), 16, load)
    _, rho_bo = ofno.macro_residual(prob, p64, bumped.cpu().numpy().astype(np.float64), 16, load)
    print(f"\n[accept] exact gpu {rho:.3e} oracle {rho_o:.3e}; bumped gpu {rho_b:.3e} oracle {rho_bo:.3e}",
          flush=True)
    assert abs(rho - rho_o) <= 1e-5 + 1e-3 * rho_o
    assert abs(rho_b - rho_bo) <= 1e-5 + 1e-3 * rho_bo
    assert rho <= 0.5e-3 < 2e-3 <= rho_b
    solver.close()


def test_fno_advance_accept_and_fallback():
    import torch
    shape = (32, 32, 32)
    batch = inputs.rve_batch(n_inst=1, seed=34, sizes=(32,))
    cfg = cases.batch_instance_cfg(batch, 0)
    p = gpu_params(seed=4)
    cond = np.random.default_rng(5).normal(size=7)
    # everything accepted: the state is the network's prediction, call after call
    s1, _ = cases.gpu_solver(cfg)
    net = binding.Fno(s1, p)
    eta0 = s1.field(binding.PF_FIELD_ETA)
    rep = net.advance(2, 16, cond, cfg["eps_bar"], cfg["sig_bar"], tol=np.inf)
    assert rep["accepted"] == 2 and rep["rejected"] == 0
    expect = net.forward(cond, net.forward(cond, eta0[0])[None][0])
    got = s1.field(binding.PF_FIELD_ETA)[0]
    assert torch.equal(got, expect)
    net.close()
    s1.close()
    # everything rejected: the state is that of plain steps
    s2, _ = cases.gpu_solver(cfg)
    net = binding.Fno(s2, p)
    rep = net.advance(2, 16, cond, cfg["eps_bar"], cfg["sig_bar"], tol=-1.0)
    assert rep["accepted"] == 0 and rep["rejected"] == 2
    got = s2.field(binding.PF_FIELD_ETA).cpu().numpy()
    net.close()
    s2.close()
    s3, _ = cases.gpu_solver(cfg)
    s3.step(32, cfg["eps_bar"], cfg["sig_bar"])
    plain = s3.field(binding.PF_FIELD_ETA).cpu().numpy()
    s3.close()
    assert np.array_equal(got, plain)
