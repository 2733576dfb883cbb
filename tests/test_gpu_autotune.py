"""GPU: the autotuner and the FFT plans it chooses from.

The tuner times, per size group, the FFT plan variants (radix split and
elements per thread) and column tiles of every column pass and keeps the
fastest. Plans differ in rounding only, so:
* every plan variant of every pass, forced through pf_batch_set_plan,
  transforms like the FP64 FFT (y passes and the plain z pass, every axis
  length) or steps like the FP64 oracle (Green z pass, spectral z pass);
* a tuned batch matches an untuned one to FP32 round-off on the spectral and
  fixed-point paths, and a tuned polycrystal does as well;
* the cache file holds one entry per size group with every candidate's
  time; a second context applies the cached plan without timing (and then
  computes bit for bit what the tuned context did), unless asked to time
  again."""

import itertools
import json

import numpy as np
import pytest

from paper_2302_13612_amd import binding, inputs
from tests import cases
from tests.test_gpu_batch import small_batch

pytestmark = pytest.mark.gpu

TUNED_TOL = 1e-5   # order parameter, tuned vs default plans (FP32 round-off of a few steps)


def log(msg):
    print(msg, flush=True)


def run(batch, idx, variants, steps, tune=None, fixed_point=False):
    bs = cases.gpu_batch(batch, idx, variants)
    timed = None
    if tune is not None:
        timed = bs.autotune(**tune)
    plans = [bs.plan(k) for k in range(len(idx))]
    eb = np.stack([batch["instances"][i]["eps_bar"] for i in idx])
    bs.step(steps, eb, fixed_point=fixed_point)
    etas = [bs.field(k, binding.PF_FIELD_ETA).cpu().numpy() for k in range(len(idx))]
    bs.close()
    return etas, plans, timed


def valid_plan(p):
    return (p["ytile"] in (8, 16) and p["yplan"] in (0, 1, 2) and p["ztile_ms"] in (8, 16)
            and p["zplan_ms"] in (0, 1) and p["zplan_ac"] in (0, 1, 2) and p["ztile_kh"] in (8, 16)
            and p["zplan_kh"] in (0, 1))


def test_fft_plan_variants_are_factorisations():
    for n in (32, 48, 64, 96, 128, 192, 256, 384, 512):
        for k in range(3):
            e, r = binding.fft_plan(n, k)
            assert int(np.prod(r)) == n and all(e % x == 0 for x in r), (n, k, e, r)
        assert binding.fft_plan(n, 1)[0] < binding.fft_plan(n, 0)[0] < binding.fft_plan(n, 2)[0]
    with pytest.raises(binding.PfError):
        binding.fft_plan(80, 0)
    with pytest.raises(binding.PfError):
        binding.fft_plan(64, 3)


# (nz, ny, nx): every supported length once as y and once as z
TRANSFORM_SHAPES = [(32, 48, 32), (48, 64, 32), (64, 96, 32), (96, 128, 32), (128, 192, 32),
                    (192, 256, 32), (256, 384, 32), (384, 512, 32), (512, 32, 32)]


def fits(n, k, tile):
    e, _ = binding.fft_plan(n, k)
    return tile * (n // e) <= 1024


@pytest.mark.parametrize("shape", TRANSFORM_SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_every_plan_variant_transforms_like_fp64(shape):
    import torch
    cfg = inputs.single_crystal_sphere(n=32)
    nz, ny, nx = shape
    cfg = dict(cfg, shape=shape, eta0=np.zeros((1,) + shape, np.float32))
    solver, _ = cases.gpu_solver(cfg)
    rng = np.random.default_rng(sum(shape))
    real = rng.standard_normal((2,) + shape).astype(np.float32)
    ref = np.fft.rfftn(real.astype(np.float64), axes=(1, 2, 3))
    base = solver.plan()
    worst = 0.0
    for yk, yt, zk in itertools.product(range(3), (8, 16), range(3)):
        if not (fits(ny, yk, yt) and fits(nz, zk, 16)):
            continue
        solver.set_plan(dict(base, yplan=yk, ytile=yt, zplan_ac=zk))
        spec = solver.fft_forward(torch.from_numpy(real).cuda()).cpu().numpy()
        err = np.abs(spec - ref).max() / np.abs(ref).max()
        back = solver.fft_inverse(torch.from_numpy(spec).cuda()).cpu().numpy()
        err_b = np.abs(back - real).max() / np.abs(real).max()
        worst = max(worst, err, err_b)
        assert err <= 2e-6 and err_b <= 2e-6, (shape, yk, yt, zk, err, err_b)
    log(f"\n[plans] {shape}: worst relative error over the plan variants {worst:.2e}")
    solver.close()


def test_green_z_pass_plans_step_like_the_oracle():
    cfg = cases.small_polycrystal()
    steps = 2
    eta_o, sig_o, _ = cases.oracle_run(cfg, steps)
    for zk, zt in itertools.product(range(2), (8, 16)):
        if not fits(cfg["shape"][0], zk, zt):
            continue
        solver, epsp = cases.gpu_solver(cfg)
        solver.set_plan(dict(solver.plan(), zplan_ms=zk, ztile_ms=zt))
        for n in range(steps):
            e, s = cases.loads(cfg, n)
            solver.step(1, e, s, eps_p=epsp if n == 0 else None, save_stress=n == steps - 1)
        eta = solver.field(binding.PF_FIELD_ETA).cpu().numpy()
        sig = solver.field(binding.PF_FIELD_STRESS).cpu().numpy()
        solver.close()
        d, r = np.abs(eta - eta_o).max(), cases.stress_rel_l2(sig, sig_o)
        log(f"\n[plans] Green z pass variant {zk} tile {zt}: eta {d:.2e}, stress rel-L2 {r:.2e}")
        assert d <= 1e-4 and r <= 1e-5


def test_spectral_z_pass_plans_step_like_the_oracle():
    cfg = inputs.single_crystal_sphere()
    steps = 20
    eta_o, _, _ = cases.oracle_run(cfg, steps)
    for zk, zt in itertools.product(range(2), (8, 16)):
        solver, _ = cases.gpu_solver(cfg)
        solver.set_plan(dict(solver.plan(), zplan_kh=zk, ztile_kh=zt))
        for n in range(steps):
            e, s = cases.loads(cfg, n)
            solver.step(1, e, s)
        eta = solver.field(binding.PF_FIELD_ETA).cpu().numpy()
        solver.close()
        d = np.abs(eta - eta_o).max()
        log(f"\n[plans] spectral z pass variant {zk} tile {zt}: eta {d:.2e}")
        assert d <= 1e-4


def test_set_plan_rejects_plans_that_do_not_exist():
    cfg = cases.small_polycrystal()
    solver, _ = cases.gpu_solver(cfg)
    p = solver.plan()
    for bad in (dict(p, ytile=12), dict(p, yplan=3), dict(p, zplan_ms=2), dict(p, ztile_kh=4)):
        with pytest.raises(binding.PfError) as ei:
            solver.set_plan(bad)
        assert ei.value.code == binding.PF_EINVAL
    solver.close()


def test_tuned_batch_matches_untuned_and_is_cached(tmp_path):
    batch, idx, variants = small_batch()
    sizes = sorted({batch["instances"][i]["shape"][0] for i in idx})
    log(f"\n[autotune] sizes {sizes}")
    ref, plans0, _ = run(batch, idx, variants, 10)
    cache = tmp_path / "plans.jsonl"
    tuned, plans, timed = run(batch, idx, variants, 10, tune=dict(cache=cache))
    log(f"  default plans {plans0[0]}\n  tuned plans {plans}\n  groups timed {timed}")
    assert timed == len(sizes)
    assert all(valid_plan(p) for p in plans)
    d = max(np.abs(a - b).max() for a, b in zip(ref, tuned))
    log(f"  tuned vs default: eta max-abs {d:.2e}")
    assert d <= TUNED_TOL
    lines = [json.loads(l) for l in cache.read_text().splitlines()]
    assert sorted(l["nx"] for l in lines) == sizes
    for l in lines:
        assert len(l["us_y"]) == 6 and len(l["us_zkh"]) == 4
        assert min(t for t in l["us_y"] if t >= 0) > 0
        assert min(t for t in l["us_zkh"] if t >= 0) > 0
        # the chosen y plan is the fastest candidate timed
        k = [(0, 8), (0, 16), (1, 8), (1, 16), (2, 8), (2, 16)].index((l["yplan"], l["ytile"]))
        assert l["us_y"][k] == min(t for t in l["us_y"] if t >= 0)
    # a second context takes the cached plan without timing
    again, plans2, timed2 = run(batch, idx, variants, 10, tune=dict(cache=cache))
    assert timed2 == 0 and plans2 == plans
    for a, b in zip(tuned, again):
        assert np.array_equal(a, b)
    # unless asked to time again (one more entry per group)
    _, _, timed3 = run(batch, idx, variants, 1, tune=dict(cache=cache, retime=True))
    assert timed3 == len(sizes)
    assert len(cache.read_text().splitlines()) == 2 * len(sizes)


def test_tuned_fixed_point_path_matches_untuned():
    batch, idx, variants = small_batch()
    ref, _, _ = run(batch, idx, variants, 4, fixed_point=True)
    tuned, plans, timed = run(batch, idx, variants, 4, tune={}, fixed_point=True)
    d = max(np.abs(a - b).max() for a, b in zip(ref, tuned))
    log(f"\n[autotune] fixed-point path: plans {plans}, eta max-abs {d:.2e}")
    assert d <= TUNED_TOL


def test_single_polycrystal_tuned_matches_untuned(tmp_path):
    cfg = cases.small_polycrystal()
    s0, eta0, _ = cases.gpu_run(cfg, 2, save_stress_last=False)
    s0.close()
    solver, epsp = cases.gpu_solver(cfg)
    cache = tmp_path / "poly.jsonl"
    timed = solver.autotune(cache=cache)
    plan = solver.plan()
    for n in range(2):
        e, s = cases.loads(cfg, n)
        solver.step(1, e, s, eps_p=epsp if n == 0 else None)
    eta1 = solver.field(binding.PF_FIELD_ETA).cpu().numpy()
    solver.close()
    d = np.abs(eta0 - eta1).max()
    entry = json.loads(cache.read_text().splitlines()[0])
    log(f"\n[autotune] polycrystal 32^3: plan {plan}, groups timed {timed}, eta max-abs {d:.2e}\n"
        f"  candidate times: y {entry['us_y']} Green z {entry['us_zms']} Allen-Cahn z {entry['us_zac']}")
    assert timed == 1 and valid_plan(plan)
    assert min(t for t in entry["us_zms"] if t >= 0) > 0 and min(t for t in entry["us_zac"] if t >= 0) > 0
    assert d <= TUNED_TOL
