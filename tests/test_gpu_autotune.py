"""GPU: the autotuner (launch tiles of a batch of uneven RVEs picked by timing
on the device). The tile changes no arithmetic, so a tuned batch reproduces
an untuned one bit for bit, on the spectral path and on the fixed-point path;
the plan is one of the candidates; the cache file holds one entry per size
group and a second context reads its plan from there without timing, unless
asked to time again."""

import json

import numpy as np
import pytest

from paper_2302_13612_amd import binding, inputs
from tests import cases
from tests.test_gpu_batch import small_batch

pytestmark = pytest.mark.gpu


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


def test_tuned_batch_is_bit_identical_and_cached(tmp_path):
    batch, idx, variants = small_batch()
    sizes = sorted({batch["instances"][i]["shape"][0] for i in idx})
    log(f"\n[autotune] sizes {sizes}")
    ref, plans0, _ = run(batch, idx, variants, 10)
    cache = tmp_path / "plans.jsonl"
    tuned, plans, timed = run(batch, idx, variants, 10, tune=dict(cache=cache))
    log(f"  default plans {sorted(set(plans0))}, tuned plans {plans}, groups timed {timed}")
    assert timed == len(sizes)
    for p in plans:
        assert p[0] in (8, 16) and p[1] in (8, 16)
    for a, b in zip(ref, tuned):
        assert np.array_equal(a, b)
    lines = [json.loads(l) for l in cache.read_text().splitlines()]
    assert sorted(l["nx"] for l in lines) == sizes
    for l in lines:
        assert l["ytile"] in (8, 16) and len(l["us"]) == 4 and min(l["us"]) > 0
    # a second context takes the cached plan without timing
    again, plans2, timed2 = run(batch, idx, variants, 10, tune=dict(cache=cache))
    assert timed2 == 0 and plans2 == plans
    for a, b in zip(ref, again):
        assert np.array_equal(a, b)
    # unless asked to time again (one more entry per group)
    _, _, timed3 = run(batch, idx, variants, 1, tune=dict(cache=cache, retime=True))
    assert timed3 == len(sizes)
    assert len(cache.read_text().splitlines()) == 2 * len(sizes)


def test_tuned_fixed_point_path_is_bit_identical():
    batch, idx, variants = small_batch()
    ref, _, _ = run(batch, idx, variants, 4, fixed_point=True)
    tuned, plans, timed = run(batch, idx, variants, 4, tune={}, fixed_point=True)
    log(f"\n[autotune] fixed-point path: plans {plans}")
    for a, b in zip(ref, tuned):
        assert np.array_equal(a, b)


def test_single_polycrystal_tuned_matches_untuned():
    cfg = cases.small_polycrystal()
    s0, eta0, _ = cases.gpu_run(cfg, 2, save_stress_last=False)
    s0.close()
    solver, epsp = cases.gpu_solver(cfg)
    timed = solver.autotune()
    plan = solver.plan()
    for n in range(2):
        e, s = cases.loads(cfg, n)
        solver.step(1, e, s, eps_p=epsp if n == 0 else None)
    eta1 = solver.field(binding.PF_FIELD_ETA).cpu().numpy()
    solver.close()
    log(f"\n[autotune] polycrystal 32^3: plan {plan} (0: no spectral path), groups timed {timed}")
    assert timed == 1 and plan[0] in (8, 16) and plan[1] == 0
    assert np.array_equal(eta0, eta1)
