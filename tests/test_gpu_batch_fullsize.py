"""GPU: the batched RVE ensemble at the benchmark's full size and launch
configuration: 256 independent instances of 32^3 to 96^3 in one batch,
autotuned launch tiles, one warm-up step that captures the step graph, the
order parameters set back to the initial state, then graph-replayed steps.
One instance of each grid size is compared element by element with the FP64
oracle's run of that instance alone (order parameter max-abs <= 1e-4, and
the step's reductions)."""

import numpy as np
import pytest

from paper_2302_13612_amd import binding, inputs
from tests import cases
from tests.test_gpu_batch import ETA_TOL, check_stats, log

pytestmark = pytest.mark.gpu

STEPS = 16


# the FP64 oracle side takes about half a minute (16 steps up to 96^3)
@pytest.mark.timeout(600)
def test_rve_batch_full_size_vs_oracle():
    batch = inputs.rve_batch()
    insts = batch["instances"]
    idx = list(range(len(insts)))
    variants = [cases.max_sf_variant(inst["rotation"]) for inst in insts]
    first = {}
    for i, inst in enumerate(insts):
        first.setdefault(inst["shape"][0], i)
    log(f"\n[batch full size] {len(insts)} instances, sizes {sorted(first)}; checked: {first}")
    bs = cases.gpu_batch(batch, idx, variants)
    bs.autotune()
    plans = {n: bs.plan(i) for n, i in first.items()}
    eb = np.stack([inst["eps_bar"] for inst in insts])
    bs.step(1, eb)
    import torch
    for i, inst in enumerate(insts):
        bs.set_field(i, binding.PF_FIELD_ETA, torch.from_numpy(inst["eta0"]).cuda())
    bs.step(STEPS, eb)
    got = {n: bs.field(i, binding.PF_FIELD_ETA).cpu().numpy() for n, i in first.items()}
    stats = {n: bs.stats(i) for n, i in first.items()}
    bs.close()
    log(f"  plans per size: {plans}")
    for n, i in sorted(first.items()):
        cfg = cases.batch_instance_cfg(batch, i, variants[i])
        eta_o, sig_o, stats_o = cases.oracle_run(cfg, STEPS)
        d = np.abs(got[n] - eta_o).max()
        moved = np.abs(eta_o - cfg["eta0"]).max()
        log(f"  instance {i} {cfg['shape']}: eta max-abs {d:.2e} (the run moves eta by {moved:.2f})")
        assert np.isfinite(got[n]).all()
        assert d <= ETA_TOL
        assert moved > 10 * ETA_TOL
        check_stats(stats[n], stats_o[-1], np.abs(sig_o).max())
