"""GPU: the full-size ramped single-crystal lamellae run (128 x 128 x 256,
parent/twin stiffness contrast, Gaussian-random-field plastic strain, load
ramped along z) against the FP64 oracle's stored trajectory.

tests/golden/lamellae_trajectory.npz is written by
tests/golden/make_lamellae_trajectory.py (oracle only, fixed-point tolerance
1e-9): the order parameter at 2048 fixed random voxels and at up to 2048
interface voxels every 50 steps, the stress of the first step at the random
voxels, and the reductions. The library runs the same recipe (tolerance 1e-6)
and is compared at every stored checkpoint: order parameter max-abs <= 1e-4,
stress relative L2 <= 1e-5 over the sampled voxels."""

import os

import numpy as np
import pytest

from paper_2302_13612_amd import binding, inputs
from tests import cases

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "lamellae_trajectory.npz")


def test_lamellae_trajectory_vs_stored_oracle():
    g = np.load(GOLDEN)
    steps = [int(s) for s in g["steps"]]
    last = max(steps)
    cfg = inputs.single_crystal_lamellae()
    assert tuple(g["shape"]) == tuple(cfg["shape"])
    print(f"\n[trajectory] checkpoints {steps}", flush=True)
    solver, epsp = cases.gpu_solver(cfg)
    rand_idx = g["rand_idx"]
    k = 0
    for n in range(last + 1):
        e, s = cases.loads(cfg, n)
        solver.step(1, e, s, eps_p=epsp if n == 0 else None, save_stress=(n == 0))
        if n == 0:
            sig = solver.field(binding.PF_FIELD_STRESS).cpu().numpy().reshape(6, -1)[:, rand_idx]
            ref = g["sig_rand"][0]
            r = cases.stress_rel_l2(sig, ref)
            print(f"  step 0 stress rel-L2 {r:.2e}", flush=True)
            assert r <= 1e-5
        if n == steps[k]:
            eta = solver.field(binding.PF_FIELD_ETA).cpu().numpy()[0].ravel()
            d_rand = np.abs(eta[rand_idx] - g["eta_rand"][k]).max()
            idx = g["iface_idx"][k]
            sel = idx >= 0
            d_if = np.abs(eta[idx[sel]] - g["iface_eta"][k][sel]).max() if sel.any() else 0.0
            st = solver.stats()
            print(f"  step {n}: eta max-abs random {d_rand:.2e}, interface ({sel.sum()} voxels) {d_if:.2e}, "
                  f"ms_iters {st['ms_iters']} (oracle {int(g['ms_iters'][k])})", flush=True)
            assert d_rand <= 1e-4 and d_if <= 1e-4
            k += 1
    solver.close()
