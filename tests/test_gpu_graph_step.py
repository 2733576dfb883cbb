"""GPU: fixed-point steps replayed as one graph, the fixed point converging on
the device.

From the fifth fixed-point step on, pf_step replays a step as one captured
graph: as many Moulinec-Suquet iterations as the last step took (iterations
past an instance's convergence return at once), then the update, which runs
only if every instance of its group converged; the host reads the flags once
per step and finishes a step that needs more iterations itself. The kernels
and their order are those of the step driven iteration by iteration (forced
here by per-launch profiling), so the results are identical bit for bit: on
a polycrystal, on a batch that mixes iterating groups with a spectral one,
and when a jump of the load makes a step need more iterations than the one
before."""

import numpy as np
import pytest

from paper_2302_13612_amd import binding, inputs
from tests import cases

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


def poly_run(cfg, steps, host_driven, jump_at=None):
    solver, epsp = cases.gpu_solver(cfg)
    if host_driven:
        solver.profile(True)
    iters = []
    for n in range(steps):
        e, s = cases.loads(cfg, n)
        if jump_at is not None and n >= jump_at:
            e = 2.0 * np.asarray(e)
        solver.step(1, e, s, eps_p=epsp if n == 0 else None)
        iters.append(solver.stats()["ms_iters"])
    eta = solver.field(binding.PF_FIELD_ETA).cpu().numpy()
    st = solver.stats()
    solver.close()
    return eta, st, iters


@pytest.mark.parametrize("jump_at", [None, 8], ids=["steady", "load-jump"])
def test_polycrystal_graph_steps_match_host_driven(jump_at):
    cfg = cases.small_polycrystal()
    steps = 12
    eta_g, st_g, it_g = poly_run(cfg, steps, False, jump_at)
    eta_h, st_h, it_h = poly_run(cfg, steps, True, jump_at)
    log(f"\n[graph step] polycrystal 32^3 {steps} steps (jump {jump_at}): iterations {it_g}, "
        f"replayed {st_g['steps_replayed']}, host-driven replayed {st_h['steps_replayed']}")
    assert st_g["steps_replayed"] >= steps - 5 and st_h["steps_replayed"] == 0
    assert it_g == it_h
    if jump_at is not None:
        assert it_g[jump_at] > it_g[jump_at - 1]   # the host finished that step
    assert np.array_equal(eta_g, eta_h)
    for k in ("G_dw", "G_gd", "G_me"):
        assert st_g[k] == st_h[k], k


def test_per_grain_tensors_graph_steps_match_host_driven():
    # the remainder's passes (gradient, flux, divergence) inside the replayed step graph,
    # the update guarded by the fixed point's flag
    cfg = dict(cases.small_polycrystal(n_var=2), aniso_grains=dict(c2n=2.81e-7, c2s=2.81e-6))
    steps = 10
    eta_g, st_g, it_g = poly_run(cfg, steps, False)
    eta_h, st_h, it_h = poly_run(cfg, steps, True)
    log(f"\n[graph step] per-grain tensors 32^3 {steps} steps: iterations {it_g}, "
        f"replayed {st_g['steps_replayed']}")
    assert st_g["steps_replayed"] >= steps - 5 and st_h["steps_replayed"] == 0
    assert it_g == it_h
    assert np.array_equal(eta_g, eta_h)
    for k in ("G_dw", "G_gd", "G_me"):
        assert st_g[k] == st_h[k], k


def mixed_batch():
    """Sizes 32 and 48 with a parent/twin contrast in one instance of each
    (those groups iterate), size 64 homogeneous (spectral path)."""
    import torch
    batch = inputs.rve_batch(n_inst=6, seed=21, sizes=(32, 48, 64))
    insts, shapes = [], []
    for i, inst in enumerate(batch["instances"]):
        v = cases.max_sf_variant(inst["rotation"])
        Cg, Cv, e0 = binding.mg_twin_tables(np.eye(3)[None], [v])
        contrast = inst["shape"][0] in (32, 48) and i % 2 == 0
        if not contrast:
            Cv = np.broadcast_to(Cg[:, None], Cv.shape).copy()
        insts.append(dict(eta0=torch.from_numpy(inst["eta0"]).cuda(), tables=(Cg, Cv, e0),
                          rotation=inst["rotation"]))
        shapes.append((inst["shape"][0], contrast))
    return batch, insts, shapes


def batch_run(steps, host_driven):
    batch, insts, shapes = mixed_batch()
    bs = binding.BatchSolver(insts, batch["dx"], batch["A"], batch["kappa"], batch["L"], batch["dt"],
                             batch["stress_mask"], ms_tol=1e-6, ms_max_iter=60)
    if host_driven:
        bs.profile(True)
    eb = np.stack([inst["eps_bar"] for inst in batch["instances"]])
    for _ in range(steps):
        bs.step(1, eb)
    etas = [bs.field(k, binding.PF_FIELD_ETA).cpu().numpy() for k in range(len(insts))]
    stats = [bs.stats(k) for k in range(len(insts))]
    bs.close()
    return etas, stats, shapes


def test_mixed_batch_graph_steps_match_host_driven():
    steps = 10
    eg, sg, shapes = batch_run(steps, False)
    eh, sh, _ = batch_run(steps, True)
    log(f"\n[graph step] mixed batch {shapes}: replayed {sg[0]['steps_replayed']}, "
        f"iterations {[s['ms_iters'] for s in sg]}")
    assert sg[0]["steps_replayed"] >= steps - 5
    assert any(s["ms_iters"] > 1 for s in sg)
    for a, b in zip(eg, eh):
        assert np.array_equal(a, b)
