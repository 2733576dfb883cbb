"""Benchmark of the FFT phase-field twin step on one MI355X.

Default workload: the synthetic polycrystal -- 256^3 periodic grid, 64
Voronoi grains with uniformly random orientations, all six {10-12}<-1011>
twin variants per voxel, nuclei at 5% of the grain-pair interfaces,
Gaussian-random-field plastic strain (RMS 2e-3), uniaxial applied strain -5e-3
along x, mixed mean-stress condition, fixed-point tolerance 1e-6. Inputs are
resident in HBM before timing. One step = equilibrium fixed point + driving
forces + spectral Allen-Cahn update + FP64 reductions.

--workload rve-batch: 256 independent single-crystal cubes of edge 32, 48, 64
or 96 (one twin variant each, homogeneous stiffness, own orientation and
load) advanced together for 512 steps, the order parameters of every
instance copied to a trajectory buffer every 16th step; graph replay of the
batched step.

--workload pillar | lamellae: the 128 x 128 x 256 single crystal with the
parent/twin contrast and a ramped load, inside a pad layer of low mobility
or (lamellae) without one. --workload vmap: the FE <-> FFT transfer of a
pillar mesh. --workload surrogate: the learned macro stepper, trained in the
library's kernels, then 512 steps of held-out 128^3 instances with and
without it.

Prints one JSON line on stdout; progress goes to stderr.
"""

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PF-FFT voxel-updates/s at 256³ & %HBM peak; surrogate speedup at ≤1e-3 err"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# first fixed-point iteration of a step: the forward x pass reads three more
# strain fields (the cubic extrapolated warm start) and stores the
# extrapolated iterate, which the inverse pass reads in place of the strain
EXTRAPOLATION_BYTES_PER_VOXEL = {"ms_x_forward": 96}
# stages of a polycrystal step; the dominant one is timed in the timed region
STAGES = ("ms_x_forward", "ms_y_forward", "ms_z_green", "ms_y_inverse", "ms_x_inverse",
          "ac_x_forward", "ac_y_forward", "ac_z_update", "ac_y_inverse", "ac_x_inverse")
DOMINANT = "ms_x_forward"
# Table 5: gradient coefficient c2 along the twin-plane normal / shear direction
C2N, C2S = 2.81e-7, 2.81e-6


# the sources the phase-field step's kernels and their launches are built from
STEP_SOURCES = ("fft_engine.hpp", "pf_common.hpp", "pf_device.hpp", "pf_kernels.hip", "pf_xv.hip", "pf_api.cpp")


def sources_digest():
    """SHA-256 over the sources of the step's kernels: counter-based traffic
    is only reported for the kernels it was measured on."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2302_13612_amd", "csrc")
    for name in STEP_SOURCES:
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel, grid, n_var, window):
    """HBM bytes per launch of a stage from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, calibrated by a device copy), or None
    if absent, or taken on other sources, on another grid or variant count, or
    over another window of steps (warm-up, timed): the per-launch average
    depends on the window through the share of first iterations."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256") != sources_digest():
        return None
    if t.get("grid") != list(grid) or t.get("n_var") != n_var or t.get("window") != list(window):
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k["fetch_bytes"] + k["write_bytes"]


def kernel_bytes(name, nx, ny, nz, V, multigrain, save_stress=False):
    """Algorithmic HBM bytes of one launch of a named stage (compulsory reads
    and writes of fields and spectra; tables and partials are negligible)."""
    nvox = nx * ny * nz
    nspec = (nx // 2 + 1) * ny * nz
    fields_in = (6 + V + 6) * 4 * nvox + (nvox if multigrain else 0)
    table = {
        "ms_x_forward": fields_in + 6 * 8 * nspec,
        "ms_y_forward": 2 * 6 * 8 * nspec,
        "ms_z_green": 2 * 6 * 8 * nspec,
        "ms_y_inverse": 2 * 6 * 8 * nspec,
        "ms_x_inverse": 6 * 8 * nspec + 2 * 6 * 4 * nvox,
        "ac_x_forward": fields_in + V * 8 * nspec + (6 * 4 * nvox if save_stress else 0),
        "ac_y_forward": 2 * V * 8 * nspec,
        "ac_z_update": 2 * V * 8 * nspec,
        "ac_y_inverse": 2 * V * 8 * nspec,
        "ac_x_inverse": V * 8 * nspec + V * 4 * nvox,
        # fixed point over the update: the base f^n + L dt m mech kept by the
        # first forward pass, the order parameter and base read by a further
        # one, the overwritten values read by the inverse pass (max change)
        "ac_x_forward+base": fields_in + V * 8 * nspec + V * 4 * nvox,
        "pc_x_forward": 2 * V * 4 * nvox + V * 8 * nspec,
        "ac_x_inverse+change": V * 8 * nspec + 2 * V * 4 * nvox,
        # per-grain gradient tensors: the explicit remainder's passes (gradient
        # V -> 3V spectra, flux 3V, divergence 3V added into the update's V)
        "rem_x_forward": V * 4 * nvox + V * 8 * nspec,
        "rem_y_forward": 2 * V * 8 * nspec,
        "rem_z_gradient": 4 * V * 8 * nspec,
        "rem_y_inverse3": 2 * 3 * V * 8 * nspec,
        "rem_x_flux": 2 * 3 * V * 8 * nspec + (nvox if multigrain else 0),
        "rem_y_forward3": 2 * 3 * V * 8 * nspec,
        "rem_z_divergence": 5 * V * 8 * nspec,
    }
    return table.get(name, 0)


def copy_bandwidth(torch, dev, nbytes=1 << 30, reps=10, own=False):
    """Device-to-device copy rate (bytes read + written per second) of a
    1 GiB buffer, by torch's copy or (own) by the library's streaming copy
    kernel (16 bytes per lane, nontemporal hints): the bandwidth a kernel
    that only moves bytes reaches on this device, reported beside the
    datasheet peak. Events on the stream both copies run on."""
    from paper_2302_13612_amd import binding
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)

    def copy():
        if own:
            binding.stream_copy(dst, src)
        else:
            dst.copy_(src)
    copy()
    s = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        copy()
    e1.record(s)
    e1.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def cpu_info():
    cores = len(os.sched_getaffinity(0))
    model = "unknown"
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    return cores, model


def library_load_variants(binding, n_var):
    """variant_for of the polycrystal recipe through the library's Mg tables:
    per grain the variant whose eigenstrain does the most work against the
    applied mean strain, eps_bar : eps0_a (for uniaxial compression the
    largest Schmid factor)."""
    def pick(R, eps_bar):
        _, _, e0 = binding.mg_twin_tables(np.asarray(R), list(range(n_var)))   # (G, V, 6) tensor-Voigt
        w = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 2.0]) * np.asarray(eps_bar, dtype=np.float64)
        return np.argmax(e0 @ w, axis=1)
    return pick


def oracle_load_variants(n_var):
    """The same choice from the oracle's crystallography (CPU baseline leg)."""
    from oracle import crystal as cr
    from oracle import mech

    def pick(R, eps_bar):
        _, _, e0 = cr.mg_tables(np.asarray(R), list(range(n_var)))
        eb = mech.voigt6_to_tensor(np.asarray(eps_bar, dtype=np.float64))
        return np.argmax(np.einsum("gaij,ij->ga", e0, eb), axis=1)
    return pick


def cpu_baseline(n=256, iters_per_step=None, pf_max_iter=1, pf_tol=1e-6, aniso=False):
    """The FP64 oracle, as it stands, on the same recipe at n^3: one step with
    a single fixed-point iteration (that iteration, the stress of the result,
    the driving forces, the update and the statistics), and one more
    iteration of the fixed point alone (constitutive law, forward transform,
    Green's operator, inverse transform). The oracle's step time is formed
    with the fixed-point iterations per step the GPU measured in the same run,
    step = t_step(1 iteration) + (K - 1) t_iteration, so both sides are priced
    for the same work."""
    from oracle import crystal as cr
    from oracle import mech
    from oracle import phasefield as opf
    from paper_2302_13612_amd import inputs
    cfg = inputs.polycrystal(shape=(n, n, n), variant_for=oracle_load_variants(6))
    tabs = cr.mg_tables(cfg["rotations"], cfg["variant_ids"])
    C0 = opf.reference_stiffness_average(tabs[0], tabs[1])
    kg = cr.twin_gradient_tensors(cfg["rotations"], cfg["variant_ids"]) if aniso else None
    prob = opf.Problem(cfg["shape"], cfg["dx"], tabs, cfg["A"], cfg["kappa"], cfg["L"], cfg["dt"], C0,
                       gid=cfg["gid"], ms_tol=cfg["ms_tol"], ms_max_iter=1,
                       pf_tol=pf_tol, pf_max_iter=pf_max_iter, kappa_grain=kg)
    st = opf.State.initial(cfg["eta0"].astype(np.float64), np.zeros(6))
    epsp6 = cfg["eps_p"].astype(np.float64)
    ld = dict(eps_bar=cfg["eps_bar"], sig_bar=cfg["sig_bar"], stress_mask=cfg["stress_mask"])
    t0 = time.perf_counter()
    new, stats, _ = opf.step(prob, st, epsp6, ld)
    t_step1 = time.perf_counter() - t0
    # one more iteration of the fixed point from the strain the step reached
    eps_p = mech.voigt6_to_tensor(epsp6)
    t0 = time.perf_counter()
    _, _, sigma = mech.eigenstrain_and_stress(new.eps, st.eta, eps_p, prob.gid, *prob.tables, prob.h_kind)
    deps = -mech.ifft_tensor(prob.green.apply(mech.fft_tensor(sigma)), prob.shape)
    t_iter = time.perf_counter() - t0
    del deps, sigma
    K = float(iters_per_step) if iters_per_step else 1.0
    t_step = t_step1 + (K - 1.0) * t_iter
    cores, model = cpu_info()
    return {
        "value": n ** 3 / t_step, "unit": "voxel-updates/s", "cores": cores, "kind": "oracle",
        "sample": f"the oracle on the same polycrystal recipe at {n}^3 (64 grains, 6 variants): one step with one "
                  f"fixed-point iteration {t_step1:.1f} s and one further iteration {t_iter:.1f} s, "
                  f"priced at the GPU's {K:.2f} iterations per step ({t_step:.1f} s per step)"
                  + (f", update fixed point tol {pf_tol:g}, {stats['pf_iters']} solves" if pf_max_iter > 1 else "")
                  + (", anisotropic gradient energy per grain" if aniso else "")
                  + f", on {model}",
        "s_per_iteration": round(t_iter, 2), "s_per_step_one_iteration": round(t_step1, 2),
        "iterations_per_step": round(K, 3),
    }


def kh_bytes(name, groups, V=1):
    """Algorithmic HBM bytes of one step of a spectral-path stage, summed over
    the size groups of a batch: groups = [(edge, n_instances)]."""
    tot = 0
    for n, k in groups:
        nvox = n ** 3 * k
        nspec = (n // 2 + 1) * n * n * k
        tot += {
            "kh_x_forward": V * 4 * nvox + 2 * V * 8 * nspec,
            "kh_y_forward": 2 * 2 * V * 8 * nspec,
            "kh_z_update": 2 * V * 8 * nspec + V * 8 * nspec,
            "kh_y_inverse": 2 * V * 8 * nspec,
            "kh_x_inverse": V * 8 * nspec + V * 4 * nvox,
        }.get(name, 0)
    return tot


def oracle_rve_baseline(batch, variants, sizes_count, aniso=False):
    """Oracle per-step time of one instance of each size, extrapolated to the
    batch (sum over instances of the per-size time)."""
    from oracle import crystal as cr
    from oracle import phasefield as opf
    t_size = {}
    for n in sorted(sizes_count):
        i = next(k for k, inst in enumerate(batch["instances"]) if inst["shape"][0] == n)
        inst = batch["instances"][i]
        Cg, Cv, e0 = cr.mg_tables(inst["rotation"][None], [variants[i]])
        Cv = np.broadcast_to(Cg[:, None], Cv.shape).copy()
        C0 = opf.reference_stiffness_average(Cg, Cv)
        kv = cr.twin_gradient_tensors(inst["rotation"][None], [variants[i]], c2n=C2N, c2s=C2S)[0] if aniso else None
        prob = opf.Problem(inst["shape"], batch["dx"], (Cg, Cv, e0), batch["A"], batch["kappa"], batch["L"],
                           batch["dt"], C0, ms_tol=batch["ms_tol"], ms_max_iter=batch["ms_max_iter"],
                           kappa_var=kv)
        st = opf.State.initial(inst["eta0"].astype(np.float64), np.zeros(6))
        ld = dict(eps_bar=inst["eps_bar"], sig_bar=batch["sig_bar"], stress_mask=batch["stress_mask"])
        opf.step(prob, st, None, ld)  # warm (plans, caches)
        t0 = time.perf_counter()
        opf.step(prob, st, None, ld)
        t_size[n] = time.perf_counter() - t0
    t_batch = sum(t_size[n] * c for n, c in sizes_count.items())
    nvox = sum(n ** 3 * c for n, c in sizes_count.items())
    cores, model = cpu_info()
    return {
        "value": nvox / t_batch, "unit": "voxel-updates/s", "cores": cores, "kind": "oracle",
        "sample": "one oracle step per instance size (" +
                  ", ".join(f"{n}^3: {t_size[n]:.2f} s" for n in sorted(t_size)) +
                  f") on {model}, extrapolated to the batch's instance counts",
    }


def bench_rve_batch(args):
    import torch
    from paper_2302_13612_amd import binding, inputs
    batch = inputs.rve_batch()
    insts = batch["instances"]
    nb = len(insts)
    # twin variant most favoured by compression along x: the most negative
    # sample-frame eps0_xx among the six (library tables)
    variants = []
    for inst in insts:
        _, _, e0 = binding.mg_twin_tables(inst["rotation"][None], list(range(6)))
        variants.append(int(np.argmin(e0[0, :, 0])))
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    specs = []
    for inst, v in zip(insts, variants):
        Cg, Cv, e0 = binding.mg_twin_tables(np.eye(3)[None], [v])
        Cv = np.broadcast_to(Cg[:, None], Cv.shape).copy()
        sp = dict(eta0=torch.from_numpy(inst["eta0"]).to(dev), tables=(Cg, Cv, e0), rotation=inst["rotation"])
        if args.aniso:
            # gradient tensors of Table 5 (c2 along the normal and the shear
            # direction of the instance's variant), sample frame
            sp["kappa_var"] = binding.mg_twin_gradient(inst["rotation"][None], [v], c2n=C2N, c2s=C2S)[0]
        specs.append(sp)
    offs = np.cumsum([0] + [inst["eta0"].size for inst in insts])
    nvox = int(offs[-1])
    log(f"batch of {nb} instances, {nvox / 1e6:.1f} M voxels")
    bs = binding.BatchSolver(specs, batch["dx"], batch["A"], batch["kappa"], batch["L"], batch["dt"],
                             batch["stress_mask"], ms_tol=batch["ms_tol"], ms_max_iter=batch["ms_max_iter"])
    eta0_all = [sp["eta0"] for sp in specs]
    del specs
    log(f"workspace {bs.workspace.numel() / 2**30:.2f} GiB")
    plans, timed, tune_ms = {}, 0, 0.0
    if not args.no_tune:
        t0 = time.perf_counter()
        timed = bs.autotune(cache=args.tune_cache)
        tune_ms = 1e3 * (time.perf_counter() - t0)
        for i, inst in enumerate(insts):
            plans.setdefault(str(inst["shape"][0]), bs.plan(i))
        log(f"autotuned {timed} size groups in {tune_ms:.0f} ms: plans {plans}")
    eb = np.stack([inst["eps_bar"] for inst in insts])
    steps = args.steps if args.steps_given else batch["steps"]
    every = batch["save_every"]
    nsnap = steps // every + 1
    traj = torch.empty((nsnap, nvox), dtype=torch.float32, device=dev)
    log(f"trajectory buffer {traj.numel() * 4 / 2**30:.2f} GiB ({nsnap} snapshots)")

    def snapshot(k):
        for i in range(nb):
            bs.field(i, binding.PF_FIELD_ETA, out=traj[k, offs[i]:offs[i + 1]])

    # warm-up (captures the step graph), then back to the initial state
    bs.step(max(1, args.warmup), eb)
    for i in range(nb):
        bs.set_field(i, binding.PF_FIELD_ETA, eta0_all[i])
    torch.cuda.synchronize()
    log(f"timing {steps} steps, snapshot every {every}")
    t0 = time.perf_counter()
    snapshot(0)
    for k in range(1, nsnap):
        bs.step(every, eb)
        snapshot(k)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    value = nvox * steps / elapsed
    log(f"{1e3 * elapsed / steps:.3f} ms/step, {value:.3e} voxel-updates/s")
    fin = [bs.stats(i) for i in (0, nb - 1)]
    # per-kernel times: a few more steps with events (direct launches, no graph)
    bs.profile(True)
    nprof = 8
    bs.step(nprof, eb)
    prof = bs.profile_read()
    bs.profile(False)
    bs.close()
    sizes_count = {}
    for inst in insts:
        sizes_count[inst["shape"][0]] = sizes_count.get(inst["shape"][0], 0) + 1
    groups = sorted(sizes_count.items())
    rows = []
    total_ms = sum(v[1] for v in prof.values())
    for name, (cnt, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        b = kh_bytes(name, groups) * nprof
        gbs = b / (ms * 1e-3) / 1e9 if b else 0.0
        rows.append((name, cnt, ms, gbs, b))
        log(f"  {name:22s} {cnt:5d} x {1e3 * ms / cnt:9.1f} us  {100 * ms / total_ms:5.1f}%  "
            f"{gbs:8.1f} GB/s ({100 * gbs / HBM_PEAK_GBS:5.1f}% of HBM)")
    dom = next(r for r in rows if r[4] > 0)
    step_bytes = sum(kh_bytes(nm, groups) for nm in ("kh_x_forward", "kh_y_forward", "kh_z_update",
                                                     "kh_y_inverse", "kh_x_inverse"))
    ms_step = 1e3 * elapsed / steps
    out = {
        "metric": "PF-FFT voxel-updates/s, batch of 256 RVEs (edges 32-96), graph replay" +
                  (", anisotropic gradient energy" if args.aniso else ""),
        "value": value, "unit": "voxel-updates/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"rve-batch: {nb} single-crystal cubes, " +
                               ", ".join(f"{n}^3 x{c}" for n, c in groups) +
                               f", 1 variant, homogeneous stiffness, {nsnap} snapshots of eta",
                   "voxels": nvox, "path": "homogeneous spectral",
                   "plans": plans, "groups_timed": timed, "tune_ms": round(tune_ms, 1),
                   "gradient_energy": (f"anisotropic per variant, c2 {C2N:g} (normal) / {C2S:g} (shear) N"
                                       if args.aniso else f"isotropic, kappa {batch['kappa']:g} J/m")},
        "roofline": {"bound": "hbm", "kernel": dom[0], "achieved": round(dom[3], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(dom[3] / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_step": kh_bytes(dom[0], groups),
                     "step_algorithmic_GBs": round(step_bytes / (ms_step * 1e-3) / 1e9, 1),
                     "step_frac": round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "final_eta_mean": [float(f["eta_mean"][0]) for f in fin],
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, one step per size)")
        out["cpu_baseline"] = oracle_rve_baseline(batch, variants, sizes_count, aniso=args.aniso)
    print(json.dumps(out), flush=True)


def bench_surrogate(args):
    """Learned macro stepper: train on the batched-RVE trajectories, then
    advance held-out 128^3 instances by 512 steps with the stepper (16 steps
    per call, residual check, fallback to plain steps) and without it."""
    import torch
    from paper_2302_13612_amd import binding, inputs, surrogate
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    train_batch = inputs.rve_batch()
    trajs, conds = surrogate.generate_trajectories(binding, torch, train_batch, dev, log=log)
    # trained by the library's kernels alone (forward, backward, Adam)
    trainer = surrogate.NativeTrainer(torch, binding, surrogate.init_params(), dev)
    info = surrogate.train_native(torch, trainer, trajs, conds, seconds=args.train_seconds, log=log)
    params = trainer.params()
    del trainer
    info["trainer"] = "library kernels (forward, backward, Adam)"
    del trajs
    torch.cuda.empty_cache()
    held = inputs.rve_batch(n_inst=args.eval_instances, seed=99, sizes=(128,))
    calls, per = held["steps"] // 16, 16
    results = []
    for i, inst in enumerate(held["instances"]):
        v, cond = surrogate.variant_and_cond(binding, inst["rotation"], inst["eps_bar"][0])
        Cg, Cv, e0 = binding.mg_twin_tables(inst["rotation"][None], [v])
        Cv = np.broadcast_to(Cg[:, None], Cv.shape).copy()

        def solver():
            return binding.Solver(torch.from_numpy(inst["eta0"]).to(dev), held["dx"], held["A"], held["kappa"],
                                  held["L"], held["dt"], (Cg, Cv, e0), held["stress_mask"],
                                  ms_tol=held["ms_tol"], ms_max_iter=held["ms_max_iter"])

        eb, sb = inst["eps_bar"], held["sig_bar"]
        # plain stepping (graph replay), snapshots every 16 steps
        sp = solver()
        sp.step(per, eb, sb)  # warm-up: graph capture
        sp.close()
        sp = solver()
        snaps_plain = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(calls):
            sp.step(per, eb, sb)
            snaps_plain.append(sp.field(binding.PF_FIELD_ETA))
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        sp.close()
        # learned stepper with the residual check and fallback
        sf = solver()
        net = binding.Fno(sf, params)
        warm = net.forward(cond, sf.field(binding.PF_FIELD_ETA)[0])  # warm-up
        rho0 = binding.macro_residual(sf, sf.field(binding.PF_FIELD_ETA), per, eb, sb)
        del warm, rho0
        snaps_fno, reps = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(calls):
            reps.append(net.advance(1, per, cond, eb, sb, tol=args.tol))
            snaps_fno.append(sf.field(binding.PF_FIELD_ETA))
        torch.cuda.synchronize()
        t_fno = time.perf_counter() - t0
        net.close()
        sf.close()
        # the network alone (every call accepted) for its error and cost
        sa = solver()
        net = binding.Fno(sa, params)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        net.advance(1, per, cond, eb, sb, tol=float("inf"))
        torch.cuda.synchronize()
        t_call = time.perf_counter() - t0
        err_free = [float((sa.field(binding.PF_FIELD_ETA) - snaps_plain[0]).abs().max())]
        for k in range(1, calls):
            net.advance(1, per, cond, eb, sb, tol=float("inf"))
            err_free.append(float((sa.field(binding.PF_FIELD_ETA) - snaps_plain[k]).abs().max()))
        net.close()
        sa.close()
        err = [float((a - b).abs().max()) for a, b in zip(snaps_fno, snaps_plain)]
        acc = sum(r["accepted"] for r in reps)
        rhos = [r["last_rho"] for r in reps]
        res = dict(instance=i, variant=v, eps_xx=float(eb[0]), t_plain=t_plain, t_fno=t_fno,
                   speedup=t_plain / t_fno, accepted=acc, calls=calls, max_err=max(err),
                   rho_min=float(min(rhos)), rho_median=float(np.median(rhos)),
                   fno_call_plus_check_s=t_call, plain_16_steps_s=t_plain / calls,
                   free_rollout_err_first=err_free[0], free_rollout_err_last=err_free[-1])
        log(f"instance {i}: plain {t_plain * 1e3:.1f} ms, with stepper {t_fno * 1e3:.1f} ms "
            f"(speedup {res['speedup']:.3f}), accepted {acc}/{calls}, max err {res['max_err']:.2e}, "
            f"rho min/median {res['rho_min']:.2e}/{res['rho_median']:.2e}; one call + check "
            f"{t_call * 1e3:.2f} ms vs 16 plain steps {t_plain / calls * 1e3:.2f} ms; free rollout err "
            f"{err_free[0]:.2e} -> {err_free[-1]:.2e}")
        results.append(res)
    speed = float(np.mean([r["speedup"] for r in results]))
    out = {
        "metric": "surrogate speedup at <=1e-3 err (512 steps of 128^3, 16 steps per call, residual check + fallback)",
        "value": speed, "unit": "x", "n_gpus": 1, "steps": held["steps"], "warmup": 1,
        "ms_per_step": float(np.mean([r["t_fno"] for r in results])) * 1e3 / held["steps"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f32",
        "data": "synthetic",
        "config": {"workload": f"surrogate: FNO width 32, modes 12, 4 layers trained {args.train_seconds:.0f} s "
                               f"on the 256-RVE trajectories; {len(results)} held-out 128^3 instances",
                   "tol": args.tol, "training": info},
        "max_err": max(r["max_err"] for r in results),
        "instances": results,
    }
    print(json.dumps(out), flush=True)


def bench_vmap(args):
    """FE <-> FFT coupling transfer of the paper's loop (Sec. 3, Table 1):
    a pillar mesh's Gauss points inside the 128 x 128 x 256 box with a pad
    layer; per coupling step the plastic strain (6 components) goes to the
    cells and the volume fraction back to the points."""
    import torch
    from paper_2302_13612_amd import binding, inputs
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    dx = 5e-8
    shape = (256, 128, 128)
    ncell = int(np.prod(shape))
    pts = inputs.pillar_gauss_points(shape, dx, elem=4.0)
    npts = pts.shape[0]
    log(f"pillar mesh: {npts} Gauss points, grid {shape}")
    pts_d = torch.from_numpy(pts).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vm = binding.VoronoiMap(pts_d, shape, dx)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    pv = torch.from_numpy(rng.normal(size=(6, npts)).astype(np.float32)).to(dev)
    cv = torch.empty((6,) + shape, dtype=torch.float32, device=dev)
    eta = torch.from_numpy(rng.random((1,) + shape, dtype=np.float32)).to(dev)
    back = torch.empty((1, npts), dtype=torch.float32, device=dev)
    steps = args.steps if args.steps_given else 50
    for _ in range(3):
        vm.to_cells(pv, out=cv)
        vm.to_points(eta, out=back)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        vm.to_cells(pv, out=cv)
        ev[k][1].record()
        vm.to_points(eta, out=back)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    t_cells = sum(a.elapsed_time(b) for a, b in ev) / steps * 1e-3
    value = ncell * steps / elapsed
    # algorithmic bytes of the gather: the point index and 6 values per cell,
    # the point values once
    b_cells = ncell * (4 + 6 * 4) + npts * 6 * 4
    log(f"build {t_build * 1e3:.1f} ms; {1e3 * elapsed / steps:.3f} ms per coupling step, {value:.3e} cells/s; "
        f"to_cells {t_cells * 1e6:.1f} us")
    out = {
        "metric": "FE<->FFT mapping cells/s (nearest Gauss point, 6 components in, 1 back)",
        "value": value, "unit": "cells/s", "n_gpus": 1, "steps": steps, "warmup": 3,
        "ms_per_step": 1e3 * elapsed / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 values, f64 coordinates", "data": "synthetic",
        "config": {"workload": f"vmap: pillar hex mesh (elements of 4 cells, 2x2x2 Gauss points, jittered nodes), "
                               f"{npts} points, grid {shape[2]}x{shape[1]}x{shape[0]}, pad 4 cells",
                   "build_ms": round(t_build * 1e3, 2)},
        "roofline": {"bound": "hbm", "kernel": "vmap_to_cells", "achieved": round(b_cells / t_cells / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(b_cells / t_cells / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None, "bytes_per_launch": b_cells, "avg_launch_us": round(t_cells * 1e6, 1)},
    }
    if not args.no_cpu_baseline:
        from oracle import mapping as om
        sample = rng.choice(ncell, size=400, replace=False)
        cen = om.cell_centres(shape, dx).reshape(-1, 3)[sample]
        t0 = time.perf_counter()
        for c in cen:
            d2 = (pts[:, 0] - c[0]) ** 2
            d2 = d2 + (pts[:, 1] - c[1]) ** 2
            d2 = d2 + (pts[:, 2] - c[2]) ** 2
            int(np.argmin(d2))
        dt = time.perf_counter() - t0
        cores, model = cpu_info()
        out["cpu_baseline"] = {"value": 400 / dt, "unit": "cells/s", "cores": cores, "kind": "oracle",
                               "sample": f"brute-force nearest point of 400 sampled cells over all {npts} points "
                                         f"({dt:.1f} s on {model}); the transfers themselves not timed"}
    print(json.dumps(out), flush=True)


def bench_pillar(args, pad=12):
    """The paper's specimen geometry (Sec. 4): the single crystal with the
    parent/twin contrast on the 128 x 128 x 256 grid, inside a pad layer of
    very low mobility (12 cells, about 10% of the width; m = 1e-3), plastic
    strain field, strain ramped along z; steps 11-110 of the run. pad = 0:
    the same single crystal with three lamellar nuclei and no pad (the
    ramped lamellae run of the stored trajectory)."""
    import torch
    from paper_2302_13612_amd import binding, inputs
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = inputs.single_crystal_lamellae()
    nz, ny, nx = cfg["shape"]
    mob = torch.from_numpy(inputs.pad_mobility(cfg["shape"], pad=pad, m_pad=1e-3)).to(dev) if pad else None
    Cg, Cv, e0 = binding.mg_twin_tables(cfg["rotations"], cfg["variant_ids"])
    eta0 = torch.from_numpy(cfg["eta0"]).to(dev)
    epsp = torch.from_numpy(cfg["eps_p"]).to(dev)
    solver = binding.Solver(eta0, cfg["dx"], cfg["A"], cfg["kappa"], cfg["L"], cfg["dt"], (Cg, Cv, e0),
                            cfg["stress_mask"], ms_tol=cfg["ms_tol"], ms_max_iter=cfg["ms_max_iter"], mobility=mob)
    steps = args.steps if args.steps_given else 100
    warm = args.warmup if args.warmup is not None else 10
    for n in range(warm):
        e, sg = inputs.ramp_load(cfg, n)
        solver.step(1, e, sg, eps_p=epsp if n == 0 else None)
    torch.cuda.synchronize()
    solver.profile(True, only=DOMINANT)
    t0 = time.perf_counter()
    for n in range(warm, warm + steps):
        e, sg = inputs.ramp_load(cfg, n)
        solver.step(1, e, sg)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = solver.profile_read()
    solver.profile(False)
    nvox = nx * ny * nz
    value = nvox * steps / elapsed
    cnt, ms = prof[DOMINANT]
    b = kernel_bytes(DOMINANT, nx, ny, nz, 1, False) * cnt + EXTRAPOLATION_BYTES_PER_VOXEL[DOMINANT] * nvox * steps
    gbs = b / (ms * 1e-3) / 1e9
    log(f"{1e3 * elapsed / steps:.3f} ms/step, {value:.3e} voxel-updates/s, {cnt / steps:.2f} fixed-point "
        f"iterations per step; {DOMINANT} {1e3 * ms / cnt:.1f} us ({100 * gbs / HBM_PEAK_GBS:.1f}% of HBM)")
    if pad:
        metric = "PF-FFT voxel-updates/s, pillar in a pad layer of low mobility"
        workload = (f"pillar: single crystal {nx}x{ny}x{nz} with parent/twin contrast, pad {pad} cells "
                    f"at relative mobility 1e-3, GRF plastic strain RMS 1e-3, strain ramped along z, "
                    f"fixed-point tol 1e-6")
    else:
        metric = "PF-FFT voxel-updates/s, single-crystal lamellae"
        workload = (f"lamellae: single crystal {nx}x{ny}x{nz} with parent/twin contrast, 3 lamellar nuclei, "
                    f"GRF plastic strain RMS 1e-3, strain ramped along z (0 to -4e-3 over 2000 steps), "
                    f"fixed-point tol 1e-6")
    out = {
        "metric": metric, "value": value,
        "unit": "voxel-updates/s", "n_gpus": 1, "steps": steps, "warmup": warm, "ms_per_step": 1e3 * elapsed / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload, "fixed_point_iters_per_step": round(cnt / steps, 3),
                   "timed_steps": f"{warm + 1}-{warm + steps} of the run"},
        "roofline": {"bound": "hbm", "kernel": DOMINANT, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_launch": round(b / cnt), "avg_launch_us": round(1e3 * ms / cnt, 1)},
    }
    solver.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("polycrystal", "rve-batch", "surrogate", "vmap", "pillar", "lamellae"),
                    default="polycrystal")
    ap.add_argument("--train-seconds", type=float, default=240.0)
    ap.add_argument("--eval-instances", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-3, help="acceptance residual of the learned stepper")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--n", type=int, default=256, help="grid edge (default 256)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=256, help="grid edge of the oracle's timed sample")
    ap.add_argument("--aniso", action="store_true",
                    help="anisotropic gradient energy of Table 5: rve-batch, for every instance; polycrystal, "
                         "per grain (the stabilised split)")
    ap.add_argument("--pf-max-iter", type=int, default=1,
                    help="polycrystal: solves of the fixed point over the update per step (Table 1; 1: plain step)")
    ap.add_argument("--pf-tol", type=float, default=1e-6, help="its threshold on max |f^i - f^{i-1}|")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch tiles (no autotuning)")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (one JSON object per line)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one 256 MiB device copy first (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU decomposition "
              "(z slabs with one all-to-all per 3D transform, FP64 all-reduces for the means) is not built.",
              file=sys.stderr)
        sys.exit(2)
    args.steps_given = args.steps is not None
    if args.workload == "rve-batch":
        if args.warmup is None:
            args.warmup = 3
        return bench_rve_batch(args)
    if args.workload == "surrogate":
        return bench_surrogate(args)
    if args.workload == "vmap":
        return bench_vmap(args)
    if args.workload == "pillar":
        return bench_pillar(args)
    if args.workload == "lamellae":
        return bench_pillar(args, pad=0)
    # polycrystal: steps 6-25 of the 1000-step run by default (5 warm-up
    # steps, then 20 timed). The fixed-point iteration count per step falls as
    # the run settles (about 3.5 per step here, 2 later), so the line states
    # its window, the iterations per step and the time per iteration and per
    # update, which compare across windows.
    if args.steps is None:
        args.steps = 20
    if args.warmup is None:
        args.warmup = 5

    import torch
    from paper_2302_13612_amd import binding, inputs

    n = args.n
    shape = (n, n, n)
    log(f"generating polycrystal {shape}")
    t0 = time.perf_counter()
    cfg = inputs.polycrystal(shape=shape, variant_for=library_load_variants(binding, 6))
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s ({cfg['n_nuclei']} nuclei on "
        f"{cfg['n_interfaces']} interfaces)")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_probe:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 268435456 bytes read + 268435456 bytes written")
        del src, dst
    # one crystal-frame Mg material shared by the grains, turned per grain
    Cg, Cv, e0 = binding.mg_twin_tables(np.eye(3)[None], cfg["variant_ids"])
    eta0 = torch.from_numpy(cfg["eta0"]).to(dev)
    gid = torch.from_numpy(cfg["gid"]).to(dev)
    epsp = torch.from_numpy(cfg["eps_p"]).to(dev)
    # per-grain tensors of Table 5 (c2 along the twin-plane normal and the shear direction)
    kg = binding.mg_twin_gradient(cfg["rotations"], cfg["variant_ids"]) if args.aniso else None
    solver = binding.Solver(eta0, cfg["dx"], cfg["A"], cfg["kappa"], cfg["L"], cfg["dt"], (Cg, Cv, e0),
                            cfg["stress_mask"], gid=gid, ms_tol=cfg["ms_tol"], ms_max_iter=cfg["ms_max_iter"],
                            rotations=cfg["rotations"], pf_tol=args.pf_tol, pf_max_iter=args.pf_max_iter,
                            kappa_grain=kg)
    del eta0
    plan = None
    if not args.no_tune:
        solver.autotune(cache=args.tune_cache)
        plan = solver.plan()
        log(f"autotuned plan: {plan}")
    iterated = args.pf_max_iter > 1
    # with the fixed point over the update its further forward passes are
    # timed (they and the update's passes dominate the step)
    dominant = "pc_x_forward" if iterated else DOMINANT
    log("warmup")
    solver.step(1, cfg["eps_bar"], cfg["sig_bar"], eps_p=epsp)
    for _ in range(max(0, args.warmup - 1)):
        solver.step(1, cfg["eps_bar"], cfg["sig_bar"])
    torch.cuda.synchronize()
    # The timed steps carry HIP events around the launches of the dominant
    # stage only (events around every launch cost a few per cent of the step).
    log(f"timing {args.steps} steps")
    solver.profile(True, only=dominant)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if iterated:
        # one call per step: every step's statistics carry its solve count
        solves = 0
        for _ in range(args.steps):
            solver.step(1, cfg["eps_bar"], cfg["sig_bar"])
            solves += solver.stats()["pf_iters"]
    else:
        solver.step(args.steps, cfg["eps_bar"], cfg["sig_bar"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = solver.profile_read()
    solver.profile(False)
    stats = solver.stats()
    value = n ** 3 * args.steps / elapsed
    ms_step = 1e3 * elapsed / args.steps
    n_iter = prof[dominant][0]  # one launch of each fixed-point stage per iteration
    if iterated:
        log(f"{ms_step:.3f} ms/step, {value:.3e} voxel-updates/s, {solves / args.steps:.2f} update solves per "
            f"step (last step {stats['pf_iters']}, equilibrium iterations {stats['ms_iters']})")
    else:
        log(f"{ms_step:.3f} ms/step, {value:.3e} voxel-updates/s, {n_iter / args.steps:.2f} fixed-point "
            f"iterations per step (last step {stats['ms_iters']})")

    V = cfg["n_var"]
    nvox = n ** 3

    def stage_bytes(name, cnt, steps):
        # per-launch bytes, plus the warm start's extra traffic once per step
        if iterated and name in ("ac_x_forward", "ac_x_inverse"):
            name += "+base" if name == "ac_x_forward" else "+change"
        return kernel_bytes(name, n, n, n, V, True) * cnt + EXTRAPOLATION_BYTES_PER_VOXEL.get(name, 0) * nvox * steps

    cnt, ms = prof[dominant]
    b_dom = stage_bytes(dominant, cnt, args.steps)
    dom = (dominant, cnt, ms / cnt, b_dom / (ms * 1e-3) / 1e9, b_dom / cnt)
    step_bytes = sum(stage_bytes(nm, n_iter if nm.startswith("ms_") else args.steps, args.steps)
                     for nm in STAGES) / args.steps
    # per-stage breakdown (stderr only): a few more steps with every launch timed
    nprof = min(5, args.steps)
    solver.profile(True)
    solver.step(nprof, cfg["eps_bar"], cfg["sig_bar"])
    allp = solver.profile_read()
    solver.profile(False)
    if iterated or args.aniso:
        # bytes of a step from the launches each stage made in those steps
        step_bytes = sum(stage_bytes(nm, c2, nprof) for nm, (c2, _) in allp.items()) / nprof
    total_ms = sum(v[1] for v in allp.values())
    fp_iters = allp.get("ms_x_forward", (0, 0.0))[0]
    ms_iter = sum(m2 for nm, (_, m2) in allp.items() if nm.startswith("ms_")) / max(1, fp_iters)
    ms_update = sum(m2 for nm, (_, m2) in allp.items() if nm.startswith(("ac_", "pc_", "rem_"))) / nprof
    log(f"per-stage times over {nprof} further steps ({fp_iters / nprof:.2f} iterations per step): "
        f"{ms_iter:.3f} ms per fixed-point iteration, {ms_update:.3f} ms per update")
    for name, (c2, m2) in sorted(allp.items(), key=lambda kv: -kv[1][1]):
        b = stage_bytes(name, c2, nprof)
        gbs = b / (m2 * 1e-3) / 1e9 if b else 0.0
        log(f"  {name:22s} {c2:5d} x {m2 / c2 * 1e3:9.1f} us  {100 * m2 / total_ms:5.1f}%  "
            f"{gbs:8.1f} GB/s ({100 * gbs / HBM_PEAK_GBS:5.1f}% of HBM)")
    roofline = {
        "bound": "hbm",
        "kernel": dom[0],
        "achieved": round(dom[3], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(dom[3] / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(dom[0], (n, n, n), V, (args.warmup, args.steps)),
        "bytes_per_launch": round(dom[4]),
        "avg_launch_us": round(dom[2] * 1e3, 1),
        "launches": dom[1],
        "step_algorithmic_GBs": round(step_bytes / (ms_step * 1e-3) / 1e9, 1),
        "step_frac": round(step_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
    }
    copy_gbs = copy_bandwidth(torch, dev, own=True)
    torch_gbs = copy_bandwidth(torch, dev)
    roofline["copy_GBs"] = round(copy_gbs, 1)
    roofline["torch_copy_GBs"] = round(torch_gbs, 1)
    roofline["frac_of_copy"] = round(dom[3] / copy_gbs, 4)
    log(f"streaming copy {copy_gbs:.0f} GB/s (torch copy {torch_gbs:.0f}); {dom[0]} at "
        f"{100 * dom[3] / copy_gbs:.1f}% of it")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "voxel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"polycrystal {n}^3, 64 Voronoi grains, 6 twin variants, nuclei of each grain's max-Schmid "
                        f"variant on 5% of the grain-pair interfaces, GRF plastic strain "
                        f"RMS 2e-3, uniaxial -5e-3, fixed-point tol 1e-6"
                        + (f", update iterated to max change {args.pf_tol:g} (Table 1)" if iterated else "")
                        + (", anisotropic gradient energy per grain (Table 5, stabilised split)" if args.aniso
                           else ""),
            "grid": [n, n, n], "n_var": V, "n_grains": 64,
            "ms_iters_last_step": stats["ms_iters"],
            "fixed_point_iters_per_step": round(n_iter / args.steps, 3),
            "ms_per_fixed_point_iteration": round(ms_iter, 4),
            "ms_per_update": round(ms_update, 4),
            "variant_updates_per_s": value * V,
            "timed_steps": f"{args.warmup + 1}-{args.warmup + args.steps} of the run",
            "plan": plan,
        },
        "roofline": roofline,
    }
    if args.aniso:
        out["metric"] = METRIC + ", anisotropic gradient energy per grain"
    if iterated:
        out["metric"] = METRIC + ", update iterated (Table 1)"
        out["config"]["update_solves_per_step"] = round(solves / args.steps, 3)
        out["config"]["pf_max_iter"] = args.pf_max_iter
    solver.close()
    if not args.no_cpu_baseline:
        k_fp = fp_iters / nprof if iterated else n_iter / args.steps
        log(f"cpu baseline (oracle at {args.cpu_n}^3, {k_fp:.2f} iterations per step)")
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, k_fp, pf_max_iter=args.pf_max_iter, pf_tol=args.pf_tol,
                                           aniso=args.aniso)
        log(f"cpu baseline {out['cpu_baseline']['value']:.3e} voxel-updates/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
