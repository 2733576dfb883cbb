"""Write the oracle's reference trajectory of the ramped single-crystal
lamellae workload (128 x 128 x 256, parent/twin stiffness contrast,
Gaussian-random-field plastic strain, load ramped to -4e-3 over 2000 steps).

Calls only the oracle and the seeded input generator. Run from the repository
root:

    python tests/golden/make_lamellae_trajectory.py [max_steps] [--out PATH] [--state PATH]

Checkpoints are appended as the run goes (every 50 steps, stress samples
every 250 steps and after the first step), so a partial run is usable. For
each checkpoint after step n (0-based, i.e. after n+1 steps) it stores the
order parameter at fixed random voxels and at up to 2048 voxels of the
interface (0.05 < eta < 0.95), the stress of that step's equilibrium at fixed
random voxels, and the step's reductions.

The fixed point of each step starts from the cubic extrapolation of the
four previous converged strain fields (their means extrapolated alike),
linear and quadratic while fewer are known; the converged state does not
depend on the starting point beyond the tolerance, and the extrapolation
roughly halves the iterations per step.

--out writes the trajectory somewhere else than the stored file (a long run
then never replaces it with a shorter one before it ends). --state keeps the
oracle's full state (order parameter, strain, mean strain, sampling generator
and the records so far) at every checkpoint and resumes from it when it
exists; the oracle is deterministic, so a resumed run writes the same values
as an uninterrupted one.
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import crystal as cr              # noqa: E402
from oracle import mech                        # noqa: E402
from oracle import phasefield as pf            # noqa: E402
from paper_2302_13612_amd import inputs        # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lamellae_trajectory.npz")
ETA_EVERY = 50
SIG_EVERY = 250
N_SAMPLES = 2048
ORACLE_TOL = 1e-9


def _save_state(path, n, st, rng, rec, rand_idx, hist):
    tmp = path + ".tmp.npz"
    extra = {f"hist_eps{i}": h[0] for i, h in enumerate(hist)}
    extra.update({f"hist_ebar{i}": h[1] for i, h in enumerate(hist)})
    np.savez(tmp, n=n, eta=st.eta, eps=st.eps, ebar=st.ebar, rand_idx=rand_idx,
             rng=np.array(repr(rng.bit_generator.state)), n_hist=len(hist),
             **{"rec_" + k: np.asarray(v) for k, v in rec.items()}, **extra)
    os.replace(tmp, path)


def _load_state(path, rng):
    import ast
    z = np.load(path)
    rng.bit_generator.state = ast.literal_eval(str(z["rng"]))
    rec = {k[4:]: list(z[k]) for k in z.files if k.startswith("rec_")}
    st = pf.State(z["eta"], z["eps"], z["ebar"])
    nh = int(z["n_hist"]) if "n_hist" in z.files else 0
    hist = [(z[f"hist_eps{i}"], z[f"hist_ebar{i}"]) for i in range(nh)]
    return int(z["n"]), st, rec, z["rand_idx"], hist


def _extrapolate(hist):
    """Initial guess of the next fixed point from the converged (strain, mean
    strain) pairs of the previous steps, latest last."""
    if len(hist) >= 4:
        w = (-1.0, 4.0, -6.0, 4.0)      # 4 (L + P2) - 6 P - P3
    elif len(hist) == 3:
        w = (1.0, -3.0, 3.0)            # 3 (L - P) + P2
    elif len(hist) == 2:
        w = (-1.0, 2.0)                 # 2 L - P
    else:
        return hist[-1]
    tail = hist[-len(w):]
    eps = sum(c * h[0] for c, h in zip(w, tail))
    ebar = sum(c * h[1] for c, h in zip(w, tail))
    return eps, ebar


def main(max_steps, out=OUT, state_path=None):
    cfg = inputs.single_crystal_lamellae()
    shape = cfg["shape"]
    tabs = cr.mg_tables(cfg["rotations"], cfg["variant_ids"])
    C0 = pf.reference_stiffness_average(tabs[0], tabs[1])
    prob = pf.Problem(shape, cfg["dx"], tabs, cfg["A"], cfg["kappa"], cfg["L"], cfg["dt"], C0,
                      ms_tol=ORACLE_TOL, ms_max_iter=200)
    rng = np.random.Generator(np.random.PCG64(1234))
    ntot = int(np.prod(shape))
    rand_idx = np.sort(rng.choice(ntot, size=N_SAMPLES, replace=False))
    st = pf.State.initial(cfg["eta0"].astype(np.float64), np.zeros(6))
    epsp = cfg["eps_p"].astype(np.float64)
    ld = dict(stress_mask=cfg["stress_mask"])
    rec = dict(steps=[], eta_rand=[], iface_idx=[], iface_eta=[], sig_steps=[], sig_rand=[],
               eta_mean=[], sig_mean=[], G=[], ms_iters=[])
    first = 0
    hist = []
    if state_path and os.path.exists(state_path):
        last, st, rec, rand_idx, hist = _load_state(state_path, rng)
        first = last + 1
        print(f"resumed after step {last} ({len(hist)} converged fields kept)", flush=True)
    t0 = time.time()
    for n in range(first, max_steps):
        ld["eps_bar"], ld["sig_bar"] = inputs.ramp_load(cfg, n)
        if hist:
            guess, gbar = _extrapolate(hist)
            st = pf.State(st.eta, guess, gbar)
        st, stats, sigma = pf.step(prob, st, epsp, ld)
        hist = (hist + [(st.eps, st.ebar)])[-4:]
        done = n + 1
        if done % SIG_EVERY == 0 or n == 0:
            s6 = mech.tensor_to_voigt6(sigma).reshape(6, -1)
            rec["sig_steps"].append(n)
            rec["sig_rand"].append(s6[:, rand_idx].astype(np.float64))
        if done % ETA_EVERY == 0 or n == 0:
            e = st.eta[0].ravel()
            iface = np.flatnonzero((e > 0.05) & (e < 0.95))
            if iface.size > N_SAMPLES:
                iface = np.sort(rng.choice(iface, size=N_SAMPLES, replace=False))
            pad = np.full(N_SAMPLES, -1, dtype=np.int64)
            pad[:iface.size] = iface
            vals = np.zeros(N_SAMPLES)
            vals[:iface.size] = e[iface]
            rec["steps"].append(n)
            rec["eta_rand"].append(e[rand_idx])
            rec["iface_idx"].append(pad)
            rec["iface_eta"].append(vals)
            rec["eta_mean"].append(stats["eta_mean"][0])
            rec["sig_mean"].append(stats["sig_mean"])
            rec["G"].append([stats["G_dw"], stats["G_gd"], stats["G_me"]])
            rec["ms_iters"].append(stats["ms_iters"])
            arrays = {k: np.asarray(v) for k, v in rec.items()}
            tmp = out + ".tmp.npz"
            np.savez_compressed(tmp, rand_idx=rand_idx, shape=np.array(shape), **arrays)
            os.replace(tmp, out)
            if state_path:
                _save_state(state_path, n, st, rng, rec, rand_idx, hist)
            print(f"step {n} saved ({time.time() - t0:.0f} s, ms_iters {stats['ms_iters']}, "
                  f"eta_mean {stats['eta_mean'][0]:.6f})", flush=True)


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("max_steps", nargs="?", type=int, default=2000)
    ap.add_argument("--out", default=OUT)
    ap.add_argument("--state", default=None)
    a = ap.parse_args()
    main(a.max_steps, a.out, a.state)
