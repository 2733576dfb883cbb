"""Thin ctypes binding over libpftwin.so (C ABI in include/pf.h).

Argument marshalling only: every step of the path runs in the HIP library.
PyTorch supplies device memory (caller-owned workspace and fields) and the
HIP stream. Importing this module does not load the library; ``load()`` does,
and raises if the library has not been built.
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpftwin.so")

PF_OK, PF_EINVAL, PF_ENOMEM, PF_EDEVICE, PF_ENOCONV, PF_ENONFINITE, PF_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
PF_TUNE_RETIME = 1
ERROR_NAMES = {PF_EINVAL: "PF_EINVAL", PF_ENOMEM: "PF_ENOMEM", PF_EDEVICE: "PF_EDEVICE",
               PF_ENOCONV: "PF_ENOCONV", PF_ENONFINITE: "PF_ENONFINITE",
               PF_EUNSUPPORTED: "PF_EUNSUPPORTED"}
PF_H_LINEAR, PF_H_QUINTIC = 0, 1
PF_STEP_SAVE_STRESS, PF_STEP_FIXED_POINT = 1, 2
PF_FIELD_ETA, PF_FIELD_STRAIN, PF_FIELD_STRESS = 0, 1, 2
# pf_plan fields, in order
PLAN_FIELDS = ("ytile", "yplan", "ztile_ms", "zplan_ms", "zplan_ac", "ztile_kh", "zplan_kh")

_dp = ctypes.POINTER(ctypes.c_double)


class PfProblem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("dx", ctypes.c_double),
        ("n_var", ctypes.c_int32),
        ("A", ctypes.c_double), ("kappa", ctypes.c_double), ("L", ctypes.c_double), ("dt", ctypes.c_double),
        ("h_kind", ctypes.c_int32),
        ("n_grains", ctypes.c_int32),
        ("C_grain", _dp), ("C_var", _dp), ("eps0", _dp),
        ("grain_rot", _dp),
        ("grain_id", ctypes.c_void_p),
        ("eta0", ctypes.c_void_p),
        ("C_ref", ctypes.c_double * 36),
        ("C_ref_auto", ctypes.c_int32),
        ("ms_tol", ctypes.c_double),
        ("ms_max_iter", ctypes.c_int32),
        ("bc_stress_mask", ctypes.c_uint32),
        ("kappa_var", _dp),
        ("mobility", ctypes.c_void_p),
        ("pf_tol", ctypes.c_double),
        ("pf_max_iter", ctypes.c_int32),
        ("kappa_grain", _dp),
    ]


def _kappa_var_voigt(kappa_var, V):
    """(V, 3, 3) or (V, 6) gradient tensors -> contiguous (V, 6) tensor-Voigt."""
    k = np.asarray(kappa_var, dtype=np.float64)
    if k.shape == (V, 3, 3):
        k = np.stack([k[:, 0, 0], k[:, 1, 1], k[:, 2, 2], k[:, 1, 2], k[:, 0, 2], k[:, 0, 1]], axis=1)
    if k.shape != (V, 6):
        raise ValueError("kappa_var must be (n_var, 3, 3) or (n_var, 6)")
    return np.ascontiguousarray(k)


class PfLoad(ctypes.Structure):
    _fields_ = [
        ("eps_bar", ctypes.c_double * 6),
        ("sig_bar", ctypes.c_double * 6),
        ("eps_p", ctypes.c_void_p),
        ("flags", ctypes.c_uint32),
    ]


class PfStats(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64),
        ("G_dw", ctypes.c_double), ("G_gd", ctypes.c_double), ("G_me", ctypes.c_double),
        ("sig_mean", ctypes.c_double * 6),
        ("eps_mean", ctypes.c_double * 6),
        ("eta_mean", ctypes.c_double * 6),
        ("eta_min", ctypes.c_double), ("eta_max", ctypes.c_double),
        ("ms_iters", ctypes.c_int32),
        ("ms_residual", ctypes.c_double),
        ("pf_iters", ctypes.c_int32),
        ("pf_change", ctypes.c_double),
        ("steps_replayed", ctypes.c_int64),
    ]


_lib = None


def load():
    """Load libpftwin.so (once) and declare the C signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2302_13612_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32
    lib.pf_workspace_size.argtypes = [ctypes.POINTER(PfProblem), ctypes.POINTER(ctypes.c_size_t)]
    lib.pf_init.argtypes = [ctypes.POINTER(PfProblem), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.pf_step.argtypes = [vp, i32, ctypes.POINTER(PfLoad)]
    lib.pf_fields.argtypes = [vp, i32, i32, vp]
    lib.pf_stats_get.argtypes = [vp, ctypes.POINTER(PfStats)]
    lib.pf_fft.argtypes = [vp, i32, i32, vp, vp]
    lib.pf_profile_enable.argtypes = [vp, i32]
    lib.pf_profile_read.argtypes = [vp, i32, vp, ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)]
    lib.pf_profile_select.argtypes = [vp, ctypes.c_char_p]
    lib.pf_autotune.argtypes = [vp, ctypes.c_char_p, u32, ctypes.POINTER(i32)]
    sz = ctypes.c_size_t
    lib.pf_specconv_workspace_size.argtypes = [i32] * 6 + [ctypes.POINTER(sz)]
    lib.pf_specconv_forward.argtypes = [i32] * 6 + [vp] * 6 + [sz, vp]
    lib.pf_specconv_backward.argtypes = [i32] * 6 + [vp] * 8 + [sz, vp]
    i64, f32 = ctypes.c_int64, ctypes.c_float
    lib.pf_nt_lift.argtypes = [i32, i32, i64] + [vp] * 6
    lib.pf_nt_layer_forward.argtypes = [i32, i32, i64] + [vp] * 7
    lib.pf_nt_project_forward.argtypes = [i32, i32, i32, i64, vp, vp, vp, f32, vp, vp, vp, vp, vp]
    lib.pf_nt_project_backward.argtypes = [i32, i32, i32, i64, vp, vp, vp, vp, vp, f32, vp, vp, vp, vp, vp]
    lib.pf_nt_gelu_backward.argtypes = [i64, vp, vp, vp, vp]
    lib.pf_nt_layer_input_grad.argtypes = [i32, i32, i64] + [vp] * 5
    lib.pf_nt_outer_workspace.argtypes = [i32, i32, i32, i64, ctypes.POINTER(sz)]
    lib.pf_nt_outer_sum.argtypes = [i32, i32, i32, i64, vp, vp, vp, i32, vp, sz, vp]
    lib.pf_nt_outer_sum_noalloc.argtypes = [i32, i32, i32, i64, vp, vp, vp, i32, vp]
    lib.pf_nt_cond_grad.argtypes = [i32, i32] + [vp] * 5
    lib.pf_nt_adam.argtypes = [i64, vp, vp, vp, vp, f32, f32, f32, f32, i32, vp]
    lib.pf_batch_plan.argtypes = [vp, i32, ctypes.POINTER(PfPlan)]
    lib.pf_batch_set_plan.argtypes = [vp, i32, ctypes.POINTER(PfPlan)]
    lib.pf_fft_plan.argtypes = [i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.pf_vmap_workspace_size.argtypes = [i32, i32, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.pf_vmap_build.argtypes = [i32, i32, i32, ctypes.c_double, i32, vp, vp, ctypes.c_size_t, vp, vp]
    lib.pf_vmap_to_cells.argtypes = [ctypes.c_int64, vp, i32, i32, vp, vp, vp]
    lib.pf_vmap_to_points.argtypes = [i32, i32, i32, ctypes.c_double, vp, i32, vp, i32, vp, vp, vp,
                                      ctypes.c_size_t, vp]
    lib.pf_destroy.argtypes = [vp]
    lib.pf_last_error.argtypes = [vp]
    lib.pf_last_error.restype = ctypes.c_char_p
    lib.pf_mg_twin_tables.argtypes = [_dp, ctypes.c_double, ctypes.c_double, i32, _dp, i32,
                                      ctypes.POINTER(i32), _dp, _dp, _dp]
    lib.pf_mg_twin_gradient.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        i32, _dp, i32, ctypes.POINTER(i32), _dp]
    lib.pf_batch_workspace_size.argtypes = [ctypes.POINTER(PfProblem), i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.pf_batch_init.argtypes = [ctypes.POINTER(PfProblem), i32, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.pf_batch_step.argtypes = [vp, i32, ctypes.POINTER(PfLoad)]
    lib.pf_batch_fields.argtypes = [vp, i32, i32, i32, vp]
    lib.pf_batch_stats.argtypes = [vp, i32, ctypes.POINTER(PfStats)]
    lib.pf_batch_size.argtypes = [vp]
    for name in ("pf_workspace_size", "pf_init", "pf_step", "pf_fields", "pf_stats_get", "pf_fft",
                 "pf_profile_enable", "pf_profile_read", "pf_profile_select", "pf_destroy",
                 "pf_mg_twin_tables", "pf_mg_twin_gradient", "pf_vmap_workspace_size", "pf_vmap_build",
                 "pf_vmap_to_cells", "pf_vmap_to_points",
                 "pf_batch_workspace_size", "pf_batch_init", "pf_batch_step", "pf_batch_fields",
                 "pf_batch_stats", "pf_batch_size"):
        getattr(lib, name).restype = ctypes.c_int
    _ = u32
    _lib = lib
    return lib


class PfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def _ptr(a):
    return a.ctypes.data_as(_dp)


def mg_twin_tables(rotations, variant_ids, C_hex=(59.4e9, 25.6e9, 21.4e9, 61.6e9, 16.4e9),
                   c_over_a=1.633, gamma_tw=0.129):
    """Sample-frame (C_grain, C_var, eps0) tables computed by the library."""
    lib = load()
    R = np.ascontiguousarray(np.asarray(rotations, dtype=np.float64).reshape(-1, 3, 3))
    G, V = R.shape[0], len(variant_ids)
    ids = (ctypes.c_int32 * V)(*[int(v) for v in variant_ids])
    Ch = np.ascontiguousarray(np.asarray(C_hex, dtype=np.float64))
    Cg = np.zeros((G, 6, 6))
    Cv = np.zeros((G, V, 6, 6))
    e0 = np.zeros((G, V, 6))
    rc = lib.pf_mg_twin_tables(_ptr(Ch), c_over_a, gamma_tw, G, _ptr(R), V, ids, _ptr(Cg), _ptr(Cv), _ptr(e0))
    if rc != PF_OK:
        raise PfError(rc, "pf_mg_twin_tables")
    return Cg, Cv, e0


def mg_twin_gradient(rotations, variant_ids, c2n=2.81e-7, c2s=2.81e-6, c2t=None, c_over_a=1.633):
    """Sample-frame anisotropic gradient tensors (G, V, 6) computed by the
    library (c2t defaults to c2n)."""
    lib = load()
    R = np.ascontiguousarray(np.asarray(rotations, dtype=np.float64).reshape(-1, 3, 3))
    G, V = R.shape[0], len(variant_ids)
    ids = (ctypes.c_int32 * V)(*[int(v) for v in variant_ids])
    out = np.zeros((G, V, 6))
    rc = lib.pf_mg_twin_gradient(c_over_a, c2n, c2s, c2n if c2t is None else c2t, G, _ptr(R), V, ids, _ptr(out))
    if rc != PF_OK:
        raise PfError(rc, "pf_mg_twin_gradient")
    return out


def stress_mask_bits(mask):
    return int(sum(1 << i for i, m in enumerate(mask) if m))


def _fill_load(ld, eps_bar, sig_bar, eps_p_ptr, flags):
    for i in range(6):
        ld.eps_bar[i] = float(eps_bar[i])
        ld.sig_bar[i] = 0.0 if sig_bar is None else float(sig_bar[i])
    ld.eps_p = eps_p_ptr
    ld.flags = flags


def _stats_dict(s, n_var):
    return {
        "step": s.step, "G_dw": s.G_dw, "G_gd": s.G_gd, "G_me": s.G_me,
        "G": s.G_dw + s.G_gd + s.G_me,
        "sig_mean": np.array(s.sig_mean[:]), "eps_mean": np.array(s.eps_mean[:]),
        "eta_mean": np.array(s.eta_mean[:n_var]),
        "eta_min": s.eta_min, "eta_max": s.eta_max,
        "ms_iters": s.ms_iters, "ms_residual": s.ms_residual,
        "pf_iters": s.pf_iters, "pf_change": s.pf_change, "steps_replayed": s.steps_replayed,
    }


def _autotune(obj, cache, retime):
    n = ctypes.c_int32()
    path = None if cache is None else os.fspath(cache).encode()
    obj._check(obj.lib.pf_autotune(obj.ctx, path, PF_TUNE_RETIME if retime else 0, ctypes.byref(n)), "pf_autotune")
    return n.value


class PfPlan(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in PLAN_FIELDS]


def _plan(obj, inst):
    p = PfPlan()
    obj._check(obj.lib.pf_batch_plan(obj.ctx, inst, ctypes.byref(p)), "pf_batch_plan")
    return {name: getattr(p, name) for name in PLAN_FIELDS}


def _set_plan(obj, inst, plan):
    p = PfPlan(**{name: int(plan[name]) for name in PLAN_FIELDS})
    obj._check(obj.lib.pf_batch_set_plan(obj.ctx, inst, ctypes.byref(p)), "pf_batch_set_plan")


def fft_plan(n, variant):
    """(elements per thread, radices of the stages) of FFT plan variant
    `variant` on an axis of length n."""
    lib = load()
    e, ns = ctypes.c_int32(), ctypes.c_int32()
    r = (ctypes.c_int32 * 8)()
    rc = lib.pf_fft_plan(n, variant, ctypes.byref(e), r, ctypes.byref(ns))
    if rc != PF_OK:
        raise PfError(rc, f"pf_fft_plan({n}, {variant})")
    return e.value, [r[i] for i in range(ns.value)]


class Solver:
    """One phase-field context on the current torch CUDA device and stream.

    eta0: torch float32 CUDA tensor (n_var, nz, ny, nx). gid: torch uint8 CUDA
    tensor (nz, ny, nx) or None. Tables are numpy float64 (G,6,6), (G,V,6,6),
    (G,V,6). C_ref: 6x6 numpy or None for the mean of all stiffnesses.
    rotations: optional (G,3,3) crystal->sample rotations; then the tables
    hold one crystal-frame material (leading dimension 1) shared by all grains.
    kappa_var: optional (V,3,3) or (V,6) anisotropic gradient tensors (sample
    frame; one grain only). mobility: optional float32 CUDA tensor (nz, ny, nx)
    of relative mobilities in [0, 1]. pf_max_iter > 1: the fixed point over the
    update (Table 1), stopping at max |f^i - f^{i-1}| <= pf_tol. kappa_grain:
    optional (G,V,3,3) or (G,V,6) per-grain gradient tensors of a polycrystal
    (see pf_problem.kappa_grain).
    """

    def __init__(self, eta0, dx, A, kappa, L, dt, tables, stress_mask, gid=None, C_ref=None,
                 h_kind=PF_H_LINEAR, ms_tol=1e-6, ms_max_iter=50, rotations=None, kappa_var=None,
                 mobility=None, pf_tol=1e-6, pf_max_iter=1, kappa_grain=None):
        import torch
        self.lib = load()
        self.torch = torch
        if eta0.dtype != torch.float32 or not eta0.is_cuda or eta0.dim() != 4:
            raise ValueError("eta0 must be a float32 CUDA tensor (n_var, nz, ny, nx)")
        eta0 = eta0.contiguous()
        V, nz, ny, nx = eta0.shape
        Cg, Cv, e0 = (np.ascontiguousarray(np.asarray(t, dtype=np.float64)) for t in tables)
        G = Cg.shape[0]
        if Cv.shape != (G, V, 6, 6) or e0.shape != (G, V, 6):
            raise ValueError("table shapes do not match n_var / n_grains")
        rot = None
        if rotations is not None:
            rot = np.ascontiguousarray(np.asarray(rotations, dtype=np.float64).reshape(-1, 3, 3))
            if G != 1:
                raise ValueError("with rotations the tables hold one crystal-frame material")
            G = rot.shape[0]
        self._keep = [Cg, Cv, e0, eta0, rot]
        p = PfProblem()
        p.nx, p.ny, p.nz = nx, ny, nz
        p.dx = dx
        p.n_var = V
        p.A, p.kappa, p.L, p.dt = A, kappa, L, dt
        p.h_kind = h_kind
        p.n_grains = G
        p.C_grain, p.C_var, p.eps0 = _ptr(Cg), _ptr(Cv), _ptr(e0)
        p.grain_rot = _ptr(rot) if rot is not None else None
        if gid is not None:
            if gid.dtype != torch.uint8 or not gid.is_cuda or tuple(gid.shape) != (nz, ny, nx):
                raise ValueError("gid must be a uint8 CUDA tensor (nz, ny, nx)")
            gid = gid.contiguous()
            self._keep.append(gid)
            p.grain_id = gid.data_ptr()
        else:
            p.grain_id = None
        p.eta0 = eta0.data_ptr()
        if C_ref is None:
            p.C_ref_auto = 1
        else:
            p.C_ref_auto = 0
            for i, v in enumerate(np.asarray(C_ref, dtype=np.float64).ravel()):
                p.C_ref[i] = v
        p.ms_tol = ms_tol
        p.ms_max_iter = ms_max_iter
        p.bc_stress_mask = stress_mask_bits(stress_mask)
        if kappa_var is not None:
            kv = _kappa_var_voigt(kappa_var, V)
            self._keep.append(kv)
            p.kappa_var = _ptr(kv)
        else:
            p.kappa_var = None
        if mobility is not None:
            if mobility.dtype != torch.float32 or not mobility.is_cuda or tuple(mobility.shape) != (nz, ny, nx):
                raise ValueError("mobility must be a float32 CUDA tensor (nz, ny, nx)")
            mobility = mobility.contiguous()
            self._keep.append(mobility)
            p.mobility = mobility.data_ptr()
        else:
            p.mobility = None
        p.pf_tol = pf_tol
        p.pf_max_iter = pf_max_iter
        if kappa_grain is not None:
            kg = np.asarray(kappa_grain, dtype=np.float64)
            kg = np.ascontiguousarray(_kappa_var_voigt(kg.reshape((-1,) + kg.shape[2:]), kg.shape[0] * V))
            if kg.shape[0] != G * V:
                raise ValueError("kappa_grain must be (n_grains, n_var, 3, 3) or (n_grains, n_var, 6)")
            self._keep.append(kg)
            p.kappa_grain = _ptr(kg)
        else:
            p.kappa_grain = None
        nbytes = ctypes.c_size_t()
        rc = self.lib.pf_workspace_size(ctypes.byref(p), ctypes.byref(nbytes))
        if rc != PF_OK:
            raise PfError(rc, "pf_workspace_size")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=eta0.device)
        self.shape = (nz, ny, nx)
        self.n_var = V
        self.stream = torch.cuda.current_stream(eta0.device)
        ctx = ctypes.c_void_p()
        rc = self.lib.pf_init(ctypes.byref(p), self.workspace.data_ptr(), nbytes.value,
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if rc != PF_OK:
            raise PfError(rc, "pf_init (see stderr)")
        self.ctx = ctx
        self._epsp = None

    def _check(self, rc, what):
        if rc != PF_OK:
            raise PfError(rc, f"{what}: {self.lib.pf_last_error(self.ctx).decode()}")

    def step(self, n_steps, eps_bar, sig_bar=None, eps_p=None, save_stress=False, fixed_point=False):
        ld = PfLoad()
        ptr = None
        if eps_p is not None:
            t = self.torch
            if eps_p.dtype != t.float32 or not eps_p.is_cuda or tuple(eps_p.shape) != (6,) + self.shape:
                raise ValueError("eps_p must be a float32 CUDA tensor (6, nz, ny, nx)")
            self._epsp = eps_p.contiguous()
            ptr = self._epsp.data_ptr()
        flags = (PF_STEP_SAVE_STRESS if save_stress else 0) | (PF_STEP_FIXED_POINT if fixed_point else 0)
        _fill_load(ld, eps_bar, sig_bar, ptr, flags)
        self._check(self.lib.pf_step(self.ctx, int(n_steps), ctypes.byref(ld)), "pf_step")

    def field(self, which):
        n = self.n_var if which == PF_FIELD_ETA else 6
        out = self.torch.empty((n,) + self.shape, dtype=self.torch.float32, device=self.workspace.device)
        self._check(self.lib.pf_fields(self.ctx, which, 0, out.data_ptr()), "pf_fields")
        return out

    def set_field(self, which, buf):
        buf = buf.contiguous()
        self._check(self.lib.pf_fields(self.ctx, which, 1, buf.data_ptr()), "pf_fields")
        self.stream.synchronize()

    def stats(self):
        s = PfStats()
        self._check(self.lib.pf_stats_get(self.ctx, ctypes.byref(s)), "pf_stats_get")
        return _stats_dict(s, self.n_var)

    def fft_forward(self, real):
        t = self.torch
        real = real.contiguous()
        nc = real.shape[0]
        nz, ny, nx = self.shape
        spec = t.empty((nc, nz, ny, nx // 2 + 1), dtype=t.complex64, device=real.device)
        self._check(self.lib.pf_fft(self.ctx, 1, nc, real.data_ptr(), spec.data_ptr()), "pf_fft")
        return spec

    def fft_inverse(self, spec):
        t = self.torch
        spec = spec.clone().contiguous()
        nc = spec.shape[0]
        real = t.empty((nc,) + self.shape, dtype=t.float32, device=spec.device)
        self._check(self.lib.pf_fft(self.ctx, -1, nc, real.data_ptr(), spec.data_ptr()), "pf_fft")
        return real

    def profile(self, on=True, only=None):
        """Per-launch HIP-event timing on (reset) or off; only: time just the
        launches of that stage name."""
        self._check(self.lib.pf_profile_select(self.ctx, only.encode() if only else None), "pf_profile_select")
        self._check(self.lib.pf_profile_enable(self.ctx, 1 if on else 0), "pf_profile_enable")

    def profile_read(self):
        n = ctypes.c_int32()
        maxn = 64
        names = (ctypes.c_char * 64 * maxn)()
        counts = (ctypes.c_int64 * maxn)()
        tot = (ctypes.c_double * maxn)()
        self._check(self.lib.pf_profile_read(self.ctx, maxn, names, counts, tot, ctypes.byref(n)),
                    "pf_profile_read")
        return {names[i].value.decode(): (counts[i], tot[i]) for i in range(min(n.value, maxn))}

    def autotune(self, cache=None, retime=False):
        """Pick the launch tiles by timing (see pf_autotune); returns the
        number of groups timed (0 when the cache held the plan)."""
        return _autotune(self, cache, retime)

    def plan(self):
        """Launch plan of the column passes (dict of the pf_plan fields)."""
        return _plan(self, 0)

    def set_plan(self, plan):
        _set_plan(self, 0, plan)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.pf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchSolver:
    """A batch of independent single-grain instances in one context.

    instances: list of dicts with keys
      eta0      torch float32 CUDA tensor (n_var, nz, ny, nx)
      tables    (C_grain (1,6,6), C_var (1,V,6,6), eps0 (1,V,6)) numpy float64;
                crystal frame when "rotation" is given
      rotation  optional (3,3) crystal->sample rotation
      C_ref     optional 6x6 reference medium (default: the mean stiffness)
      kappa_var optional (V,3,3) or (V,6) anisotropic gradient tensors
                (sample frame)
    The shared parameters are keyword arguments as for Solver.
    """

    def __init__(self, instances, dx, A, kappa, L, dt, stress_mask, h_kind=PF_H_LINEAR, ms_tol=1e-6,
                 ms_max_iter=50):
        import torch
        self.lib = load()
        self.torch = torch
        n = len(instances)
        probs = (PfProblem * n)()
        self._keep = []
        self.shapes = []
        self.n_var = None
        dev = None
        for i, inst in enumerate(instances):
            eta0 = inst["eta0"]
            if eta0.dtype != torch.float32 or not eta0.is_cuda or eta0.dim() != 4:
                raise ValueError("eta0 must be a float32 CUDA tensor (n_var, nz, ny, nx)")
            eta0 = eta0.contiguous()
            dev = eta0.device
            V, nz, ny, nx = eta0.shape
            if self.n_var is None:
                self.n_var = V
            Cg, Cv, e0 = (np.ascontiguousarray(np.asarray(t, dtype=np.float64)) for t in inst["tables"])
            if Cg.shape != (1, 6, 6) or Cv.shape != (1, V, 6, 6) or e0.shape != (1, V, 6):
                raise ValueError("batched instances take one-grain tables")
            rot = inst.get("rotation")
            if rot is not None:
                rot = np.ascontiguousarray(np.asarray(rot, dtype=np.float64).reshape(1, 3, 3))
            self._keep += [Cg, Cv, e0, eta0, rot]
            p = probs[i]
            p.nx, p.ny, p.nz = nx, ny, nz
            p.dx = dx
            p.n_var = V
            p.A, p.kappa, p.L, p.dt = A, kappa, L, dt
            p.h_kind = h_kind
            p.n_grains = 1
            p.C_grain, p.C_var, p.eps0 = _ptr(Cg), _ptr(Cv), _ptr(e0)
            p.grain_rot = _ptr(rot) if rot is not None else None
            p.grain_id = None
            p.eta0 = eta0.data_ptr()
            C_ref = inst.get("C_ref")
            if C_ref is None:
                p.C_ref_auto = 1
            else:
                p.C_ref_auto = 0
                for k, v in enumerate(np.asarray(C_ref, dtype=np.float64).ravel()):
                    p.C_ref[k] = v
            p.ms_tol = ms_tol
            p.ms_max_iter = ms_max_iter
            p.bc_stress_mask = stress_mask_bits(stress_mask)
            if inst.get("kappa_var") is not None:
                kv = _kappa_var_voigt(inst["kappa_var"], V)
                self._keep.append(kv)
                p.kappa_var = _ptr(kv)
            else:
                p.kappa_var = None
            self.shapes.append((nz, ny, nx))
        nbytes = ctypes.c_size_t()
        rc = self.lib.pf_batch_workspace_size(probs, n, ctypes.byref(nbytes))
        if rc != PF_OK:
            raise PfError(rc, "pf_batch_workspace_size")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
        self.stream = torch.cuda.current_stream(dev)
        ctx = ctypes.c_void_p()
        rc = self.lib.pf_batch_init(probs, n, self.workspace.data_ptr(), nbytes.value,
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(ctx))
        if rc != PF_OK:
            raise PfError(rc, "pf_batch_init (see stderr)")
        self.ctx = ctx
        self.n = n
        self._loads = (PfLoad * n)()
        self._epsp = [None] * n

    def _check(self, rc, what):
        if rc != PF_OK:
            raise PfError(rc, f"{what}: {self.lib.pf_last_error(self.ctx).decode()}")

    def step(self, n_steps, eps_bar, sig_bar=None, eps_p=None, save_stress=False, fixed_point=False):
        """eps_bar, sig_bar: (n_inst, 6) arrays; eps_p: None or a list with a
        tensor (6, nz, ny, nx) or None per instance."""
        eb = np.asarray(eps_bar, dtype=np.float64).reshape(self.n, 6)
        sb = np.zeros((self.n, 6)) if sig_bar is None else np.asarray(sig_bar, dtype=np.float64).reshape(self.n, 6)
        flags = (PF_STEP_SAVE_STRESS if save_stress else 0) | (PF_STEP_FIXED_POINT if fixed_point else 0)
        for i in range(self.n):
            ptr = None
            if eps_p is not None and eps_p[i] is not None:
                e = eps_p[i].contiguous()
                if tuple(e.shape) != (6,) + self.shapes[i]:
                    raise ValueError("eps_p[i] must be (6, nz, ny, nx)")
                self._epsp[i] = e
                ptr = e.data_ptr()
            _fill_load(self._loads[i], eb[i], sb[i], ptr, flags)
        self._check(self.lib.pf_batch_step(self.ctx, int(n_steps), self._loads), "pf_batch_step")

    def field(self, inst, which, out=None):
        n = self.n_var if which == PF_FIELD_ETA else 6
        if out is None:
            out = self.torch.empty((n,) + self.shapes[inst], dtype=self.torch.float32, device=self.workspace.device)
        self._check(self.lib.pf_batch_fields(self.ctx, int(inst), which, 0, out.data_ptr()), "pf_batch_fields")
        return out

    def set_field(self, inst, which, buf):
        buf = buf.contiguous()
        self._check(self.lib.pf_batch_fields(self.ctx, int(inst), which, 1, buf.data_ptr()), "pf_batch_fields")
        self.stream.synchronize()

    def stats(self, inst):
        s = PfStats()
        self._check(self.lib.pf_batch_stats(self.ctx, int(inst), ctypes.byref(s)), "pf_batch_stats")
        return _stats_dict(s, self.n_var)

    profile = Solver.profile
    profile_read = Solver.profile_read

    def autotune(self, cache=None, retime=False):
        """Pick each size group's launch tiles by timing (see pf_autotune);
        returns the number of groups timed."""
        return _autotune(self, cache, retime)

    def plan(self, inst):
        """Launch plan of the instance's group (dict of the pf_plan fields)."""
        return _plan(self, inst)

    def set_plan(self, inst, plan):
        _set_plan(self, inst, plan)

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.pf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PfFnoWeights(ctypes.Structure):
    _fp = ctypes.POINTER(ctypes.c_float)
    _fields_ = [
        ("width", ctypes.c_int32), ("modes", ctypes.c_int32), ("hidden", ctypes.c_int32),
        ("n_layers", ctypes.c_int32), ("n_cond", ctypes.c_int32),
        ("P", _fp), ("p", _fp), ("W", _fp), ("b", _fp), ("R", _fp),
        ("Q1", _fp), ("q1", _fp), ("Q2", _fp), ("q2", ctypes.c_float),
    ]


class PfFnoReport(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int32), ("rejected", ctypes.c_int32),
                ("rho_max_accepted", ctypes.c_double), ("rho_min_rejected", ctypes.c_double),
                ("last_rho", ctypes.c_double)]


def _declare_fno(lib):
    if getattr(lib, "_fno_declared", False):
        return
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.pf_fno_workspace_size.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.pf_fno_init.argtypes = [vp, ctypes.POINTER(PfFnoWeights), vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    lib.pf_fno_forward.argtypes = [vp, _dp, vp, vp]
    lib.pf_fno_advance.argtypes = [vp, i32, i32, _dp, ctypes.POINTER(PfLoad), ctypes.c_double,
                                   ctypes.POINTER(PfFnoReport)]
    lib.pf_fno_destroy.argtypes = [vp]
    lib.pf_macro_residual.argtypes = [vp, vp, i32, ctypes.POINTER(PfLoad), ctypes.POINTER(ctypes.c_double)]
    for name in ("pf_fno_workspace_size", "pf_fno_init", "pf_fno_forward", "pf_fno_advance", "pf_fno_destroy",
                 "pf_macro_residual"):
        getattr(lib, name).restype = ctypes.c_int
    lib._fno_declared = True


def stream_copy(dst, src):
    """Streaming device copy src -> dst (torch CUDA tensors of the same byte
    size, 16-byte multiples) on torch's current stream (pf_stream_copy)."""
    import torch
    lib = load()
    if not getattr(lib, "_stream_declared", False):
        lib.pf_stream_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        lib.pf_stream_copy.restype = ctypes.c_int
        lib._stream_declared = True
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("stream_copy needs contiguous tensors of the same byte size")
    rc = lib.pf_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes, torch.cuda.current_stream().cuda_stream)
    if rc != PF_OK:
        raise PfError(rc, "pf_stream_copy")


def macro_residual(solver, eta_prev, n_steps, eps_bar, sig_bar=None):
    """Residual max of the macro step from eta_prev to the solver's current
    order parameter (end-corrected trapezoid of the summed plain steps; see
    pf_macro_residual)."""
    lib = solver.lib
    _declare_fno(lib)
    ld = PfLoad()
    _fill_load(ld, eps_bar, sig_bar, None, 0)
    prev = eta_prev.contiguous()
    rho = ctypes.c_double()
    solver._check(lib.pf_macro_residual(solver.ctx, prev.data_ptr(), int(n_steps), ctypes.byref(ld),
                                        ctypes.byref(rho)), "pf_macro_residual")
    return rho.value


class Fno:
    """Learned macro stepper bound to a single-instance Solver.

    params: dict of float arrays (P (32, 8), p (32), W (4, 32, 32), b (4, 32),
    R complex (4, 32, 32, 2m, 2m, m), Q1 (128, 32), q1 (128), Q2 (1, 128) or
    (128,), q2 scalar) -- the layout of the checker's parameter set.
    """

    def __init__(self, solver, params):
        torch = solver.torch
        self.solver = solver
        self.lib = solver.lib
        _declare_fno(self.lib)
        R = np.asarray(params["R"])
        m = R.shape[-1]
        f32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float32))  # noqa: E731
        self._arrs = dict(P=f32(params["P"]), p=f32(params["p"]), W=f32(params["W"]), b=f32(params["b"]),
                          R=f32(np.stack([R.real, R.imag], axis=-1)), Q1=f32(params["Q1"]),
                          q1=f32(params["q1"]), Q2=f32(np.asarray(params["Q2"]).reshape(-1)))
        w = PfFnoWeights()
        w.width, w.modes, w.hidden = self._arrs["P"].shape[0], m, self._arrs["Q1"].shape[0]
        w.n_layers, w.n_cond = self._arrs["W"].shape[0], self._arrs["P"].shape[1] - 1
        for k, a in self._arrs.items():
            setattr(w, k, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
        w.q2 = float(np.asarray(params["q2"]).reshape(-1)[0])
        nbytes = ctypes.c_size_t()
        solver._check(self.lib.pf_fno_workspace_size(solver.ctx, m, ctypes.byref(nbytes)), "pf_fno_workspace_size")
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=solver.workspace.device)
        h = ctypes.c_void_p()
        solver._check(self.lib.pf_fno_init(solver.ctx, ctypes.byref(w), self.workspace.data_ptr(), nbytes.value,
                                           ctypes.byref(h)), "pf_fno_init")
        self.h = h

    def forward(self, cond, eta_in):
        t = self.solver.torch
        eta_in = eta_in.contiguous()
        out = t.empty_like(eta_in)
        c = np.ascontiguousarray(np.asarray(cond, dtype=np.float64))
        self.solver._check(self.lib.pf_fno_forward(self.h, _ptr(c), eta_in.data_ptr(), out.data_ptr()),
                           "pf_fno_forward")
        return out

    def advance(self, n_calls, steps_per_call, cond, eps_bar, sig_bar=None, tol=1e-3):
        ld = PfLoad()
        _fill_load(ld, eps_bar, sig_bar, None, 0)
        rep = PfFnoReport()
        c = np.ascontiguousarray(np.asarray(cond, dtype=np.float64))
        self.solver._check(self.lib.pf_fno_advance(self.h, int(n_calls), int(steps_per_call), _ptr(c),
                                                   ctypes.byref(ld), float(tol), ctypes.byref(rep)),
                           "pf_fno_advance")
        return {"accepted": rep.accepted, "rejected": rep.rejected, "rho_max_accepted": rep.rho_max_accepted,
                "rho_min_rejected": rep.rho_min_rejected, "last_rho": rep.last_rho}

    def close(self):
        if getattr(self, "h", None):
            self.lib.pf_fno_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class VoronoiMap:
    """FE <-> FFT mapping by nearest Gauss point on the current torch stream.

    points: torch float64 CUDA tensor (n_points, 3) in metres; shape (nz, ny,
    nx) and dx of the grid (cell centres at (i + 1/2) dx). cell_point holds
    the nearest point of every cell (int32, (nz, ny, nx)).
    """

    def __init__(self, points, shape, dx):
        import torch
        self.lib = load()
        self.torch = torch
        if points.dtype != torch.float64 or not points.is_cuda or points.dim() != 2 or points.shape[1] != 3:
            raise ValueError("points must be a float64 CUDA tensor (n, 3)")
        self.points = points.contiguous()
        self.n = points.shape[0]
        self.shape = tuple(int(v) for v in shape)
        self.dx = float(dx)
        nbytes = ctypes.c_size_t()
        nz, ny, nx = self.shape
        rc = self.lib.pf_vmap_workspace_size(nx, ny, nz, self.n, ctypes.byref(nbytes))
        if rc != PF_OK:
            raise PfError(rc, "pf_vmap_workspace_size")
        dev = points.device
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
        self.cell_point = torch.empty(self.shape, dtype=torch.int32, device=dev)
        self.stream = torch.cuda.current_stream(dev)
        self.build()

    def build(self):
        nz, ny, nx = self.shape
        rc = self.lib.pf_vmap_build(nx, ny, nz, self.dx, self.n, self.points.data_ptr(), self.workspace.data_ptr(),
                                    self.workspace.numel(), ctypes.c_void_p(self.stream.cuda_stream),
                                    self.cell_point.data_ptr())
        if rc != PF_OK:
            raise PfError(rc, "pf_vmap_build")

    def to_cells(self, point_values, out=None):
        """(ncomp, n_points) float32 -> (ncomp, nz, ny, nx)."""
        torch = self.torch
        pv = point_values.contiguous()
        if pv.dtype != torch.float32 or pv.dim() != 2 or pv.shape[1] != self.n:
            raise ValueError("point_values must be float32 (ncomp, n_points)")
        out = torch.empty((pv.shape[0],) + self.shape, dtype=torch.float32, device=pv.device) if out is None else out
        rc = self.lib.pf_vmap_to_cells(self.cell_point.numel(), self.cell_point.data_ptr(), self.n, pv.shape[0],
                                       pv.data_ptr(), out.data_ptr(), ctypes.c_void_p(self.stream.cuda_stream))
        if rc != PF_OK:
            raise PfError(rc, "pf_vmap_to_cells")
        return out

    def to_points(self, cell_values, out=None):
        """(ncomp, nz, ny, nx) float32 -> (ncomp, n_points)."""
        torch = self.torch
        cv = cell_values.contiguous()
        if cv.dtype != torch.float32 or tuple(cv.shape[1:]) != self.shape:
            raise ValueError("cell_values must be float32 (ncomp, nz, ny, nx)")
        out = torch.empty((cv.shape[0], self.n), dtype=torch.float32, device=cv.device) if out is None else out
        nz, ny, nx = self.shape
        rc = self.lib.pf_vmap_to_points(nx, ny, nz, self.dx, self.cell_point.data_ptr(), self.n,
                                        self.points.data_ptr(), cv.shape[0], cv.data_ptr(), out.data_ptr(),
                                        self.workspace.data_ptr(), self.workspace.numel(),
                                        ctypes.c_void_p(self.stream.cuda_stream))
        if rc != PF_OK:
            raise PfError(rc, "pf_vmap_to_points")
        return out


def spectral_conv(v, R, m):
    """K v of a Fourier layer through the library's training kernels, with
    their backward pass: v (B, C, nz, ny, nx) float32 CUDA, R the layer's
    (C, C, 2m, 2m, m, 2) float32 (real, imaginary) weights. Differentiable in
    v and R (pf_specconv_forward / pf_specconv_backward)."""
    return _spectral_conv_fn().apply(v, R, m)


_SPEC_FN = None


def _spectral_conv_fn():
    global _SPEC_FN
    if _SPEC_FN is not None:
        return _SPEC_FN
    import torch

    def dims(v, m):
        B, C, nz, ny, nx = v.shape
        return [int(B), int(C), int(nx), int(ny), int(nz), int(m)]

    def work_for(lib, d, dev):
        n = ctypes.c_size_t()
        rc = lib.pf_specconv_workspace_size(*d, ctypes.byref(n))
        if rc != PF_OK:
            raise PfError(rc, f"pf_specconv_workspace_size{tuple(d)}")
        return torch.empty(n.value, dtype=torch.uint8, device=dev), n.value

    class SpectralConv(torch.autograd.Function):
        @staticmethod
        def forward(ctx, v, R, m):
            lib = load()
            if v.dtype != torch.float32 or R.dtype != torch.float32 or not v.is_cuda or not R.is_cuda:
                raise ValueError("spectral_conv needs float32 CUDA tensors")
            v, R = v.contiguous(), R.contiguous()
            d = dims(v, m)
            B, C = d[0], d[1]
            work, nbytes = work_for(lib, d, v.device)
            S = torch.empty((B, C, 2 * m, 2 * m, m, 2), dtype=torch.float32, device=v.device)
            M = torch.empty_like(S)
            y = torch.empty_like(v)
            stream = torch.cuda.current_stream(v.device).cuda_stream
            rc = lib.pf_specconv_forward(*d, v.data_ptr(), R.data_ptr(), S.data_ptr(), M.data_ptr(), y.data_ptr(),
                                         work.data_ptr(), nbytes, ctypes.c_void_p(stream))
            if rc != PF_OK:
                raise PfError(rc, "pf_specconv_forward")
            ctx.save_for_backward(R, S)
            ctx.m = m
            return y

        @staticmethod
        def backward(ctx, dy):
            lib = load()
            R, S = ctx.saved_tensors
            dy = dy.contiguous()
            d = dims(dy, ctx.m)
            work, nbytes = work_for(lib, d, dy.device)
            G = torch.empty_like(S)
            M = torch.empty_like(S)
            dv = torch.empty_like(dy)
            dR = torch.empty_like(R)
            stream = torch.cuda.current_stream(dy.device).cuda_stream
            rc = lib.pf_specconv_backward(*d, dy.data_ptr(), R.data_ptr(), S.data_ptr(), G.data_ptr(),
                                          M.data_ptr(), dv.data_ptr(), dR.data_ptr(), work.data_ptr(), nbytes,
                                          ctypes.c_void_p(stream))
            if rc != PF_OK:
                raise PfError(rc, "pf_specconv_backward")
            return dv, dR, None

    _SPEC_FN = SpectralConv
    return _SPEC_FN
