"""Build the HIP library libpftwin.so in-tree for gfx950.

Usage: python -m paper_2302_13612_amd.build   (or build() from Python).
Compiles every time it is called; translation units are compiled in
parallel (the forward x-pass kernels once per number of twin variants).
"""

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpftwin.so")
ARCH = "gfx950"
# (source, extra defines, object name)
UNITS = [("pf_kernels.hip", [], "pf_kernels.o"),
         ("pf_fno.hip", [], "pf_fno.o"),
         ("pf_vmap.hip", [], "pf_vmap.o"),
         ("pf_specconv.hip", [], "pf_specconv.o"),
         ("pf_fnotrain.hip", [], "pf_fnotrain.o"),
         ("pf_stream.hip", [], "pf_stream.o"),
         ("pf_api.cpp", [], "pf_api.o"),
         ("pf_crystal.cpp", [], "pf_crystal.o")] + \
        [("pf_xv.hip", [f"-DPF_NV={v}"], f"pf_xv{v}.o") for v in range(1, 7)]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags():
    return [
        "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
        # keep the compiler off packed FP32 instructions
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-result",
    ]


def _compile(unit, outdir, extra):
    src, defs, obj = unit
    out = os.path.join(outdir, obj)
    cmd = [hipcc()] + flags() + defs + extra + ["-c", os.path.join(CSRC, src), "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True)
    return cmd, res, out


def build(verbose=False, jobs=None, extra_flags=(), out=None):
    jobs = jobs or min(len(UNITS), max(1, min(16, os.cpu_count() or 1)))
    with tempfile.TemporaryDirectory(prefix="pftwin_build_") as tmp:
        with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
            results = list(ex.map(lambda u: _compile(u, tmp, list(extra_flags)), UNITS))
        failed = False
        for cmd, res, _ in results:
            if verbose:
                print(" ".join(cmd), flush=True)
            if res.returncode != 0:
                failed = True
                sys.stderr.write(res.stdout + res.stderr)
            elif verbose and extra_flags:
                sys.stderr.write(res.stderr)
        if failed:
            raise RuntimeError("hipcc failed building libpftwin.so")
        lib = out or LIB
        out_tmp = lib + ".tmp"
        link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC"] + [r[2] for r in results] + ["-o", out_tmp]
        res = subprocess.run(link, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("link of libpftwin.so failed")
        os.replace(out_tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
