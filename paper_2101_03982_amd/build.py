"""Builds liblbm.so (HIP, gfx950) in-tree.

Every (velocity set, storage, stencil length) part of the kernel table is
its own translation unit so that the parts compile in parallel; the host API
is one more unit.  Usage: ``python -m paper_2101_03982_amd.build [-j N]``.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblbm.so")

SETS = ["D2Q9", "D2Q19", "D2Q25", "D3Q13", "D3Q21", "D3Q27", "D3V27", "D3Q45"]
DIM = {"D2Q9": 2, "D2Q19": 2, "D2Q25": 2, "D3Q13": 3, "D3Q21": 3, "D3Q27": 3, "D3V27": 3, "D3Q45": 3}
STORAGES = ["ST_F64", "ST_F32", "ST_BF16", "ST_F16"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no packed FP32 instructions (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


# Extra compiler flags per unit name prefix.  The 16-bit D3Q45 f + g kernels
# run 2.5 % (BF16) and 4.4 % (FP16) faster at 256^3 with LLVM's ILP-oriented
# machine scheduler; every other kernel measured 1-27 % slower with it.
UNIT_FLAGS = {
    "part_D3Q45_bf16_": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
    "part_D3Q45_f16_": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
}


def unit_flags(path):
    name = os.path.basename(path)
    for prefix, flags in UNIT_FLAGS.items():
        if name.startswith(prefix):
            return flags
    return []


GLC_SETS = ("D2Q9", "D3Q13", "D3Q21", "D3Q27", "D3V27")


def _unit(s, st, ns):
    return ('#include "lbm_inst.hpp"\n'
            "namespace lbm {\n"
            "template bool find_kernels_part<%s, %s, %s>(int, int, Kernels*);\n"
            "}  // namespace lbm\n" % (s, st, ns))


def parts():
    """(name, source text) of every kernel-table unit."""
    out = []
    for s in SETS:
        for st in STORAGES:
            if st in ("ST_BF16", "ST_F16") and DIM[s] == 2:
                continue
            for ns in range(1, 6):
                if ns == 1 and s not in ("D2Q9", "D3Q27"):
                    continue
                name = "part_%s_%s_%d" % (s, st[3:].lower(), ns)
                out.append((name, _unit(s, st, str(ns))))
            # the cell-wise Gauss-Lobatto-Chebyshev support, p = 4
            if s in GLC_SETS and st in ("ST_F64", "ST_F32"):
                out.append(("part_%s_%s_glc4" % (s, st[3:].lower()), _unit(s, st, "GLC_P4")))
    return out


KERNEL_HEADERS = ["lbm_kernels.hpp", "lbm_sets.hpp", "lbm_dispatch.hpp", "lbm_inst.hpp"]


def _stale(src, obj):
    if not os.path.exists(obj):
        return True
    deps = [src] + [os.path.join(CSRC, f) for f in KERNEL_HEADERS]
    if src.endswith("lbm_api.hip"):
        deps.append(os.path.join(HERE, "..", "include", "lbm.h"))
    if src.endswith("lbm_api.hip") or src.endswith("lbm_diag.hip"):
        deps.append(os.path.join(CSRC, "lbm_diag.hpp"))
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps if os.path.exists(d))


def _compile(src, obj, force=True):
    if not force and not _stale(src, obj):
        return obj, 0.0
    cmd = [HIPCC, *FLAGS, *unit_flags(src), "-I", CSRC, "-c", src, "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj, time.time() - t0


def build(jobs: int | None = None, verbose: bool = False, force: bool = True) -> str:
    """Compiles every unit (``force``) or only those older than their sources."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))
    units = []
    for name, text in parts():
        path = os.path.join(BUILD, name + ".hip")
        if not os.path.exists(path) or open(path).read() != text:
            with open(path, "w") as fh:
                fh.write(text)
        units.append((path, os.path.join(BUILD, name + ".o")))
    units.append((os.path.join(CSRC, "lbm_api.hip"), os.path.join(BUILD, "lbm_api.o")))
    units.append((os.path.join(CSRC, "lbm_diag.hip"), os.path.join(BUILD, "lbm_diag.o")))
    # longest units first (the 3D sets with many combinations)
    units.sort(key=lambda u: ("D3Q45" not in u[0], "D3" not in u[0], u[0]))
    t0 = time.time()
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, s, o, force) for s, o in units]
        for f in cf.as_completed(futs):
            obj, dt = f.result()
            objs.append(obj)
            if verbose:
                print("  %-40s %6.1fs" % (os.path.basename(obj), dt), flush=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *sorted(objs)]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    if verbose:
        print("built %s in %.1fs" % (LIB, time.time() - t0), flush=True)
    return LIB


def clean():
    shutil.rmtree(BUILD, ignore_errors=True)
    if os.path.exists(LIB):
        os.remove(LIB)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", "--jobs", type=int, default=None)
    ap.add_argument("--clean", action="store_true")
    ap.add_argument("--incremental", action="store_true", help="recompile only stale units")
    a = ap.parse_args()
    if a.clean:
        clean()
    build(a.jobs, verbose=True, force=not a.incremental)
    sys.exit(0)
