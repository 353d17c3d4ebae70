"""Build the HIP library (gfx950) in-tree with hipcc.

    python -m paper_2103_16120_amd.build

produces paper_2103_16120_amd/_lib/libmpgcr.so from csrc/*.hip.  Each source
file is compiled to an object of its own (in parallel), then they are linked.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
OBJDIR = os.path.join(ROOT, "_build")
LIBNAME = "libmpgcr.so"
ARCH = "gfx950"

# the C-ABI, the network, and one source per precision form's solve
SOURCES = ["solver.hip", "cnn.hip", "noalloc.hip", "solve_f64.hip", "solve_mixed.hip", "solve_mixed_fp64dot.hip",
           "solve_mixed_half_pc.hip", "solve_single.hip", "solve_single_polar64.hip", "si_step.hip"]
HEADERS = ["device.h", "kernels.h", "cnn.h", "cnn_internal.h", "learned.h", "solver_impl.h"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed fp32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    cand = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(cand):
        raise RuntimeError("hipcc not found")
    return cand


def lib_path() -> str:
    return os.path.join(LIBDIR, LIBNAME)


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed ({res.returncode}): {cmd[-1]}")


def build_library(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    os.makedirs(OBJDIR, exist_ok=True)
    cc = hipcc()
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmds.append([cc, *FLAGS, "-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, src), "-o", obj])
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    out = lib_path()
    tmp = out + ".tmp"
    _run([cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp], verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_library(verbose=True))
