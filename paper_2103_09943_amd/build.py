"""Build libllp.so (the HIP library behind include/llp.h) for gfx950 with hipcc.

Usage: python -m paper_2103_09943_amd.build   (or build() from Python).  The library is written next to this
file so that it travels with the source tree.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libllp.so")
SOURCES = ["llp_kernels.hip", "llp_operator.hip", "llp_fast.hip", "llp_sweep.hip", "llp_refine.hip", "llp_precond.hip",
           "llp_api.hip",
           "llp_batch.hip", "llp_tune.hip", "llp_cnn.hip",
           "llp_cnn_api.hip", "llp_noalloc.hip", "llp_prior.hip", "llp_kernel_est.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def _run(cmd):
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(line for line in proc.stdout.splitlines() if "packed-fp32-ops" not in line)
    if proc.returncode != 0:
        raise RuntimeError(f"command failed ({proc.returncode}): {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link libllp.so.  Always recompiles."""
    from concurrent.futures import ThreadPoolExecutor

    bdir = os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = [os.path.join(bdir, os.path.splitext(src)[0] + ".o") for src in SOURCES]
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", 0)) or os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(jobs) as ex:  # one hipcc process per source
        outs = list(ex.map(lambda so: _run([HIPCC, *COMMON, *DEVICE_FLAGS, "-c", os.path.join(CSRC, so[0]), "-o",
                                            so[1]]), zip(SOURCES, objs)))
    if verbose:
        for out in outs:
            if out.strip():
                print(out)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
