"""Build the HIP libraries for gfx950 in-tree.

Compiles every ``csrc/*.hip`` translation unit with hipcc and links them into
``paper_2601_00976_amd/libnmc.so`` (the solver), and ``csrc_probe/*.hip`` into
``paper_2601_00976_amd/libnmc_probe.so`` (the FP64 FMA throughput probe of the
benchmark, not part of the solver).  Always rebuilds when called.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnmc.so")
PROBE_DIR = os.path.join(HERE, "csrc_probe")
PROBE_LIB = os.path.join(HERE, "libnmc_probe.so")
BUILD_DIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 forms are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # atomics stay plain single-lane operations, so the work-queue grab's
    # result is not waited for where it is issued
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wall", "-Wno-unused-function",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def _link(objs, lib):
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"link of {os.path.basename(lib)} failed")
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    psrcs = sorted(glob.glob(os.path.join(PROBE_DIR, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs) + len(psrcs))) as ex:
        objs = list(ex.map(_compile, srcs + psrcs))
    _link(objs[:len(srcs)], LIB)
    if psrcs:
        _link(objs[len(srcs):], PROBE_LIB)
    if verbose:
        print(f"built {LIB}" + (f" and {PROBE_LIB}" if psrcs else ""))
    return LIB


if __name__ == "__main__":
    build(verbose=True)
