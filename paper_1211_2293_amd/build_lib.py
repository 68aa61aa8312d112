"""Compile the HIP sources under csrc/ into libtc.so for gfx950 (in-tree).

Flags:
  -ffp-contract=off   keys, topology, moments and opening radii must be
                      reproducible bit for bit; the force loop writes its
                      FMAs explicitly.
  -packed-fp32-ops    (target feature switched off) no packed FP32 ops.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtc.so")
SOURCES = ["api.hip", "build.hip", "force.hip", "step.hip", "closure.hip", "learned.hip", "direct.hip", "perbody.hip", "fmm.hip"]
# a benchmark program beside the library: the force loop's own throughput
PROBE_SRC = "loop_probe.hip"
PROBE = os.path.join(HERE, "loop_probe")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function",
]


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the packed-fp32 feature: drop that notice
    err = "\n".join(l for l in p.stderr.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    if err.strip() and verbose:
        print(err, file=sys.stderr)
    return obj


def _build_probe(verbose: bool) -> str:
    tmp = PROBE + ".tmp"
    cmd = [HIPCC, *CFLAGS, os.path.join(CSRC, PROBE_SRC), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in p.stderr.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"hipcc failed on {PROBE_SRC}:\n{err}")
    os.replace(tmp, PROBE)
    return PROBE


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES) + 1) as ex:
        probe = ex.submit(_build_probe, verbose)
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
        probe.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
