"""Build the gfx950 shared library ``libmi355bls.so`` next to this file.

Usage: ``python -m paper_2302_01293_amd.build`` (or ``build()`` from Python).
Compiles every HIP source with hipcc for gfx950, FP contraction off (the fold's
phase and bin arithmetic must be plain IEEE operations) and packed FP32 disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmi355bls.so")
SOURCES = ["plan.cpp", "search.hip", "rebin.hip", "snr.hip", "pp.hip", "stats.hip", "fit.hip", "noalloc.hip"]
ARCH = os.environ.get("MI355BLS_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def command(out: str) -> list[str]:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    return [hipcc(), "-O3", "--offload-arch=" + ARCH, "-std=c++17", "-fPIC", "-shared",
            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-o", out] + srcs


CEIL_LIB = os.path.join(HERE, "libmi355ceil.so")


def build_ceilings(verbose: bool = False) -> str:
    """The unit-rate microbenchmarks (``csrc/ceilings.hip``) as their own library."""
    tmp = CEIL_LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-O3", "--offload-arch=" + ARCH, "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-o", tmp,
           os.path.join(CSRC, "ceilings.hip")]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (res.stderr or "").splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    os.replace(tmp, CEIL_LIB)
    return CEIL_LIB


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (res.stderr or "").splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_ceilings(verbose=True))
