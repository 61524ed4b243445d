"""Builds libwfp.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2507_07823_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwfp.so")
SOURCES = ["wfp_kernels.hip", "wfp_plan.hip", "wfp_batch.hip", "wfp_host.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


PROBE = os.path.join(HERE, "lds_probe")


def build_library(verbose=True):
    cmd = [HIPCC] + FLAGS + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    build_probe(verbose)
    return LIB


def build_probe(verbose=True):
    """The LDS read-throughput probe that bench.py runs beside the on-the-fly
    local sum's roofline (a separate program: the library has no use for it)."""
    flags = [f for f in FLAGS if f not in ("-fPIC", "-shared")]
    cmd = [HIPCC] + flags + [os.path.join(CSRC, "lds_probe.hip"), "-o", PROBE + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(PROBE + ".tmp", PROBE)
    return PROBE


if __name__ == "__main__":
    build_library()
    sys.exit(0)
