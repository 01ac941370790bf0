"""Builds the gfx950 shared library ``libhough_tf.so`` in-tree with hipcc.

``build_library(phase_clocks=True)`` builds the measurement variant
``libhough_tf_phases.so`` instead: the same library compiled with
HOUGH_PHASE_CLOCKS, whose finder records its cycles per phase for every
event into the event-clock buffer (see ``phase_clocks.py``)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libhough_tf.so")
LIB_PHASES = os.path.join(PKG, "libhough_tf_phases.so")
SOURCES = [os.path.join(CSRC, "hough_kernels.hip"), os.path.join(CSRC, "hough_host.hip"),
           os.path.join(CSRC, "hough_serve.hip"), os.path.join(CSRC, "hough_refit.hip"),
           os.path.join(CSRC, "hough_cf.hip"), os.path.join(CSRC, "hough_probe.hip"),
           os.path.join(CSRC, "hough_tw.hip")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # the bin index must be the same rounded float expression as on the host
    "-ffp-contract=off",
    # no packed fp32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def build_library(verbose: bool = False, phase_clocks: bool = False) -> str:
    """Compiles the library (always) and returns its path."""
    out = LIB_PHASES if phase_clocks else LIB
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + (["-DHOUGH_PHASE_CLOCKS"] if phase_clocks else []) + \
        ["-I", INCLUDE, "-I", CSRC, "-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv, phase_clocks="--phase-clocks" in sys.argv))
