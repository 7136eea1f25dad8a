"""Build libms.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libms.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for every HIP object of this project.  No FP contraction:
# every float operation of the step is a separately rounded IEEE binary32 operation, in the
# order the step model writes it.  Common-code sinking is off: merging the narrowphase's
# per-shape slot writes behind pointer phis would put its register-slot arrays in scratch
# memory.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-mllvm", "-simplifycfg-sink-common=false",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def build_library(verbose: bool = False, out: str = LIB, extra=()) -> str:
    """Compile the single translation unit ms_lib.hip (kernels + host runtime) into libms.so."""
    tmp = out + ".tmp"
    cmd = [HIPCC] + FLAGS + list(extra) + [os.path.join(CSRC, "ms_lib.hip"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed to build libms.so")
    os.replace(tmp, out)
    return out


CLOCK_LIB = os.path.join(HERE, "libms_clock.so")


def build_clock_library(verbose: bool = False) -> str:
    """The per-phase clock build (libms_clock.so: the same library with -DMS_PHASE_CLOCK), a
    measurement tool; the binding loads it when MS_LIBRARY names it."""
    return build_library(verbose, out=CLOCK_LIB, extra=["-DMS_PHASE_CLOCK"])


if __name__ == "__main__":
    print(build_library(verbose=True))
    if len(sys.argv) > 1 and sys.argv[1] == "clock":
        print(build_clock_library(verbose=True))
