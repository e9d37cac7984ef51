"""Build the gfx950 shared library libehdlb.so in-tree with hipcc.

    python -m paper_2608_12868_amd.build

Packed-FP32 instructions are disabled at code generation (-packed-fp32-ops);
every other flag is standard HIP for gfx950.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libehdlb.so")
SOURCES = [os.path.join(HERE, "csrc", "ehdlb.hip")]
HEADERS = [os.path.join(HERE, "csrc", n) for n in ("kernels.h", "step.h", "lattice.h", "adjoint.h", "preset.h")] + [
    os.path.join(ROOT, "include", "ehdlb.h")]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-ffp-contract=fast",
           "-I", os.path.join(ROOT, "include"),
           "-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libehdlb.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
