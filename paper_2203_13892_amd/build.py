"""Build ``libtqsim.so`` in-tree for gfx950 with hipcc.

Usage: ``python -m paper_2203_13892_amd.build`` (or ``build()`` from Python).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libtqsim.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("host.cpp", "plan.cpp", "device.hip", "mlp.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are kept out of generated code (ordinary scalar
# float code is used instead).
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument",
         # keep switch cases on distinct tile registers: sinking their common
         # code would index the register tile dynamically (scratch memory)
         "-mllvm", "-simplifycfg-sink-common=false",
         "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc")]


def build(verbose: bool = False) -> str:
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + SOURCES + ["-lrocprofiler-sdk-roctx", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(SO)
