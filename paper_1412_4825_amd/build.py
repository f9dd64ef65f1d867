"""Build the HIP library (gfx950) in-tree: paper_1412_4825_amd/libbrng.so.

Flags:
  --offload-arch=gfx950                 MI355X only, no other targets
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                        no packed fp32 instructions
  -fno-gpu-flush-denormals-to-zero      fp32 subnormals kept (gamma shapes
                                        below 1 can produce them)
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", f) for f in ("brng.hip", "serve.hip")]
LIB = os.path.join(HERE, "libbrng.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-flush-denormals-to-zero",
    "-Wall",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    """Compile libbrng.so (always recompiles)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + SRCS + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
