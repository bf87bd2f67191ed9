"""Build libvibelsd.so for gfx950 with hipcc (in-tree)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvibelsd.so")
SOURCES = ["graph.hip", "bp.hip", "select.hip", "lsd.hip", "api.hip", "runtime.hip", "grad.hip", "probe.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile every source into one shared library at `out`; `defines` are
    extra -D settings (for example VIBE_BP_DEPTH=8)."""
    tmp = out + ".tmp"
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
           # keep the compiler from forming packed FP32 instructions
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument"] + [f"-D{d}" for d in defines] + \
          ["-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
