"""Build libgenesis_hip.so for gfx950 in-tree with hipcc.

The library is a plain C-ABI shared object (include/genesis.h); the Python
binding in this package only loads it with ctypes.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SO = os.path.join(HERE, "libgenesis_hip.so")
SRCS = [os.path.join(HERE, "csrc", f) for f in ("genesis.hip", "serving.hip", "mlp.hip")]
DEPS = SRCS + [os.path.join(HERE, "csrc", f) for f in
               ("genesis_device.h", "genesis_common.h", "voigt_rational.h", "weideman36.h")] + \
       [os.path.join(ROOT, "include", "genesis.h")]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # reproducible arithmetic: FMAs only where the source asks for them
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def build(verbose: bool = False) -> str:
    tmp = SO + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + ["-o", tmp] + SRCS
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building %s" % SO)
    os.replace(tmp, SO)
    return SO


def stale() -> bool:
    if not os.path.exists(SO):
        return True
    t = os.path.getmtime(SO)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    print(build(verbose=True))
