"""Builds the HIP library librok4e.so in-tree for gfx950 (hipcc cross-compiles without
a GPU)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "rok4e.hip")
LIB = os.path.join(HERE, "librok4e.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # contraction only within one source expression: the same expression rounds the
         # same way in every kernel variant
         "-ffp-contract=on",
         # packed FP32 ops stay off: the compiler must not form v_pk_*_f32
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def build(verbose: bool = False, defines: dict | None = None, out: str | None = None) -> str:
    """Compiles the library (to `out`, default the in-tree librok4e.so); `defines` sets
    the tuning macros (ROK4E_OCC_ROWS1, ROK4E_RX_UNROLL)."""
    lib = out or LIB
    dflags = [f"-D{k}={v}" for k, v in (defines or {}).items()]
    cmd = [HIPCC, *FLAGS, *dflags, "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc"),
           "-o", lib + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
