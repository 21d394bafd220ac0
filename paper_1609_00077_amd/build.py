"""Build libpqph.so in-tree for gfx950 (hipcc cross-compiles without a GPU).

Steps: regenerate the constant term tables from the derivation, then compile
the HIP sources into one shared library next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpqph.so")
SOURCES = ["pqph_ctx.hip", "solver_kernels.hip", "pq_residual.hip", "integrals.hip", "batched.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # packed FP32 instructions stay off (wrong results seen on this part)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def generate_tables() -> None:
    from .derive import codegen
    codegen.emit_pq_header(codegen.build_pq_tables(), os.path.join(CSRC, "pq_tables.h"))


def build(verbose: bool = False) -> str:
    generate_tables()
    cmd = [HIPCC] + FLAGS + ["-o", LIB + ".tmp"] + [os.path.join(CSRC, s) for s in SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libpqph.so")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
