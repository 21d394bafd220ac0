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
SOURCES = ["pqph_ctx.hip", "solver_kernels.hip", "pq_residual.hip", "pq_lane.hip", "pq_lane_adj.hip",
           "integrals.hip", "batched.hip", "ph_residual.hip", "ceilings.hip", "spin.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         # packed FP32 instructions stay off (wrong results seen on this part)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
OBJDIR = os.path.join(HERE, "_build")


def generate_tables() -> None:
    from .derive import codegen
    tb = codegen.build_pq_tables()
    codegen.emit_pq_header(tb, os.path.join(CSRC, "pq_tables.h"))
    codegen.emit_lane_code(tb, os.path.join(CSRC, "pq_lane_code.h"))
    codegen.emit_lane_adj_code(tb, os.path.join(CSRC, "pq_lane_adj_code.h"))


PH_TERMS = os.path.join(HERE, "ph_terms.bin")
PH_INPUTS = [os.path.join(HERE, "derive", f) for f in ("algebra.py", "terms.py", "codegen.py",
                                                       "ph_tables.py")]


def _ph_key() -> str:
    import hashlib
    h = hashlib.sha256()
    for path in PH_INPUTS:
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def ensure_ph_terms() -> str:
    """The PH term tables (ph_terms.bin beside the library), regenerated when
    the derivation sources changed since they were written.  Enumerating the
    three-pair classes takes several CPU-minutes on 8 cores, so a current
    file is kept."""
    key = _ph_key()
    keyfile = PH_TERMS + ".key"
    if os.path.exists(PH_TERMS) and os.path.exists(keyfile):
        with open(keyfile) as fh:
            if fh.read().strip() == key:
                return PH_TERMS
    from .derive import ph_tables
    ph_tables.main([PH_TERMS])
    with open(keyfile, "w") as fh:
        fh.write(key + "\n")
    return PH_TERMS


def build(verbose: bool = False) -> str:
    """Regenerate the tables, compile every source to an object in parallel
    (the generated straight-line kernel dominates), link the shared library."""
    generate_tables()
    ensure_ph_terms()
    os.makedirs(OBJDIR, exist_ok=True)
    procs = []
    for src in SOURCES:
        obj = os.path.join(OBJDIR, src.replace(".hip", ".o"))
        cmd = [HIPCC] + FLAGS + ["-c", "-o", obj, os.path.join(CSRC, src)]
        procs.append((src, obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                                 text=True)))
    objs, failed = [], []
    for src, obj, pr in procs:
        out, err = pr.communicate()
        if pr.returncode != 0:
            failed.append(src)
            sys.stderr.write(out + err)
        elif verbose:
            sys.stderr.write(err)
        objs.append(obj)
    if failed:
        raise RuntimeError("hipcc failed on " + ", ".join(failed))
    cmd = [HIPCC, "--offload-arch=gfx950", "-fPIC", "-shared", "-o", LIB + ".tmp"] + objs + ["-ldl", "-lz"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libpqph.so")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
