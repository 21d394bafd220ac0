"""The C ABI library loads on the host and exports every function declared in
include/pqph.h (no compute call is made without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pqph.h")
LIB = os.path.join(ROOT, "paper_1609_00077_amd", "libpqph.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_]+\s*\**\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("defined",)))


def test_header_declares_the_path():
    names = declared()
    for n in ("pq_residual", "pq_solve", "pq_energy", "pqph_integrals", "pqph_create",
              "ph_residual", "ph_energy", "ph_solve"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpqph.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpqph.so not built")
def test_host_side_size_queries():
    from paper_1609_00077_amd import _lib
    lib = _lib.load()
    assert lib.pq_amp_len(70) == 70245
    assert lib.pq_eri_len(70) == 104265
    assert lib.ph_amp_len(20) == 350990
    assert lib.ph_eri_len(20) == 104050
    assert lib.pq_amp_len(0) == 0


def test_bench_refuses_multi_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stdout


def _struct_fields(name):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + ";", text).group(1)
    return re.findall(r"(int|double)\s+(\w+);", body)


def test_binding_structs_match_the_header():
    """The ctypes mirrors of the option and report structs list the header's
    fields in the header's order with the same types."""
    from paper_1609_00077_amd import _lib
    ctype = {"int": ctypes.c_int, "double": ctypes.c_double}
    for cls, name in ((_lib.SolveOpts, "pqph_solve_opts"), (_lib.SolveInfo, "pqph_solve_info")):
        want = [(n, ctype[t]) for t, n in _struct_fields(name)]
        assert list(cls._fields_) == want, name


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpqph.so not built")
def test_default_options():
    from paper_1609_00077_amd import _lib
    lib = _lib.load()
    o = _lib.SolveOpts()
    o.spin_adapted = 7
    lib.pqph_default_opts(ctypes.byref(o))
    assert (o.max_iter, o.tol, o.diis_dim, o.diis_start, o.stall_window) == (200, 1e-8, 8, 2, 40)
    assert (o.max_rank, o.solver, o.spin_adapted) == (0, 0, 0)
