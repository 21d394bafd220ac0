"""ctypes binding of libpqph.so: argument marshalling only.

The library must have been built in-tree (paper_1609_00077_amd/build.py).
Nothing here computes any part of the method; a missing library is an error.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpqph.so")


class SolveOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int), ("tol", C.c_double), ("diis_dim", C.c_int),
                ("diis_start", C.c_int), ("level_shift", C.c_double),
                ("diverge_factor", C.c_double), ("stall_window", C.c_int), ("max_rank", C.c_int),
                ("solver", C.c_int), ("spin_adapted", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("rnorm", C.c_double), ("status", C.c_int),
                ("solve_ms", C.c_double)]


STATUS = {0: "OK", -1: "INVALID_ARG", -2: "DEVICE", -3: "OOM", -4: "NONFINITE",
          -5: "NOT_CONVERGED", -6: "DIVERGED"}

# every exported symbol and its signature (restype, argtypes)
P = C.c_void_p
SIGNATURES = {
    "pqph_default_opts": (None, [C.POINTER(SolveOpts)]),
    "pqph_create": (C.c_int, [C.POINTER(P), C.c_int, P]),
    "pqph_destroy": (None, [P]),
    "pqph_last_error": (C.c_char_p, [P]),
    "pq_amp_len": (C.c_size_t, [C.c_int]),
    "ph_amp_len": (C.c_size_t, [C.c_int]),
    "pq_eri_len": (C.c_size_t, [C.c_int]),
    "ph_eri_len": (C.c_size_t, [C.c_int]),
    "pqph_integrals": (C.c_int, [P, C.c_int, C.c_int, P, P, P, P, P]),
    "pq_residual": (C.c_int, [P, C.c_int, P, P, P, P]),
    "ph_residual": (C.c_int, [P, C.c_int, P, P, P, P]),
    "pq_residual_noalloc": (C.c_int, [P, C.c_int, P, P, P, P]),
    "ph_energy": (C.c_int, [P, C.c_int, P, P, P, C.POINTER(C.c_double)]),
    "pq_energy": (C.c_int, [P, C.c_int, P, P, P, C.POINTER(C.c_double)]),
    "pq_solve": (C.c_int, [P, C.c_int, P, P, C.POINTER(SolveOpts), P, C.POINTER(C.c_double),
                           C.POINTER(SolveInfo)]),
    "ph_solve": (C.c_int, [P, C.c_int, P, P, C.POINTER(SolveOpts), P, C.POINTER(C.c_double),
                           C.POINTER(SolveInfo)]),
    "pqph_denominators": (C.c_int, [P, C.c_int, C.c_int, P, C.c_double, P]),
    "pq_residual_profile": (C.c_int, [P, C.c_int, P, P, P, P, C.POINTER(C.c_double), C.c_int,
                                      C.POINTER(C.c_int)]),
    "pq_residual_phase_name": (C.c_char_p, [C.c_int]),
    "pqph_measure_ceilings": (C.c_int, [P, C.POINTER(C.c_double)]),
    "pqph_autotune": (C.c_int, [P, C.c_int, P, P, P, P, C.POINTER(C.c_int)]),
    "pqph_set_variant": (C.c_int, [P, C.c_int, C.c_int]),
    "pqph_set_s1_mode": (C.c_int, [P, C.c_int, C.c_int]),
    "pqph_set_pq_intermediates": (C.c_int, [P, C.c_int, C.c_int]),
    "pqph_tuning": (C.c_int, [P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "pqph_set_batch_mode": (C.c_int, [P, C.c_int]),
    "pqph_set_solve_mode": (C.c_int, [P, C.c_int]),
    "pq_vjp": (C.c_int, [P, C.c_int, P, P, P, P, C.c_double, P, P, P]),
    "pq_energy_grad": (C.c_int, [P, C.c_int, P, P, P, C.POINTER(SolveOpts), C.POINTER(C.c_double),
                                 P, P, P, C.POINTER(SolveInfo)]),
    "pq_densities": (C.c_int, [P, C.c_int, P, P, P, C.POINTER(SolveOpts), C.POINTER(C.c_double),
                               P, P, C.POINTER(C.c_double), C.POINTER(SolveInfo)]),
    "pq_solve_batched": (C.c_int, [P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_int64), C.POINTER(C.c_int64), P, P,
                                   C.POINTER(SolveOpts), P, C.POINTER(C.c_double),
                                   C.POINTER(SolveInfo)]),
}

_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1609_00077_amd.build` (no CPU fallback exists)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class PQPHError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
