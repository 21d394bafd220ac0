"""Algorithmic work of the PQ residual kernels (counted, not measured).

Flops are the arithmetic of each kernel's formula in the factorisation the
library uses: one multiplication per factor of a term plus one addition per
term for the interpreted classes, 2 per multiply-add of a contraction, with
spectators restricted to labels distinct from the outputs.  The byte counts
are the compulsory HBM traffic of a residual: read t (packed), the packed
integrals and f once, write r once.
"""
from __future__ import annotations

from functools import lru_cache
from math import comb

import numpy as np


@lru_cache(maxsize=1)
def _tables():
    from .derive.codegen import build_pq_tables
    return build_pq_tables()


def _class_cost(tab):
    nf = (tab.fac != 0).sum(axis=1)
    return float((nf + 1).sum())


def _spec_cost(specs):
    return float(sum(len(s) for s in specs))


def pq_kernel_flops(N: int) -> dict:
    tb = _tables()
    np2 = comb(N, 2)
    c = tb.classes
    out = {}
    nsym1 = sum(len(e) for e in tb.h1_sym)
    nsym2 = sum(len(e) for e in tb.h2_sym)
    out["k_vertex1"] = 2.0 * nsym1 * N
    out["k_vertex2"] = 2.0 * nsym2 * N * (N - 1)
    out["k_unpack_t2"] = 29.0 * N * (N - 1) / 2          # one sign multiply per mirrored entry
    out["k_spec_w"] = _spec_cost(tb.r2s2_w) * N * (N - 1)
    out["k_spec_lam"] = _spec_cost(tb.r2s2_lam) * N * (N - 1)
    out["k_dress"] = 2.0 * len(tb.r2s2_dress) * N * N * N
    # one-spectator contraction over A != P, Q; its sides X, Y (products of
    # factors) are materialised (k_spec_xy) or formed while staging
    out["k_spec_xy"] = (_spec_cost(tb.r2s1_x) + _spec_cost(tb.r2s1_y)) * N * (N - 1)
    out["k_gemm_s1"] = 2.0 * len(tb.r2s1_pairs) * np2 * max(N - 2, 0)
    # two spectators: per output pair and (w, a) group: L_a on N-2 labels, the
    # (N-2)x(N-2) vertex contraction, then per b: L_b and a dot over N-2 labels
    lsum = 0.0
    for (wi, ai), lst in tb.r2s2_groups:
        lsum += len(tb.r2s2_l[ai]) * (N - 2) + 2.0 * (N - 2) ** 2
        for bi, _, _ in lst:
            lsum += (len(tb.r2s2_l[bi]) + 2.0) * (N - 2)
    out["k_r2s2"] = lsum * np2
    out["k_r2c"] = (_class_cost(c["R2S0"]) + _class_cost(c["R2S1"])) * np2
    out["k_r1"] = N * _class_cost(c["R1S0"])
    out["k_r1c"] = N * (N - 1) * _class_cost(c["R1S1"])
    # factorised one-pair two-spectator terms: products X, Y, Z (and Z^T) over
    # ordered label pairs, then per group and output pair one row of a
    # contraction over N labels and a dot per closing product
    r1f = tb.r1s2_x + tb.r1s2_y + tb.r1s2_z
    out["k_spec_r1"] = _spec_cost(r1f) * N * (N - 1)
    out["k_r1s2"] = 2.0 * len(tb.r1s2_groups) * N * N * N          # M = G Mid per group
    out["k_r1s2_close"] = 2.0 * N * N * sum(len(l) for _, l in tb.r1s2_groups)
    out["k_final"] = float((3 * N + 29 * np2) * 4)
    return out


def pq_compulsory_bytes(N: int) -> float:
    """8 * (2 * amplitudes + integrals + f): read t and the integrals once, write r."""
    amps = 3 * N + 29 * comb(N, 2)
    eri = 6 * N + 43 * comb(N, 2)
    return 8.0 * (2 * amps + eri + 4 * N * N)


def integral_flops(N: int, k: int = 2) -> float:
    """Integral transformation of a chain of n = 2N sites: Y over every orbital
    pair (2 n^2 n(n+1)/2), f = C^T (F C) (2 x 2 n^3) and one dot of length n
    per stored integral (2 n each)."""
    n = 2 * N
    npq = n * (n + 1) // 2
    stored = 6 * N + 43 * comb(N, 2) + (84 * comb(N, 3) if k == 3 else 0)
    return 2.0 * n * n * npq + 4.0 * n ** 3 + 2.0 * n * stored


# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_FP64_MATRIX_TFLOPS = 78.6
