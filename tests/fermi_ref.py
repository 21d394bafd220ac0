"""A second, deliberately different fermion implementation used only to pin
the oracle: determinants are sorted tuples of spin orbitals in interleaved
order (2*spatial + spin), states are dicts, and every operator is applied one
at a time.  It shares nothing with oracle/determinants.py."""
from __future__ import annotations

import itertools

import numpy as np


def so(spatial: int, spin: int) -> int:
    return 2 * spatial + spin


def apply_op(state: dict, create: bool, orb: int) -> dict:
    out = {}
    for det, c in state.items():
        occ = orb in det
        if create == occ:
            continue
        sign = -1.0 if sum(1 for x in det if x < orb) % 2 else 1.0
        nd = tuple(sorted(det + (orb,))) if create else tuple(x for x in det if x != orb)
        out[nd] = out.get(nd, 0.0) + sign * c
    return out


def apply_string(state: dict, ops) -> dict:
    """ops: list of (create, spin-orbital), leftmost first."""
    for cre, o in reversed(ops):
        state = apply_op(state, cre, o)
    return state


def reference(npair: int) -> dict:
    return {tuple(sorted(so(p, s) for p in range(npair) for s in (0, 1))): 1.0}


def slot_ops(npair: int, labels, tup):
    ops = []
    for P, e in zip(labels, tup):
        if e & 1:
            ops.append((False, so(P, 0)))
        if e & 2:
            ops.append((False, so(P, 1)))
        if e & 4:
            ops.append((True, so(npair + P, 0)))
        if e & 8:
            ops.append((True, so(npair + P, 1)))
    return ops


def overlap(a: dict, b: dict) -> float:
    return sum(c * b.get(d, 0.0) for d, c in a.items())


def antisym(eri: np.ndarray, p, q, r, s) -> float:
    """<pq||rs> over spin orbitals from chemists' spatial integrals."""
    P, sp = divmod(p, 2)
    Q, sq = divmod(q, 2)
    R, sr = divmod(r, 2)
    S, ss = divmod(s, 2)
    v = 0.0
    if sp == sr and sq == ss:
        v += eri[P, R, Q, S]
    if sp == ss and sq == sr:
        v -= eri[P, S, Q, R]
    return v


def hn_on_reference(npair: int, f: np.ndarray, eri: np.ndarray) -> dict:
    """H_N |0> = sum f_ai a+_a a_i |0> + 1/4 sum <ab||ij> a+_a a+_b a_j a_i |0>."""
    occ = [so(p, s) for p in range(npair) for s in (0, 1)]
    vir = [so(npair + p, s) for p in range(npair) for s in (0, 1)]
    ref = reference(npair)
    out: dict = {}

    def add(st, c):
        for d, x in st.items():
            out[d] = out.get(d, 0.0) + c * x

    for a in vir:
        for i in occ:
            if a % 2 == i % 2 and f[a // 2, i // 2] != 0.0:
                add(apply_string(ref, [(True, a), (False, i)]), f[a // 2, i // 2])
    for a, b in itertools.permutations(vir, 2):
        for i, j in itertools.permutations(occ, 2):
            v = antisym(eri, a, b, i, j)
            if v != 0.0:
                add(apply_string(ref, [(True, a), (True, b), (False, j), (False, i)]), 0.25 * v)
    return out


def diagonal_one_body(det, f: np.ndarray) -> float:
    """<det| sum_p f_pp a+_p a_p |det> for a determinant of spin orbitals."""
    return float(sum(f[x // 2, x // 2] for x in det))


def pair_label(spatial: int, npair: int) -> int:
    """Pair of a spatial orbital in the mirror numbering (o_P = P, v_P = N+P)."""
    return spatial if spatial < npair else spatial - npair


def restricted_mp2(npair: int, k: int, f: np.ndarray, eri: np.ndarray) -> float:
    """-sum_{i<j, a<b} |<ij||ab>|^2 / (f_aa + f_bb - f_ii - f_jj) over the
    spin-orbital doubles whose four orbitals lie in at most k pairs."""
    occ = [so(p, s) for p in range(npair) for s in (0, 1)]
    vir = [so(npair + p, s) for p in range(npair) for s in (0, 1)]
    e = 0.0
    for i, j in itertools.combinations(occ, 2):
        for a, b in itertools.combinations(vir, 2):
            labels = {pair_label(x // 2, npair) for x in (i, j, a, b)}
            if len(labels) > k:
                continue
            v = antisym(eri, i, j, a, b)
            d = f[a // 2, a // 2] + f[b // 2, b // 2] - f[i // 2, i // 2] - f[j // 2, j // 2]
            e -= v * v / d
    return e


def restricted_mp2_zdo(npair: int, k: int, f: np.ndarray, C: np.ndarray, V: np.ndarray) -> float:
    """restricted_mp2 for a zero-differential-overlap Hamiltonian at sizes where
    the dense integral tensor does not fit: every label set S of at most k
    pairs is visited once, its local chemists' integrals formed from the MO
    coefficients, (pq|rs) = sum_xy C_xp C_xq V_xy C_yr C_ys, and only the
    doubles whose four orbitals cover exactly S are summed."""
    e = 0.0
    for size in range(1, k + 1):
        sets = list(itertools.combinations(range(npair), size))
        if not sets:
            continue
        # local spatial orbitals of a set: o_P for P in S, then v_P
        orbs = np.array([[P for P in s] + [npair + P for P in s] for s in sets])
        Cs = C[:, orbs].transpose(1, 0, 2)                     # (sets, n, 2*size)
        m = 2 * size
        X = (Cs[:, :, :, None] * Cs[:, :, None, :]).reshape(len(sets), C.shape[0], m * m)
        Y = np.einsum("xy,syk->sxk", V, X)
        G = np.einsum("sxk,sxl->skl", X, Y).reshape(len(sets), m, m, m, m)   # (pq|rs)
        label = np.array(list(range(size)) * 2)                 # local orbital -> role
        occ = [(p, s) for p in range(size) for s in (0, 1)]
        vir = [(size + p, s) for p in range(size) for s in (0, 1)]
        fd = np.array([[f[o, o] for o in row] for row in orbs])  # (sets, 2*size)
        for (i, si), (j, sj) in itertools.combinations(occ, 2):
            for (a, sa), (b, sb) in itertools.combinations(vir, 2):
                if len({label[i], label[j], label[a], label[b]}) != size:
                    continue
                # <ij||ab> = (ia|jb) d(si,sa) d(sj,sb) - (ib|ja) d(si,sb) d(sj,sa)
                v = np.zeros(len(sets))
                if si == sa and sj == sb:
                    v = v + G[:, i, a, j, b]
                if si == sb and sj == sa:
                    v = v - G[:, i, b, j, a]
                d = fd[:, a] + fd[:, b] - fd[:, i] - fd[:, j]
                e -= float(np.sum(v * v / d))
    return e
