"""Packed layouts of amplitudes and pair-block integrals, written from the
definitions in include/pqph.h.

Orbitals.  N pairs; spatial orbital P is o_P (occupied, HOMO-P) and N+P is
v_P (virtual, LUMO+P), the mirror numbering of Fig. 1.

Local excitation patterns.  Each pair carries four excitation generators,
numbered by bit: 0 = a(o_P alpha), 1 = a(o_P beta), 2 = a+(v_P alpha),
3 = a+(v_P beta).  A pattern e in 1..15 is a set of these bits and g_P^e is
the product of its generators in ascending bit order.  The pattern's charge
per spin is (#particles - #holes) of that spin.

Amplitudes.  The excitation with label set {P0 < P1 < ...} and patterns
(e0, e1, ...) (all nonempty, total charge zero per spin) is the operator
g_{P0}^{e0} g_{P1}^{e1} ...; T is the sum over packed slots of amplitude times
operator.  Slots are grouped by the size of the label set (Eq. (1) and its PH
extension: rank-1, rank-2 and rank-3 subtensors), class-major:

  [ t1: 3 x N ]  [ t2: 29 x C(N,2) ]  [ t3: 303 x C(N,3) (PH only) ]

with the pattern tuples of one label-set size enumerated lexicographically,
pairs P<Q indexed Q(Q-1)/2 + P and triples P<Q<R indexed
R(R-1)(R-2)/6 + Q(Q-1)/2 + P.

Integrals.  Chemists' (pq|rs) with 8-fold symmetry, each unique integral
stored once, grouped by its label set (label sets of <= 2 pairs for PQ, <= 3
for PH; Table I caption).  Within a set with ascending labels the local
orbitals are numbered 2*role + type (type 0 = o, 1 = v); the stored quadruples
are p>=q, r>=s, pq>=rs (pq = p(p+1)/2 + q) in lexicographic (pq, rs) order,
keeping those whose labels cover the whole set: 6, 43 and 84 per set.

  [ e1: 6 x N ]  [ e2: 43 x C(N,2) ]  [ e3: 84 x C(N,3) (PH only) ]
"""
from __future__ import annotations

import itertools
from functools import lru_cache
from math import comb

import numpy as np


def pattern_charge(e: int):
    """(alpha, beta) charge: particles minus holes of each spin."""
    return ((e >> 2) & 1) - (e & 1), ((e >> 3) & 1) - ((e >> 1) & 1)


@lru_cache(maxsize=None)
def pattern_tuples(nlab: int):
    """All tuples of nonempty patterns over nlab labels with zero total charge."""
    out = []
    for tup in itertools.product(range(1, 16), repeat=nlab):
        ca = sum(pattern_charge(e)[0] for e in tup)
        cb = sum(pattern_charge(e)[1] for e in tup)
        if ca == 0 and cb == 0:
            out.append(tup)
    return tuple(out)


def pair_index(P: int, Q: int) -> int:
    assert P < Q
    return Q * (Q - 1) // 2 + P


def triple_index(P: int, Q: int, R: int) -> int:
    assert P < Q < R
    return R * (R - 1) * (R - 2) // 6 + Q * (Q - 1) // 2 + P


def label_sets(npair: int, size: int):
    """Label sets of one size in packed order (ascending packed index)."""
    sets = list(itertools.combinations(range(npair), size))
    if size == 2:
        sets.sort(key=lambda s: pair_index(*s))
    elif size == 3:
        sets.sort(key=lambda s: triple_index(*s))
    return sets


def set_index(labels) -> int:
    if len(labels) == 1:
        return labels[0]
    if len(labels) == 2:
        return pair_index(*labels)
    return triple_index(*labels)


def amp_count(npair: int, k: int) -> int:
    n = 3 * npair
    if k >= 2:
        n += 29 * comb(npair, 2)
    if k >= 3:
        n += 303 * comb(npair, 3)
    return n


def amp_block_offset(npair: int, size: int) -> int:
    if size == 1:
        return 0
    if size == 2:
        return 3 * npair
    return 3 * npair + 29 * comb(npair, 2)


def amp_slot(npair: int, labels, m: int) -> int:
    """Packed position of pattern-tuple number m on the sorted label set."""
    size = len(labels)
    nsets = comb(npair, size)
    return amp_block_offset(npair, size) + m * nsets + set_index(labels)


def iter_amp_slots(npair: int, k: int):
    """Yield (packed position, labels, pattern tuple) for every slot."""
    for size in range(1, k + 1):
        tuples = pattern_tuples(size)
        for labels in label_sets(npair, size):
            for m, tup in enumerate(tuples):
                yield amp_slot(npair, labels, m), labels, tup


# ---------------------------------------------------------------- integrals
@lru_cache(maxsize=None)
def eri_quads(size: int):
    """Stored local quadruples (p, q, r, s) for a label set of the given size."""
    norb = 2 * size
    pairs = [(p, q) for p in range(norb) for q in range(p + 1)]   # compound order
    out = []
    for ipq, (p, q) in enumerate(pairs):
        for irs in range(ipq + 1):
            r, s = pairs[irs]
            roles = {p // 2, q // 2, r // 2, s // 2}
            if len(roles) == size:
                out.append((p, q, r, s))
    return tuple(out)


def eri_count(npair: int, k: int) -> int:
    n = 6 * npair
    if k >= 2:
        n += 43 * comb(npair, 2)
    if k >= 3:
        n += 84 * comb(npair, 3)
    return n


def eri_block_offset(npair: int, size: int) -> int:
    if size == 1:
        return 0
    if size == 2:
        return 6 * npair
    return 6 * npair + 43 * comb(npair, 2)


def local_to_global(labels, npair: int, loc: int) -> int:
    role, typ = divmod(loc, 2)
    return labels[role] + (npair if typ else 0)


def pack_eri(eri_full: np.ndarray, npair: int, k: int) -> np.ndarray:
    """Packed pair-block vector from a dense (2N)^4 integral tensor."""
    out = np.zeros(eri_count(npair, k))
    for size in range(1, k + 1):
        quads = eri_quads(size)
        nsets = comb(npair, size)
        off = eri_block_offset(npair, size)
        for labels in label_sets(npair, size):
            si = set_index(labels)
            for u, (p, q, r, s) in enumerate(quads):
                g = [local_to_global(labels, npair, x) for x in (p, q, r, s)]
                out[off + u * nsets + si] = eri_full[g[0], g[1], g[2], g[3]]
    return out


def unpack_eri(packed: np.ndarray, npair: int, k: int) -> np.ndarray:
    """Dense (2N)^4 tensor holding the packed integrals at all 8 symmetric
    positions and zero for every label set of more than k pairs."""
    n = 2 * npair
    full = np.zeros((n, n, n, n), dtype=np.asarray(packed).dtype)
    for size in range(1, k + 1):
        quads = eri_quads(size)
        nsets = comb(npair, size)
        off = eri_block_offset(npair, size)
        for labels in label_sets(npair, size):
            si = set_index(labels)
            for u, (p, q, r, s) in enumerate(quads):
                a, b, c, d = (local_to_global(labels, npair, x) for x in (p, q, r, s))
                val = packed[off + u * nsets + si]
                for (w, x, y, z) in ((a, b, c, d), (b, a, c, d), (a, b, d, c), (b, a, d, c),
                                     (c, d, a, b), (d, c, a, b), (c, d, b, a), (d, c, b, a)):
                    full[w, x, y, z] = val
    return full


def eri_slot_multiplicity(npair: int, k: int) -> np.ndarray:
    """Number of distinct (p,q,r,s) positions each packed integral stands for."""
    out = np.zeros(eri_count(npair, k))
    for size in range(1, k + 1):
        quads = eri_quads(size)
        nsets = comb(npair, size)
        off = eri_block_offset(npair, size)
        for u, (p, q, r, s) in enumerate(quads):
            imgs = {(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                    (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)}
            out[off + u * nsets: off + (u + 1) * nsets] = len(imgs)
    return out


def spin_flip(e: int) -> int:
    """The pattern with alpha and beta exchanged (bits 0 <-> 1, 2 <-> 3)."""
    return ((e & 1) << 1) | ((e >> 1) & 1) | ((e & 4) << 1) | ((e >> 1) & 4)


def spin_flip_sign(e: int) -> int:
    """Sign of writing the spin-exchanged generators of g^e (taken in the
    order of g^e) in ascending bit order."""
    fl = [b ^ 1 for b in range(4) if e >> b & 1]
    inv = sum(1 for i in range(len(fl)) for j in range(i + 1, len(fl)) if fl[i] > fl[j])
    return -1 if inv % 2 else 1


def spin_partner(npair: int, k: int):
    """(partner slot, sign) of every packed slot: the excitation with alpha
    and beta exchanged on every pair, and the product over its pairs of the
    reordering signs.  A closed-shell (spin-free) problem keeps
    t[partner] = sign * t and R[partner] = sign * R."""
    n = amp_count(npair, k)
    partner = np.zeros(n, dtype=np.int64)
    sign = np.zeros(n)
    for pos, labels, tup in iter_amp_slots(npair, k):
        ft = tuple(spin_flip(e) for e in tup)
        m = pattern_tuples(len(labels)).index(ft)
        partner[pos] = amp_slot(npair, labels, m)
        sign[pos] = np.prod([spin_flip_sign(e) for e in tup])
    return partner, sign
