"""Exterior-algebra form of the pair-truncated CC similarity transform.

Generators.  Pair role r carries generators 4r+b, b = 0: a(o alpha),
1: a(o beta), 2: a+(v alpha), 3: a+(v beta).  They anticommute and square to
zero, and every excited determinant is (monomial)|0>.  The de-excitation
operators a+(o), a(v) act as left derivatives d/dg.

Normal-ordered Hamiltonian (Sec. II; f whole, v truncated to <= k pairs):
    H_N = sum_pq f_pq {p+ q} + 1/4 sum_pqrs <pq||rs> {p+ q+ s r}
becomes sum_h c_h g_{I_h} d_{J_h}.  Because g's commute through e^{T} up to
sign and d_J e^{T} = P_J(T) e^{T}, with P_J a signed sum over set partitions
of J of products of derivatives of T,
    e^{-T} H_N e^{T} = sum_h c_h g_{I_h} P_{J_h}(T).
"""
from __future__ import annotations

import itertools
from functools import lru_cache

# ----------------------------------------------------------------- monomials


def sort_sign(seq):
    """(sign, sorted tuple) of a product of anticommuting symbols; sign 0 if
    a symbol repeats."""
    seq = list(seq)
    if len(set(seq)) != len(seq):
        return 0, ()
    sign = 1
    # bubble sort counting transpositions (sequences are short)
    for i in range(len(seq)):
        for j in range(len(seq) - 1 - i):
            if seq[j] > seq[j + 1]:
                seq[j], seq[j + 1] = seq[j + 1], seq[j]
                sign = -sign
    return sign, tuple(seq)


def derive_monomial(K, mono):
    """d_K applied to the monomial mono (sorted tuple); d_K = d_K[0] d_K[1] ...
    acts right to left.  Returns (sign, remaining tuple) or (0, ())."""
    cur = list(mono)
    sign = 1
    for x in reversed(K):
        if x not in cur:
            return 0, ()
        pos = cur.index(x)
        if pos % 2:
            sign = -sign
        cur.pop(pos)
    return sign, tuple(cur)


def pattern_gens(role: int, e: int):
    return tuple(4 * role + b for b in range(4) if e >> b & 1)


def slot_monomial(roles, pats):
    out = ()
    for r, e in zip(roles, pats):
        out += pattern_gens(r, e)
    return out


def pattern_charge(e: int):
    return ((e >> 2) & 1) - (e & 1), ((e >> 3) & 1) - ((e >> 1) & 1)


@lru_cache(maxsize=None)
def pattern_tuples(nlab: int):
    """Nonempty pattern tuples with zero total charge, lexicographic (the
    packed amplitude order)."""
    out = []
    for tup in itertools.product(range(1, 16), repeat=nlab):
        if sum(pattern_charge(e)[0] for e in tup) == 0 and \
           sum(pattern_charge(e)[1] for e in tup) == 0:
            out.append(tup)
    return tuple(out)


# -------------------------------------------------------------- Hamiltonian
# spatial orbital of a role: 2*role + type (type 0 = o, 1 = v)
# spin orbital: (role, type, spin)


def _op_of(spin_orb, creation: bool):
    """('g' | 'd', generator) of a+ (creation) or a of a spin orbital."""
    role, typ, spin = spin_orb
    if typ == 0:      # occupied: a = g (hole), a+ = d
        return ("g" if not creation else "d", 4 * role + spin)
    return ("g" if creation else "d", 4 * role + 2 + spin)


def normal_order(ops):
    """{X1 ... Xn} as (sign, I, J): all g's moved left of all d's."""
    n = len(ops)
    gs = [i for i in range(n) if ops[i][0] == "g"]
    ds = [i for i in range(n) if ops[i][0] == "d"]
    perm = gs + ds
    # parity of perm
    sign = 1
    p = list(perm)
    for i in range(n):
        for j in range(i + 1, n):
            if p[i] > p[j]:
                sign = -sign
    return sign, tuple(ops[i][1] for i in gs), tuple(ops[i][1] for i in ds)


def eri_canon(p, q, r, s):
    """Canonical representative of (pq|rs) under the 8-fold symmetry."""
    imgs = [(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
            (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)]
    return min(imgs)


@lru_cache(maxsize=None)
def hamiltonian_terms(roles: tuple, k: int):
    """Normal-ordered H_N terms whose spin orbitals span exactly `roles`.

    Returns {(I, J): {symbol: weight}} with I, J sorted generator tuples and
    symbols ('f', p, q) (spatial orbitals 2*role+type, general matrix) or
    ('v', p, q, r, s) (chemists' integral, canonical image).
    """
    rs = set(roles)
    sos = [(r, t, s) for r in roles for t in (0, 1) for s in (0, 1)]
    acc = {}

    def add(ops, sym, w):
        sg, I, J = normal_order(ops)
        s1, I2 = sort_sign(I)
        s2, J2 = sort_sign(J)
        if s1 == 0 or s2 == 0:
            return
        key = (I2, J2)
        d = acc.setdefault(key, {})
        d[sym] = d.get(sym, 0.0) + sg * s1 * s2 * w
    # one-body
    for p in sos:
        for q in sos:
            if p[2] != q[2] or {p[0], q[0]} != rs:
                continue
            ops = [_op_of(p, True), _op_of(q, False)]
            add(ops, ("f", 2 * p[0] + p[1], 2 * q[0] + q[1]), 1.0)
    # two-body: 1/4 <pq||rs> {p+ q+ s r}
    if len(roles) <= k:
        for p, q, r, s in itertools.product(sos, repeat=4):
            if {p[0], q[0], r[0], s[0]} != rs:
                continue
            ops = [_op_of(p, True), _op_of(q, True), _op_of(s, False), _op_of(r, False)]
            sp = lambda x: 2 * x[0] + x[1]
            if p[2] == r[2] and q[2] == s[2]:
                add(ops, ("v",) + eri_canon(sp(p), sp(r), sp(q), sp(s)), 0.25)
            if p[2] == s[2] and q[2] == r[2]:
                add(ops, ("v",) + eri_canon(sp(p), sp(s), sp(q), sp(r)), -0.25)
    out = {}
    for key, d in acc.items():
        d = {s: w for s, w in d.items() if abs(w) > 1e-14}
        if d:
            out[key] = d
    return out


# ------------------------------------------------------ connected derivative


@lru_cache(maxsize=None)
def partition_products(J: tuple):
    """e^{-T} d_J e^{T} = sum sign * D_{K1} D_{K2} ... with D_K = d_K T.

    Returns a tuple of (sign, (K1, K2, ...)); each K keeps the order of J.
    """
    if not J:
        return ((1, ()),)
    j, rest = J[0], J[1:]
    out = {}
    for sign, blocks in partition_products(rest):
        # d_j acting on D_{K1} ... D_{Km}: derivation with grading
        par = 0
        for i, K in enumerate(blocks):
            nb = list(blocks)
            nb[i] = (j,) + K
            key = tuple(nb)
            out[key] = out.get(key, 0) + sign * (-1) ** par
            par += len(K)
        # (-1)^{|rest|} P_rest D_(j)
        key = tuple(blocks) + ((j,),)
        out[key] = out.get(key, 0) + sign * (-1) ** len(rest)
    return tuple((s, b) for b, s in out.items() if s != 0)
