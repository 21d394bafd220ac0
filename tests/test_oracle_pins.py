"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test fails for a plausible mistake in the oracle: a dropped term, a
wrong sign or index, a transposed operand or a wrong truncation.
"""
import itertools
from math import comb

import numpy as np
import pytest

from inputs import chain_problem, random_amplitudes, random_bfactors, random_fock
from oracle import integrals, layout, solver, tier_a, tier_b
import fermi_ref as fr


def _solve_tier_a(N, k, f, eri_packed, tol=1e-12):
    ta = tier_a.TierA(N, k)
    eri_t = layout.unpack_eri(eri_packed, N, k)
    D = solver.denominators(f, N, k)
    res = solver.solve(lambda t: ta.residual(f, eri_t, t)[0],
                       lambda t: ta.energy(f, eri_t, t), D, tol=tol, max_iter=300)
    assert res.converged
    return res


# ------------------------------------------------------------- counts (Table II)
def test_manifold_counts():
    # unique excitations per label set: 3, 29, 303 (and 6, 43, 84 unique integrals)
    assert [len(layout.pattern_tuples(n)) for n in (1, 2, 3)] == [3, 29, 303]
    assert [len(layout.eri_quads(n)) for n in (1, 2, 3)] == [6, 43, 84]
    # PQ at N=2 and PH at N=3 span the whole determinant space but the reference
    assert layout.amp_count(2, 2) == comb(4, 2) ** 2 - 1
    assert layout.amp_count(3, 3) == comb(6, 3) ** 2 - 1

    def rank(tup):
        return sum(bin(e & 3).count("1") for e in tup)
    # Table II, rank-1 column: T1 has 2 subtensors (alpha, beta), T2 has 1
    r1 = [rank(t) for t in layout.pattern_tuples(1)]
    assert r1.count(1) == 2 and r1.count(2) == 1
    # rank-2 singles: t_P^Q alpha and beta, 2 subtensors, each both orders unique
    r2 = [rank(t) for t in layout.pattern_tuples(2)]
    assert r2.count(1) == 2 * 2
    assert max(r2) == 4 and r2.count(4) == 1
    r3 = [rank(t) for t in layout.pattern_tuples(3)]
    assert max(r3) == 6 and r3.count(6) == 1


# ------------------------------------------------------- exactness (Sec. I, Table VI)
def test_pq_exact_for_4e4o():
    prob = chain_problem(4, U=4.0, seed=4)
    f = integrals.mo_fock(prob.F_site, prob.C)
    eri = integrals.eri_dense_zdo(prob.C, prob.V)
    res = _solve_tier_a(2, 2, f, layout.pack_eri(eri, 2, 2))
    efci, eref = tier_a.TierA(2, 2).fci(f, eri)
    assert abs(res.energy - efci) < 1e-10
    assert abs(eref + prob.E_core - prob.E_rhf) < 1e-10


def test_ph_exact_for_6e6o():
    prob = chain_problem(6, U=4.0, seed=6)
    f = integrals.mo_fock(prob.F_site, prob.C)
    eri = integrals.eri_dense_zdo(prob.C, prob.V)
    res = _solve_tier_a(3, 3, f, layout.pack_eri(eri, 3, 3))
    efci, _ = tier_a.TierA(3, 3).fci(f, eri)
    assert abs(res.energy - efci) < 1e-10


def test_pq_not_exact_for_6e6o():
    # PQ truncates integrals and amplitudes at three pairs: not FCI there
    prob = chain_problem(6, U=4.0, seed=6)
    f = integrals.mo_fock(prob.F_site, prob.C)
    eri = integrals.eri_dense_zdo(prob.C, prob.V)
    res = _solve_tier_a(3, 2, f, layout.pack_eri(eri, 3, 2))
    efci, _ = tier_a.TierA(3, 3).fci(f, eri)
    assert abs(res.energy - efci) > 1e-5


def test_dimer_closed_form():
    # 2-site chain: covalent/ionic 2x2 problem; core-charge form shifts by -V
    prob = chain_problem(2, U=4.0, seed=2)
    t = prob.h_site[0, 1]
    U = prob.U
    V = prob.V[0, 1]
    exact = 0.5 * (U + V) - np.sqrt((0.5 * (U - V)) ** 2 + 4 * t * t) - V
    f = integrals.mo_fock(prob.F_site, prob.C)
    eri = integrals.eri_dense_zdo(prob.C, prob.V)
    for k in (1, 2, 3):
        res = _solve_tier_a(1, k, f, layout.pack_eri(eri, 1, k))
        assert abs(prob.E_rhf + res.energy - exact) < 1e-10


def test_pp_is_sum_of_pair_fci():
    # k=1 with a diagonal Fock matrix: independent pairs (Sec. II on PP)
    prob = chain_problem(6, U=3.0, seed=11)
    f = integrals.mo_fock(prob.F_site, prob.C)
    assert np.abs(f - np.diag(np.diag(f))).max() < 1e-9
    f = np.diag(np.diag(f))
    eri = integrals.eri_dense_zdo(prob.C, prob.V)
    res = _solve_tier_a(3, 1, f, layout.pack_eri(eri, 3, 1))
    total = 0.0
    for P in range(3):
        orbs = [P, 3 + P]
        fs = f[np.ix_(orbs, orbs)]
        es = eri[np.ix_(orbs, orbs, orbs, orbs)]
        total += tier_a.TierA(1, 1).fci(fs, es)[0]
    assert abs(res.energy - total) < 1e-10


# ------------------------------------------------------------- closed forms
def _random_system(N, k, seed):
    f = random_fock(N, seed=seed)
    B = random_bfactors(N, seed=seed + 1)
    eri_full = integrals.eri_dense_from_b(B)
    packed = integrals.eri_packed_from_b(B, N, k)
    return f, eri_full, packed


@pytest.mark.parametrize("N,k", [(2, 2), (3, 2), (3, 3)])
def test_residual_at_zero_amplitudes(N, k):
    """R(t=0)_mu = <g^mu 0| H_N |0>: f_ai for singles, <ab||ij> for doubles,
    zero for triples and up; built here with a separate fermion code."""
    f, eri_full, packed = _random_system(N, k, 7)
    eri_t = layout.unpack_eri(packed, N, k)
    R, E = tier_a.TierA(N, k).residual(f, eri_t, np.zeros(layout.amp_count(N, k)))
    assert abs(E) < 1e-14
    hn0 = fr.hn_on_reference(N, f, eri_t)
    for pos, labels, tup in layout.iter_amp_slots(N, k):
        d = fr.apply_string(fr.reference(N), fr.slot_ops(N, labels, tup))
        assert abs(R[pos] - fr.overlap(d, hn0)) < 1e-13


@pytest.mark.parametrize("N,k", [(2, 2), (3, 2), (3, 3)])
def test_energy_formula(N, k):
    """E_c = sum f_ia t_i^a + 1/4 sum <ij||ab> t_ij^ab + 1/2 sum <ij||ab> t_i^a t_j^b
    (Eqs. (2)-(3) give its doubles part), with the slot signs found by applying
    the slot operators to the reference."""
    f, eri_full, packed = _random_system(N, k, 9)
    eri_t = layout.unpack_eri(packed, N, k)
    t = random_amplitudes(N, "pq" if k == 2 else "ph", seed=10, scale=0.2)
    E = tier_a.TierA(N, k).energy(f, eri_t, t)
    ref = fr.reference(N)
    occ = [fr.so(p, s) for p in range(N) for s in (0, 1)]
    vir = [fr.so(N + p, s) for p in range(N) for s in (0, 1)]
    t1 = {}
    t2 = {}
    for pos, labels, tup in layout.iter_amp_slots(N, k):
        st = fr.apply_string(ref, fr.slot_ops(N, labels, tup))
        (det, c), = st.items()
        refdet = set(next(iter(ref)))
        holes = sorted(refdet - set(det))
        parts = sorted(set(det) - refdet)
        if len(holes) == 1:
            # a+_a a_i |0> has the same determinant; its sign fixes t_i^a
            s = fr.apply_string(ref, [(True, parts[0]), (False, holes[0])])[det]
            t1[holes[0], parts[0]] = c * s * t[pos]
        elif len(holes) == 2:
            i, j = holes
            a, b = parts
            s = fr.apply_string(ref, [(True, a), (True, b), (False, j), (False, i)])[det]
            t2[i, j, a, b] = c * s * t[pos]
    e = 0.0
    for (i, a), v in t1.items():
        e += f[i // 2, a // 2] * v if i % 2 == a % 2 else 0.0
    for (i, j, a, b), v in t2.items():          # i<j, a<b: the 1/4 cancels
        e += fr.antisym(eri_t, i, j, a, b) * v
    for (i, a), v in t1.items():
        for (j, b), w in t1.items():
            e += 0.5 * fr.antisym(eri_t, i, j, a, b) * v * w
    assert abs(E - e) < 1e-13


# ------------------------------------------------------------- invariants
def test_residual_polynomial_degree_four():
    N, k = 3, 2
    f, _, packed = _random_system(N, k, 13)
    eri_t = layout.unpack_eri(packed, N, k)
    ta = tier_a.TierA(N, k)
    t = random_amplitudes(N, "pq", seed=14, scale=0.1)
    d = random_amplitudes(N, "pq", seed=15, scale=0.1)
    vals = [ta.residual(f, eri_t, t + s * d)[0] for s in range(6)]
    fifth = sum((-1) ** (5 - s) * comb(5, s) * vals[s] for s in range(6))
    fourth = sum((-1) ** (4 - s) * comb(4, s) * vals[s] for s in range(5))
    assert np.abs(fifth).max() < 1e-11
    assert np.abs(fourth).max() > 1e-6       # the quartic terms are there


def test_residual_linear_in_hamiltonian():
    N, k = 3, 2
    f1, _, p1 = _random_system(N, k, 17)
    f2, _, p2 = _random_system(N, k, 19)
    ta = tier_a.TierA(N, k)
    t = random_amplitudes(N, "pq", seed=20, scale=0.1)
    a, b = 0.7, -1.3
    R1 = ta.residual(f1, layout.unpack_eri(p1, N, k), t)[0]
    R2 = ta.residual(f2, layout.unpack_eri(p2, N, k), t)[0]
    R12 = ta.residual(a * f1 + b * f2, layout.unpack_eri(a * p1 + b * p2, N, k), t)[0]
    assert np.abs(R12 - a * R1 - b * R2).max() < 1e-12


def _permute_system(N, k, perm, f, packed, t):
    """Relabel pairs P -> perm[P] in f, integrals and amplitudes."""
    orb = np.concatenate([perm, N + np.asarray(perm)])
    fp = np.zeros_like(f)
    fp[np.ix_(orb, orb)] = f
    full = layout.unpack_eri(packed, N, k)
    fullp = np.zeros_like(full)
    fullp[np.ix_(orb, orb, orb, orb)] = full
    packed_p = layout.pack_eri(fullp, N, k)
    tp = np.zeros_like(t)
    for pos, labels, tup in layout.iter_amp_slots(N, k):
        new = [(perm[P], e) for P, e in zip(labels, tup)]
        order = sorted(range(len(new)), key=lambda i: new[i][0])
        # sign of reordering the pair factors g^e (parity |e|)
        sgn = 1.0
        par = [bin(e).count("1") % 2 for _, e in new]
        for i in range(len(order)):
            for j in range(i + 1, len(order)):
                if order[i] > order[j] and par[order[i]] and par[order[j]]:
                    sgn = -sgn
        nl = tuple(new[i][0] for i in order)
        nt = tuple(new[i][1] for i in order)
        m = layout.pattern_tuples(len(nl)).index(nt)
        tp[layout.amp_slot(N, nl, m)] = sgn * t[pos]
    return fp, packed_p, tp


@pytest.mark.parametrize("k", [2, 3])
def test_pair_relabelling_invariance(k):
    N = 4 if k == 2 else 3
    f, _, packed = _random_system(N, k, 23)
    t = random_amplitudes(N, "pq" if k == 2 else "ph", seed=24, scale=0.1)
    perm = [2, 0, 3, 1] if N == 4 else [2, 0, 1]
    ta = tier_a.TierA(N, k)
    R, E = ta.residual(f, layout.unpack_eri(packed, N, k), t)
    fp, pp, tp = _permute_system(N, k, perm, f, packed, t)
    Rp, Ep = ta.residual(fp, layout.unpack_eri(pp, N, k), tp)
    _, _, Rmapped = _permute_system(N, k, perm, f, packed, R)
    assert abs(E - Ep) < 1e-12
    assert np.abs(Rp - Rmapped).max() < 1e-12


def test_not_invariant_to_occupied_rotation():
    # rotating o_0 with o_1 changes the PQ energy at N>=3 (Sec. II)
    prob = chain_problem(6, U=4.0, seed=6)
    f = integrals.mo_fock(prob.F_site, prob.C)
    eri = integrals.eri_dense_zdo(prob.C, prob.V)
    e0 = _solve_tier_a(3, 2, f, layout.pack_eri(eri, 3, 2)).energy
    th = 0.3
    C2 = prob.C.copy()
    c, s = np.cos(th), np.sin(th)
    C2[:, [0, 1]] = prob.C[:, [0, 1]] @ np.array([[c, -s], [s, c]])
    f2 = integrals.mo_fock(prob.F_site, C2)
    eri2 = integrals.eri_dense_zdo(C2, prob.V)
    e1 = _solve_tier_a(3, 2, f2, layout.pack_eri(eri2, 3, 2)).energy
    assert abs(e1 - e0) > 1e-6


def test_size_consistency():
    """Two non-interacting 4-site chains with fragment-local pairs:
    E_PQ(A+B) = E_PQ(A) + E_PQ(B) (size extensivity, Sec. II)."""
    pa = chain_problem(4, U=4.0, seed=31)
    pb = chain_problem(4, U=3.0, seed=32)
    fa, fb = (integrals.mo_fock(p.F_site, p.C) for p in (pa, pb))
    ea, eb = (integrals.eri_dense_zdo(p.C, p.V) for p in (pa, pb))
    N = 4
    # pairs 0,1 from A and 2,3 from B; orbitals [o0..o3, v0..v3]
    oa = [0, 1, 4, 5]
    ob = [2, 3, 6, 7]
    f = np.zeros((8, 8))
    f[np.ix_(oa, oa)] = fa
    f[np.ix_(ob, ob)] = fb
    eri = np.zeros((8,) * 4)
    eri[np.ix_(oa, oa, oa, oa)] = ea
    eri[np.ix_(ob, ob, ob, ob)] = eb
    res = _solve_tier_a(N, 2, f, layout.pack_eri(eri, N, 2))
    efa = tier_a.TierA(2, 2).fci(fa, ea)[0]
    efb = tier_a.TierA(2, 2).fci(fb, eb)[0]
    assert abs(res.energy - efa - efb) < 1e-10


def test_tier_b_equals_tier_a_beyond_cluster_size():
    """The sub-cluster sum is complete: at N=5 (PQ) every residual block and
    the energy agree with the full determinant-space evaluation."""
    N, k = 5, 2
    f, _, packed = _random_system(N, k, 41)
    t = random_amplitudes(N, "pq", seed=42, scale=0.1)
    RA, EA = tier_a.TierA(N, k).residual(f, layout.unpack_eri(packed, N, k), t)
    tb = tier_b.TierB(N, k, f, packed)
    for L in [(0,), (3,), (0, 4), (1, 2), (2, 4)]:
        for s, v in tb.residual_block(L, t).items():
            assert abs(RA[s] - v) < 1e-13
    assert abs(tb.energy(t) - EA) < 1e-13


def test_tier_b_swapped_sums_equal_block_sums():
    """residual_all (each sub-system once, Moebius weights per label-set size)
    equals the determinant-space residual at N=5 and the block-by-block
    inclusion-exclusion at N=6."""
    for N, seed in ((5, 43), (6, 45)):
        f, _, packed = _random_system(N, 2, seed)
        t = random_amplitudes(N, "pq", seed=seed + 1, scale=0.1)
        tb = tier_b.TierB(N, 2, f, packed)
        R = tb.residual_all(t, workers=2)
        if N == 5:
            RA, _ = tier_a.TierA(N, 2).residual(f, layout.unpack_eri(packed, N, 2), t)
            assert np.abs(R - RA).max() < 1e-13
        else:
            for L in [(0,), (5,), (0, 5), (2, 3)]:
                for s, v in tb.residual_block(L, t).items():
                    assert abs(R[s] - v) < 1e-13


def test_packed_integrals_match_dense():
    prob = chain_problem(8, U=4.0, seed=8)
    eri = integrals.eri_dense_zdo(prob.C, prob.V)
    for k in (2, 3):
        assert np.abs(integrals.eri_packed_zdo(prob.C, prob.V, 4, k)
                      - layout.pack_eri(eri, 4, k)).max() < 1e-13
    # 8-fold symmetry of the site-basis transformation
    assert np.abs(eri - eri.transpose(1, 0, 2, 3)).max() < 1e-13
    assert np.abs(eri - eri.transpose(2, 3, 0, 1)).max() < 1e-13


# ------------------------------------------------ denominators (Table IV)
@pytest.mark.parametrize("N,k", [(2, 2), (3, 3)])
def test_denominators_from_diagonal_fock_operator(N, k):
    """D_mu is the change of <F_d> = sum_p f_pp <a+_p a_p> from the reference to
    the excited determinant tau_mu|0>, found by applying the slot's operator
    string with the separate fermion code (a wrong orbital, spin or sign in
    the oracle's bit-pattern sum fails it).  A non-symmetric diagonal pattern
    is used so that occupied and virtual entries cannot be confused."""
    rng = np.random.default_rng(51 + N)
    f = random_fock(N, seed=51)
    f[np.diag_indices(2 * N)] = rng.uniform(-3.0, 3.0, 2 * N)
    D = solver.denominators(f, N, k)
    ref = fr.reference(N)
    e0 = fr.diagonal_one_body(next(iter(ref)), f)
    for pos, labels, tup in layout.iter_amp_slots(N, k):
        (det, _), = fr.apply_string(ref, fr.slot_ops(N, labels, tup)).items()
        assert abs(D[pos] - (fr.diagonal_one_body(det, f) - e0)) < 1e-13
    # closed form for the pair double o_P(alpha beta) -> v_P(alpha beta)
    m = layout.pattern_tuples(1).index((15,))
    for P in range(N):
        assert abs(D[layout.amp_slot(N, (P,), m)] - 2 * (f[N + P, N + P] - f[P, P])) < 1e-13
    # the level shift adds to every slot
    assert np.abs(solver.denominators(f, N, k, shift=0.25) - D - 0.25).max() < 1e-15


# ------------------------------------------------ weak coupling (Sec. II)
@pytest.mark.parametrize("N,k", [(3, 2), (3, 3), (4, 2)])
def test_first_jacobi_step_gives_pair_restricted_mp2(N, k):
    """With a diagonal f, one Jacobi step from t = 0 gives t = -<ab||ij>/D on
    the doubles of the manifold, and its energy is the MP2 energy restricted to
    the doubles whose orbitals lie in at most k pairs, summed here over spin
    orbitals with the untruncated integrals."""
    f = np.diag(np.diag(random_fock(N, seed=61 + N)))
    B = random_bfactors(N, seed=62 + N, scale=0.2)
    eri_full = integrals.eri_dense_from_b(B)
    packed = integrals.eri_packed_from_b(B, N, k)
    eri_t = layout.unpack_eri(packed, N, k)
    ta = tier_a.TierA(N, k)
    R0, _ = ta.residual(f, eri_t, np.zeros(layout.amp_count(N, k)))
    t1 = -R0 / solver.denominators(f, N, k)
    e1 = ta.energy(f, eri_t, t1)
    emp2 = fr.restricted_mp2(N, k, f, eri_full)
    assert emp2 < -1e-4
    assert abs(e1 - emp2) < 1e-13 * max(1.0, abs(emp2))
    # PQ keeps fewer doubles than PH: the restriction is really applied
    if k == 3:
        assert fr.restricted_mp2(N, 2, f, eri_full) > emp2 + 1e-6


def test_weak_coupling_limit_of_solved_energy():
    """U -> 0 on the 8-site chain: E_c / E_MP2(pair-restricted) -> 1 with an
    error of first order in U (the third-order energy over the second)."""
    devs = []
    for U in (0.02, 0.01):
        prob = chain_problem(8, U=U, seed=8)
        f = integrals.mo_fock(prob.F_site, prob.C)
        eri = integrals.eri_dense_zdo(prob.C, prob.V)
        res = _solve_tier_a(4, 2, f, layout.pack_eri(eri, 4, 2))
        emp2 = fr.restricted_mp2(4, 2, np.diag(np.diag(f)), eri)
        devs.append(abs(res.energy / emp2 - 1.0))
    assert devs[0] < 0.1
    assert 1.6 < devs[0] / devs[1] < 2.4


# ------------------------------------------------ size consistency, PH (Sec. II)
def test_size_consistency_ph():
    """Two non-interacting 4-site chains (2 pairs each) with fragment-local
    pairs at k = 3: the three-pair amplitudes that span both fragments must
    vanish and E_PH(A+B) = E(A) + E(B), each exact (FCI) for two pairs."""
    pa = chain_problem(4, U=4.5, seed=33)
    pb = chain_problem(4, U=2.5, seed=34)
    fa, fb = (integrals.mo_fock(p.F_site, p.C) for p in (pa, pb))
    ea, eb = (integrals.eri_dense_zdo(p.C, p.V) for p in (pa, pb))
    oa = [0, 1, 4, 5]
    ob = [2, 3, 6, 7]
    f = np.zeros((8, 8))
    f[np.ix_(oa, oa)] = fa
    f[np.ix_(ob, ob)] = fb
    eri = np.zeros((8,) * 4)
    eri[np.ix_(oa, oa, oa, oa)] = ea
    eri[np.ix_(ob, ob, ob, ob)] = eb
    res = _solve_tier_a(4, 3, f, layout.pack_eri(eri, 4, 3))
    efa = tier_a.TierA(2, 2).fci(fa, ea)[0]
    efb = tier_a.TierA(2, 2).fci(fb, eb)[0]
    assert abs(res.energy - efa - efb) < 1e-10
    # amplitudes on label sets mixing the fragments vanish
    for pos, labels, _ in layout.iter_amp_slots(4, 3):
        if {0, 1} & set(labels) and {2, 3} & set(labels):
            assert abs(res.t[pos]) < 1e-9


# ------------------------------------------------ excitation-rank limits (Sec. V)
def test_rank_limit_counts():
    rk = solver.slot_ranks(3, 3)
    assert rk.max() == 6 and rk.min() == 1
    # per pair: 2 singles (o -> v alpha, beta) and 1 double; per pair of pairs
    # 4 singles, 16 doubles, 8 triples, 1 quadruple (Table II's rank columns)
    r2 = solver.slot_ranks(2, 2)
    assert np.bincount(r2).tolist() == [0, 2 * 2 + 4, 2 + 16, 8, 1]


def test_rank_two_is_exact_for_two_electron_fragments():
    """Two non-interacting 2-site chains (one pair, two electrons each):
    coupled cluster with singles and doubles only is exact for two
    electrons and size-extensive, so the rank-2 limit of PQ on the union is
    FCI(A) + FCI(B), while rank 1 is not."""
    pa = chain_problem(2, U=4.0, seed=35)
    pb = chain_problem(2, U=2.5, seed=36)
    fa, fb = (integrals.mo_fock(p.F_site, p.C) for p in (pa, pb))
    ea, eb = (integrals.eri_dense_zdo(p.C, p.V) for p in (pa, pb))
    oa, ob = [0, 2], [1, 3]
    f = np.zeros((4, 4))
    f[np.ix_(oa, oa)] = fa
    f[np.ix_(ob, ob)] = fb
    eri = np.zeros((4,) * 4)
    eri[np.ix_(oa, oa, oa, oa)] = ea
    eri[np.ix_(ob, ob, ob, ob)] = eb
    N, k = 2, 2
    packed = layout.pack_eri(eri, N, k)
    ta = tier_a.TierA(N, k)
    et = layout.unpack_eri(packed, N, k)
    D = solver.denominators(f, N, k)
    rk = solver.slot_ranks(N, k)
    exact = tier_a.TierA(1, 1).fci(fa, ea)[0] + tier_a.TierA(1, 1).fci(fb, eb)[0]
    res = solver.solve(lambda t: ta.residual(f, et, t)[0], lambda t: ta.energy(f, et, t), D,
                       tol=1e-12, max_iter=300, keep=rk <= 2)
    assert res.converged and abs(res.energy - exact) < 1e-10
    assert np.abs(res.t[rk > 2]).max() == 0.0
    r1 = solver.solve(lambda t: ta.residual(f, et, t)[0], lambda t: ta.energy(f, et, t), D,
                      tol=1e-12, max_iter=300, keep=rk <= 1)
    assert abs(r1.energy - exact) > 1e-4


def test_rank_limit_changes_ph_energy():
    """PH restricted to doubles (local CCSD on three-pair clusters) differs
    from PH-SDTQ and the full PH; SDTQ on three pairs misses only the rank-5
    and rank-6 excitations, so it lies closest to PH."""
    prob = chain_problem(6, U=4.0, seed=6)
    f = integrals.mo_fock(prob.F_site, prob.C)
    eri = layout.pack_eri(integrals.eri_dense_zdo(prob.C, prob.V), 3, 3)
    N, k = 3, 3
    ta = tier_a.TierA(N, k)
    et = layout.unpack_eri(eri, N, k)
    D = solver.denominators(f, N, k)
    rk = solver.slot_ranks(N, k)
    e = {}
    for r in (2, 4, 6):
        res = solver.solve(lambda t: ta.residual(f, et, t)[0], lambda t: ta.energy(f, et, t), D,
                           tol=1e-11, max_iter=300, keep=rk <= r)
        assert res.converged
        e[r] = res.energy
    assert abs(e[6] - e[4]) < abs(e[6] - e[2])
    assert abs(e[4] - e[2]) > 1e-5


# ------------------------------------------------ Newton's method (Sec. IV.B)
def test_newton_reaches_the_jacobi_diis_fixed_point():
    """Where Jacobi/DIIS converges (6-site chain, U = 4), Newton's method with
    the complex-step Jacobian finds the same amplitudes and energy; two
    different iterations agree on the root of the definitional residual."""
    prob = chain_problem(6, U=4.0, seed=6)
    f, eri = integrals.chain_integrals(prob, 2)
    ta = tier_a.TierA(3, 2)
    et = layout.unpack_eri(eri, 3, 2)
    R = lambda t: ta.residual(f, et, t)[0]
    E = lambda t: ta.energy(f, et, t)
    D = solver.denominators(f, 3, 2)
    ref = solver.solve(R, E, D, tol=1e-12, max_iter=300)
    nw = solver.newton(R, lambda t: ta.jacobian(f, et, t), E, np.zeros_like(D), tol=1e-12)
    assert ref.converged and nw.converged and nw.iterations < 10
    assert abs(nw.energy - ref.energy) < 1e-11
    assert np.abs(nw.t - ref.t).max() < 1e-9


def test_newton_solves_a_chain_where_jacobi_diis_stalls():
    """8-site chain at U = 10: Jacobi/DIIS is still far from converged after
    60 iterations (and after 1000, ||R|| ~ 0.09); Newton from its last iterate
    reaches ||R|| <= 1e-11 in a few steps."""
    prob = chain_problem(8, U=10.0, seed=8)
    f, eri = integrals.chain_integrals(prob, 2)
    ta = tier_a.TierA(4, 2)
    et = layout.unpack_eri(eri, 4, 2)
    R = lambda t: ta.residual(f, et, t)[0]
    E = lambda t: ta.energy(f, et, t)
    D = solver.denominators(f, 4, 2)
    jd = solver.solve(R, E, D, tol=1e-8, max_iter=60)
    assert not jd.converged and jd.rnorm > 1e-2
    nw = solver.newton(R, lambda t: ta.jacobian(f, et, t), E, jd.t, tol=1e-11)
    assert nw.converged and nw.iterations <= 6
    assert np.linalg.norm(R(nw.t)) <= 1e-11


# ------------------------------------------------ closed-shell spin symmetry (Sec. V)
@pytest.mark.parametrize("N,k", [(4, 2), (3, 3)])
def test_spin_symmetry_of_closed_shell_solutions(N, k):
    """With a spin-free Hamiltonian and the closed-shell reference the
    residual maps spin-symmetric amplitudes (t[partner] = sign t) to a
    spin-symmetric residual, and the solved amplitudes are spin-symmetric;
    amplitudes breaking the symmetry give a residual that breaks it."""
    f, _, packed = _random_system(N, k, 57)
    et = layout.unpack_eri(packed, N, k)
    ta = tier_a.TierA(N, k)
    partner, sign = layout.spin_partner(N, k)
    assert np.all(partner[partner] == np.arange(len(partner)))
    assert np.all(sign * sign[partner] == 1.0)
    # orbits: 2 per pair, 16 per pair of pairs, 155 per triple (header counts)
    orbits = np.sum(partner >= np.arange(len(partner)))
    assert orbits == 2 * N + 16 * comb(N, 2) + (155 * comb(N, 3) if k == 3 else 0)
    rng = np.random.default_rng(58)
    t = rng.uniform(-0.1, 0.1, len(partner))
    t_sym = 0.5 * (t + sign * t[partner])
    R, _ = ta.residual(f, et, t_sym)
    assert np.abs(R[partner] - sign * R).max() < 1e-13
    Rb, _ = ta.residual(f, et, t)
    assert np.abs(Rb[partner] - sign * Rb).max() > 1e-4
    res = solver.solve(lambda x: ta.residual(f, et, x)[0], lambda x: ta.energy(f, et, x),
                       solver.denominators(f, N, k), tol=1e-12, max_iter=300)
    assert np.abs(res.t[partner] - sign * res.t).max() < 1e-12


@pytest.mark.parametrize("N,k", [(3, 2), (4, 3)])
def test_restricted_mp2_by_label_sets(N, k):
    """The label-set MP2 sum used at full size equals the spin-orbital sum
    over the dense integrals of the same chain."""
    prob = chain_problem(2 * N, U=4.0, seed=70 + N)
    f = integrals.mo_fock(prob.F_site, prob.C)
    eri = np.einsum("xp,xq,xy,yr,ys->pqrs", prob.C, prob.C, prob.V, prob.C, prob.C)
    e_dense = fr.restricted_mp2(N, k, np.diag(np.diag(f)), eri)
    e_sets = fr.restricted_mp2_zdo(N, k, f, prob.C, prob.V)
    assert e_dense < -1e-3
    assert abs(e_dense - e_sets) < 1e-13
