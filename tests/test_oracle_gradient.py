"""Pins of the oracle gradient: central finite differences of the solved
energy (independent of the Lagrangian route), homogeneity
<f, dE/df> + <v, dE/dv> = E_c (R and E_c are linear in H, so t is unchanged
under H -> sH) and tr(dE/df) restricted to... invariance of E_c under f -> f + c I."""
import numpy as np
import pytest

from inputs import random_amplitudes, random_bfactors, random_fock, random_vector
from oracle import gradient, integrals, layout, solver, tier_a


def _solve(N, k, f, eri):
    ta = tier_a.TierA(N, k)
    et = layout.unpack_eri(eri, N, k)
    res = solver.solve(lambda t: ta.residual(f, et, t)[0], lambda t: ta.energy(f, et, t),
                       solver.denominators(f, N, k), tol=1e-13, max_iter=400)
    assert res.converged
    return res


@pytest.mark.parametrize("N,k", [(2, 2), (3, 2)])
def test_lagrangian_gradient_against_finite_differences(N, k):
    f = random_fock(N, seed=71, offdiag=0.05)
    eri = integrals.eri_packed_from_b(random_bfactors(N, seed=72, scale=0.2), N, k)
    res = _solve(N, k, f, eri)
    gf, ge, lam = gradient.lagrangian_gradient(N, k, f, eri, res.t)
    rng = np.random.default_rng(73)
    for _ in range(3):
        df = rng.normal(size=f.shape)
        df = 0.5 * (df + df.T)
        de = rng.normal(size=eri.shape)
        s = 1e-5
        ep = _solve(N, k, f + s * df, eri + s * de).energy
        em = _solve(N, k, f - s * df, eri - s * de).energy
        fd = (ep - em) / (2 * s)
        an = np.sum(gf * df) + np.sum(ge * de)
        assert abs(fd - an) < 1e-7 * max(1.0, abs(an))


def test_gradient_identities():
    N, k = 3, 2
    f = random_fock(N, seed=81, offdiag=0.05)
    eri = integrals.eri_packed_from_b(random_bfactors(N, seed=82, scale=0.2), N, k)
    res = _solve(N, k, f, eri)
    gf, ge, _ = gradient.lagrangian_gradient(N, k, f, eri, res.t)
    # homogeneity: E_c(sf, sv) = s E_c(f, v) with the same t
    assert abs(np.sum(gf * f) + np.sum(ge * eri) - res.energy) < 1e-10
    # f -> f + c I changes no denominator difference nor any residual: E_c invariant
    assert abs(np.trace(gf)) < 1e-10


def _phi(N, k, f, eri, t, lam, w):
    ta = tier_a.TierA(N, k)
    R, E = ta.residual(f, layout.unpack_eri(eri, N, k), t)
    return lam @ R + w * E


def test_vjp_against_finite_differences():
    """Transposed-residual contraction of the oracle vs central differences of
    lam . R + w E_c along random directions (real arithmetic, no complex step)."""
    N, k, w = 2, 2, 0.7
    f = random_fock(N, seed=91, offdiag=0.05)
    eri = integrals.eri_packed_from_b(random_bfactors(N, seed=92, scale=0.2), N, k)
    t = random_amplitudes(N, seed=93, scale=0.1)
    lam = random_vector(len(t), seed=94)
    tbar, hbar, eribar = gradient.vjp(N, k, f, eri, t, lam, w)
    rng = np.random.default_rng(95)
    for _ in range(3):
        dt, df, de = rng.normal(size=t.shape), rng.normal(size=f.shape), rng.normal(size=eri.shape)
        s = 1e-4
        fd = (_phi(N, k, f + s * df, eri + s * de, t + s * dt, lam, w)
              - _phi(N, k, f - s * df, eri - s * de, t - s * dt, lam, w)) / (2 * s)
        an = tbar @ dt + np.sum(hbar * df) + eribar @ de
        assert abs(fd - an) < 1e-7 * max(1.0, abs(an))


def test_subcluster_directional_vjp_matches_determinant_space():
    """The any-size directional form (sub-cluster sums) equals the
    determinant-space contraction dotted with the same directions."""
    N, k, w = 3, 2, 0.3
    f = random_fock(N, seed=101, offdiag=0.05)
    eri = integrals.eri_packed_from_b(random_bfactors(N, seed=102, scale=0.2), N, k)
    t = random_amplitudes(N, seed=103, scale=0.1)
    lam = random_vector(len(t), seed=104)
    tbar, hbar, eribar = gradient.vjp(N, k, f, eri, t, lam, w)
    blocks = {}
    import itertools
    for size in (1, 2):
        for L in itertools.combinations(range(N), size):
            slots = [layout.amp_slot(N, L, m) for m in range(len(layout.pattern_tuples(size)))]
            blocks[L] = {s: float(lam[s]) for s in slots}
    rng = np.random.default_rng(105)
    dt, df, de = rng.normal(size=t.shape), rng.normal(size=f.shape), rng.normal(size=eri.shape)
    d = gradient.directional_vjp_blocks(N, k, f, eri, t, blocks, w, dt, df, de, keep_cache=True)
    an = tbar @ dt + np.sum(hbar * df) + eribar @ de
    assert abs(d - an) < 1e-10 * max(1.0, abs(an))


def test_densities_equal_fci_density_where_the_model_is_exact():
    """PQ is exact for two pairs, so its response density equals the FCI
    one-particle density <Psi|E_pq|Psi> of the ground state (Hellmann-Feynman),
    built here from the FCI eigenvector in the determinant space; the trace is
    the electron count and the natural occupations lie in [0, 2]."""
    from oracle.tier_a import TierA
    N, k = 2, 2
    f = random_fock(N, seed=131, offdiag=0.05)
    B = random_bfactors(N, seed=132, scale=0.3)
    eri_full = integrals.eri_dense_from_b(B)
    eri = integrals.eri_packed_from_b(B, N, k)
    res = _solve(N, k, f, eri)
    gamma, Gamma, noons = gradient.densities(N, k, f, eri, res.t)
    ta = TierA(N, k)
    hb = ta.bare_onebody(f, eri_full)
    ns = ta.shape[0] * ta.shape[1]
    Hm = np.zeros((ns, ns))
    e = np.zeros(ta.shape)
    for i in range(ns):
        e.flat[i] = 1.0
        Hm[:, i] = ta.sigma(hb, eri_full, e).reshape(-1)
        e.flat[i] = 0.0
    w, v = np.linalg.eigh(0.5 * (Hm + Hm.T))
    psi = v[:, 0].reshape(ta.shape)
    n = 2 * N
    g_fci = np.array([[np.sum(psi * ta._e(p, q, psi)) for q in range(n)] for p in range(n)])
    assert np.abs(gamma - g_fci).max() < 1e-9
    assert abs(np.trace(gamma) - 2 * N) < 1e-10
    assert noons.min() > -1e-12 and noons.max() < 2 + 1e-12
    assert abs(noons.sum() - 2 * N) < 1e-10


def test_density_trace_and_occupations_pq_three_pairs():
    N, k = 3, 2
    f = random_fock(N, seed=141, offdiag=0.05)
    eri = integrals.eri_packed_from_b(random_bfactors(N, seed=142, scale=0.2), N, k)
    res = _solve(N, k, f, eri)
    gamma, _, noons = gradient.densities(N, k, f, eri, res.t)
    assert abs(np.trace(gamma) - 2 * N) < 1e-10
    # strongly occupied and weakly occupied halves
    assert noons[:N].min() > 1.0 > noons[N:].max()
