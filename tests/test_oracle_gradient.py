"""Pins of the oracle gradient: central finite differences of the solved
energy (independent of the Lagrangian route), homogeneity
<f, dE/df> + <v, dE/dv> = E_c (R and E_c are linear in H, so t is unchanged
under H -> sH) and tr(dE/df) restricted to... invariance of E_c under f -> f + c I."""
import numpy as np
import pytest

from inputs import random_amplitudes, random_bfactors, random_fock
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
