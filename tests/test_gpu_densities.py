"""Densities of the PQ Lagrangian and natural occupation numbers on the GPU
(Table IV caption: after lambda the densities are formed; Sec. IV.B, Fig. 7:
natural occupations) against the oracle's complex-step densities, and their
invariants at the benchmark size."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from inputs import chain_problem, random_bfactors, random_fock
from oracle import gradient, layout, solver, tier_a
from oracle import integrals as oint

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def pq():
    import paper_1609_00077_amd as pq
    pq._lib.load()
    return pq


def _d(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("N", [2, 3])
def test_densities_match_oracle(pq, N):
    f = random_fock(N, seed=160 + N, offdiag=0.05)
    eri = oint.eri_packed_from_b(random_bfactors(N, seed=170 + N, scale=0.2), N, 2)
    ta = tier_a.TierA(N, 2)
    et = layout.unpack_eri(eri, N, 2)
    ref = solver.solve(lambda t: ta.residual(f, et, t)[0], lambda t: ta.energy(f, et, t),
                       solver.denominators(f, N, 2), tol=1e-13, max_iter=400)
    assert ref.converged
    gamma, Gamma, noons = gradient.densities(N, 2, f, eri, ref.t)
    d = pq.pq_densities(_d(f), _d(eri), tol=1e-13)
    assert d.status == "OK"
    assert np.abs(d.gamma.cpu().numpy() - gamma).max() < 1e-9
    assert np.abs(d.Gamma.cpu().numpy() - Gamma).max() < 1e-9
    assert np.abs(np.array(d.noons) - noons).max() < 1e-9


def test_densities_140_sites(pq):
    """The benchmark chain: tr gamma = 140 electrons, the natural occupations
    sum to it, lie near [0, 2] and split into 70 strongly and 70 weakly
    occupied orbitals."""
    prob = chain_problem(140, U=4.0, seed=140)
    f, eri = pq.integrals(_d(prob.F_site), _d(prob.V), _d(prob.C), k=2)
    d = pq.pq_densities(f, eri, tol=1e-10)
    assert d.status == "OK"
    n = np.array(d.noons)
    assert abs(float(torch.trace(d.gamma)) - 140.0) < 1e-8
    assert abs(n.sum() - 140.0) < 1e-8
    assert n.max() < 2.05 and n.min() > -0.05
    assert n[69] > 1.0 > n[70]
    print("140-site PQ natural occupations around the gap:", np.round(n[64:76], 5).tolist())
