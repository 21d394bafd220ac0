"""GPU parity of the PQ path (HIP kernels through the C ABI) against the FP64
oracle.  Tolerances: residual max|R_gpu - R_cpu| <= 1e-12 * max(1, max|R|);
energies 1e-10 Eh; amplitudes 1e-9 at ||R|| <= 1e-12 (tolerances derived in
the design doc from FP64 rounding of O(1e4)-term sums)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from inputs import chain_problem, random_amplitudes, random_bfactors, random_fock
from oracle import integrals as oint
from oracle import layout, solver, tier_a

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def pq():
    import paper_1609_00077_amd as pq
    pq._lib.load()
    return pq


def _d(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _random_system(N, seed):
    f = random_fock(N, seed=seed)
    B = random_bfactors(N, seed=seed + 1)
    return f, oint.eri_packed_from_b(B, N, 2)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_residual_matches_definitional_oracle(pq, N):
    f, eri = _random_system(N, 100 + N)
    t = random_amplitudes(N, "pq", seed=200 + N, scale=0.1)
    RA, EA = tier_a.TierA(N, 2).residual(f, layout.unpack_eri(eri, N, 2), t)
    R = pq.pq_residual(_d(f), _d(eri), _d(t)).cpu().numpy()
    tol = 1e-12 * max(1.0, np.abs(RA).max())
    assert np.abs(R - RA).max() <= tol, (N, np.abs(R - RA).max())
    E = pq.pq_energy(_d(f), _d(eri), _d(t))
    assert abs(E - EA) <= 1e-12


def test_residual_ppp_chain_with_device_integrals(pq):
    prob = chain_problem(8, U=4.0, seed=8)
    N = 4
    f_dev, eri_dev = pq.integrals(_d(prob.F_site), _d(prob.V), _d(prob.C), k=2)
    f_ref, eri_ref = oint.chain_integrals(prob, 2)
    assert np.abs(f_dev.cpu().numpy() - f_ref).max() < 1e-12
    assert np.abs(eri_dev.cpu().numpy() - eri_ref).max() < 1e-12
    t = random_amplitudes(N, "pq", seed=81, scale=0.05)
    RA, _ = tier_a.TierA(N, 2).residual(f_ref, layout.unpack_eri(eri_ref, N, 2), t)
    R = pq.pq_residual(f_dev, eri_dev, _d(t)).cpu().numpy()
    assert np.abs(R - RA).max() <= 1e-12 * max(1.0, np.abs(RA).max())


@pytest.mark.parametrize("nsites", [40, 140])
def test_integrals_match_oracle(pq, nsites):
    prob = chain_problem(nsites, U=4.0, seed=nsites)
    f_dev, eri_dev = pq.integrals(_d(prob.F_site), _d(prob.V), _d(prob.C), k=2)
    f_ref, eri_ref = oint.chain_integrals(prob, 2)
    assert np.abs(f_dev.cpu().numpy() - f_ref).max() < 1e-11
    assert np.abs(eri_dev.cpu().numpy() - eri_ref).max() < 1e-12


def test_solve_4e4o_is_fci(pq):
    prob = chain_problem(4, U=4.0, seed=4)
    f, eri = oint.chain_integrals(prob, 2)
    res = pq.pq_solve(_d(f), _d(eri), tol=1e-12)
    efci, _ = tier_a.TierA(2, 2).fci(f, oint.eri_dense_zdo(prob.C, prob.V))
    assert abs(res.energy - efci) < 1e-10


def test_solve_8_sites_matches_oracle_solve(pq):
    prob = chain_problem(8, U=4.0, seed=8)
    N = 4
    f, eri = oint.chain_integrals(prob, 2)
    res = pq.pq_solve(_d(f), _d(eri), tol=1e-12)
    ta = tier_a.TierA(N, 2)
    eri_t = layout.unpack_eri(eri, N, 2)
    ref = solver.solve(lambda t: ta.residual(f, eri_t, t)[0], lambda t: ta.energy(f, eri_t, t),
                       solver.denominators(f, N, 2), tol=1e-12)
    assert ref.converged
    assert abs(res.energy - ref.energy) < 1e-10
    assert np.abs(res.t.cpu().numpy() - ref.t).max() < 1e-9
