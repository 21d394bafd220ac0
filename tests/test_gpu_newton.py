"""Newton-Krylov amplitude solves (pqph_solve_opts.solver 1 and 2) for the
systems where Jacobi/DIIS stalls or diverges (Sec. IV.B), against the
oracle's Newton iteration with the exact (complex-step) Jacobian: the same
root, energies to 1e-10 Eh and amplitudes to 1e-9."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from inputs import chain_problem
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


@pytest.fixture(scope="module")
def stalled_chain():
    """8-site chain at U = 10: Jacobi/DIIS stalls; the oracle's Newton root."""
    prob = chain_problem(8, U=10.0, seed=8)
    f, eri = oint.chain_integrals(prob, 2)
    ta = tier_a.TierA(4, 2)
    et = layout.unpack_eri(eri, 4, 2)
    R = lambda t: ta.residual(f, et, t)[0]
    E = lambda t: ta.energy(f, et, t)
    D = solver.denominators(f, 4, 2)
    jd = solver.solve(R, E, D, tol=1e-8, max_iter=60)
    ref = solver.newton(R, lambda t: ta.jacobian(f, et, t), E, jd.t, tol=1e-12)
    assert ref.converged
    return f, eri, ref


def test_jacobi_diis_stalls(pq, stalled_chain):
    f, eri, _ = stalled_chain
    res = pq.pq_solve(_d(f), _d(eri), tol=1e-8, raise_on_failure=False)
    assert res.status == "NOT_CONVERGED"


@pytest.mark.parametrize("solver_mode", [1, 2])
def test_newton_krylov_reaches_the_oracle_root(pq, stalled_chain, solver_mode):
    f, eri, ref = stalled_chain
    res = pq.pq_solve(_d(f), _d(eri), tol=1e-11, solver=solver_mode)
    assert res.status == "OK", (res.status, res.rnorm, res.iterations)
    assert abs(res.energy - ref.energy) < 1e-10
    assert np.abs(res.t.cpu().numpy() - ref.t).max() < 1e-9


def test_newton_krylov_equals_jacobi_diis_where_both_converge(pq):
    """A 40-site chain at U = 4 (20 pairs): Newton-Krylov from zero and
    Jacobi/DIIS reach the same amplitudes."""
    prob = chain_problem(40, U=4.0, seed=40)
    f, eri = pq.integrals(_d(prob.F_site), _d(prob.V), _d(prob.C), k=2)
    a = pq.pq_solve(f, eri, tol=1e-11)
    b = pq.pq_solve(f, eri, tol=1e-11, solver=1)
    assert a.status == "OK" and b.status == "OK"
    assert abs(a.energy - b.energy) < 1e-10
    assert (a.t - b.t).abs().max().item() < 1e-9


def test_newton_krylov_ph(pq):
    """PH (three pairs of 8 sites: 4 pairs) by Newton-Krylov against the
    oracle's Jacobi/DIIS root."""
    prob = chain_problem(8, U=4.0, seed=8)
    f, eri = oint.chain_integrals(prob, 3)
    ta = tier_a.TierA(4, 3)
    et = layout.unpack_eri(eri, 4, 3)
    ref = solver.solve(lambda t: ta.residual(f, et, t)[0], lambda t: ta.energy(f, et, t),
                       solver.denominators(f, 4, 3), tol=1e-11)
    assert ref.converged
    res = pq.ph_solve(_d(f), _d(eri), tol=1e-11, solver=1)
    assert res.status == "OK"
    assert abs(res.energy - ref.energy) < 1e-10
    assert np.abs(res.t.cpu().numpy() - ref.t).max() < 1e-8


def test_batched_solver_2_converges_the_stalled_chain(pq, stalled_chain):
    """A batch holding the stalled chain and two ordinary ones: with solver 2
    every chain converges and each energy equals its single solve."""
    f, eri, ref = stalled_chain
    hs, es = [_d(f)], [_d(eri)]
    for n in (12, 20):
        p = chain_problem(n, U=4.0, seed=n)
        fd, ed = pq.integrals(_d(p.F_site), _d(p.V), _d(p.C), k=2)
        hs.append(fd)
        es.append(ed)
    plain = pq.pq_solve_batched(hs, es, tol=1e-10)
    assert plain.statuses[0] == "NOT_CONVERGED" and plain.statuses[1:] == ["OK", "OK"]
    res = pq.pq_solve_batched(hs, es, tol=1e-10, solver=2)
    assert res.statuses == ["OK", "OK", "OK"]
    assert abs(res.energies[0] - ref.energy) < 1e-9
    for i in (1, 2):
        single = pq.pq_solve(hs[i], es[i], tol=1e-10)
        assert abs(res.energies[i] - single.energy) < 1e-10
