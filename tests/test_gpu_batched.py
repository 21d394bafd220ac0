"""Batched PQ solves (HIP) against single solves and the oracle."""
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


def _chains(specs):
    out = []
    for n, U, seed in specs:
        prob = chain_problem(n, U=U, seed=seed)
        out.append((prob, *oint.chain_integrals(prob, 2)))
    return out


SPECS = [(8, 4.0, 1), (4, 3.0, 2), (12, 2.5, 3), (6, 5.0, 4), (20, 4.0, 5), (10, 6.0, 6)]


def test_batched_matches_single_and_oracle(pq):
    chains = _chains(SPECS)
    res = pq.pq_solve_batched([_d(f) for _, f, _ in chains], [_d(e) for _, _, e in chains], tol=1e-11)
    assert all(s == "OK" for s in res.statuses), res.statuses
    for i, (prob, f, eri) in enumerate(chains):
        single = pq.pq_solve(_d(f), _d(eri), tol=1e-11)
        assert abs(single.energy - res.energies[i]) < 1e-10
        N = prob.npair
        t_b = res.t[res.t_off[i]: res.t_off[i] + layout.amp_count(N, 2)].cpu().numpy()
        assert np.abs(t_b - single.t.cpu().numpy()).max() < 1e-9
        if N <= 3:
            ta = tier_a.TierA(N, 2)
            et = layout.unpack_eri(eri, N, 2)
            ref = solver.solve(lambda t: ta.residual(f, et, t)[0], lambda t: ta.energy(f, et, t),
                               solver.denominators(f, N, 2), tol=1e-12)
            assert abs(ref.energy - res.energies[i]) < 1e-10


def test_batched_is_order_independent_and_deterministic(pq):
    chains = _chains(SPECS)
    hs = [_d(f) for _, f, _ in chains]
    es = [_d(e) for _, _, e in chains]
    a = pq.pq_solve_batched(hs, es, tol=1e-10)
    perm = [3, 0, 5, 1, 4, 2]
    b = pq.pq_solve_batched([hs[i] for i in perm], [es[i] for i in perm], tol=1e-10)
    c = pq.pq_solve_batched(hs, es, tol=1e-10)
    for j, i in enumerate(perm):
        assert b.energies[j] == a.energies[i]          # bitwise
        assert b.iterations[j] == a.iterations[i]
    assert a.energies == c.energies


def test_batched_flags_a_bad_chain_without_stopping_others(pq):
    chains = _chains(SPECS[:3])
    hs = [_d(f) for _, f, _ in chains]
    es = [_d(e) for _, _, e in chains]
    bad = es[1].clone()
    bad[0] = float("nan")
    res = pq.pq_solve_batched([hs[0], hs[1], hs[2]], [es[0], bad, es[2]], tol=1e-10)
    assert res.statuses[1] == "NONFINITE"
    assert res.statuses[0] == "OK" and res.statuses[2] == "OK"


def test_graph_and_lockstep_modes_agree(pq):
    """The device-resident, graph-replayed iterations reach the same solutions
    as the host-driven lockstep iterations (same Jacobi/DIIS steps; the DIIS
    solve runs on the device in one mode and on the host in the other)."""
    chains = _chains(SPECS)
    hs = [_d(f) for _, f, _ in chains]
    es = [_d(e) for _, _, e in chains]
    g = pq.pq_solve_batched(hs, es, tol=1e-11, mode="graph")
    s = pq.pq_solve_batched(hs, es, tol=1e-11, mode="lockstep")
    assert g.statuses == s.statuses
    for a, b in zip(g.energies, s.energies):
        assert abs(a - b) < 1e-10
    for a, b in zip(g.iterations, s.iterations):
        assert abs(a - b) <= 1


def test_batched_iteration_limit(pq):
    """Chains stopped by the iteration limit report NOT_CONVERGED with the
    limit as their iteration count, in both modes."""
    chains = _chains(SPECS[:3])
    hs = [_d(f) for _, f, _ in chains]
    es = [_d(e) for _, _, e in chains]
    for mode in ("graph", "lockstep"):
        res = pq.pq_solve_batched(hs, es, tol=1e-14, max_iter=3, mode=mode)
        assert all(st == "NOT_CONVERGED" for st in res.statuses), res.statuses
        assert res.iterations == [3, 3, 3]
