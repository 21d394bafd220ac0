"""Device-driven against host-driven Jacobi/DIIS iterations of the PQ solve.

The device-driven loop (opt-in) takes the norm test, the convergence, stall
and divergence decisions and the DIIS coefficients on the device and enqueues
the next iteration before the host reads the last one; a finished solve
gates off the iteration queued beyond its end.  The host-driven loop (the
default) synchronises once per iteration and solves the DIIS system on the host.
Both take the same steps and tests (Sec. III: Jacobi steps with DIIS
extrapolation), so they reach the same amplitudes and outcomes; only the
rounding of the DIIS coefficients differs.  Also: the residual graphs cached
for several buffer sets give the residual of the buffers they are called
with."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from inputs import chain_problem, random_amplitudes, random_bfactors, random_fock
from oracle import integrals as oint
from oracle import layout, tier_a

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def pq():
    import paper_1609_00077_amd as pq
    pq._lib.load()
    yield pq
    pq.set_solve_mode("host")


def _d(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _both(pq, f, eri, t0=None, **kw):
    out = []
    for mode in ("host", "device"):
        pq.set_solve_mode(mode)
        out.append(pq.pq_solve(f, eri, t0, raise_on_failure=False, **kw))
    pq.set_solve_mode("host")
    return out


@pytest.mark.parametrize("sites", [6, 24, 74, 140])
def test_modes_reach_the_same_solution(pq, sites):
    prob = chain_problem(sites, U=4.0, seed=sites)
    f, eri = pq.integrals(_d(prob.F_site), _d(prob.V), _d(prob.C), k=2)
    a, b = _both(pq, f, eri, tol=1e-10)
    assert a.status == b.status == "OK"
    assert abs(a.iterations - b.iterations) <= 1, (a.iterations, b.iterations)
    assert abs(a.energy - b.energy) < 1e-11
    assert (a.t - b.t).abs().max().item() < 1e-9
    assert b.rnorm <= 1e-10


def test_plain_jacobi_iterates_are_bitwise_equal(pq):
    """Without DIIS both loops apply t <- t - R/D with the same arithmetic:
    after a fixed number of steps the amplitudes agree bit for bit."""
    prob = chain_problem(24, U=4.0, seed=24)
    f, eri = pq.integrals(_d(prob.F_site), _d(prob.V), _d(prob.C), k=2)
    a, b = _both(pq, f, eri, tol=1e-14, diis_dim=0, max_iter=6)
    assert a.status == b.status == "NOT_CONVERGED"
    assert a.iterations == b.iterations == 6
    assert torch.equal(a.t, b.t)
    assert abs(a.rnorm - b.rnorm) <= 1e-12 * a.rnorm


def test_iteration_limit(pq):
    N = 4
    f = random_fock(N, seed=935)
    eri = oint.eri_packed_from_b(random_bfactors(N, seed=936), N, 2)
    a, b = _both(pq, _d(f), _d(eri), tol=1e-14, max_iter=3)
    assert a.status == b.status == "NOT_CONVERGED"
    assert a.iterations == b.iterations == 3
    assert (a.t - b.t).abs().max().item() < 1e-13
    pq.set_solve_mode("device")
    with pytest.raises(pq.PQPHError, match="not converged in 3 iterations"):
        pq.pq_solve(_d(f), _d(eri), tol=1e-14, max_iter=3)
    pq.set_solve_mode("host")


def test_nonfinite_and_divergence(pq):
    N = 4
    f = random_fock(N, seed=910)
    eri = oint.eri_packed_from_b(random_bfactors(N, seed=911), N, 2)
    t0 = random_amplitudes(N, "pq", seed=912, scale=0.05)
    t0[5] = np.nan
    a, b = _both(pq, _d(f), _d(eri), _d(t0))
    assert a.status == b.status == "NONFINITE"
    assert a.iterations == b.iterations == 1
    big = random_amplitudes(N, "pq", seed=913, scale=10.0)
    a, b = _both(pq, _d(f), _d(eri), _d(big))
    assert a.status == b.status == "DIVERGED"
    assert a.iterations == b.iterations
    assert b.rnorm > 1e3
    pq.set_solve_mode("device")
    with pytest.raises(pq.PQPHError, match="diverged at iteration"):
        pq.pq_solve(_d(f), _d(eri), _d(big))
    pq.set_solve_mode("host")


def test_stall_and_newton_fallback(pq):
    """8-site chain at U = 10, where Jacobi/DIIS stalls: both loops stop on
    the stall test; with solver 2 both hand their best iterate to
    Newton-Krylov and reach the same root."""
    prob = chain_problem(8, U=10.0, seed=8)
    f, eri = oint.chain_integrals(prob, 2)
    a, b = _both(pq, _d(f), _d(eri), tol=1e-8)
    assert a.status == b.status == "NOT_CONVERGED"
    pq.set_solve_mode("device")
    with pytest.raises(pq.PQPHError, match="stalled"):
        pq.pq_solve(_d(f), _d(eri), tol=1e-8)
    pq.set_solve_mode("host")
    a, b = _both(pq, _d(f), _d(eri), tol=1e-11, solver=2)
    assert a.status == b.status == "OK"
    assert abs(a.energy - b.energy) < 1e-10
    ta = tier_a.TierA(4, 2)
    R = ta.residual(f, layout.unpack_eri(eri, 4, 2), b.t.cpu().numpy())[0]
    assert np.abs(R).max() < 1e-10


def test_spin_adapted_modes_agree(pq):
    prob = chain_problem(24, U=4.0, seed=24)
    f, eri = pq.integrals(_d(prob.F_site), _d(prob.V), _d(prob.C), k=2)
    a, b = _both(pq, f, eri, tol=1e-10, spin_adapted=1)
    assert a.status == b.status == "OK"
    assert abs(a.energy - b.energy) < 1e-11
    assert (a.t - b.t).abs().max().item() < 1e-9


def test_energy_gradient_after_device_driven_solve(pq):
    """pq_energy_grad's amplitude solve follows the solve mode, its lambda
    solve is always host-driven: the energy and dE/dh agree."""
    prob = chain_problem(24, U=4.0, seed=24)
    f, eri = pq.integrals(_d(prob.F_site), _d(prob.V), _d(prob.C), k=2)
    out = []
    for mode in ("host", "device"):
        pq.set_solve_mode(mode)
        out.append(pq.pq_energy_grad(f, eri, tol=1e-11))
    pq.set_solve_mode("host")
    a, b = out
    assert abs(a.energy - b.energy) < 1e-11
    assert (a.dE_dh - b.dE_dh).abs().max().item() < 1e-8


def test_residual_graphs_for_many_buffer_sets(pq):
    """More buffer sets than cached graphs, called in an interleaved order:
    every residual equals the first one computed for its amplitudes."""
    N = 12
    prob = chain_problem(2 * N, U=4.0, seed=77)
    f, eri = pq.integrals(_d(prob.F_site), _d(prob.V), _d(prob.C), k=2)
    ts = [_d(random_amplitudes(N, "pq", seed=780 + i, scale=0.05)) for i in range(6)]
    outs = [torch.empty_like(t) for t in ts]
    ref = [pq.pq_residual(f, eri, t).clone() for t in ts]
    for order in ([0, 1, 2, 3, 4, 5], [5, 3, 1, 0, 2, 4], [1, 1, 4, 0, 5, 2, 3]):
        for i in order:
            pq.pq_residual(f, eri, ts[i], out=outs[i])
            torch.cuda.synchronize()
            assert torch.equal(outs[i], ref[i]), i


def test_solve_mode_rejects_other_values(pq):
    lib, ctx = pq._ctx(torch.device(DEV))
    assert lib.pqph_set_solve_mode(ctx, 2) == -1
    with pytest.raises(ValueError):
        pq.set_solve_mode("fast")


@pytest.mark.parametrize("max_rank", [2, 3])
def test_rank_limited_modes_agree(pq, max_rank):
    """Excitation-rank limits mask the residual inside both loops alike, so
    the rank-limited solutions agree."""
    prob = chain_problem(24, U=4.0, seed=24)
    f, eri = pq.integrals(_d(prob.F_site), _d(prob.V), _d(prob.C), k=2)
    a, b = _both(pq, f, eri, tol=1e-10, max_rank=max_rank)
    assert a.status == b.status == "OK"
    assert abs(a.iterations - b.iterations) <= 1
    assert abs(a.energy - b.energy) < 1e-11
    assert (a.t - b.t).abs().max().item() < 1e-9
