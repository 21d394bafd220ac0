"""Closed-shell spin adaptation of the solves (pqph_solve_opts.spin_adapted,
Sec. V: spin summation for closed shells): the reduced space of one value
per alpha/beta exchange orbit reaches the full-space solution (energies to
1e-10 Eh, amplitudes to 1e-9) and the oracle's, with every solved amplitude
obeying t[partner] = sign * t of the oracle's exchange map."""
import ctypes as C

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


def _symmetric(t, N, k):
    partner, sign = layout.spin_partner(N, k)
    return np.abs(t[partner] - sign * t).max()


@pytest.mark.parametrize("N,k", [(3, 2), (4, 2), (3, 3)])
def test_spin_adapted_solve_matches_oracle(pq, N, k):
    prob = chain_problem(2 * N, U=4.0, seed=2 * N + k)
    f, eri = oint.chain_integrals(prob, k)
    ta = tier_a.TierA(N, k)
    et = layout.unpack_eri(eri, N, k)
    ref = solver.solve(lambda t: ta.residual(f, et, t)[0], lambda t: ta.energy(f, et, t),
                       solver.denominators(f, N, k), tol=1e-11, max_iter=300)
    assert ref.converged
    solve = pq.pq_solve if k == 2 else pq.ph_solve
    res = solve(_d(f), _d(eri), tol=1e-11, spin_adapted=1)
    assert res.status == "OK"
    assert abs(res.energy - ref.energy) < 1e-10
    t = res.t.cpu().numpy()
    assert np.abs(t - ref.t).max() < 1e-9
    assert _symmetric(t, N, k) < 1e-15


@pytest.mark.parametrize("N,k", [(24, 2), (70, 2), (8, 3)])
def test_spin_adapted_equals_full_space(pq, N, k):
    """Same iteration in exact arithmetic: same energy, amplitudes and
    (up to rounding) iteration count; the reduced history is the smaller."""
    prob = chain_problem(2 * N, U=4.0, seed=N)
    f, eri = oint.chain_integrals(prob, k)
    solve = pq.pq_solve if k == 2 else pq.ph_solve
    full = solve(_d(f), _d(eri), tol=1e-10)
    red = solve(_d(f), _d(eri), tol=1e-10, spin_adapted=1)
    assert full.status == "OK" and red.status == "OK"
    assert abs(full.energy - red.energy) < 1e-10
    assert (full.t - red.t).abs().max().item() < 1e-9
    assert abs(full.iterations - red.iterations) <= 2, (full.iterations, red.iterations)
    assert _symmetric(red.t.cpu().numpy(), N, k) < 1e-15


def test_spin_adapted_projects_the_start(pq):
    """A start that breaks the symmetry is projected: the solve from it ends
    at the solution of the symmetric start."""
    N = 10
    prob = chain_problem(2 * N, U=4.0, seed=31)
    f, eri = oint.chain_integrals(prob, 2)
    ref = pq.pq_solve(_d(f), _d(eri), tol=1e-11)
    t0 = np.random.default_rng(32).uniform(-0.02, 0.02, pq.amp_len(N))
    assert _symmetric(t0, N, 2) > 1e-3
    red = pq.pq_solve(_d(f), _d(eri), _d(t0), tol=1e-11, spin_adapted=1)
    assert red.status == "OK"
    assert abs(red.energy - ref.energy) < 1e-10
    assert (red.t - ref.t).abs().max().item() < 1e-9


@pytest.mark.parametrize("k,r", [(2, 2), (3, 2), (3, 4)])
def test_spin_adapted_rank_limited(pq, k, r):
    N = 6 if k == 3 else 12
    prob = chain_problem(2 * N, U=4.0, seed=40 + k)
    f, eri = oint.chain_integrals(prob, k)
    solve = pq.pq_solve if k == 2 else pq.ph_solve
    full = solve(_d(f), _d(eri), tol=1e-11, max_rank=r)
    red = solve(_d(f), _d(eri), tol=1e-11, max_rank=r, spin_adapted=1)
    assert full.status == "OK" and red.status == "OK"
    assert abs(full.energy - red.energy) < 1e-10
    assert (full.t - red.t).abs().max().item() < 1e-9


def test_spin_adapted_gradient(pq):
    """The lambda equations in the reduced space give the same gradient."""
    N = 16
    prob = chain_problem(2 * N, U=4.0, seed=50)
    f, eri = oint.chain_integrals(prob, 2)
    full = pq.pq_energy_grad(_d(f), _d(eri), tol=1e-11)
    red = pq.pq_energy_grad(_d(f), _d(eri), tol=1e-11, spin_adapted=1)
    assert full.status == "OK" and red.status == "OK"
    assert abs(full.energy - red.energy) < 1e-10
    scale = max(1.0, full.dE_deri.abs().max().item())
    assert (full.dE_dh - red.dE_dh).abs().max().item() < 1e-9 * scale
    assert (full.dE_deri - red.dE_deri).abs().max().item() < 1e-9 * scale
    assert _symmetric(red.lam.cpu().numpy(), N, 2) < 1e-14


def test_spin_adapted_newton(pq):
    """Newton-Krylov in the reduced space on the strongly correlated chain
    where Jacobi/DIIS stalls reaches the full-space Newton root."""
    prob = chain_problem(8, U=10.0, seed=8)
    f, eri = oint.chain_integrals(prob, 2)
    full = pq.pq_solve(_d(f), _d(eri), tol=1e-11, solver=2)
    red = pq.pq_solve(_d(f), _d(eri), tol=1e-11, solver=2, spin_adapted=1)
    assert full.status == "OK" and red.status == "OK", (full.status, red.status)
    assert abs(full.energy - red.energy) < 1e-10
    assert (full.t - red.t).abs().max().item() < 1e-9


def test_spin_adapted_rejected_where_unsupported(pq):
    from paper_1609_00077_amd import _lib
    lib, ctx = pq._ctx(torch.device(DEV))
    prob = chain_problem(6, U=4.0, seed=6)
    f, eri = oint.chain_integrals(prob, 2)
    fd, ed = _d(f), _d(eri)
    t = torch.zeros(pq.amp_len(3), dtype=torch.float64, device=DEV)
    opts = _lib.SolveOpts()
    lib.pqph_default_opts(C.byref(opts))
    opts.spin_adapted = 2
    e = C.c_double()
    st = lib.pq_solve(ctx, 3, C.c_void_p(fd.data_ptr()), C.c_void_p(ed.data_ptr()), C.byref(opts),
                      C.c_void_p(t.data_ptr()), C.byref(e), None)
    assert _lib.STATUS[st] == "INVALID_ARG"
    opts.spin_adapted = 1
    en = (C.c_double * 1)()
    infos = (_lib.SolveInfo * 1)()
    st = lib.pq_solve_batched(ctx, 1, (C.c_int * 1)(3), (C.c_int64 * 1)(0), (C.c_int64 * 1)(0),
                              (C.c_int64 * 1)(0), C.c_void_p(fd.data_ptr()),
                              C.c_void_p(ed.data_ptr()), C.byref(opts), C.c_void_p(t.data_ptr()),
                              en, infos)
    assert _lib.STATUS[st] == "INVALID_ARG"
