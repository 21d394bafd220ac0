"""Failure handling of the solvers and argument checks of the C ABI, forced
from the host so that every kernel still runs to its normal end.

A solve reports its outcome as a status code, never by aborting: NaN in the
iterates is NONFINITE, a growing residual norm (Sec. IV.B: the PQ/PH
iterations can diverge at stretched geometries) is DIVERGED, a vanishing
orbital-energy denominator (Table IV's denominator application) and bad sizes
or null pointers are INVALID_ARG.  After each failure the context must still
give correct results."""
import ctypes as C

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
    return pq


def _d(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def _system(N, k, seed):
    f = random_fock(N, seed=seed)
    return f, oint.eri_packed_from_b(random_bfactors(N, seed=seed + 1), N, k)


def _still_correct(pq, N=3):
    """A residual on the same context after a failure matches the oracle."""
    f, eri = _system(N, 2, 900)
    t = random_amplitudes(N, "pq", seed=901, scale=0.1)
    RA, _ = tier_a.TierA(N, 2).residual(f, layout.unpack_eri(eri, N, 2), t)
    R = pq.pq_residual(_d(f), _d(eri), _d(t)).cpu().numpy()
    assert np.abs(R - RA).max() <= 1e-12 * max(1.0, np.abs(RA).max())


@pytest.mark.parametrize("model", ["pq", "ph"])
def test_nan_in_amplitudes_is_nonfinite(pq, model):
    N = 4
    k = 2 if model == "pq" else 3
    f, eri = _system(N, k, 910)
    t0 = random_amplitudes(N, model, seed=911, scale=0.05)
    t0[7] = np.nan
    solve = pq.pq_solve if model == "pq" else pq.ph_solve
    res = solve(_d(f), _d(eri), _d(t0), raise_on_failure=False)
    assert res.status == "NONFINITE"
    assert res.iterations == 1
    with pytest.raises(pq.PQPHError, match="NONFINITE"):
        solve(_d(f), _d(eri), _d(t0))
    _still_correct(pq)


def test_nan_energy_is_nonfinite(pq):
    N = 3
    f, eri = _system(N, 2, 915)
    t = random_amplitudes(N, "pq", seed=916, scale=0.05)
    t[layout.amp_slot(N, (0, 1), 5)] = np.nan
    with pytest.raises(pq.PQPHError, match="NONFINITE"):
        pq.pq_energy(_d(f), _d(eri), _d(t))


@pytest.mark.parametrize("model", ["pq", "ph"])
def test_large_start_diverges(pq, model):
    """Amplitudes of order ten make the quartic residual huge: the norm test
    (above 1e3, or diverge_factor times the smallest norm) stops the solve."""
    N = 4
    k = 2 if model == "pq" else 3
    f, eri = _system(N, k, 920)
    t0 = random_amplitudes(N, model, seed=921, scale=10.0)
    solve = pq.pq_solve if model == "pq" else pq.ph_solve
    res = solve(_d(f), _d(eri), _d(t0), raise_on_failure=False)
    assert res.status == "DIVERGED"
    assert np.isfinite(res.rnorm) and res.rnorm > 1e3
    _still_correct(pq)


def test_growth_factor_diverges(pq):
    """Without DIIS and with a negative level shift close to the smallest
    denominator, the Jacobi step overshoots and the norm grows geometrically;
    a growth factor of 2 over the smallest norm is then DIVERGED, not a
    silent NaN or NOT_CONVERGED."""
    N = 3
    f, eri = _system(N, 2, 925)
    dmin = float(pq.denominators(_d(f)).abs().min())
    res = pq.pq_solve(_d(f), _d(eri), diis_dim=0, level_shift=-0.97 * dmin,
                      diverge_factor=2.0, max_iter=500, raise_on_failure=False)
    assert res.status == "DIVERGED", (res.status, res.iterations, res.rnorm)
    assert res.iterations > 1


@pytest.mark.parametrize("model", ["pq", "ph"])
def test_vanishing_denominator_is_invalid(pq, model):
    """f_oo = f_vv for one pair makes its single o_P -> v_P denominator zero."""
    N = 3
    k = 2 if model == "pq" else 3
    f, eri = _system(N, k, 930)
    f[N + 1, N + 1] = f[1, 1]
    solve = pq.pq_solve if model == "pq" else pq.ph_solve
    res = solve(_d(f), _d(eri), raise_on_failure=False)
    assert res.status == "INVALID_ARG"
    with pytest.raises(pq.PQPHError, match="denominator"):
        solve(_d(f), _d(eri))
    _still_correct(pq)


def test_iteration_limit_is_not_converged(pq):
    N = 4
    f, eri = _system(N, 2, 935)
    res = pq.pq_solve(_d(f), _d(eri), max_iter=3, tol=1e-14, raise_on_failure=False)
    assert res.status == "NOT_CONVERGED" and res.iterations == 3


def test_invalid_arguments(pq):
    lib, ctx = pq._ctx(torch.device(DEV))
    f, eri = _system(3, 2, 940)
    h, e = _d(f), _d(eri)
    t = _d(np.zeros(layout.amp_count(3, 2)))
    r = torch.empty_like(t)
    p = lambda x: C.c_void_p(x.data_ptr())
    for npair in (0, -1, 257):
        assert lib.pq_residual(ctx, npair, p(h), p(e), p(t), p(r)) == -1
        assert lib.ph_residual(ctx, npair, p(h), p(e), p(t), p(r)) == -1
        assert b"npair" in lib.pqph_last_error(ctx)
    assert lib.pq_residual(ctx, 3, None, p(e), p(t), p(r)) == -1
    assert lib.pq_residual(ctx, 3, p(h), p(e), p(t), None) == -1
    assert lib.pq_residual(None, 3, p(h), p(e), p(t), p(r)) == -1
    en = C.c_double()
    assert lib.pq_energy(ctx, 3, p(h), p(e), p(t), None) == -1
    assert lib.pqph_denominators(ctx, 3, 4, p(h), 0.0, p(r)) == -1
    assert lib.pqph_set_variant(ctx, 120, 2) == -1
    assert lib.pqph_set_s1_mode(ctx, 3, 7) == -1
    assert lib.pqph_set_batch_mode(ctx, 5) == -1
    bad = pq._lib.SolveOpts(0, 1e-8, 8, 2, 0.0, 1e4, 40)          # max_iter 0
    assert lib.pq_solve(ctx, 3, p(h), p(e), C.byref(bad), p(t), C.byref(en), None) == -1
    bad = pq._lib.SolveOpts(10, 1e-8, 17, 2, 0.0, 1e4, 40)        # diis_dim above 16
    assert lib.pq_solve(ctx, 3, p(h), p(e), C.byref(bad), p(t), C.byref(en), None) == -1
    bad = pq._lib.SolveOpts(10, 1e-8, 8, 2, 0.0, 1.0, 40)         # diverge_factor not > 1
    assert lib.pq_solve(ctx, 3, p(h), p(e), C.byref(bad), p(t), C.byref(en), None) == -1
    _still_correct(pq)
