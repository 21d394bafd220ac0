"""MI355X-native perfect quadruples (PQ) and perfect hextuples (PH) library.

The hot path of the paper's method -- the pair-truncated coupled-cluster
amplitude residuals over dense pair-indexed tensors inside Jacobi/DIIS
iterations (Sec. II-III of arXiv:1609.00077) -- runs in hand-written HIP
kernels behind the C ABI of include/pqph.h.  This module only marshals torch
tensors (device memory and the current HIP stream) into those calls.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib

__all__ = ["pq_residual", "pq_residual_noalloc", "pq_energy", "pq_solve", "pq_solve_batched", "pq_vjp",
           "pq_energy_grad", "pq_densities", "PQEnergy", "pq_energy_autograd", "integrals", "denominators",
           "amp_len", "eri_len", "SolveResult", "GradResult", "BatchResult", "PQPHError"]

PQPHError = _lib.PQPHError
_ctx_cache: dict = {}


def _ctx(device: torch.device):
    lib = _lib.load()
    idx = device.index if device.index is not None else torch.cuda.current_device()
    stream = torch.cuda.current_stream(idx).cuda_stream
    key = (idx, stream)
    ctx = _ctx_cache.get(key)
    if ctx is None:
        h = C.c_void_p()
        st = lib.pqph_create(C.byref(h), idx, C.c_void_p(stream))
        if st != 0:
            raise PQPHError(st, lib.pqph_last_error(None).decode())
        ctx = h
        _ctx_cache[key] = ctx
    return lib, ctx


def _check(lib, ctx, st):
    if st != 0:
        raise PQPHError(st, lib.pqph_last_error(ctx).decode())


def _dev(x: torch.Tensor, name: str, n: int | None = None):
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != torch.float64 or not x.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor")
    if n is not None and x.numel() != n:
        raise ValueError(f"{name} has {x.numel()} elements, expected {n}")
    return C.c_void_p(x.data_ptr())


def amp_len(npair: int, model: str = "pq") -> int:
    lib = _lib.load()
    return int(lib.pq_amp_len(npair) if model == "pq" else lib.ph_amp_len(npair))


def eri_len(npair: int, model: str = "pq") -> int:
    lib = _lib.load()
    return int(lib.pq_eri_len(npair) if model == "pq" else lib.ph_eri_len(npair))


def integrals(F: torch.Tensor, V: torch.Tensor, Cmo: torch.Tensor, k: int = 2):
    """(f, packed eri) of a ZDO site Hamiltonian; see pqph_integrals."""
    n = F.shape[0]
    npair = n // 2
    lib, ctx = _ctx(F.device)
    f = torch.empty((n, n), dtype=torch.float64, device=F.device)
    eri = torch.empty(eri_len(npair, "pq" if k == 2 else "ph"), dtype=torch.float64, device=F.device)
    _check(lib, ctx, lib.pqph_integrals(ctx, npair, k, _dev(F, "F", n * n), _dev(V, "V", n * n),
                                        _dev(Cmo, "C", n * n), _dev(f, "f"), _dev(eri, "eri")))
    return f, eri


def pq_residual(h: torch.Tensor, eri: torch.Tensor, t: torch.Tensor, out: torch.Tensor | None = None):
    """Packed PQ residual r(t) (no host sync)."""
    npair = h.shape[0] // 2
    lib, ctx = _ctx(h.device)
    na = amp_len(npair)
    if out is None:
        out = torch.empty(na, dtype=torch.float64, device=h.device)
    _check(lib, ctx, lib.pq_residual(ctx, npair, _dev(h, "h", 4 * npair * npair),
                                     _dev(eri, "eri", eri_len(npair)), _dev(t, "t", na),
                                     _dev(out, "out", na)))
    return out


def pq_residual_noalloc(h: torch.Tensor, eri: torch.Tensor, t: torch.Tensor, out: torch.Tensor):
    """Packed PQ residual into out with no device allocation by the library
    (its workspace is a static per-GPU array; npair <= 32; calls on one GPU
    must not overlap).  out must be given."""
    npair = h.shape[0] // 2
    lib, ctx = _ctx(h.device)
    na = amp_len(npair)
    _check(lib, ctx, lib.pq_residual_noalloc(ctx, npair, _dev(h, "h", 4 * npair * npair),
                                             _dev(eri, "eri", eri_len(npair)), _dev(t, "t", na),
                                             _dev(out, "out", na)))
    return out


def pq_residual_profile(h: torch.Tensor, eri: torch.Tensor, t: torch.Tensor):
    """One residual with per-kernel HIP-event times: (r, [(kernel, ms), ...])."""
    npair = h.shape[0] // 2
    lib, ctx = _ctx(h.device)
    na = amp_len(npair)
    out = torch.empty(na, dtype=torch.float64, device=h.device)
    ms = (C.c_double * 24)()
    n = C.c_int()
    _check(lib, ctx, lib.pq_residual_profile(ctx, npair, _dev(h, "h", 4 * npair * npair),
                                             _dev(eri, "eri", eri_len(npair)), _dev(t, "t", na),
                                             _dev(out, "out", na), ms, 24, C.byref(n)))
    names = [lib.pq_residual_phase_name(i).decode() for i in range(16)]
    if n.value == 13:      # npair == 2: no one-pair two-spectator terms
        names = [x for x in names if x not in ("k_spec_r1", "k_r1s2", "k_r1s2_close")]
    elif n.value == 4:     # npair == 1: no two-pair outputs
        names = ["k_vertex1", "k_r1", "k_r1c", "k_final"]
    return out, list(zip(names, [ms[i] for i in range(n.value)]))


def measure_ceilings(device: str | torch.device = "cuda:0") -> dict:
    """Measured HBM bandwidth (STREAM copy, triad), FP64 FMA and FP64 MFMA
    rates of the device (diagnostic for roofline fractions)."""
    lib, ctx = _ctx(torch.device(device))
    out = (C.c_double * 4)()
    _check(lib, ctx, lib.pqph_measure_ceilings(ctx, out))
    return {"stream_copy_GBs": out[0], "stream_triad_GBs": out[1], "fp64_fma_TFLOPs": out[2],
            "fp64_mfma_TFLOPs": out[3]}


def autotune(h: torch.Tensor, eri: torch.Tensor, t: torch.Tensor) -> int:
    """Pick the fastest two-spectator kernel variant for this size (kept on
    the context of the current stream); returns the variant number."""
    npair = h.shape[0] // 2
    lib, ctx = _ctx(h.device)
    na = amp_len(npair)
    out = torch.empty(na, dtype=torch.float64, device=h.device)
    ch = C.c_int()
    _check(lib, ctx, lib.pqph_autotune(ctx, npair, _dev(h, "h", 4 * npair * npair),
                                       _dev(eri, "eri", eri_len(npair)), _dev(t, "t", na),
                                       _dev(out, "out", na), C.byref(ch)))
    return ch.value


def set_variant(npair: int, variant: int, device: str | torch.device = "cuda:0") -> None:
    """Force the two-spectator kernel variant (1 or 2; 0 = default) for npair
    on the context of the current stream."""
    lib, ctx = _ctx(torch.device(device))
    _check(lib, ctx, lib.pqph_set_variant(ctx, npair, variant))


def set_s1_mode(npair: int, mode: int, device: str | torch.device = "cuda:0") -> None:
    """Force how the one-spectator GEMM gets its sides for npair (1 formed
    while staging, 2 materialised, 3 formed while staging with the loads
    pipelined, npair <= 128, 4 materialised with the loads pipelined;
    0 = default) on the context of the current stream."""
    lib, ctx = _ctx(torch.device(device))
    _check(lib, ctx, lib.pqph_set_s1_mode(ctx, npair, mode))


def set_solve_mode(mode: str, device: str | torch.device = "cuda:0") -> None:
    """How PQ amplitude solves iterate on the context of the current stream:
    "host" (default: one host synchronisation per iteration, DIIS solved on
    the host) or "device" (the Jacobi/DIIS decisions taken on the device, the
    next iteration enqueued before the host reads the last one)."""
    if mode not in ("device", "host"):
        raise ValueError("mode must be 'device' or 'host'")
    lib, ctx = _ctx(torch.device(device))
    _check(lib, ctx, lib.pqph_set_solve_mode(ctx, 0 if mode == "device" else 1))


def set_pq_intermediates(npair: int, labels: int, device: str | torch.device = "cuda:0") -> None:
    """PQ model for npair on the context of the current stream: labels = 3
    (exact projection, the default) or 2 (two-pair intermediates: the
    doubly-mixed two-spectator terms left out)."""
    lib, ctx = _ctx(torch.device(device))
    _check(lib, ctx, lib.pqph_set_pq_intermediates(ctx, npair, labels))


def tuning(npair: int, device: str | torch.device = "cuda:0") -> dict:
    """The kernel choices in effect for npair: two-spectator variant and
    one-spectator mode."""
    lib, ctx = _ctx(torch.device(device))
    v, m = C.c_int(), C.c_int()
    _check(lib, ctx, lib.pqph_tuning(ctx, npair, C.byref(v), C.byref(m)))
    return {"s2_variant": v.value, "s1_mode": m.value}


def pq_energy(h: torch.Tensor, eri: torch.Tensor, t: torch.Tensor) -> float:
    npair = h.shape[0] // 2
    lib, ctx = _ctx(h.device)
    e = C.c_double()
    _check(lib, ctx, lib.pq_energy(ctx, npair, _dev(h, "h", 4 * npair * npair),
                                   _dev(eri, "eri", eri_len(npair)), _dev(t, "t", amp_len(npair)),
                                   C.byref(e)))
    return e.value


def denominators(h: torch.Tensor, k: int = 2, shift: float = 0.0) -> torch.Tensor:
    npair = h.shape[0] // 2
    lib, ctx = _ctx(h.device)
    D = torch.empty(amp_len(npair, "pq" if k == 2 else "ph"), dtype=torch.float64, device=h.device)
    _check(lib, ctx, lib.pqph_denominators(ctx, npair, k, _dev(h, "h", 4 * npair * npair),
                                           float(shift), _dev(D, "D")))
    return D


@dataclass
class BatchResult:
    t: torch.Tensor            # packed amplitudes of every chain, concatenated
    t_off: list
    energies: list
    iterations: list
    rnorms: list
    statuses: list
    solve_ms: float


def pq_solve_batched(hs, eris, *, tol: float = 1e-8, max_iter: int = 200, diis_dim: int = 8,
                     diis_start: int = 2, level_shift: float = 0.0,
                     diverge_factor: float = 1e4, stall_window: int = 40,
                     max_rank: int = 0, solver: int = 0,
                     mode: str = "graph") -> BatchResult:
    """Solve many PQ problems together.  hs, eris: lists of per-chain Fock
    matrices and packed integrals (device tensors), packed here into one
    buffer each.  mode: "graph" (device-resident iterations replayed from a
    HIP graph) or "lockstep" (host-driven)."""
    dev = hs[0].device
    lib, ctx = _ctx(dev)
    if mode not in ("graph", "lockstep"):
        raise ValueError("mode must be 'graph' or 'lockstep'")
    _check(lib, ctx, lib.pqph_set_batch_mode(ctx, 0 if mode == "graph" else 1))
    nb = len(hs)
    npairs = [h.shape[0] // 2 for h in hs]
    h_all = torch.cat([h.reshape(-1) for h in hs]).contiguous()
    e_all = torch.cat([e.reshape(-1) for e in eris]).contiguous()
    h_off, e_off, t_off = [], [], []
    a = b = c = 0
    for h, e, n in zip(hs, eris, npairs):
        if e.numel() != eri_len(n):
            raise ValueError("integral vector of the wrong length in the batch")
        h_off.append(a); e_off.append(b); t_off.append(c)
        a += h.numel(); b += e.numel(); c += amp_len(n)
    t = torch.zeros(c, dtype=torch.float64, device=dev)
    opts = _lib.SolveOpts(max_iter, tol, diis_dim, diis_start, level_shift, diverge_factor,
                          stall_window, max_rank, solver)
    infos = (_lib.SolveInfo * nb)()
    en = (C.c_double * nb)()
    st = lib.pq_solve_batched(ctx, nb, (C.c_int * nb)(*npairs), (C.c_int64 * nb)(*h_off),
                              (C.c_int64 * nb)(*e_off), (C.c_int64 * nb)(*t_off),
                              _dev(h_all, "h"), _dev(e_all, "eri"), C.byref(opts), _dev(t, "t"),
                              en, infos)
    if st not in (0, -4, -5, -6):
        _check(lib, ctx, st)
    return BatchResult(t, t_off, [en[i] for i in range(nb)], [infos[i].iterations for i in range(nb)],
                       [infos[i].rnorm for i in range(nb)],
                       [_lib.STATUS.get(infos[i].status, str(infos[i].status)) for i in range(nb)],
                       infos[0].solve_ms if nb else 0.0)


@dataclass
class SolveResult:
    t: torch.Tensor
    energy: float
    iterations: int
    rnorm: float
    status: str
    solve_ms: float


def pq_solve(h: torch.Tensor, eri: torch.Tensor, t0: torch.Tensor | None = None, *,
             tol: float = 1e-8, max_iter: int = 200, diis_dim: int = 8, diis_start: int = 2,
             level_shift: float = 0.0, diverge_factor: float = 1e4, stall_window: int = 40,
             max_rank: int = 0, solver: int = 0, spin_adapted: int = 0,
             raise_on_failure: bool = True) -> SolveResult:
    npair = h.shape[0] // 2
    lib, ctx = _ctx(h.device)
    na = amp_len(npair)
    t = torch.zeros(na, dtype=torch.float64, device=h.device) if t0 is None else t0.clone()
    opts = _lib.SolveOpts(max_iter, tol, diis_dim, diis_start, level_shift, diverge_factor,
                          stall_window, max_rank, solver, spin_adapted)
    info = _lib.SolveInfo()
    e = C.c_double()
    st = lib.pq_solve(ctx, npair, _dev(h, "h", 4 * npair * npair), _dev(eri, "eri", eri_len(npair)),
                      C.byref(opts), _dev(t, "t", na), C.byref(e), C.byref(info))
    if st != 0 and raise_on_failure:
        _check(lib, ctx, st)
    return SolveResult(t, e.value, info.iterations, info.rnorm, _lib.STATUS.get(st, str(st)),
                       info.solve_ms)


def ph_residual(h: torch.Tensor, eri: torch.Tensor, t: torch.Tensor, out: torch.Tensor | None = None):
    """Packed PH (three-pair) residual r(t) (no host sync)."""
    npair = h.shape[0] // 2
    lib, ctx = _ctx(h.device)
    na = amp_len(npair, "ph")
    if out is None:
        out = torch.empty(na, dtype=torch.float64, device=h.device)
    _check(lib, ctx, lib.ph_residual(ctx, npair, _dev(h, "h", 4 * npair * npair),
                                     _dev(eri, "eri", eri_len(npair, "ph")), _dev(t, "t", na),
                                     _dev(out, "out", na)))
    return out


def ph_energy(h: torch.Tensor, eri: torch.Tensor, t: torch.Tensor) -> float:
    npair = h.shape[0] // 2
    lib, ctx = _ctx(h.device)
    e = C.c_double()
    _check(lib, ctx, lib.ph_energy(ctx, npair, _dev(h, "h", 4 * npair * npair),
                                   _dev(eri, "eri", eri_len(npair, "ph")),
                                   _dev(t, "t", amp_len(npair, "ph")), C.byref(e)))
    return e.value


def ph_solve(h: torch.Tensor, eri: torch.Tensor, t0: torch.Tensor | None = None, *,
             tol: float = 1e-8, max_iter: int = 200, diis_dim: int = 8, diis_start: int = 2,
             level_shift: float = 0.0, diverge_factor: float = 1e4, stall_window: int = 40,
             max_rank: int = 0, solver: int = 0, spin_adapted: int = 0,
             raise_on_failure: bool = True) -> SolveResult:
    npair = h.shape[0] // 2
    lib, ctx = _ctx(h.device)
    na = amp_len(npair, "ph")
    t = torch.zeros(na, dtype=torch.float64, device=h.device) if t0 is None else t0.clone()
    opts = _lib.SolveOpts(max_iter, tol, diis_dim, diis_start, level_shift, diverge_factor,
                          stall_window, max_rank, solver, spin_adapted)
    info = _lib.SolveInfo()
    e = C.c_double()
    st = lib.ph_solve(ctx, npair, _dev(h, "h", 4 * npair * npair),
                      _dev(eri, "eri", eri_len(npair, "ph")), C.byref(opts), _dev(t, "t", na),
                      C.byref(e), C.byref(info))
    if st != 0 and raise_on_failure:
        _check(lib, ctx, st)
    return SolveResult(t, e.value, info.iterations, info.rnorm, _lib.STATUS.get(st, str(st)),
                       info.solve_ms)


def pq_vjp(h: torch.Tensor, eri: torch.Tensor, t: torch.Tensor, lam: torch.Tensor,
           energy_weight: float = 0.0, with_hamiltonian: bool = True):
    """Transposed residual contraction (no host sync): returns (tbar, hbar,
    eribar) with tbar = lam . dR/dt + w dE_c/dt and hbar, eribar the same
    with respect to f and the packed integrals (None unless with_hamiltonian)."""
    npair = h.shape[0] // 2
    lib, ctx = _ctx(h.device)
    na, ne = amp_len(npair), eri_len(npair)
    tbar = torch.empty(na, dtype=torch.float64, device=h.device)
    hbar = eribar = None
    hp = ep = None
    if with_hamiltonian:
        hbar = torch.empty_like(h)
        eribar = torch.empty(ne, dtype=torch.float64, device=h.device)
        hp, ep = _dev(hbar, "hbar"), _dev(eribar, "eribar")
    _check(lib, ctx, lib.pq_vjp(ctx, npair, _dev(h, "h", 4 * npair * npair), _dev(eri, "eri", ne),
                                _dev(t, "t", na), _dev(lam, "lam", na), float(energy_weight),
                                _dev(tbar, "tbar"), hp, ep))
    return tbar, hbar, eribar


@dataclass
class GradResult:
    energy: float
    dE_dh: torch.Tensor        # 2N x 2N, f read as a general matrix
    dE_deri: torch.Tensor      # packed integral layout
    lam: torch.Tensor          # de-excitation amplitudes of the Lagrangian
    iterations: int            # lambda iterations
    rnorm: float
    status: str
    solve_ms: float


def pq_energy_grad(h: torch.Tensor, eri: torch.Tensor, t: torch.Tensor | None = None, *,
                   tol: float = 1e-8, max_iter: int = 200, diis_dim: int = 8, diis_start: int = 2,
                   level_shift: float = 0.0, diverge_factor: float = 1e4, stall_window: int = 40,
                   max_rank: int = 0, solver: int = 0, spin_adapted: int = 0,
                   raise_on_failure: bool = True) -> GradResult:
    """PQ correlation energy and dE/dh, dE/d(packed eri) through the lambda
    equations; t: converged amplitudes, or None to solve them here."""
    npair = h.shape[0] // 2
    lib, ctx = _ctx(h.device)
    na, ne = amp_len(npair), eri_len(npair)
    gh = torch.empty_like(h)
    ge = torch.empty(ne, dtype=torch.float64, device=h.device)
    lam = torch.empty(na, dtype=torch.float64, device=h.device)
    opts = _lib.SolveOpts(max_iter, tol, diis_dim, diis_start, level_shift, diverge_factor,
                          stall_window, max_rank, solver, spin_adapted)
    info = _lib.SolveInfo()
    e = C.c_double()
    st = lib.pq_energy_grad(ctx, npair, _dev(h, "h", 4 * npair * npair), _dev(eri, "eri", ne),
                            None if t is None else _dev(t, "t", na), C.byref(opts), C.byref(e),
                            _dev(gh, "dE_dh"), _dev(ge, "dE_deri"), _dev(lam, "lambda"),
                            C.byref(info))
    if st != 0 and raise_on_failure:
        _check(lib, ctx, st)
    return GradResult(e.value, gh, ge, lam, info.iterations, info.rnorm,
                      _lib.STATUS.get(st, str(st)), info.solve_ms)


@dataclass
class DensityResult:
    energy: float
    gamma: torch.Tensor        # 2N x 2N, <E_pq>: reference occupation + dE/dh
    Gamma: torch.Tensor        # packed integral layout, dE/d(eri)
    noons: list                # natural occupation numbers, descending
    iterations: int            # lambda iterations
    rnorm: float
    status: str
    solve_ms: float


def pq_densities(h: torch.Tensor, eri: torch.Tensor, t: torch.Tensor | None = None, *,
                 tol: float = 1e-8, max_iter: int = 200, diis_dim: int = 8, diis_start: int = 2,
                 level_shift: float = 0.0, diverge_factor: float = 1e4, stall_window: int = 40,
                 max_rank: int = 0, solver: int = 0, spin_adapted: int = 0,
                 raise_on_failure: bool = True) -> DensityResult:
    """Unrelaxed densities gamma, Gamma of the PQ Lagrangian and the natural
    occupation numbers; t: converged amplitudes, or None to solve them here."""
    npair = h.shape[0] // 2
    lib, ctx = _ctx(h.device)
    na, ne = amp_len(npair), eri_len(npair)
    g1 = torch.empty_like(h)
    g2 = torch.empty(ne, dtype=torch.float64, device=h.device)
    noons = (C.c_double * (2 * npair))()
    opts = _lib.SolveOpts(max_iter, tol, diis_dim, diis_start, level_shift, diverge_factor,
                          stall_window, max_rank, solver, spin_adapted)
    info = _lib.SolveInfo()
    e = C.c_double()
    st = lib.pq_densities(ctx, npair, _dev(h, "h", 4 * npair * npair), _dev(eri, "eri", ne),
                          None if t is None else _dev(t, "t", na), C.byref(opts), C.byref(e),
                          _dev(g1, "gamma"), _dev(g2, "Gamma"), noons, C.byref(info))
    if st != 0 and raise_on_failure:
        _check(lib, ctx, st)
    return DensityResult(e.value, g1, g2, [noons[i] for i in range(2 * npair)], info.iterations,
                         info.rnorm, _lib.STATUS.get(st, str(st)), info.solve_ms)


class PQEnergy(torch.autograd.Function):
    """E_c(f, eri) of the converged PQ model as a differentiable function.

    Forward solves the amplitudes; backward solves the lambda equations at
    the saved amplitudes and returns grad_E * (dE/dh, dE/deri)."""

    @staticmethod
    def forward(ctx, h, eri, tol=1e-10, max_iter=200):
        h = h.detach().contiguous()
        eri = eri.detach().contiguous()
        res = pq_solve(h, eri, tol=tol, max_iter=max_iter)
        ctx.save_for_backward(h, eri, res.t)
        ctx.tol, ctx.max_iter = tol, max_iter
        return torch.tensor(res.energy, dtype=torch.float64, device=h.device)

    @staticmethod
    def backward(ctx, gE):
        h, eri, t = ctx.saved_tensors
        g = pq_energy_grad(h, eri, t, tol=ctx.tol, max_iter=ctx.max_iter)
        return gE * g.dE_dh, gE * g.dE_deri, None, None


def pq_energy_autograd(h: torch.Tensor, eri: torch.Tensor, tol: float = 1e-10,
                       max_iter: int = 200) -> torch.Tensor:
    return PQEnergy.apply(h, eri, tol, max_iter)
