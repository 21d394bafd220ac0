// Batched PQ solves: many Hamiltonians of uneven pair counts iterated together.
//
// Every chain keeps its own Jacobi/DIIS state (Sec. III) and converges on its
// own.  Chains are spread over several HIP streams in longest-processing-time
// order so their kernels run concurrently; chains sharing a stream share its
// residual workspace.
//
// Default (graph) mode: the whole iteration of every chain runs on the device
// -- the residual, then the single solve's device-driven kernels: one pass for
// the norm, the Jacobi step into the DIIS history and the Gram row; one
// workgroup for the convergence/stall/divergence tests and the (m+1)x(m+1)
// DIIS solve; the extrapolation -- with the chain's state (flags, counters,
// B matrix, coefficients, best-norm ring) in device memory.  One iteration of
// the whole batch is captured once into a HIP graph and replayed; a finished
// chain closes its gate flag and all of its later kernels return at once.
// The host only polls the gate flags every few replays.
//
// Lockstep mode (pqph_set_batch_mode 1): the same iteration driven from the
// host, with three host synchronisations per iteration for the whole batch.
#include "pqph_internal.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace {

constexpr int kMaxStreams = 8;

struct Chain {
    int N = 0, stream = 0;
    size_t n = 0;
    int nblk = 0;
    const double *h = nullptr, *eri = nullptr;
    double* t = nullptr;
    double *D, *r, *e, *tn, *th, *eh, *part;
    double* vtx = nullptr;        // the chain's bare vertices, formed once per batch
    int stored = 0, next = 0;
    bool active = true;
    int iters = 0;
    double rn = INFINITY, rmin = INFINITY;
    pqph_status st = PQPH_NOT_CONVERGED;
    std::vector<double> B;
    std::vector<double> best;     // smallest norm so far, per iteration
};

pqph_status make_streams(pqph_ctx* ctx, int ns) {
    while ((int)ctx->bstreams.size() < ns) {
        hipStream_t s;
        PQPH_HIP(ctx, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        ctx->bstreams.push_back(s);
        hipEvent_t e;
        PQPH_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->bevents.push_back(e);
    }
    if (!ctx->fork) PQPH_HIP(ctx, hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
    return PQPH_OK;
}

// make every batch stream wait for work already issued on the context stream
pqph_status fork(pqph_ctx* ctx, int ns) {
    PQPH_HIP(ctx, hipEventRecord(ctx->fork, ctx->stream));
    for (int i = 0; i < ns; ++i) PQPH_HIP(ctx, hipStreamWaitEvent(ctx->bstreams[i], ctx->fork, 0));
    return PQPH_OK;
}

// make the context stream wait for all batch streams
pqph_status join(pqph_ctx* ctx, int ns) {
    for (int i = 0; i < ns; ++i) {
        PQPH_HIP(ctx, hipEventRecord(ctx->bevents[i], ctx->bstreams[i]));
        PQPH_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->bevents[i], 0));
    }
    return PQPH_OK;
}


// ------------------------------------------------- device-resident iteration
// Each chain's Jacobi/DIIS state lives in device memory (the single solve's
// device-driven state, dev_solve_doubles() doubles per chain); its active
// flag gates every kernel of the chain, residual included.
}  // namespace

namespace {

struct Batch {
    int nb, ns, m;
    pqph_solve_opts o;
    std::vector<Chain> ch;
    std::vector<int> order;
    std::vector<double*> ws;
    double *norms, *gram, *coef, *edev, *dmin;
    double* dstate;               // nb device-resident chain states, dsd doubles apart
    size_t dsd;
    SolveHead* head(int c) const { return reinterpret_cast<SolveHead*>(dstate + (size_t)c * dsd); }
};

pqph_status lockstep(pqph_ctx* ctx, Batch& b) {
    const pqph_solve_opts& o = b.o;
    const int nbatch = b.nb, ns = b.ns, m = b.m;
    auto& ch = b.ch;
    double* hst = ctx->host;
    auto S = [&](const Chain& x) { return ctx->bstreams[x.stream]; };
    pqph_status st;
    std::vector<double> cvec;
    int nactive = nbatch;
    for (int it = 1; it <= o.max_iter && nactive > 0; ++it) {
        // residuals and their norms
        if ((st = fork(ctx, ns))) return st;
        for (int c : b.order) {
            Chain& x = ch[c];
            if (!x.active) continue;
            if ((st = pq_residual_ws(ctx, S(x), x.N, x.h, x.eri, x.t, x.r, b.ws[x.stream], nullptr, -1, false,
                                     x.vtx)))
                return st;
            launch_norm2(S(x), x.r, x.n, x.part, x.nblk, b.norms + c);
        }
        if ((st = join(ctx, ns))) return st;
        PQPH_HIP(ctx, hipMemcpyAsync(hst, b.norms, nbatch * sizeof(double), hipMemcpyDeviceToHost,
                                     ctx->stream));
        PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
        for (int c = 0; c < nbatch; ++c) {
            Chain& x = ch[c];
            if (!x.active) continue;
            x.iters = it;
            x.rn = std::sqrt(hst[c]);
            x.rmin = std::min(x.rmin, x.rn);
            x.best.push_back(x.rmin);
            const bool stalled = o.stall_window > 0 && it > o.stall_window &&
                                 x.rmin > 0.5 * x.best[it - 1 - o.stall_window];
            // the single solve's order: non-finite, converged, stalled, diverged, limit
            if (!std::isfinite(x.rn)) x.st = PQPH_NONFINITE;
            else if (x.rn <= o.tol) x.st = PQPH_OK;
            else if (stalled) x.st = PQPH_NOT_CONVERGED;
            else if (x.rn > 1e3 || x.rn > o.diverge_factor * x.rmin) x.st = PQPH_DIVERGED;
            else if (it == o.max_iter) x.st = PQPH_NOT_CONVERGED;
            else continue;
            x.active = false;
            --nactive;
        }
        if (nactive == 0) break;
        // Jacobi step, DIIS history and Gram rows
        if ((st = fork(ctx, ns))) return st;
        for (int c : b.order) {
            Chain& x = ch[c];
            if (!x.active) continue;
            launch_jacobi(S(x), x.t, x.r, x.D, x.n, x.tn, x.e);
            if (o.diis_dim == 0) continue;
            const int slot = x.next;
            PQPH_HIP(ctx, hipMemcpyAsync(x.th + (size_t)slot * x.n, x.tn, x.n * sizeof(double),
                                         hipMemcpyDeviceToDevice, S(x)));
            PQPH_HIP(ctx, hipMemcpyAsync(x.eh + (size_t)slot * x.n, x.e, x.n * sizeof(double),
                                         hipMemcpyDeviceToDevice, S(x)));
            launch_gram(S(x), x.eh, m, x.eh + (size_t)slot * x.n, x.n, x.part, x.nblk,
                        b.gram + (size_t)c * m);
        }
        if ((st = join(ctx, ns))) return st;
        std::vector<char> use(nbatch, 0);
        if (o.diis_dim > 0) {
            PQPH_HIP(ctx, hipMemcpyAsync(hst, b.gram, (size_t)nbatch * m * sizeof(double),
                                         hipMemcpyDeviceToHost, ctx->stream));
            PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
            std::vector<double> cm((size_t)nbatch * m, 0.0);
            for (int c = 0; c < nbatch; ++c) {
                Chain& x = ch[c];
                if (!x.active) continue;
                const int slot = x.next;
                x.next = (x.next + 1) % m;
                x.stored = std::min(x.stored + 1, m);
                for (int j = 0; j < m; ++j) {
                    x.B[(size_t)slot * 16 + j] = hst[(size_t)c * m + j];
                    x.B[(size_t)j * 16 + slot] = hst[(size_t)c * m + j];
                }
                if (it >= o.diis_start && x.stored >= 2) {
                    std::vector<double> Bs(16 * 16, 0.0);
                    for (int a = 0; a < x.stored; ++a)
                        for (int q = 0; q < x.stored; ++q) Bs[(size_t)a * 16 + q] = x.B[(size_t)a * 16 + q];
                    if (diis_solve(Bs, x.stored, cvec)) {
                        for (int a = 0; a < x.stored; ++a) cm[(size_t)c * m + a] = cvec[a];
                        use[c] = 1;
                    }
                }
            }
            for (size_t i = 0; i < cm.size(); ++i) hst[i] = cm[i];
            PQPH_HIP(ctx, hipMemcpyAsync(b.coef, hst, cm.size() * sizeof(double), hipMemcpyHostToDevice,
                                         ctx->stream));
        }
        if ((st = fork(ctx, ns))) return st;
        for (int c : b.order) {
            Chain& x = ch[c];
            if (!x.active) continue;
            if (use[c])
                launch_combine(S(x), x.th, b.coef + (size_t)c * m, x.stored, x.n, x.t);
            else
                PQPH_HIP(ctx, hipMemcpyAsync(x.t, x.tn, x.n * sizeof(double), hipMemcpyDeviceToDevice,
                                             S(x)));
        }
        if ((st = join(ctx, ns))) return st;
        // the pinned coefficients must stay untouched until the copy has run
        PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    return PQPH_OK;
}

// one iteration of every chain, enqueued on the batch streams (captured): the
// residual, then the single solve's device-driven step, decision and update
pqph_status enqueue_iteration(pqph_ctx* ctx, Batch& b, const DevSolveOpts& dopts) {
    pqph_status st;
    for (int c : b.order) {
        Chain& x = b.ch[c];
        hipStream_t s = ctx->bstreams[x.stream];
        double* state = b.dstate + (size_t)c * b.dsd;
        const int* gate = &b.head(c)->active;
        if ((st = pq_residual_ws(ctx, s, x.N, x.h, x.eri, x.t, x.r, b.ws[x.stream], gate, -1, false,
                                 x.vtx)))
            return st;
        launch_dsolve_step(s, state, x.t, x.r, x.D, x.n, x.th, x.eh, b.m, x.part, x.nblk);
        launch_dsolve_decide(s, state, x.part, x.nblk, dopts);
        launch_dsolve_update(s, state, x.th, x.n, x.t, nullptr, nullptr);
    }
    PQPH_HIP(ctx, hipGetLastError());
    return PQPH_OK;
}

pqph_status graph_mode(pqph_ctx* ctx, Batch& b) {
    const int ns = b.ns, nb = b.nb;
    DevSolveOpts dopts;
    dopts.max_iter = b.o.max_iter;
    dopts.m = b.m;
    dopts.diis_on = b.o.diis_dim > 0;
    dopts.diis_start = b.o.diis_start;
    dopts.stall_window = b.o.stall_window;
    dopts.tol = b.o.tol;
    dopts.diverge_factor = b.o.diverge_factor;
    hipStream_t s0 = ctx->bstreams[0];
    pqph_status st;
    for (int c = 0; c < nb; ++c) launch_dsolve_init(ctx->stream, b.dstate + (size_t)c * b.dsd);
    PQPH_HIP(ctx, hipGetLastError());
    // s0 starts after everything already on the context stream
    PQPH_HIP(ctx, hipEventRecord(ctx->fork, ctx->stream));
    PQPH_HIP(ctx, hipStreamWaitEvent(s0, ctx->fork, 0));
    PQPH_HIP(ctx, hipStreamBeginCapture(s0, hipStreamCaptureModeRelaxed));
    // fork the other streams from s0, enqueue, join them back into s0
    bool capturing = true;
    auto body = [&]() -> pqph_status {
        PQPH_HIP(ctx, hipEventRecord(ctx->fork, s0));
        for (int i = 1; i < ns; ++i) PQPH_HIP(ctx, hipStreamWaitEvent(ctx->bstreams[i], ctx->fork, 0));
        pqph_status e = enqueue_iteration(ctx, b, dopts);
        if (e) return e;
        for (int i = 1; i < ns; ++i) {
            PQPH_HIP(ctx, hipEventRecord(ctx->bevents[i], ctx->bstreams[i]));
            PQPH_HIP(ctx, hipStreamWaitEvent(s0, ctx->bevents[i], 0));
        }
        return PQPH_OK;
    };
    st = body();
    hipGraph_t graph = nullptr;
    hipError_t ec = hipStreamEndCapture(s0, &graph);
    capturing = false;
    (void)capturing;
    if (st) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (ec != hipSuccess || !graph)
        return pqph_fail(ctx, PQPH_DEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
    hipGraphExec_t exec = nullptr;
    ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ec != hipSuccess)
        return pqph_fail(ctx, PQPH_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ec));
    // replay; poll the gate flags after a few replays, then every other one
    int* flags = reinterpret_cast<int*>(ctx->host);
    pqph_status result = PQPH_OK;
    int launched = 0;
    int next_poll = std::min(b.o.max_iter, 8);
    while (launched < b.o.max_iter) {
        ec = hipGraphLaunch(exec, s0);
        if (ec != hipSuccess) {
            result = pqph_fail(ctx, PQPH_DEVICE, std::string("graph launch: ") + hipGetErrorString(ec));
            break;
        }
        ++launched;
        if (launched < next_poll && launched < b.o.max_iter) continue;
        ec = hipMemcpy2DAsync(flags, sizeof(int), &b.head(0)->active, b.dsd * sizeof(double), sizeof(int),
                              nb, hipMemcpyDeviceToHost, s0);
        if (ec == hipSuccess) ec = hipStreamSynchronize(s0);
        if (ec != hipSuccess) {
            result = pqph_fail(ctx, PQPH_DEVICE, std::string("poll: ") + hipGetErrorString(ec));
            break;
        }
        int any = 0;
        for (int c = 0; c < nb; ++c) any |= flags[c];
        if (!any) break;
        next_poll = launched + 2;
    }
    (void)hipGraphExecDestroy(exec);
    if (result) return result;
    PQPH_HIP(ctx, hipEventRecord(ctx->bevents[0], s0));
    PQPH_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->bevents[0], 0));
    return PQPH_OK;
}

}  // namespace

extern "C" pqph_status pqph_set_batch_mode(pqph_ctx* ctx, int mode) {
    if (!ctx) return pqph_fail(nullptr, PQPH_INVALID_ARG, "null context");
    if (mode != 0 && mode != 1) return pqph_fail(ctx, PQPH_INVALID_ARG, "batch mode must be 0 or 1");
    ctx->batch_mode = mode;
    return PQPH_OK;
}

extern "C" pqph_status pq_solve_batched(pqph_ctx* ctx, int nbatch, const int* npair,
                                        const int64_t* h_off, const int64_t* eri_off,
                                        const int64_t* t_off, const double* h, const double* eri,
                                        const pqph_solve_opts* opts_in, double* t,
                                        double* energies, pqph_solve_info* infos) {
    if (!ctx) return pqph_fail(nullptr, PQPH_INVALID_ARG, "null context");
    if (nbatch < 1 || !npair || !h_off || !eri_off || !t_off || !h || !eri || !t || !energies)
        return pqph_fail(ctx, PQPH_INVALID_ARG, "invalid batch arguments");
    for (int c = 0; c < nbatch; ++c)
        if (npair[c] < 1 || npair[c] > 256 || h_off[c] < 0 || eri_off[c] < 0 || t_off[c] < 0)
            return pqph_fail(ctx, PQPH_INVALID_ARG,
                             "chain " + std::to_string(c) + ": npair must be in [1, 256], offsets >= 0");
    Batch b;
    pqph_solve_opts& o = b.o;
    pqph_default_opts(&o);
    if (opts_in) o = *opts_in;
    if (o.max_iter < 1 || !(o.tol > 0.0) || o.diis_dim < 0 || o.diis_dim > 16 ||
        !(o.diverge_factor > 1.0) || o.stall_window < 0 || o.stall_window >= kSolveRing || o.max_rank != 0 ||
        (o.solver != 0 && o.solver != 2) || o.spin_adapted != 0)
        return pqph_fail(ctx, PQPH_INVALID_ARG,
                         "invalid solver options (batched: stall_window < 257, max_rank 0, solver 0 or 2, "
                         "spin_adapted 0)");
    PQPH_HIP(ctx, hipSetDevice(ctx->device));
    const int m = b.m = std::max(o.diis_dim, 1);
    const int ns = b.ns = std::min(kMaxStreams, nbatch);
    b.nb = nbatch;
    pqph_status st = make_streams(ctx, ns);
    if (st) return st;

    // longest processing time first: the two-spectator work grows as N^4
    auto& ch = b.ch;
    auto& order = b.order;
    ch.resize(nbatch);
    order.resize(nbatch);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int a, int q) { return npair[a] > npair[q]; });
    std::vector<double> load(ns, 0.0);
    std::vector<size_t> ws_need(ns, 0);
    for (int c : order) {
        const int s = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        const double N = npair[c];
        load[s] += N * N * N * N;
        Chain& x = ch[c];
        x.N = npair[c];
        x.stream = s;
        x.n = pq_amp_len(x.N);
        x.nblk = stream_blocks(x.n);
        x.h = h + h_off[c];
        x.eri = eri + eri_off[c];
        x.t = t + t_off[c];
        x.B.assign(16 * 16, 0.0);
        ws_need[s] = std::max(ws_need[s], pq_ws_doubles(x.N) + 8);
    }
    // device memory: per-stream residual workspace, per-chain solver state,
    // the batch-wide arrays of norms, Gram rows, coefficients, energies, and
    // the device-resident chain states
    size_t total = 0;
    for (int s = 0; s < ns; ++s) total += ws_need[s];
    for (auto& x : ch) total += x.n * (4 + 2 * (size_t)m) + (size_t)x.nblk * (m + 1) + pq_vertex_doubles(x.N);
    const size_t nsmall = (size_t)nbatch * (2 * m + 4);
    total += nsmall;
    b.dsd = dev_solve_doubles();
    total += b.dsd * nbatch + 32;
    st = pqph_ensure_sv(ctx, total * sizeof(double));
    if (st) return st;
    st = pqph_ensure_host(ctx, nsmall);
    if (st) return st;
    double* p = ctx->sv;
    b.ws.resize(ns);
    for (int s = 0; s < ns; ++s) { b.ws[s] = p; p += ws_need[s]; }
    for (auto& x : ch) {
        x.D = p; p += x.n;
        x.r = p; p += x.n;
        x.e = p; p += x.n;
        x.tn = p; p += x.n;
        x.th = p; p += (size_t)m * x.n;
        x.eh = p; p += (size_t)m * x.n;
        x.part = p; p += (size_t)x.nblk * (m + 1);
        x.vtx = p; p += pq_vertex_doubles(x.N);
    }
    b.norms = p; p += nbatch;
    b.gram = p; p += (size_t)nbatch * m;
    b.coef = p; p += (size_t)nbatch * m;
    b.edev = p; p += nbatch;
    b.dmin = p; p += nbatch;
    p = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(p) + 255) & ~uintptr_t(255));
    b.dstate = p;
    double* hst = ctx->host;
    auto S = [&](const Chain& x) { return ctx->bstreams[x.stream]; };

    PQPH_HIP(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    if ((st = fork(ctx, ns))) return st;
    for (int c : order) {
        Chain& x = ch[c];
        if ((st = pq_denominators_dev(ctx, S(x), x.N, x.h, o.level_shift, x.D))) return st;
        launch_absmin(S(x), x.D, x.n, x.part, x.nblk, b.dmin + c);
        // the vertices depend on the chain's integrals only: formed once
        if ((st = pq_vertices_into(ctx, S(x), x.N, x.h, x.eri, x.vtx))) return st;
    }
    if ((st = join(ctx, ns))) return st;
    PQPH_HIP(ctx, hipMemcpyAsync(hst, b.dmin, nbatch * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int c = 0; c < nbatch; ++c)
        if (!(hst[c] > 1e-12))
            return pqph_fail(ctx, PQPH_INVALID_ARG,
                             "chain " + std::to_string(c) + ": vanishing orbital-energy denominator");

    if (ctx->batch_mode == 1) {
        if ((st = lockstep(ctx, b))) return st;
    } else {
        if ((st = graph_mode(ctx, b))) return st;
        // per-chain reports from the device states
        std::vector<SolveHead> hs(nbatch);
        PQPH_HIP(ctx, hipMemcpy2DAsync(hs.data(), sizeof(SolveHead), b.head(0), b.dsd * sizeof(double),
                                       sizeof(SolveHead), nbatch, hipMemcpyDeviceToHost, ctx->stream));
        PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
        for (int c = 0; c < nbatch; ++c) {
            ch[c].iters = hs[c].iters;
            ch[c].rn = hs[c].rn;
            ch[c].st = hs[c].active ? PQPH_NOT_CONVERGED : hs[c].status;
        }
    }
    // energies of the last iterates
    if ((st = fork(ctx, ns))) return st;
    for (int c : order) {
        Chain& x = ch[c];
        if ((st = pq_energy_ws(ctx, S(x), x.N, x.h, x.eri, x.t, b.edev + c, b.ws[x.stream]))) return st;
    }
    if ((st = join(ctx, ns))) return st;
    PQPH_HIP(ctx, hipMemcpyAsync(hst, b.edev, nbatch * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    PQPH_HIP(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    std::vector<double> en(hst, hst + nbatch);
    // solver 2: chains the batched Jacobi/DIIS left unconverged are solved
    // again alone (Jacobi/DIIS, then Newton-Krylov from its best iterate); the
    // batch's device state is no longer needed, so pq_solve may reuse it
    if (o.solver == 2) {
        pqph_solve_opts o2 = o;
        for (int c = 0; c < nbatch; ++c) {
            if (ch[c].st != PQPH_NOT_CONVERGED && ch[c].st != PQPH_DIVERGED) continue;
            Chain& x = ch[c];
            PQPH_HIP(ctx, hipMemsetAsync(x.t, 0, x.n * sizeof(double), ctx->stream));
            pqph_solve_info inf{};
            double e = 0.0;
            const pqph_status sc = pq_solve(ctx, x.N, x.h, x.eri, &o2, x.t, &e, &inf);
            if (sc != PQPH_OK && sc != PQPH_NOT_CONVERGED && sc != PQPH_DIVERGED && sc != PQPH_NONFINITE)
                return sc;
            x.st = sc;
            x.iters += inf.iterations;
            x.rn = inf.rnorm;
            en[c] = e;
            ms += (float)inf.solve_ms;      // pq_solve times itself on the context stream
        }
    }
    pqph_status worst = PQPH_OK;
    for (int c = 0; c < nbatch; ++c) {
        energies[c] = en[c];
        if (ch[c].st == PQPH_OK && !std::isfinite(en[c])) ch[c].st = PQPH_NONFINITE;
        if (infos) {
            infos[c].iterations = ch[c].iters;
            infos[c].rnorm = ch[c].rn;
            infos[c].status = ch[c].st;
            infos[c].solve_ms = ms;
        }
        if (ch[c].st != PQPH_OK && worst == PQPH_OK) worst = ch[c].st;
    }
    if (worst != PQPH_OK) pqph_fail(ctx, worst, "some chains of the batch did not converge (see infos)");
    return worst;
}
