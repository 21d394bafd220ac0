// Batched PQ solves: many Hamiltonians of uneven pair counts iterated together.
//
// Every chain keeps its own Jacobi/DIIS state (Sec. III) and converges on its
// own; all chains advance in lockstep, spread over several HIP streams in
// longest-processing-time order so their kernels run concurrently, and the
// per-chain norms and DIIS Gram rows are reduced on the device into one array
// each, so the whole batch needs three host synchronisations per iteration
// (norms, Gram rows, DIIS coefficients) instead of three per chain.  Chains
// sharing a stream share its residual workspace.
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
    int stored = 0, next = 0;
    bool active = true;
    int iters = 0;
    double rn = INFINITY, rmin = INFINITY;
    pqph_status st = PQPH_NOT_CONVERGED;
    std::vector<double> B;
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

}  // namespace

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
    pqph_solve_opts o;
    pqph_default_opts(&o);
    if (opts_in) o = *opts_in;
    if (o.max_iter < 1 || !(o.tol > 0.0) || o.diis_dim < 0 || o.diis_dim > 16 ||
        !(o.diverge_factor > 1.0))
        return pqph_fail(ctx, PQPH_INVALID_ARG, "invalid solver options");
    PQPH_HIP(ctx, hipSetDevice(ctx->device));
    const int m = std::max(o.diis_dim, 1);
    const int ns = std::min(kMaxStreams, nbatch);
    pqph_status st = make_streams(ctx, ns);
    if (st) return st;

    // longest processing time first: the two-spectator work grows as N^4
    std::vector<Chain> ch(nbatch);
    std::vector<int> order(nbatch);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return npair[a] > npair[b]; });
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
    // and the batch-wide arrays of norms, Gram rows, coefficients, energies
    size_t total = 0;
    for (int s = 0; s < ns; ++s) total += ws_need[s];
    for (auto& x : ch) total += x.n * (4 + 2 * (size_t)m) + (size_t)x.nblk * (m + 1);
    const size_t nsmall = (size_t)nbatch * (2 * m + 4);
    total += nsmall;
    st = pqph_ensure_sv(ctx, total * sizeof(double));
    if (st) return st;
    st = pqph_ensure_host(ctx, nsmall);
    if (st) return st;
    double* p = ctx->sv;
    std::vector<double*> ws(ns);
    for (int s = 0; s < ns; ++s) { ws[s] = p; p += ws_need[s]; }
    for (auto& x : ch) {
        x.D = p; p += x.n;
        x.r = p; p += x.n;
        x.e = p; p += x.n;
        x.tn = p; p += x.n;
        x.th = p; p += (size_t)m * x.n;
        x.eh = p; p += (size_t)m * x.n;
        x.part = p; p += (size_t)x.nblk * (m + 1);
    }
    double* norms = p; p += nbatch;
    double* gram = p; p += (size_t)nbatch * m;
    double* coef = p; p += (size_t)nbatch * m;
    double* edev = p; p += nbatch;
    double* dmin = p; p += nbatch;
    double* hst = ctx->host;
    auto S = [&](const Chain& x) { return ctx->bstreams[x.stream]; };

    PQPH_HIP(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    if ((st = fork(ctx, ns))) return st;
    for (int c : order) {
        Chain& x = ch[c];
        if ((st = pq_denominators_dev(ctx, S(x), x.N, x.h, o.level_shift, x.D))) return st;
        launch_absmin(S(x), x.D, x.n, x.part, x.nblk, dmin + c);
    }
    if ((st = join(ctx, ns))) return st;
    PQPH_HIP(ctx, hipMemcpyAsync(hst, dmin, nbatch * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int c = 0; c < nbatch; ++c)
        if (!(hst[c] > 1e-12))
            return pqph_fail(ctx, PQPH_INVALID_ARG,
                             "chain " + std::to_string(c) + ": vanishing orbital-energy denominator");

    std::vector<double> cvec;
    int nactive = nbatch;
    for (int it = 1; it <= o.max_iter && nactive > 0; ++it) {
        // residuals and their norms
        if ((st = fork(ctx, ns))) return st;
        for (int c : order) {
            Chain& x = ch[c];
            if (!x.active) continue;
            if ((st = pq_residual_ws(ctx, S(x), x.N, x.h, x.eri, x.t, x.r, ws[x.stream]))) return st;
            launch_norm2(S(x), x.r, x.n, x.part, x.nblk, norms + c);
        }
        if ((st = join(ctx, ns))) return st;
        PQPH_HIP(ctx, hipMemcpyAsync(hst, norms, nbatch * sizeof(double), hipMemcpyDeviceToHost,
                                     ctx->stream));
        PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
        for (int c = 0; c < nbatch; ++c) {
            Chain& x = ch[c];
            if (!x.active) continue;
            x.iters = it;
            x.rn = std::sqrt(hst[c]);
            x.rmin = std::min(x.rmin, x.rn);
            if (!std::isfinite(x.rn)) x.st = PQPH_NONFINITE;
            else if (x.rn <= o.tol) x.st = PQPH_OK;
            else if (x.rn > 1e3 || x.rn > o.diverge_factor * x.rmin) x.st = PQPH_DIVERGED;
            else if (it == o.max_iter) x.st = PQPH_NOT_CONVERGED;
            else continue;
            x.active = false;
            --nactive;
        }
        if (nactive == 0) break;
        // Jacobi step, DIIS history and Gram rows
        if ((st = fork(ctx, ns))) return st;
        for (int c : order) {
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
                        gram + (size_t)c * m);
        }
        if ((st = join(ctx, ns))) return st;
        std::vector<char> use(nbatch, 0);
        if (o.diis_dim > 0) {
            PQPH_HIP(ctx, hipMemcpyAsync(hst, gram, (size_t)nbatch * m * sizeof(double),
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
                        for (int b = 0; b < x.stored; ++b) Bs[(size_t)a * 16 + b] = x.B[(size_t)a * 16 + b];
                    if (diis_solve(Bs, x.stored, cvec)) {
                        for (int a = 0; a < x.stored; ++a) cm[(size_t)c * m + a] = cvec[a];
                        use[c] = 1;
                    }
                }
            }
            for (size_t i = 0; i < cm.size(); ++i) hst[i] = cm[i];
            PQPH_HIP(ctx, hipMemcpyAsync(coef, hst, cm.size() * sizeof(double), hipMemcpyHostToDevice,
                                         ctx->stream));
        }
        if ((st = fork(ctx, ns))) return st;
        for (int c : order) {
            Chain& x = ch[c];
            if (!x.active) continue;
            if (use[c])
                launch_combine(S(x), x.th, coef + (size_t)c * m, m, x.n, x.t);
            else
                PQPH_HIP(ctx, hipMemcpyAsync(x.t, x.tn, x.n * sizeof(double), hipMemcpyDeviceToDevice,
                                             S(x)));
        }
        if ((st = join(ctx, ns))) return st;
        // the pinned coefficients must stay untouched until the copy has run
        PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    // energies of the last iterates
    if ((st = fork(ctx, ns))) return st;
    for (int c : order) {
        Chain& x = ch[c];
        if ((st = pq_energy_ws(ctx, S(x), x.N, x.h, x.eri, x.t, edev + c, ws[x.stream]))) return st;
    }
    if ((st = join(ctx, ns))) return st;
    PQPH_HIP(ctx, hipMemcpyAsync(hst, edev, nbatch * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    PQPH_HIP(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    pqph_status worst = PQPH_OK;
    for (int c = 0; c < nbatch; ++c) {
        energies[c] = hst[c];
        if (ch[c].st == PQPH_OK && !std::isfinite(hst[c])) ch[c].st = PQPH_NONFINITE;
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
