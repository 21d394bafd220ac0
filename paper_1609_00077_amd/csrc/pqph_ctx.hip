// Context, workspace and the C ABI entry points of libpqph.
#include "pqph_internal.h"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <vector>

namespace {

thread_local std::string g_no_ctx_error;

}  // namespace

// ------------------------------------------- scratch of pq_residual_noalloc
// A file-scope device array: every GPU the library runs on holds its own
// copy from module load until the process ends.  Host code never uses the
// array's name as an address; the device address of each GPU's copy is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and kept in g_scratch_dev.  48 MiB holds the carved residual workspace up
// to 32 pairs.
constexpr size_t kScratchDoubles = (size_t)6 << 20;
constexpr int kScratchMaxPairs = 32;
constexpr int kScratchMaxDevices = 64;
static __device__ __align__(256) double scratch[kScratchDoubles];
static std::mutex g_scratch_mu;
static double* g_scratch_dev[kScratchMaxDevices] = {};

// Called with ctx->device current.
static pqph_status scratch_lookup(pqph_ctx* ctx) {
    if (ctx->device >= kScratchMaxDevices) return PQPH_OK;   // the entry point reports it
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[ctx->device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return pqph_fail(ctx, PQPH_DEVICE, std::string("scratch symbol lookup: ") +
                                                   hipGetErrorString(e));
        }
        g_scratch_dev[ctx->device] = (double*)p;
    }
    ctx->scratch = g_scratch_dev[ctx->device];
    return PQPH_OK;
}

// ----------------------------------------------------------------- helpers
pqph_status pqph_fail(pqph_ctx* ctx, pqph_status st, const std::string& msg) {
    if (ctx)
        ctx->err = msg;
    else
        g_no_ctx_error = msg;
    return st;
}

static pqph_status ensure_dev(pqph_ctx* ctx, double*& buf, size_t& have, size_t bytes) {
    if (bytes <= have) return PQPH_OK;
    if (buf) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(buf);
        buf = nullptr;
        have = 0;
    }
    size_t want = std::max(bytes, have + have / 4);
    if (hipMalloc((void**)&buf, want) != hipSuccess) {
        buf = nullptr;
        (void)hipGetLastError();
        if (hipMalloc((void**)&buf, bytes) != hipSuccess) {
            buf = nullptr;
            (void)hipGetLastError();
            return pqph_fail(ctx, PQPH_OOM, "device workspace allocation of " +
                                                std::to_string(bytes) + " bytes failed");
        }
        want = bytes;
    }
    have = want;
    return PQPH_OK;
}

pqph_status pqph_ensure_ws(pqph_ctx* ctx, size_t bytes) {
    return ensure_dev(ctx, ctx->ws, ctx->ws_bytes, bytes);
}
pqph_status pqph_ensure_sv(pqph_ctx* ctx, size_t bytes) {
    return ensure_dev(ctx, ctx->sv, ctx->sv_bytes, bytes);
}
pqph_status pqph_ensure_host(pqph_ctx* ctx, size_t n) {
    if (n <= ctx->host_n) return PQPH_OK;
    if (ctx->host) (void)hipHostFree(ctx->host);
    ctx->host = nullptr;
    ctx->host_n = 0;
    if (hipHostMalloc((void**)&ctx->host, n * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        ctx->host = nullptr;
        (void)hipGetLastError();
        return pqph_fail(ctx, PQPH_OOM, "pinned host allocation failed");
    }
    ctx->host_n = n;
    return PQPH_OK;
}

int pq_intermediates(const pqph_ctx* ctx, int npair) {
    return (npair >= 0 && npair <= 256 && ctx->pq_int[npair] == 2) ? 2 : 3;
}

int pq_s2_variant(const pqph_ctx* ctx, int npair) {
    if (npair >= 0 && npair <= 256 && ctx->s2_variant[npair]) return ctx->s2_variant[npair];
    return 1;
}

pqph_status pq_residual_graph(pqph_ctx* ctx, int N, const double* h, const double* eri,
                              const double* t, double* r, double* ws, const int* gate,
                              bool vertices) {
    if (ctx->profiling) return pq_residual_ws(ctx, ctx->stream, N, h, eri, t, r, ws, gate, -1, vertices);
    const int s1 = pq_s1_mode(ctx, N), s2 = pq_s2_variant(ctx, N), li = pq_intermediates(ctx, N);
    using G = pqph_ctx::ResidualGraph;
    auto same = [&](const G& g) {
        return g.exec && g.N == N && g.h == h && g.eri == eri && g.t == t && g.r == r && g.ws == ws &&
               g.s1 == s1 && g.s2 == s2 && g.li == li && g.gate == gate && g.vertices == vertices;
    };
    G* hit = nullptr;
    for (G& g : ctx->rgraph)
        if (same(g)) hit = &g;
    if (!hit) {
        // an empty entry, else the least recently used one
        hit = &ctx->rgraph[0];
        for (G& g : ctx->rgraph)
            if (!g.exec || (hit->exec && g.used < hit->used)) hit = &g;
        if (hit->exec) {
            PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));    // the old graph may still run
            (void)hipGraphExecDestroy(hit->exec);
            *hit = G();
        }
        // capture on a stream of our own (the context's may be the legacy default
        // stream, which cannot be captured), forked to the side streams, then
        // replay on the context's stream
        if (pqph_status e = pq_residual_prepare(ctx)) return e;
        if (pqph_status e = pqph_ensure_side(ctx)) return e;
        if (!ctx->cap) PQPH_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
        PQPH_HIP(ctx, hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeRelaxed));
        const pqph_status st = pq_residual_ws(ctx, ctx->cap, N, h, eri, t, r, ws, gate, 1, vertices);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(ctx->cap, &graph);
        if (st) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (ec != hipSuccess || !graph)
            return pqph_fail(ctx, PQPH_DEVICE, std::string("residual capture: ") + hipGetErrorString(ec));
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess)
            return pqph_fail(ctx, PQPH_DEVICE, std::string("residual instantiate: ") + hipGetErrorString(ei));
        hit->exec = exec;
        hit->N = N;
        hit->h = h;
        hit->eri = eri;
        hit->t = t;
        hit->r = r;
        hit->ws = ws;
        hit->s1 = s1;
        hit->s2 = s2;
        hit->li = li;
        hit->gate = gate;
        hit->vertices = vertices;
    }
    hit->used = ++ctx->rgraph_clock;
    PQPH_HIP(ctx, hipGraphLaunch(hit->exec, ctx->stream));
    return PQPH_OK;
}

pqph_status pqph_ensure_side(pqph_ctx* ctx) {
    for (hipStream_t& st : ctx->side)
        if (!st) PQPH_HIP(ctx, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    for (hipEvent_t& e : ctx->sev)
        if (!e) PQPH_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return PQPH_OK;
}

int pq_s1_mode(const pqph_ctx* ctx, int npair) {
    if (npair >= 0 && npair <= 256 && ctx->s1_mode[npair]) return ctx->s1_mode[npair];
    // untuned: the materialised sides with pipelined staging (mode 4; measured:
    // equal to the other modes within noise below 50 pairs, 1.1x-1.4x faster
    // residuals from 60 to 120 pairs)
    return 4;
}

void pqph_mark(pqph_ctx* ctx) {
    if (!ctx->profiling || ctx->prof_n >= 24) return;
    (void)hipEventRecord(ctx->prof[ctx->prof_n++], ctx->stream);
}

static pqph_status check_pq(pqph_ctx* ctx, int npair) {
    if (!ctx) return pqph_fail(nullptr, PQPH_INVALID_ARG, "null context");
    if (npair < 1 || npair > 256)
        return pqph_fail(ctx, PQPH_INVALID_ARG, "npair must be in [1, 256]");
    PQPH_HIP(ctx, hipSetDevice(ctx->device));
    return PQPH_OK;
}

// ================================================================== C ABI
extern "C" {

void pqph_default_opts(pqph_solve_opts* o) {
    if (!o) return;
    o->max_iter = 200;
    o->tol = 1e-8;
    o->diis_dim = 8;
    o->diis_start = 2;
    o->level_shift = 0.0;
    o->diverge_factor = 1e4;
    o->stall_window = 40;
    o->max_rank = 0;
    o->solver = 0;
    o->spin_adapted = 0;
}

pqph_status pqph_set_solve_mode(pqph_ctx* ctx, int mode) {
    if (!ctx) return pqph_fail(nullptr, PQPH_INVALID_ARG, "null context");
    if (mode != 0 && mode != 1) return pqph_fail(ctx, PQPH_INVALID_ARG, "solve mode must be 0 or 1");
    ctx->solve_mode = mode;
    return PQPH_OK;
}

pqph_status pqph_create(pqph_ctx** out, int device, void* hip_stream) {
    if (!out) return pqph_fail(nullptr, PQPH_INVALID_ARG, "null output pointer");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return pqph_fail(nullptr, PQPH_INVALID_ARG, "no such HIP device");
    pqph_ctx* ctx = new pqph_ctx();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess || hipEventCreate(&ctx->ev0) != hipSuccess ||
        hipEventCreate(&ctx->ev1) != hipSuccess) {
        delete ctx;
        return pqph_fail(nullptr, PQPH_DEVICE, "device setup failed");
    }
    if (scratch_lookup(ctx) != PQPH_OK || pq_residual_prepare(ctx) != PQPH_OK) {
        const std::string msg = ctx->err;
        pqph_destroy(ctx);
        return pqph_fail(nullptr, PQPH_DEVICE, msg);
    }
    *out = ctx;
    return PQPH_OK;
}

void pqph_destroy(pqph_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->sv) (void)hipFree(ctx->sv);
    if (ctx->host) (void)hipHostFree(ctx->host);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    for (hipEvent_t e : ctx->prof)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->bevents) (void)hipEventDestroy(e);
    for (hipStream_t st : ctx->bstreams) (void)hipStreamDestroy(st);
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    for (pqph_ctx::ResidualGraph& g : ctx->rgraph)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    for (hipEvent_t e : ctx->dsev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    for (hipEvent_t e : ctx->sev)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t st : ctx->side)
        if (st) (void)hipStreamDestroy(st);
    ph_tables_free(ctx);
    delete ctx;
}

const char* pqph_last_error(const pqph_ctx* ctx) {
    return ctx ? ctx->err.c_str() : g_no_ctx_error.c_str();
}

size_t pq_amp_len(int n) {
    if (n < 1) return 0;
    return 3 * (size_t)n + 29 * ((size_t)n * (n - 1) / 2);
}
size_t ph_amp_len(int n) {
    if (n < 1) return 0;
    return pq_amp_len(n) + 303 * ((size_t)n * (n - 1) * (n - 2) / 6);
}
size_t pq_eri_len(int n) {
    if (n < 1) return 0;
    return 6 * (size_t)n + 43 * ((size_t)n * (n - 1) / 2);
}
size_t ph_eri_len(int n) {
    if (n < 1) return 0;
    return pq_eri_len(n) + 84 * ((size_t)n * (n - 1) * (n - 2) / 6);
}

pqph_status pq_residual(pqph_ctx* ctx, int npair, const double* h, const double* eri,
                        const double* t, double* r) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (!h || !eri || !t || !r) return pqph_fail(ctx, PQPH_INVALID_ARG, "null array");
    st = pqph_ensure_ws(ctx, pq_ws_doubles(npair) * sizeof(double));
    if (st) return st;
    return pq_residual_graph(ctx, npair, h, eri, t, r, ctx->ws);
}

pqph_status pq_residual_noalloc(pqph_ctx* ctx, int npair, const double* h, const double* eri,
                                const double* t, double* r) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (!h || !eri || !t || !r) return pqph_fail(ctx, PQPH_INVALID_ARG, "null array");
    if (npair > kScratchMaxPairs || pq_ws_doubles(npair) > kScratchDoubles)
        return pqph_fail(ctx, PQPH_INVALID_ARG,
                         "npair above the allocation-free limit of " +
                             std::to_string(kScratchMaxPairs) + " pairs");
    if (!ctx->scratch)
        return pqph_fail(ctx, PQPH_DEVICE, "no scratch array on this device");
    if ((st = pq_residual_prepare(ctx))) return st;
    // the same kernels as pq_residual, serially on the context's stream, with
    // the workspace carved from this GPU's scratch array; every workspace
    // value a kernel reads is written earlier in the same call, so nothing
    // needs clearing between calls
    return pq_residual_ws(ctx, ctx->stream, npair, h, eri, t, r, ctx->scratch, nullptr, 0);
}

static const char* kPhaseNames[] = {"k_vertex1",  "k_vertex2", "k_unpack_t2", "k_spec_w",
                                    "k_spec_lam", "k_dress",   "k_spec_xy",   "k_gemm_s1",
                                    "k_r2s2",     "k_r2c",     "k_spec_r1",   "k_r1s2",
                                    "k_r1s2_close", "k_r1",    "k_r1c",       "k_final"};
constexpr int kNPhase = (int)(sizeof(kPhaseNames) / sizeof(kPhaseNames[0]));

const char* pq_residual_phase_name(int i) {
    return (i >= 0 && i < kNPhase) ? kPhaseNames[i] : "";
}

pqph_status pq_residual_profile(pqph_ctx* ctx, int npair, const double* h, const double* eri,
                                const double* t, double* r, double* phase_ms, int nphase,
                                int* nphase_out) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (!h || !eri || !t || !r || !phase_ms || !nphase_out)
        return pqph_fail(ctx, PQPH_INVALID_ARG, "null array");
    st = pqph_ensure_ws(ctx, pq_ws_doubles(npair) * sizeof(double));
    if (st) return st;
    for (int i = 0; i < 24; ++i)
        if (!ctx->prof[i]) PQPH_HIP(ctx, hipEventCreate(&ctx->prof[i]));
    ctx->prof_n = 0;
    ctx->profiling = true;
    pqph_mark(ctx);   // start event
    st = pq_residual_ws(ctx, ctx->stream, npair, h, eri, t, r, ctx->ws);
    ctx->profiling = false;
    if (st) return st;
    PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const int n = ctx->prof_n - 1;
    if (n > nphase) return pqph_fail(ctx, PQPH_INVALID_ARG, "phase_ms too short");
    for (int i = 0; i < n; ++i) {
        float ms = 0.f;
        PQPH_HIP(ctx, hipEventElapsedTime(&ms, ctx->prof[i], ctx->prof[i + 1]));
        phase_ms[i] = ms;
    }
    *nphase_out = n;
    return PQPH_OK;
}

pqph_status pqph_set_variant(pqph_ctx* ctx, int npair, int variant) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (variant < 0 || variant > 2 || (variant == 2 && (npair + 15) / 16 > 6))
        return pqph_fail(ctx, PQPH_INVALID_ARG, "variant must be 0, 1, or 2 (2 needs npair <= 96)");
    ctx->s2_variant[npair] = variant;
    return PQPH_OK;
}

pqph_status pqph_set_s1_mode(pqph_ctx* ctx, int npair, int mode) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (mode < 0 || mode > 4 || (mode == 3 && npair > 128))
        return pqph_fail(ctx, PQPH_INVALID_ARG, "mode must be 0, 1, 2, 3 or 4 (3 needs npair <= 128)");
    ctx->s1_mode[npair] = mode;
    return PQPH_OK;
}

pqph_status pqph_set_pq_intermediates(pqph_ctx* ctx, int npair, int labels) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (labels != 2 && labels != 3)
        return pqph_fail(ctx, PQPH_INVALID_ARG, "intermediates must span 2 or 3 pairs");
    ctx->pq_int[npair] = labels;
    return PQPH_OK;
}

pqph_status pqph_tuning(pqph_ctx* ctx, int npair, int* s2_variant, int* s1_mode) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (s2_variant) *s2_variant = pq_s2_variant(ctx, npair);
    if (s1_mode) *s1_mode = pq_s1_mode(ctx, npair);
    return PQPH_OK;
}

pqph_status pqph_autotune(pqph_ctx* ctx, int npair, const double* h, const double* eri,
                          const double* t, double* r, int* choice) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (!h || !eri || !t || !r) return pqph_fail(ctx, PQPH_INVALID_ARG, "null array");
    st = pqph_ensure_ws(ctx, pq_ws_doubles(npair) * sizeof(double));
    if (st) return st;
    const int nvar = (npair + 15) / 16 <= 6 ? 2 : 1;
    float best = 1e30f;
    int bestv = 1, bestm = 1;
    // the default mode 4 first (near-ties keep it, below), then 1, 2 and,
    // up to 128 pairs, 3 (not built above)
    const int modes[4] = {4, 1, 2, 3};
    const int nmode = npair <= 128 ? 4 : 3;
    for (int combo = 0; combo < nmode * nvar; ++combo) {
        const int var = 1 + combo % nvar, mode = modes[combo / nvar];
        ctx->s2_variant[npair] = var;
        ctx->s1_mode[npair] = mode;
        for (int rep = 0; rep < 2; ++rep) {      // first run warms up
            PQPH_HIP(ctx, hipEventRecord(ctx->ev0, ctx->stream));
            for (int k = 0; k < 3; ++k) {
                st = pq_residual_ws(ctx, ctx->stream, npair, h, eri, t, r, ctx->ws);
                if (st) return st;
            }
            PQPH_HIP(ctx, hipEventRecord(ctx->ev1, ctx->stream));
            PQPH_HIP(ctx, hipEventSynchronize(ctx->ev1));
            float ms = 0.f;
            PQPH_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
            // a later (non-default) choice must win by 3 %: near-ties keep the
            // default, so the choice is stable from run to run
            if (rep == 1 && (combo == 0 || ms < 0.97f * best)) {
                best = ms;
                bestv = var;
                bestm = mode;
            }
        }
    }
    ctx->s2_variant[npair] = bestv;
    ctx->s1_mode[npair] = bestm;
    if (choice) *choice = bestv;
    return PQPH_OK;
}

pqph_status pq_energy(pqph_ctx* ctx, int npair, const double* h, const double* eri,
                      const double* t, double* energy) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (!h || !eri || !t || !energy) return pqph_fail(ctx, PQPH_INVALID_ARG, "null array");
    const size_t wsd = pq_ws_doubles(npair);
    st = pqph_ensure_ws(ctx, (wsd + 8) * sizeof(double));
    if (st) return st;
    double* dst = ctx->ws + wsd;
    st = pq_energy_ws(ctx, ctx->stream, npair, h, eri, t, dst, ctx->ws);
    if (st) return st;
    PQPH_HIP(ctx, hipMemcpyAsync(energy, dst, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (!std::isfinite(*energy)) return pqph_fail(ctx, PQPH_NONFINITE, "non-finite energy");
    return PQPH_OK;
}

pqph_status pqph_denominators(pqph_ctx* ctx, int npair, int k, const double* h, double shift,
                              double* D) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (k != 2 && k != 3) return pqph_fail(ctx, PQPH_INVALID_ARG, "k must be 2 (PQ) or 3 (PH)");
    if (!h || !D) return pqph_fail(ctx, PQPH_INVALID_ARG, "null array");
    if (k == 3) return ph_denominators_dev(ctx, ctx->stream, npair, h, shift, D);
    return pq_denominators_dev(ctx, ctx->stream, npair, h, shift, D);
}

}  // extern "C"

// ------------------------------------------------------ Jacobi/DIIS driver
// x <- x - r/D with DIIS on the last m iterates (Sec. III; Table IV), where
// resid(x, r) enqueues r = F(x) on the context stream.  bufs holds
// n*(3 + 2m) + nblk*(m+1) + 64 doubles.  One host sync per iteration.
namespace {
size_t driver_doubles(size_t n, int m) {
    return n * (3 + 2 * (size_t)m) + (size_t)stream_blocks(n) * (m + 1) + 64 + dev_solve_doubles();
}

// The Jacobi/DIIS iteration with every decision on the device (k_ds_* in the
// solver kernels): the norm test, the history bookkeeping, the Gram row and
// the DIIS coefficients.  The host enqueues iteration it + 1 before it waits
// for the state of iteration it, so the GPU never idles while the host reads
// a norm; the state's active flag is the residual's gate (ctx->solve_gate,
// for closures that pass it on) and every step kernel obeys it, so the one
// iteration enqueued beyond the end changes nothing.  Same steps, tests and
// messages as the host-driven loop below; the DIIS coefficients are solved
// on the device (same elimination, rounding may differ in the last bits).
pqph_status jacobi_diis_device(pqph_ctx* ctx, size_t n, const double* D, double* x,
                               const pqph_solve_opts& o,
                               const std::function<pqph_status(const double*, double*)>& resid,
                               double* bufs, int& iters, double& rn, pqph_status& result,
                               const double* rank, double* best) {
    const int m = std::max(o.diis_dim, 1);
    const int nblk = stream_blocks(n);
    double* r = bufs;
    double* th = r + 3 * n;                         // the host loop's layout: r, e, xn, xh, eh, part, scal
    double* eh = th + (size_t)m * n;
    double* part = eh + (size_t)m * n;
    double* state = part + (size_t)nblk * (m + 1) + 64;
    const SolveHead* head = reinterpret_cast<const SolveHead*>(state);
    hipStream_t s = ctx->stream;
    PQPH_HIP(ctx, hipStreamSynchronize(s));          // no copy into the host staging is pending
    if (pqph_status e = pqph_ensure_host(ctx, 64)) return e;
    for (hipEvent_t& e : ctx->dsev)
        if (!e) PQPH_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // two slots by iteration parity in the pinned staging, written by the
    // update kernel of every iteration (device address hd)
    SolveHead* hh = reinterpret_cast<SolveHead*>(ctx->host);
    static_assert(2 * sizeof(SolveHead) <= 64 * sizeof(double), "host staging too small");
    SolveHead* hd = nullptr;
    PQPH_HIP(ctx, hipHostGetDevicePointer((void**)&hd, ctx->host, 0));
    hh[0].active = hh[1].active = 1;
    hh[0].iters = hh[1].iters = 0;
    const char* venv = getenv("PQPH_VERBOSE");
    const bool verbose = venv && venv[0] && venv[0] != '0';
    const auto t_start = std::chrono::steady_clock::now();
    int printed = 0;
    auto report = [&](const SolveHead& hd) {
        if (!verbose || hd.iters <= printed) return;
        printed = hd.iters;
        fprintf(stderr, "pqph: iteration %d  ||R|| = %.3e  (%.1f s)\n", hd.iters, hd.rn,
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count());
    };
    DevSolveOpts dopts;
    dopts.max_iter = o.max_iter;
    dopts.m = m;
    dopts.diis_on = o.diis_dim > 0;
    dopts.diis_start = o.diis_start;
    dopts.stall_window = o.stall_window;
    dopts.tol = o.tol;
    dopts.diverge_factor = o.diverge_factor;
    const bool masked = rank != nullptr && o.max_rank > 0;
    launch_dsolve_init(s, state);
    if (masked) launch_rank_mask(s, x, rank, o.max_rank, n);
    // The gate is published only while this loop runs.  On every way out the
    // stream is drained first: iterations queued ahead write the mirror slots
    // in the pinned staging, which a later call may reallocate.
    struct GateScope {
        pqph_ctx* c;
        ~GateScope() {
            (void)hipStreamSynchronize(c->stream);
            c->solve_gate = nullptr;
        }
    } scope{ctx};
    ctx->solve_gate = &head->active;
    for (int it = 1; it <= o.max_iter; ++it) {
        if (pqph_status e = resid(x, r)) return e;
        if (masked) launch_rank_mask(s, r, rank, o.max_rank, n);
        launch_dsolve_step(s, state, x, r, D, n, th, eh, m, part, nblk);
        launch_dsolve_decide(s, state, part, nblk, dopts);
        launch_dsolve_update(s, state, th, n, x, best, hd + (it & 1));
        PQPH_HIP(ctx, hipEventRecord(ctx->dsev[it & 1], s));
        if (it > 1) {       // the state after iteration it - 1 (iteration it is already queued)
            PQPH_HIP(ctx, hipEventSynchronize(ctx->dsev[(it - 1) & 1]));
            const SolveHead prev = hh[(it - 1) & 1];
            report(prev);
            // the iteration that ended the solve wrote its own count (an
            // iteration gated off copies the unchanged state)
            if (!prev.active && prev.iters == it - 1) break;
        }
    }
    PQPH_HIP(ctx, hipMemcpyAsync(&hh[0], head, sizeof(SolveHead), hipMemcpyDeviceToHost, s));
    PQPH_HIP(ctx, hipStreamSynchronize(s));
    const SolveHead fin = hh[0];
    report(fin);
    iters = fin.iters;
    rn = fin.rn;
    result = fin.active ? PQPH_NOT_CONVERGED : (pqph_status)fin.status;
    if (result == PQPH_NONFINITE) {
        pqph_fail(ctx, result, "non-finite residual at iteration " + std::to_string(fin.iters));
    } else if (result == PQPH_DIVERGED) {
        pqph_fail(ctx, result, "residual norm diverged at iteration " + std::to_string(fin.iters));
    } else if (result == PQPH_NOT_CONVERGED && fin.stalled) {
        pqph_fail(ctx, result, "stalled: ||R|| did not halve in " + std::to_string(o.stall_window) +
                                   " iterations (iteration " + std::to_string(fin.iters) + ")");
    } else if (result == PQPH_NOT_CONVERGED) {
        pqph_fail(ctx, result, "not converged in " + std::to_string(o.max_iter) + " iterations");
    }
    return PQPH_OK;
}

// pipelined: the caller's residual is cheap next to a host round trip and
// obeys ctx->solve_gate, so the device-driven loop above may run it
pqph_status jacobi_diis(pqph_ctx* ctx, size_t n, const double* D, double* x,
                        const pqph_solve_opts& o,
                        const std::function<pqph_status(const double*, double*)>& resid,
                        double* bufs, int& iters, double& rn, pqph_status& result,
                        const double* rank = nullptr, double* best = nullptr,
                        bool pipelined = false) {
    if (pipelined && ctx->solve_mode == 0 && o.max_iter >= 1 && o.diis_dim <= 16 &&
        o.stall_window <= kSolveRing - 1)
        return jacobi_diis_device(ctx, n, D, x, o, resid, bufs, iters, rn, result, rank, best);
    const int m = std::max(o.diis_dim, 1);
    const int nblk = stream_blocks(n);
    double* r = bufs;
    double* e = r + n;
    double* xn = e + n;
    double* xh = xn + n;
    double* eh = xh + (size_t)m * n;
    double* part = eh + (size_t)m * n;
    double* hst = ctx->host;
    hipStream_t s = ctx->stream;
    std::vector<double> B(16 * 16, 0.0), c;
    int stored = 0, next = 0, it = 0;
    double rmin = INFINITY;
    std::vector<double> hist_min;  // hist_min[i]: smallest norm up to iteration i + 1
    rn = INFINITY;
    result = PQPH_NOT_CONVERGED;
    // One host synchronisation per iteration: the Jacobi step, the history
    // copies and the DIIS Gram row are enqueued right behind the residual norm
    // (if the iteration turns out to be the last they are simply unused), and
    // the norm and the Gram row come back together, written by the reduction
    // kernel straight into the pinned staging (hdev: its device address).
    // The DIIS coefficients go to the device as kernel arguments.
    double* hdev = nullptr;
    PQPH_HIP(ctx, hipHostGetDevicePointer((void**)&hdev, hst, 0));
    const bool diis = o.diis_dim > 0;
    // PQPH_VERBOSE=1: one line per iteration on stderr (long solves report progress)
    const char* venv = getenv("PQPH_VERBOSE");
    const bool verbose = venv && venv[0] && venv[0] != '0';
    const auto t_start = std::chrono::steady_clock::now();
    // excitations above max_rank: t stays zero, their residuals are not solved for
    const bool masked = rank != nullptr && o.max_rank > 0;
    if (masked) launch_rank_mask(s, x, rank, o.max_rank, n);
    for (it = 1; it <= o.max_iter; ++it) {
        pqph_status st = resid(x, r);
        if (st) return st;
        if (masked) launch_rank_mask(s, r, rank, o.max_rank, n);
        const bool step = it < o.max_iter;
        const int slot = next;
        if (step && diis) {      // norm, step and Gram row in one pass, into the history slot
            launch_step(s, x, r, D, n, xh + (size_t)slot * n, eh, m, slot, part, nblk, hdev);
        } else {
            launch_norm2(s, r, n, part, nblk, hdev);
            if (step) launch_jacobi(s, x, r, D, n, xn, e);
        }
        PQPH_HIP(ctx, hipStreamSynchronize(s));
        rn = std::sqrt(hst[0]);
        if (verbose)
            fprintf(stderr, "pqph: iteration %d  ||R|| = %.3e  (%.1f s)\n", it, rn,
                    std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count());
        if (!std::isfinite(rn)) {
            result = PQPH_NONFINITE;
            pqph_fail(ctx, result, "non-finite residual at iteration " + std::to_string(it));
            break;
        }
        if (best && rn < rmin)      // keep the iterate of smallest ||R|| (x is unchanged so far)
            PQPH_HIP(ctx, hipMemcpyAsync(best, x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        rmin = std::min(rmin, rn);
        hist_min.push_back(rmin);
        if (rn <= o.tol) {
            result = PQPH_OK;
            break;
        }
        if (o.stall_window > 0 && it > o.stall_window && rmin > 0.5 * hist_min[it - 1 - o.stall_window]) {
            pqph_fail(ctx, result, "stalled: ||R|| did not halve in " + std::to_string(o.stall_window) +
                                       " iterations (iteration " + std::to_string(it) + ")");
            iters = it;
            return PQPH_OK;
        }
        if (rn > 1e3 || rn > o.diverge_factor * rmin) {
            result = PQPH_DIVERGED;
            pqph_fail(ctx, result, "residual norm diverged at iteration " + std::to_string(it));
            break;
        }
        if (!step) break;
        if (!diis) {
            PQPH_HIP(ctx, hipMemcpyAsync(x, xn, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            continue;
        }
        next = (next + 1) % m;
        stored = std::min(stored + 1, m);
        for (int j = 0; j < m; ++j) {
            B[(size_t)slot * 16 + j] = hst[1 + j];
            B[(size_t)j * 16 + slot] = hst[1 + j];
        }
        if (it >= o.diis_start && stored >= 2) {
            std::vector<double> Bs(16 * 16, 0.0);
            for (int a = 0; a < stored; ++a)
                for (int b = 0; b < stored; ++b) Bs[(size_t)a * 16 + b] = B[(size_t)a * 16 + b];
            if (diis_solve(Bs, stored, c)) {
                launch_combine_host(s, xh, c.data(), stored, n, x);   // only written slots
                continue;
            }
        }
        PQPH_HIP(ctx, hipMemcpyAsync(x, xh + (size_t)slot * n, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
    iters = std::min(it, o.max_iter);
    if (result == PQPH_NOT_CONVERGED)
        pqph_fail(ctx, result, "not converged in " + std::to_string(o.max_iter) + " iterations");
    return PQPH_OK;
}

// Inexact Newton-Krylov solve of R(x) = 0, the same fixed point as the
// Jacobi/DIIS iteration, for the systems where that iteration stalls or
// diverges (Sec. IV.B: strongly correlated geometries; the paper suggests a
// better preconditioner).  Each Newton step solves J dx = -R by GMRES with up
// to KRYLOV Arnoldi vectors (no restart), right-preconditioned by the orbital-energy
// denominators (J M^-1 y = -R, dx = M^-1 y, M = diag(D)); J v comes from
// central differences of the residual, R(x + e v) - R(x - e v) = 2 e J v +
// O(e^3) (R is a quartic polynomial in t); classical Gram-Schmidt with one
// reorthogonalisation; the step is backtracked until ||R|| decreases.
// Every residual is evaluated on the same two buffers (xin -> rout), so a
// captured residual graph is reused.  iters counts residual evaluations.
constexpr int KRYLOV = 100;       // 30 vectors stalled near the root on strongly correlated chains
constexpr int NEWTON_MAX_STEPS = 60;

size_t newton_doubles(size_t n) {
    return n * (5 + KRYLOV + 1) + (size_t)stream_blocks(n) * (KRYLOV + 1) + KRYLOV + 64;
}

pqph_status newton_krylov(pqph_ctx* ctx, size_t n, const double* D, double* x,
                          const pqph_solve_opts& o,
                          const std::function<pqph_status(const double*, double*)>& resid,
                          double* nbuf, int& iters, double& rn, pqph_status& result,
                          const double* rank) {
    const int nblk = stream_blocks(n);
    double* r = nbuf;
    double* xin = r + n;
    double* rout = xin + n;
    double* w = rout + n;
    double* z = w + n;
    double* V = z + n;                                   // KRYLOV + 1 vectors
    double* part = V + (size_t)(KRYLOV + 1) * n;
    double* scal = part + (size_t)nblk * (KRYLOV + 1);
    hipStream_t s = ctx->stream;
    // host staging: Gram rows (KRYLOV + 1) and, apart, the Krylov coefficients
    PQPH_HIP(ctx, hipStreamSynchronize(s));      // no copy from the old buffer is pending
    if (pqph_status e = pqph_ensure_host(ctx, 2 * KRYLOV + 64)) return e;
    double* hst = ctx->host;
    double* hy = hst + KRYLOV + 32;
    const bool masked = rank != nullptr && o.max_rank > 0;
    const char* venv = getenv("PQPH_VERBOSE");
    const bool verbose = venv && venv[0] && venv[0] != '0';
    auto R = [&]() -> pqph_status {                      // rout = R(xin), masked
        if (pqph_status e = resid(xin, rout)) return e;
        if (masked) launch_rank_mask(s, rout, rank, o.max_rank, n);
        ++iters;
        return PQPH_OK;
    };
    auto fetch = [&](int cnt) -> pqph_status {           // scal[0..cnt) -> hst
        PQPH_HIP(ctx, hipMemcpyAsync(hst, scal, cnt * sizeof(double), hipMemcpyDeviceToHost, s));
        PQPH_HIP(ctx, hipStreamSynchronize(s));
        return PQPH_OK;
    };
    auto norm = [&](const double* v, double& out) -> pqph_status {
        launch_norm2(s, v, n, part, nblk, scal);
        if (pqph_status e = fetch(1)) return e;
        out = std::sqrt(hst[0]);
        return PQPH_OK;
    };
    pqph_status st;
    result = PQPH_NOT_CONVERGED;
    if (masked) launch_rank_mask(s, x, rank, o.max_rank, n);
    PQPH_HIP(ctx, hipMemcpyAsync(xin, x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if ((st = R())) return st;
    PQPH_HIP(ctx, hipMemcpyAsync(r, rout, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    double beta = 0.0;
    for (int step = 0; step < NEWTON_MAX_STEPS; ++step) {
        if ((st = norm(r, beta))) return st;
        rn = beta;
        if (verbose) fprintf(stderr, "pqph: Newton step %d  ||R|| = %.3e\n", step, beta);
        if (!std::isfinite(beta)) {
            result = PQPH_NONFINITE;
            pqph_fail(ctx, result, "non-finite residual in the Newton-Krylov solve");
            return PQPH_OK;
        }
        if (beta <= o.tol) {
            result = PQPH_OK;
            return PQPH_OK;
        }
        double xnorm = 0.0;
        if ((st = norm(x, xnorm))) return st;
        launch_axpby(s, V, -1.0 / beta, r, 0.0, nullptr, nullptr, n);      // V_0 = -R / beta
        std::vector<double> H((size_t)(KRYLOV + 1) * KRYLOV, 0.0), g(KRYLOV + 1, 0.0), cs(KRYLOV),
            sn(KRYLOV);
        auto Hat = [&](int i, int j) -> double& { return H[(size_t)i * KRYLOV + j]; };
        g[0] = beta;
        const double eta = std::min(0.1, std::sqrt(beta));                 // forcing term
        int k = 0;
        for (int j = 0; j < KRYLOV; ++j) {
            const double* Vj = V + (size_t)j * n;
            launch_axpby(s, z, 0.0, Vj, 1.0, Vj, D, n);                     // z = M^-1 V_j
            double zn = 0.0;
            if ((st = norm(z, zn))) return st;
            if (!(zn > 0.0)) break;
            const double e = 1e-5 * (1.0 + xnorm) / zn;
            launch_axpby(s, xin, 1.0, x, e, z, nullptr, n);
            if ((st = R())) return st;
            PQPH_HIP(ctx, hipMemcpyAsync(w, rout, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            launch_axpby(s, xin, 1.0, x, -e, z, nullptr, n);
            if ((st = R())) return st;
            launch_axpby(s, w, 0.5 / e, w, -0.5 / e, rout, nullptr, n);    // w = J z
            for (int pass = 0; pass < 2; ++pass) {                           // CGS2
                launch_gram(s, V, j + 1, w, n, part, nblk, scal);
                launch_sub_combine(s, w, V, scal, j + 1, n);
                if ((st = fetch(j + 1))) return st;
                for (int i = 0; i <= j; ++i) Hat(i, j) += hst[i];
            }
            double hn = 0.0;
            if ((st = norm(w, hn))) return st;
            Hat(j + 1, j) = hn;
            if (hn > 0.0) launch_axpby(s, V + (size_t)(j + 1) * n, 1.0 / hn, w, 0.0, nullptr, nullptr, n);
            for (int i = 0; i < j; ++i) {                                    // earlier rotations
                const double a = cs[i] * Hat(i, j) + sn[i] * Hat(i + 1, j);
                Hat(i + 1, j) = -sn[i] * Hat(i, j) + cs[i] * Hat(i + 1, j);
                Hat(i, j) = a;
            }
            const double den = std::hypot(Hat(j, j), Hat(j + 1, j));
            if (!(den > 0.0)) break;
            cs[j] = Hat(j, j) / den;
            sn[j] = Hat(j + 1, j) / den;
            Hat(j, j) = den;
            Hat(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            if (std::fabs(g[j + 1]) <= eta * beta || !(hn > 0.0)) break;
        }
        if (k == 0) {
            pqph_fail(ctx, result, "Newton-Krylov: no Krylov direction");
            return PQPH_OK;
        }
        std::vector<double> y(k, 0.0);                                       // H y = g
        for (int i = k - 1; i >= 0; --i) {
            double a = g[i];
            for (int l = i + 1; l < k; ++l) a -= Hat(i, l) * y[l];
            y[i] = a / Hat(i, i);
        }
        for (int i = 0; i < k; ++i) hy[i] = y[i];
        PQPH_HIP(ctx, hipMemcpyAsync(scal, hy, k * sizeof(double), hipMemcpyHostToDevice, s));
        launch_combine(s, V, scal, k, n, w);                                 // w = sum y_i V_i
        launch_axpby(s, z, 0.0, w, 1.0, w, D, n);                            // dx = M^-1 w
        // the host rewrites hy only after the copy above has completed
        PQPH_HIP(ctx, hipStreamSynchronize(s));
        bool moved = false;
        double lam = 1.0;
        for (int ls = 0; ls < 12 && !moved; ++ls, lam *= 0.5) {
            launch_axpby(s, xin, 1.0, x, lam, z, nullptr, n);
            if ((st = R())) return st;
            double rt = 0.0;
            if ((st = norm(rout, rt))) return st;
            if (std::isfinite(rt) && rt < (1.0 - 1e-4 * lam) * beta) {
                PQPH_HIP(ctx, hipMemcpyAsync(x, xin, n * sizeof(double), hipMemcpyDeviceToDevice, s));
                PQPH_HIP(ctx, hipMemcpyAsync(r, rout, n * sizeof(double), hipMemcpyDeviceToDevice, s));
                moved = true;
            }
        }
        if (!moved) {
            pqph_fail(ctx, result, "Newton-Krylov: the line search found no decrease of ||R||");
            return PQPH_OK;
        }
    }
    if ((st = norm(r, beta))) return st;
    rn = beta;
    if (beta <= o.tol)
        result = PQPH_OK;
    else
        pqph_fail(ctx, result, "Newton-Krylov: not converged in " + std::to_string(NEWTON_MAX_STEPS) +
                                   " steps");
    return PQPH_OK;
}

// The amplitude solve of pq_solve / ph_solve / pq_energy_grad by opts.solver:
// 0 Jacobi/DIIS; 1 Newton-Krylov from x; 2 Jacobi/DIIS, then Newton-Krylov
// from its iterate of smallest ||R|| when it stalls, diverges or runs out of
// iterations.  sbuf: solver_doubles(n, m, solver) doubles.
size_t solver_doubles(size_t n, int m, int solver) {
    size_t d = driver_doubles(n, m);
    if (solver >= 1) d = std::max(d, newton_doubles(n));
    if (solver == 2) d += n;                             // the best Jacobi/DIIS iterate
    return d;
}

pqph_status amplitude_solve(pqph_ctx* ctx, size_t n, const double* D, double* x,
                            const pqph_solve_opts& o,
                            const std::function<pqph_status(const double*, double*)>& resid,
                            double* sbuf, int& iters, double& rn, pqph_status& result,
                            const double* rank, bool pipelined) {
    iters = 0;
    if (o.solver == 1) return newton_krylov(ctx, n, D, x, o, resid, sbuf, iters, rn, result, rank);
    double* best = o.solver == 2 ? sbuf + solver_doubles(n, std::max(o.diis_dim, 1), 1) : nullptr;
    pqph_status st = jacobi_diis(ctx, n, D, x, o, resid, sbuf, iters, rn, result, rank, best, pipelined);
    if (st || o.solver != 2 || (result != PQPH_NOT_CONVERGED && result != PQPH_DIVERGED)) return st;
    PQPH_HIP(ctx, hipMemcpyAsync(x, best, n * sizeof(double), hipMemcpyDeviceToDevice, ctx->stream));
    int it2 = 0;
    st = newton_krylov(ctx, n, D, x, o, resid, sbuf, it2, rn, result, rank);
    iters += it2;
    return st;
}

// The solve in the space opts.spin_adapted selects: the full packed space,
// or the reduced closed-shell space of one value per alpha/beta exchange
// orbit (the residual runs on full vectors unpacked from it, its result is
// projected back).  jd_only: Jacobi/DIIS whatever opts.solver says (the
// lambda equations).  x and rank are full-length; sbuf holds
// space_doubles(...) doubles.
size_t space_doubles(size_t n, int npair, int k, int m, const pqph_solve_opts& o) {
    if (!o.spin_adapted) return solver_doubles(n, m, o.solver);
    const size_t nred = spin_len(npair, k);
    return 3 * nred + 2 * n + solver_doubles(nred, m, o.solver);
}

pqph_status space_solve(pqph_ctx* ctx, int npair, int k, size_t n, const double* D, double* x,
                        const pqph_solve_opts& o,
                        const std::function<pqph_status(const double*, double*)>& resid,
                        double* sbuf, int& iters, double& rn, pqph_status& result, const double* rank,
                        bool jd_only = false, bool pipelined = false) {
    auto core = [&](size_t len, const double* Dv, double* xv,
                    const std::function<pqph_status(const double*, double*)>& rf, double* b,
                    const double* rk) -> pqph_status {
        if (jd_only) return jacobi_diis(ctx, len, Dv, xv, o, rf, b, iters, rn, result, rk, nullptr, pipelined);
        return amplitude_solve(ctx, len, Dv, xv, o, rf, b, iters, rn, result, rk, pipelined);
    };
    if (!o.spin_adapted) return core(n, D, x, resid, sbuf, rank);
    const size_t nred = spin_len(npair, k);
    double* xr = sbuf;
    double* Dr = xr + nred;
    double* rk = Dr + nred;
    double* tf = rk + nred;
    double* rf = tf + n;
    double* b = rf + n;
    hipStream_t s = ctx->stream;
    launch_spin_pack(s, x, xr, npair, k, 0);
    launch_spin_pack(s, D, Dr, npair, k, 1);
    const double* rkp = nullptr;
    if (rank) {
        launch_spin_pack(s, rank, rk, npair, k, 1);
        rkp = rk;
    }
    auto reduced = [&](const double* xin, double* rout) -> pqph_status {
        launch_spin_unpack(s, xin, tf, npair, k);
        if (pqph_status e = resid(tf, rf)) return e;
        launch_spin_pack(s, rf, rout, npair, k, 0);
        return PQPH_OK;
    };
    if (pqph_status st = core(nred, Dr, xr, reduced, b, rkp)) return st;
    launch_spin_unpack(s, xr, x, npair, k);
    PQPH_HIP(ctx, hipGetLastError());
    return PQPH_OK;
}

// Eigenvalues of the symmetric n x n matrix A (row-major, overwritten) by
// cyclic Jacobi rotations (the symmetric Schur decomposition): each rotation
// zeroes one off-diagonal pair; sweeps stop once the off-diagonal Frobenius
// norm is below 1e-15 of the whole norm.  Host code for the small natural
// occupation problem (n = 2N <= 512).
void symmetric_eigenvalues(std::vector<double>& A, int n, std::vector<double>& w) {
    auto at = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
    double total = 0.0;
    for (double x : A) total += x * x;
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += 2.0 * at(p, q) * at(p, q);
        if (off <= 1e-30 * total || off == 0.0) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const double apq = at(p, q);
                if (apq == 0.0) continue;
                // rotation angle: tan(2 theta) = 2 a_pq / (a_qq - a_pp), smaller root
                const double tau = (at(q, q) - at(p, p)) / (2.0 * apq);
                const double tn = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + tn * tn), sn = tn * c;
                for (int k = 0; k < n; ++k) {      // columns p, q
                    const double akp = at(k, p), akq = at(k, q);
                    at(k, p) = c * akp - sn * akq;
                    at(k, q) = sn * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {      // rows p, q
                    const double apk = at(p, k), aqk = at(q, k);
                    at(p, k) = c * apk - sn * aqk;
                    at(q, k) = sn * apk + c * aqk;
                }
                at(p, q) = at(q, p) = 0.0;
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = at(i, i);
    std::sort(w.begin(), w.end(), [](double a, double b) { return a > b; });
}

// Excitation rank (number of holes) of every packed slot, through the
// denominator kernels with f = diag(-1 occupied, 0 virtual); fs holds 4N^2
// doubles of scratch.  Only when o.max_rank truncates the manifold.
pqph_status slot_ranks(pqph_ctx* ctx, const pqph_solve_opts& o, int npair, int k, double* fs,
                       double* rank, const double*& out) {
    out = nullptr;
    if (o.max_rank <= 0) return PQPH_OK;
    launch_rank_fock(ctx->stream, fs, npair);
    pqph_status st = k == 3 ? ph_denominators_dev(ctx, ctx->stream, npair, fs, 0.0, rank)
                            : pq_denominators_dev(ctx, ctx->stream, npair, fs, 0.0, rank);
    if (st) return st;
    out = rank;
    return PQPH_OK;
}

pqph_status read_opts(pqph_ctx* ctx, const pqph_solve_opts* in, pqph_solve_opts& o) {
    pqph_default_opts(&o);
    if (in) o = *in;
    if (o.max_iter < 1 || !(o.tol > 0.0) || o.diis_dim < 0 || o.diis_dim > 16 ||
        !(o.diverge_factor > 1.0) || o.stall_window < 0 || o.max_rank < 0 || o.max_rank > 6 ||
        o.solver < 0 || o.solver > 2 || o.spin_adapted < 0 || o.spin_adapted > 1)
        return pqph_fail(ctx, PQPH_INVALID_ARG, "invalid solver options");
    return PQPH_OK;
}

pqph_status check_denominators(pqph_ctx* ctx, const double* D, size_t n, double* part) {
    launch_absmin(ctx->stream, D, n, part, stream_blocks(n), part + stream_blocks(n));
    PQPH_HIP(ctx, hipMemcpyAsync(ctx->host, part + stream_blocks(n), sizeof(double),
                                 hipMemcpyDeviceToHost, ctx->stream));
    PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (!(ctx->host[0] > 1e-12))
        return pqph_fail(ctx, PQPH_INVALID_ARG, "vanishing orbital-energy denominator");
    return PQPH_OK;
}
}  // namespace

extern "C" {

pqph_status pq_solve(pqph_ctx* ctx, int npair, const double* h, const double* eri,
                     const pqph_solve_opts* opts_in, double* t, double* energy,
                     pqph_solve_info* info) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (!h || !eri || !t || !energy) return pqph_fail(ctx, PQPH_INVALID_ARG, "null array");
    pqph_solve_opts o;
    if ((st = read_opts(ctx, opts_in, o))) return st;
    const size_t n = pq_amp_len(npair);
    const int m = std::max(o.diis_dim, 1);
    const size_t nr = 2 * n + 4 * (size_t)npair * npair;     // D, ranks, rank Fock matrix
    if ((st = pqph_ensure_sv(ctx, (nr + space_doubles(n, npair, 2, m, o)) * sizeof(double)))) return st;
    const size_t wsd = pq_ws_doubles(npair);
    if ((st = pqph_ensure_ws(ctx, (wsd + 8) * sizeof(double)))) return st;
    if ((st = pqph_ensure_host(ctx, 64))) return st;
    double* D = ctx->sv;
    double* bufs = D + nr;
    const double* rank = nullptr;
    hipStream_t s = ctx->stream;
    PQPH_HIP(ctx, hipEventRecord(ctx->ev0, s));
    if ((st = pq_denominators_dev(ctx, s, npair, h, o.level_shift, D))) return st;
    if ((st = check_denominators(ctx, D, n, bufs))) return st;
    if ((st = slot_ranks(ctx, o, npair, 2, D + 2 * n, D + n, rank))) return st;
    int iters = 0;
    double rn = 0.0;
    pqph_status result = PQPH_OK;
    // the vertices depend on h and eri only: formed once, read by every
    // residual of the solve (nothing else writes ws meanwhile)
    if ((st = pq_vertices_ws(ctx, s, npair, h, eri, ctx->ws))) return st;
    auto resid = [&](const double* x, double* r) {
        return pq_residual_graph(ctx, npair, h, eri, x, r, ctx->ws, ctx->solve_gate, false);
    };
    if ((st = space_solve(ctx, npair, 2, n, D, t, o, resid, bufs, iters, rn, result, rank, false, true)))
        return st;
    double* edst = ctx->ws + wsd;
    if ((st = pq_energy_ws(ctx, s, npair, h, eri, t, edst, ctx->ws))) return st;
    PQPH_HIP(ctx, hipMemcpyAsync(ctx->host, edst, sizeof(double), hipMemcpyDeviceToHost, s));
    PQPH_HIP(ctx, hipEventRecord(ctx->ev1, s));
    PQPH_HIP(ctx, hipStreamSynchronize(s));
    *energy = ctx->host[0];
    if (info) {
        info->iterations = iters;
        info->rnorm = rn;
        info->status = result;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
        info->solve_ms = ms;
    }
    if (result == PQPH_OK && !std::isfinite(*energy)) {
        result = PQPH_NONFINITE;
        pqph_fail(ctx, result, "non-finite energy");
    }
    return result;
}

pqph_status ph_residual(pqph_ctx* ctx, int npair, const double* h, const double* eri,
                        const double* t, double* r) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (!h || !eri || !t || !r) return pqph_fail(ctx, PQPH_INVALID_ARG, "null array");
    size_t wsd = 0;
    if ((st = ph_residual_ws_doubles(ctx, npair, &wsd))) return st;
    if ((st = pqph_ensure_ws(ctx, (wsd + 8) * sizeof(double)))) return st;
    return ph_residual_dev(ctx, ctx->stream, npair, h, eri, t, r, ctx->ws);
}

pqph_status ph_energy(pqph_ctx* ctx, int npair, const double* h, const double* eri,
                      const double* t, double* energy) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (!h || !eri || !t || !energy) return pqph_fail(ctx, PQPH_INVALID_ARG, "null array");
    const size_t wsd = ph_energy_ws_doubles();
    if ((st = pqph_ensure_ws(ctx, (wsd + 8) * sizeof(double)))) return st;
    if ((st = ph_energy_dev(ctx, ctx->stream, npair, h, eri, t, ctx->ws + wsd, ctx->ws))) return st;
    PQPH_HIP(ctx, hipMemcpyAsync(energy, ctx->ws + wsd, sizeof(double), hipMemcpyDeviceToHost,
                                 ctx->stream));
    PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (!std::isfinite(*energy)) return pqph_fail(ctx, PQPH_NONFINITE, "non-finite energy");
    return PQPH_OK;
}

pqph_status ph_solve(pqph_ctx* ctx, int npair, const double* h, const double* eri,
                     const pqph_solve_opts* opts_in, double* t, double* energy,
                     pqph_solve_info* info) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (!h || !eri || !t || !energy) return pqph_fail(ctx, PQPH_INVALID_ARG, "null array");
    pqph_solve_opts o;
    if ((st = read_opts(ctx, opts_in, o))) return st;
    if ((st = ph_tables_load(ctx))) return st;
    const size_t n = ph_amp_len(npair);
    const int m = std::max(o.diis_dim, 1);
    const size_t nr = 2 * n + 4 * (size_t)npair * npair;     // D, ranks, rank Fock matrix
    if ((st = pqph_ensure_sv(ctx, (nr + space_doubles(n, npair, 3, m, o)) * sizeof(double)))) return st;
    const size_t wsd = ph_energy_ws_doubles();
    size_t rwsd = 0;      // the residual's partial sums share the workspace (same stream)
    if ((st = ph_residual_ws_doubles(ctx, npair, &rwsd))) return st;
    if ((st = pqph_ensure_ws(ctx, (std::max(wsd, rwsd) + 8) * sizeof(double)))) return st;
    if ((st = pqph_ensure_host(ctx, 64))) return st;
    double* D = ctx->sv;
    double* bufs = D + nr;
    const double* rank = nullptr;
    hipStream_t s = ctx->stream;
    PQPH_HIP(ctx, hipEventRecord(ctx->ev0, s));
    if ((st = ph_denominators_dev(ctx, s, npair, h, o.level_shift, D))) return st;
    if ((st = check_denominators(ctx, D, n, bufs))) return st;
    if ((st = slot_ranks(ctx, o, npair, 3, D + 2 * n, D + n, rank))) return st;
    int iters = 0;
    double rn = 0.0;
    pqph_status result = PQPH_OK;
    auto resid = [&](const double* x, double* r) {
        // the spin-adapted solve hands the residual spin-symmetric amplitudes
        return ph_residual_dev(ctx, s, npair, h, eri, x, r, ctx->ws, o.spin_adapted != 0);
    };
    if ((st = space_solve(ctx, npair, 3, n, D, t, o, resid, bufs, iters, rn, result, rank))) return st;
    double* edst = ctx->ws + wsd;
    if ((st = ph_energy_dev(ctx, s, npair, h, eri, t, edst, ctx->ws))) return st;
    PQPH_HIP(ctx, hipMemcpyAsync(ctx->host, edst, sizeof(double), hipMemcpyDeviceToHost, s));
    PQPH_HIP(ctx, hipEventRecord(ctx->ev1, s));
    PQPH_HIP(ctx, hipStreamSynchronize(s));
    *energy = ctx->host[0];
    if (info) {
        info->iterations = iters;
        info->rnorm = rn;
        info->status = result;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
        info->solve_ms = ms;
    }
    if (result == PQPH_OK && !std::isfinite(*energy)) {
        result = PQPH_NONFINITE;
        pqph_fail(ctx, result, "non-finite energy");
    }
    return result;
}

pqph_status pq_vjp(pqph_ctx* ctx, int npair, const double* h, const double* eri, const double* t,
                   const double* lam, double energy_weight, double* tbar, double* hbar,
                   double* eribar) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (!h || !eri || !t || !lam || !tbar) return pqph_fail(ctx, PQPH_INVALID_ARG, "null array");
    if ((hbar == nullptr) != (eribar == nullptr))
        return pqph_fail(ctx, PQPH_INVALID_ARG, "hbar and eribar must both be given or both NULL");
    const size_t wsd = pq_ws_doubles(npair), ad = pq_adj_doubles(npair);
    if ((st = pqph_ensure_ws(ctx, (wsd + ad) * sizeof(double)))) return st;
    return pq_vjp_ws(ctx, ctx->stream, npair, h, eri, t, lam, energy_weight, tbar, hbar, eribar,
                     ctx->ws, ctx->ws + wsd);
}

pqph_status pq_energy_grad(pqph_ctx* ctx, int npair, const double* h, const double* eri,
                           const double* t_in, const pqph_solve_opts* opts_in, double* energy,
                           double* dE_dh, double* dE_deri, double* lambda_out,
                           pqph_solve_info* info) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (!h || !eri || !energy || !dE_dh || !dE_deri)
        return pqph_fail(ctx, PQPH_INVALID_ARG, "null array");
    pqph_solve_opts o;
    if ((st = read_opts(ctx, opts_in, o))) return st;
    const size_t n = pq_amp_len(npair);
    const int m = std::max(o.diis_dim, 1);
    // solver memory: D, t (when solved here), lambda, tbar scratch, ranks, the
    // rank Fock matrix, driver buffers
    const size_t nr = 5 * n + 4 * (size_t)npair * npair;
    if ((st = pqph_ensure_sv(ctx, (nr + space_doubles(n, npair, 2, m, o)) * sizeof(double)))) return st;
    const size_t wsd = pq_ws_doubles(npair), ad = pq_adj_doubles(npair);
    if ((st = pqph_ensure_ws(ctx, (wsd + ad + 8) * sizeof(double)))) return st;
    if ((st = pqph_ensure_host(ctx, 64))) return st;
    double* D = ctx->sv;
    double* tl = D + n;
    double* lam = tl + n;
    double* tbar = lam + n;
    double* rankv = tbar + n;
    double* bufs = D + nr;
    const double* rank = nullptr;
    double* aws = ctx->ws + wsd;
    hipStream_t s = ctx->stream;
    PQPH_HIP(ctx, hipEventRecord(ctx->ev0, s));
    if ((st = pq_denominators_dev(ctx, s, npair, h, o.level_shift, D))) return st;
    if ((st = check_denominators(ctx, D, n, bufs))) return st;
    if ((st = slot_ranks(ctx, o, npair, 2, rankv + n, rankv, rank))) return st;
    int iters = 0;
    double rn = 0.0;
    pqph_status result = PQPH_OK;
    const double* t = t_in;
    if (!t) {
        PQPH_HIP(ctx, hipMemsetAsync(tl, 0, n * sizeof(double), s));
        if ((st = pq_vertices_ws(ctx, s, npair, h, eri, ctx->ws))) return st;   // once per solve
        auto resid = [&](const double* x, double* r) {
            return pq_residual_graph(ctx, npair, h, eri, x, r, ctx->ws, ctx->solve_gate, false);
        };
        if ((st = space_solve(ctx, npair, 2, n, D, tl, o, resid, bufs, iters, rn, result, rank, false,
                              true)))
            return st;
        if (result != PQPH_OK) return result;
        t = tl;
    }
    double* edst = aws + ad;
    if ((st = pq_energy_ws(ctx, s, npair, h, eri, t, edst, ctx->ws))) return st;
    PQPH_HIP(ctx, hipMemcpyAsync(ctx->host + 32, edst, sizeof(double), hipMemcpyDeviceToHost, s));
    PQPH_HIP(ctx, hipStreamSynchronize(s));
    *energy = ctx->host[32];
    // lambda equations: J^T lambda + dE/dt = 0, solved like the amplitudes
    // start from lambda = t, its first-order value (both solve equations with
    // the same leading part D); the converged lambda does not depend on it
    PQPH_HIP(ctx, hipMemcpyAsync(lam, t, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    // t is fixed from here on: the forward intermediates the adjoint reads are
    // computed by the first VJP and reused by the later ones (only the VJPs
    // write ws and aws during the lambda solve)
    bool fwd_ready = false;
    auto lres = [&](const double* x, double* r) {
        pqph_status e = pq_vjp_ws(ctx, s, npair, h, eri, t, x, 1.0, r, nullptr, nullptr, ctx->ws, aws,
                                  fwd_ready);
        fwd_ready = fwd_ready || e == PQPH_OK;
        return e;
    };
    if ((st = space_solve(ctx, npair, 2, n, D, lam, o, lres, bufs, iters, rn, result, rank, true)))
        return st;
    if ((st = pq_vjp_ws(ctx, s, npair, h, eri, t, lam, 1.0, tbar, dE_dh, dE_deri, ctx->ws, aws, fwd_ready)))
        return st;
    if (lambda_out)
        PQPH_HIP(ctx, hipMemcpyAsync(lambda_out, lam, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    PQPH_HIP(ctx, hipEventRecord(ctx->ev1, s));
    PQPH_HIP(ctx, hipStreamSynchronize(s));
    if (info) {
        info->iterations = iters;
        info->rnorm = rn;
        info->status = result;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
        info->solve_ms = ms;
    }
    return result;
}

pqph_status pq_densities(pqph_ctx* ctx, int npair, const double* h, const double* eri,
                         const double* t, const pqph_solve_opts* opts, double* energy, double* gamma,
                         double* Gamma, double* noons, pqph_solve_info* info) {
    pqph_status st = check_pq(ctx, npair);
    if (st) return st;
    if (!gamma || !Gamma) return pqph_fail(ctx, PQPH_INVALID_ARG, "null array");
    if (npair > 256) return pqph_fail(ctx, PQPH_INVALID_ARG, "npair must be in [1, 256]");
    const pqph_status res = pq_energy_grad(ctx, npair, h, eri, t, opts, energy, gamma, Gamma, nullptr, info);
    if (res != PQPH_OK && res != PQPH_NOT_CONVERGED) return res;
    launch_add_reference_occupation(ctx->stream, gamma, npair);
    PQPH_HIP(ctx, hipGetLastError());
    if (noons) {
        const int n = 2 * npair;
        if ((st = pqph_ensure_host(ctx, (size_t)n * n))) return st;
        PQPH_HIP(ctx, hipMemcpyAsync(ctx->host, gamma, (size_t)n * n * sizeof(double),
                                     hipMemcpyDeviceToHost, ctx->stream));
        PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
        std::vector<double> A((size_t)n * n), w;
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q)
                A[(size_t)p * n + q] = 0.5 * (ctx->host[(size_t)p * n + q] + ctx->host[(size_t)q * n + p]);
        symmetric_eigenvalues(A, n, w);
        std::copy(w.begin(), w.end(), noons);
    } else {
        PQPH_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    return res;
}


}  // extern "C"
