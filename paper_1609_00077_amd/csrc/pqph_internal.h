// Internal declarations shared by the translation units of libpqph.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pqph.h"

struct pqph_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // one growable device workspace, carved per call
    double* ws = nullptr;
    size_t ws_bytes = 0;
    // persistent solver buffers (separate so residual calls can reuse ws)
    double* sv = nullptr;
    size_t sv_bytes = 0;
    // pinned host staging for small reductions
    double* host = nullptr;
    size_t host_n = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // per-kernel timing of one residual (diagnostic entry point only)
    hipEvent_t prof[24] = {};
    int prof_n = 0;       // events recorded so far
    bool profiling = false;
    // autotuned kernel variants per npair (two-spectator contraction):
    // 1 = K-chunked staging, 2 = vertex resident in LDS; 0 = not tuned
    int s2_variant[257] = {};
    // one-spectator GEMM sides per npair: 1 = formed while staging (fused),
    // 2 = materialised X, Y read by the GEMM, 3 = fused with the staging
    // software-pipelined (npair <= 128); 0 = not tuned
    int s1_mode[257] = {};
    // PQ intermediates per npair: 3 (0 = default) = the exact projection; 2 =
    // the two-pair-intermediate model without the doubly-mixed two-spectator
    // terms (the only ones whose contraction needs a three-label intermediate)
    int pq_int[257] = {};
    // streams and events of batched solves (default priority), created on first use
    std::vector<hipStream_t> bstreams;
    std::vector<hipEvent_t> bevents;
    hipEvent_t fork = nullptr;
    // side streams (default priority) and fork/join events of one residual:
    // its independent branches run concurrently with the main chain
    hipStream_t side[2] = {};
    hipEvent_t sev[4] = {};
    // the residual captured as HIP graphs, each with what it was captured
    // for (a few are kept: callers alternate between buffer sets)
    struct ResidualGraph {
        hipGraphExec_t exec = nullptr;
        int N = 0, s1 = 0, s2 = 0, li = 0;
        const double *h = nullptr, *eri = nullptr, *t = nullptr;
        double *r = nullptr, *ws = nullptr;
        const int* gate = nullptr;
        bool vertices = true;
        unsigned long long used = 0;     // last use, for replacement
    };
    static constexpr int kResidualGraphs = 4;
    hipStream_t cap = nullptr;
    ResidualGraph rgraph[kResidualGraphs];
    unsigned long long rgraph_clock = 0;
    // PQ amplitude solves: 0 = device-driven iterations enqueued ahead of
    // the host, 1 = host-driven (default; one host synchronisation per iteration)
    int solve_mode = 1;
    // while a device-driven solve runs: its active flag, the gate the
    // residual kernels obey (NULL otherwise)
    const int* solve_gate = nullptr;
    hipEvent_t dsev[2] = {};
    // batched solves: 0 = device-resident iterations captured in a HIP graph,
    // 1 = host-driven lockstep (three host synchronisations per iteration)
    int batch_mode = 0;
    // PH term tables in device memory, read from file on first PH call
    struct PhTables* ph = nullptr;
    // device address of this GPU's static scratch array (allocation-free
    // residual), looked up once per device at pqph_create
    double* scratch = nullptr;
};

// PH (k = 3) path: term tables, residual, energy, denominators on stream s
pqph_status ph_tables_load(pqph_ctx* ctx);
void ph_tables_free(pqph_ctx* ctx);
// ws: ph_residual_ws_doubles (the work units' partial sums)
pqph_status ph_residual_ws_doubles(pqph_ctx* ctx, int N, size_t* out);
// spin_sym: t is spin-symmetric (t[partner] = sign t under the alpha/beta
// exchange): only the orbit representatives are evaluated, the partners are
// copied with their sign
pqph_status ph_residual_dev(pqph_ctx* ctx, hipStream_t s, int N, const double* h,
                            const double* eri, const double* t, double* r, double* ws,
                            bool spin_sym = false);
size_t ph_energy_ws_doubles();
pqph_status ph_energy_dev(pqph_ctx* ctx, hipStream_t s, int N, const double* h, const double* eri,
                          const double* t, double* out, double* ws);
pqph_status ph_denominators_dev(pqph_ctx* ctx, hipStream_t s, int N, const double* h, double shift,
                                double* D);

// variant of the two-spectator contraction for this npair (tuned or default)
int pq_s2_variant(const pqph_ctx* ctx, int npair);
// labels of the largest PQ intermediate for this npair: 3 (exact) or 2
int pq_intermediates(const pqph_ctx* ctx, int npair);
// one-spectator side formation for this npair (tuned, forced, or by size)
int pq_s1_mode(const pqph_ctx* ctx, int npair);

// records an event after a launch when the context is profiling
void pqph_mark(pqph_ctx* ctx);

// error helpers -----------------------------------------------------------
pqph_status pqph_fail(pqph_ctx* ctx, pqph_status st, const std::string& msg);
#define PQPH_HIP(ctx, call)                                                       \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess)                                                     \
            return pqph_fail(ctx, PQPH_DEVICE, std::string(#call) + ": " +        \
                                                   hipGetErrorString(e_));        \
    } while (0)

pqph_status pqph_ensure_ws(pqph_ctx* ctx, size_t bytes);
pqph_status pqph_ensure_sv(pqph_ctx* ctx, size_t bytes);
pqph_status pqph_ensure_host(pqph_ctx* ctx, size_t n);
// side streams and events of the residual's concurrent branches (created on first use)
pqph_status pqph_ensure_side(pqph_ctx* ctx);

// output pair index ip = Q(Q-1)/2 + P (P < Q) -> (P, Q)
__device__ inline void decode_pair(long ip, int& P, int& Q) {
    int q = (int)((1.0 + sqrt(1.0 + 8.0 * (double)ip)) * 0.5);
    while ((long)q * (q - 1) / 2 > ip) --q;
    while ((long)(q + 1) * q / 2 <= ip) ++q;
    Q = q;
    P = (int)(ip - (long)q * (q - 1) / 2);
}

// no- and one-spectator terms of the two-pair outputs (pq_lane.hip): chunk
// partial sums part[chunk][pq]; h2K, SK k-major over output pairs
void launch_r2_lane(hipStream_t s, int npair, const double* t, const double* h1, const double* h2K,
                    const double* SK, double* part, const int* gate);

// one-spectator terms of the one-pair outputs (pq_lane.hip): chunk sums
// part[chunk][k][P]; t2 the mirrored [29][N][N], h2 [key][N][N]
void launch_r1_lane(hipStream_t s, int npair, const double* t, const double* t2, const double* h1,
                    const double* h2, double* part, const int* gate);
int r1_lane_chunks();
// adjoint of the two-pair local terms (pq_lane_adj.hip): Sbar_p (p-major) and
// h2bar(P,Q) written by their owning lane, the rest added atomically
void launch_r2_lane_adj(hipStream_t s, int npair, const double* t, const double* h1, const double* h2K,
                        const double* SK, const double* lam, double* tb1, double* tb2, double* hb1,
                        double* hb2, double* SbK);
// adjoint of those terms, lam-weighted, into the amplitude and vertex adjoints
void launch_r1_lane_adj(hipStream_t s, int npair, const double* t, const double* t2, const double* h1,
                        const double* h2, const double* lam, double* tb1, double* tb2, double* hb1,
                        double* hb2);

// PQ residual pieces (pq_residual.hip) --------------------------------------
size_t pq_ws_doubles(int npair);
// residual into r on stream s using workspace ws (already large enough); no host sync
// gate: device flag; when it reads 0 every kernel returns at once (NULL: always run)
// fork: 1 = run the independent branches on the context's side streams, 0 =
// serially on s, -1 = fork when s is the context's stream, no gate is given
// and no per-kernel timing is taken
// vertices: false when ws already holds the bare vertices of h and eri
// (pq_vertices_ws, nothing written over them since): they depend on the
// integrals only, so a solve forms them once
// vtx: a private vertex block (pq_vertices_into) read instead of ws's vertices
pqph_status pq_residual_ws(pqph_ctx* ctx, hipStream_t s, int npair, const double* h,
                           const double* eri, const double* t, double* r, double* ws,
                           const int* gate = nullptr, int fork = -1, bool vertices = true,
                           const double* vtx = nullptr);
// the bare vertices of h and eri into ws (where pq_residual_ws reads them)
pqph_status pq_vertices_ws(pqph_ctx* ctx, hipStream_t s, int npair, const double* h,
                           const double* eri, double* ws);
// the same into a private block of pq_vertex_doubles(npair) doubles (batched
// chains that share a workspace keep their vertices apart)
size_t pq_vertex_doubles(int npair);
pqph_status pq_vertices_into(pqph_ctx* ctx, hipStream_t s, int npair, const double* h,
                             const double* eri, double* vtx);
// one-time kernel attributes of the residual (outside any stream capture)
pqph_status pq_residual_prepare(pqph_ctx* ctx);
// the residual on the context's stream replayed from a HIP graph captured for
// these arguments and kernel choices (captured again when they change)
// gate, vertices: as for pq_residual_ws (part of what the graph is captured for)
pqph_status pq_residual_graph(pqph_ctx* ctx, int npair, const double* h, const double* eri,
                              const double* t, double* r, double* ws, const int* gate = nullptr,
                              bool vertices = true);
// energy: writes one double to dst (device) on stream s, no sync
pqph_status pq_energy_ws(pqph_ctx* ctx, hipStream_t s, int npair, const double* h,
                         const double* eri, const double* t, double* dst, double* ws);
pqph_status pq_denominators_dev(pqph_ctx* ctx, hipStream_t s, int npair, const double* h,
                                double shift, double* D);

// adjoint (pq_residual.hip): tbar = lam . dR/dt + ew dE/dt and, when hbar and
// eribar are given, the same pulled back to f and the packed integrals.
// aws: pq_adj_doubles(npair) doubles of adjoint workspace.  fwd_ready: ws and
// aws still hold the forward intermediates of a previous call with the same
// h, eri and t (nothing else wrote them since), so they are not recomputed.
size_t pq_adj_doubles(int npair);
pqph_status pq_vjp_ws(pqph_ctx* ctx, hipStream_t s, int npair, const double* h, const double* eri,
                      const double* t, const double* lam, double ew, double* tbar, double* hbar,
                      double* eribar, double* ws, double* aws, bool fwd_ready = false);

// streaming kernels of the solver (solver_kernels.hip) ---------------------
int stream_blocks(size_t n);
// (m+1)x(m+1) DIIS system from the Gram matrix B (row stride 16); false if singular
bool diis_solve(const std::vector<double>& B, int m, std::vector<double>& c);
// out[0] = ||r||^2 (fixed-order reduction over nblk partials); out may be the
// device address of pinned host memory (launch_step's too)
void launch_norm2(hipStream_t s, const double* r, size_t n, double* part, int nblk, double* out);
// e = -r/D, tn = t + e
void launch_jacobi(hipStream_t s, const double* t, const double* r, const double* D, size_t n,
                   double* tn, double* e);
// out[j] = eh[j] . enew for j < m (part holds m*nblk partials)
void launch_gram(hipStream_t s, const double* eh, int m, const double* enew, size_t n, double* part,
                 int nblk, double* out);
// out[0] = min |a_i|
void launch_absmin(hipStream_t s, const double* a, size_t n, double* part, int nblk, double* out);
// one Jacobi/DIIS step: tn = t - r/D, eh[slot] = -r/D; out[0] = ||r||^2 and
// out[1 + j] = eh[j] . eh[slot] for j < m (m <= 16; part holds (m+1)*nblk)
void launch_step(hipStream_t s, const double* t, const double* r, const double* D, size_t n, double* tn,
                 double* eh, int m, int slot, double* part, int nblk, double* out);
// t = sum_j c[j] th[j]
void launch_combine(hipStream_t s, const double* th, const double* c, int m, size_t n, double* t);
// the same with c on the host (m <= 16, passed as a kernel argument)
void launch_combine_host(hipStream_t s, const double* th, const double* c, int m, size_t n, double* t);
// Pulay's bordered DIIS system [B/scale -1; -1 0] [c; l] = [0; -1] for k
// stored vectors (B: Gram matrix, row stride 16; scale: its largest
// diagonal), Gauss-Jordan elimination with partial pivoting; false when B is
// zero, the system is (near) singular or a coefficient is not finite (the
// caller then takes the plain Jacobi step).  Called by every thread of one
// workgroup of at least 32 threads: thread i keeps row i in registers and
// eliminates it with the same operations, in the same order, as the host
// solve (diis_solve); the pivot column and row pass through LDS.  On success
// thread 0 writes coef[0..16) (zero beyond k); every thread returns the same
// flag.
__device__ inline bool diis_coefficients(const double* B, int k, double* coef) {
    constexpr int W = 18;                       // k <= 16: n = k + 1 <= 17 rows, n + 1 columns
    __shared__ double colv[W], prow[W], crow[W], cv[16];
    const int n = k + 1, tid = threadIdx.x;
    double scale = 0.0;
    for (int i = 0; i < k; ++i) scale = fmax(scale, fabs(B[i * 16 + i]));
    if (!(scale > 0.0)) return false;
    double a[W], p[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        double v = 0.0;
        if (tid < n && j <= n) {
            if (j == n) v = (tid == k) ? -1.0 : 0.0;
            else if (tid < k && j < k) v = B[tid * 16 + j] / scale;
            else if (tid == k && j == k) v = 0.0;
            else v = -1.0;
        }
        a[j] = v;
    }
    for (int col = 0; col < n; ++col) {
        double acol = 0.0;
#pragma unroll
        for (int j = 0; j < W; ++j)
            if (j == col) acol = a[j];
        if (tid < n) colv[tid] = acol;
        __syncthreads();
        int piv = col;
        double pv = fabs(colv[col]);
#pragma unroll
        for (int i = 1; i < W - 1; ++i) {
            if (i > col && i < n) {
                const double x = fabs(colv[i]);
                if (x > pv) {
                    pv = x;
                    piv = i;
                }
            }
        }
        if (pv < 1e-300) return false;          // same values in every thread
        if (tid == piv) {
#pragma unroll
            for (int j = 0; j < W; ++j) prow[j] = a[j];
        }
        if (tid == col && piv != col) {
#pragma unroll
            for (int j = 0; j < W; ++j) crow[j] = a[j];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < W; ++j) p[j] = prow[j];
        if (tid == col) {
#pragma unroll
            for (int j = 0; j < W; ++j) a[j] = p[j];
        } else if (tid == piv) {
#pragma unroll
            for (int j = 0; j < W; ++j) a[j] = crow[j];
        }
        if (tid < n && tid != col) {
            double ac = 0.0, pc = 0.0;
#pragma unroll
            for (int j = 0; j < W; ++j)
                if (j == col) {
                    ac = a[j];
                    pc = p[j];
                }
            const double fct = ac / pc;
#pragma unroll
            for (int j = 0; j < W; ++j)
                if (j >= col && j <= n) a[j] -= fct * p[j];
        }
        __syncthreads();                        // prow, crow and colv are rewritten next
    }
    if (tid < k) {
        double rhs = 0.0, diag = 0.0;
#pragma unroll
        for (int j = 0; j < W; ++j) {
            if (j == n) rhs = a[j];
            if (j == tid) diag = a[j];
        }
        cv[tid] = rhs / diag;
    }
    __syncthreads();
    bool ok = true;
    for (int i = 0; i < k; ++i) ok = ok && isfinite(cv[i]);
    if (ok && tid == 0)
        for (int i = 0; i < 16; ++i) coef[i] = i < k ? cv[i] : 0.0;
    return ok;
}

// Device-driven Jacobi/DIIS solve (one system): the norm test, the
// convergence / stall / divergence decisions, the Gram row and the DIIS
// coefficients are all taken on the device, so the host can enqueue
// iterations ahead and only follow the state.  SolveHead opens the
// device-resident state; the host copies it back.
struct SolveHead {
    int active;     // 1 while iterating, 0 once a decision ended the solve
    int iters;      // residual norms tested so far
    int next;       // history slot of the next Jacobi iterate
    int stored;     // history slots written (at most the DIIS dimension)
    int use;        // 1: the update extrapolates with the DIIS coefficients
    int last;       // slot of the latest Jacobi iterate
    int status;     // PQPH_* once inactive
    int stalled;    // ended by the stall test
    int improved;   // the last tested norm was below every earlier one
    int pad;
    double rn, rmin;
};
constexpr int kSolveRing = 257;   // smallest-norm history: stall_window <= kSolveRing - 1
struct DevSolveOpts {
    int max_iter, m, diis_on, diis_start, stall_window;
    double tol, diverge_factor;
};
// doubles of device memory the state takes (SolveHead first)
size_t dev_solve_doubles();
void launch_dsolve_init(hipStream_t s, double* state);
// when active: e = -r/D into eh[next], x + e into th[next]; block partials of
// ||r||^2 (row 0) and of e . eh[j] (rows 1..m) into part ((m+1) nblk doubles)
void launch_dsolve_step(hipStream_t s, const double* state, const double* x, const double* r,
                        const double* D, size_t n, double* th, double* eh, int m, double* part,
                        int nblk);
// when active: sums the partials, tests the norm, updates the Gram matrix and
// solves for the DIIS coefficients (one workgroup)
void launch_dsolve_decide(hipStream_t s, double* state, const double* part, int nblk,
                          const DevSolveOpts& o);
// when active: x = sum_j c_j th[j] (DIIS) or th[last]; best (may be NULL)
// takes x first when the last norm was the smallest so far.  Always: the
// head is copied to mirror (device address of pinned host memory; may be NULL)
void launch_dsolve_update(hipStream_t s, const double* state, const double* th, size_t n,
                          double* x, double* best, SolveHead* mirror);

// f = diag(-1 occupied, 0 virtual): through the denominator kernels, the slot ranks
void launch_rank_fock(hipStream_t s, double* f, int npair);
// r[i] = 0 where rank[i] > max_rank
void launch_rank_mask(hipStream_t s, double* r, const double* rank, int max_rank, size_t n);
// out = a x + b y (y may be null; with D, y is divided elementwise by D)
void launch_axpby(hipStream_t s, double* out, double a, const double* x, double b, const double* y,
                  const double* D, size_t n);
// y -= sum_j c[j] V[j] (c on the device)
void launch_sub_combine(hipStream_t s, double* y, const double* V, const double* c, int m, size_t n);
// gamma (2N x 2N) += 2 on the occupied diagonal (p < npair)
void launch_add_reference_occupation(hipStream_t s, double* gamma, int npair);
// closed-shell spin adaptation: reduced length (one value per alpha/beta
// exchange orbit of the packed slots, label sets of up to k pairs), the
// projection v -> x (mode 0: sqrt-weighted, symmetrising; mode 1: the
// representative's value) and its inverse x -> v
size_t spin_len(int npair, int k);
void launch_spin_pack(hipStream_t s, const double* v, double* x, int npair, int k, int mode);
void launch_spin_unpack(hipStream_t s, const double* x, double* v, int npair, int k);
// per pattern m of a label set of n pairs: its orbit representative rep[m]
// and t[m] = sgn[m] * t[rep[m]] (rep[m] = m, sgn = 1 for a representative)
void spin_pattern_reps(int n, int* rep, int* sgn);
