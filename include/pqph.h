/*
 * pqph.h -- C ABI of the MI355X (gfx950) library for the perfect quadruples
 * (PQ) and perfect hextuples (PH) pair-truncated coupled-cluster models
 * (Lehtola, Parkhill, Head-Gordon, arXiv:1609.00077).
 *
 * Everything is FP64.  Matrices are row-major.  Unless marked "host", every
 * pointer is a device pointer, and all work is issued on the stream given to
 * pqph_create; calls that return results to host memory synchronise that
 * stream.  The caller owns every array.  The context owns only its workspace,
 * which it grows on demand and frees in pqph_destroy.  Errors are returned
 * as status codes and never abort; pqph_last_error gives the message of the
 * last failure on the context.  Device errors surface at the next call that
 * synchronises.  Use one context per stream and do not call one context from
 * two threads at once.
 *
 * ---------------------------------------------------------------- orbitals
 * The active space has N pairs (Sec. II, Fig. 1).  Pair P is the orbital
 * quartet of the occupied orbital o_P (HOMO-P) and the virtual v_P (LUMO+P),
 * both spins.  Spatial orbital index P is o_P and N+P is v_P.
 *
 * ----------------------------------------------------- amplitude layout (t, r)
 * Each pair carries four excitation generators, by bit: 0 = a(o_P alpha),
 * 1 = a(o_P beta), 2 = a+(v_P alpha), 3 = a+(v_P beta).  A local pattern e in
 * 1..15 is a set of these bits; g_P^e is the product of its generators in
 * ascending bit order; its charge per spin is particles minus holes.  The
 * excitation on labels P0 < P1 < ... with patterns (e0, e1, ...) (each
 * nonempty, total charge zero per spin) is the operator g_P0^e0 g_P1^e1 ...,
 * and T = sum over slots of t(slot) times that operator.  The model keeps the
 * excitations on at most k pairs (Sec. II: k = 2 for PQ, 3 for PH; Eq. (1)
 * lists the eight opposite-spin doubles subtensors of PQ).  Packed vector,
 * class-major, unique excitations only (3, 29 and 303 per label set):
 *     [ 3 x N ][ 29 x C(N,2) ][ 303 x C(N,3), PH only ]
 * Pattern tuples of one label-set size run lexicographically; pairs P<Q are
 * indexed Q(Q-1)/2+P and triples P<Q<R by R(R-1)(R-2)/6+Q(Q-1)/2+P.  The
 * residual r has the same layout: r(slot) is the coefficient of the slot's
 * operator in e^{-T} H_N e^{T}, i.e. <g^mu 0| e^{-T} H_N e^{T} |0>, not divided
 * by any denominator.
 *
 * ---------------------------------------------------- integral layout (eri)
 * Chemists' (pq|rs), real, 8-fold symmetric, each unique integral stored
 * once, grouped by its label set; only label sets of at most k pairs are
 * stored (Table I caption: PQ keeps rank-1 and rank-2 integral subtensors,
 * PH up to rank 3).  Within a set with ascending labels, local orbital
 * 2*role+type (type 0 = o, 1 = v) is numbered; the stored quadruples are
 * p>=q, r>=s, pq>=rs with pq = p(p+1)/2+q, in lexicographic (pq, rs) order,
 * keeping those whose orbitals cover every label of the set (6, 43, 84):
 *     [ 6 x N ][ 43 x C(N,2) ][ 84 x C(N,3), PH only ]
 *
 * ------------------------------------------------------ Hamiltonian (h)
 * h is the 2N x 2N Fock matrix f in the paired MO order, whole (the paper
 * truncates the two-electron integrals, not f; Sec. III takes f from the SCF).
 * The model Hamiltonian is H_N = sum_pq f_pq {p+ q} + 1/4 sum <pq||rs> {p+ q+ s r}
 * with <pq||rs> built from the stored integrals; f is read as a general matrix.
 *
 * Energies returned are correlation energies E_c = <0|H_N e^T|0> (Eqs. (2)-(3)
 * give its doubles part in subtensor form), not total energies.
 */
#ifndef PQPH_H
#define PQPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int pqph_status;
#define PQPH_OK 0
#define PQPH_INVALID_ARG (-1)    /* bad size, null pointer, unsupported option */
#define PQPH_DEVICE (-2)         /* a HIP call failed                          */
#define PQPH_OOM (-3)            /* device workspace could not be allocated    */
#define PQPH_NONFINITE (-4)      /* NaN/Inf in the inputs or the iterates      */
#define PQPH_NOT_CONVERGED (-5)  /* max_iter reached                           */
#define PQPH_DIVERGED (-6)       /* residual norm grew past the allowed bound  */

typedef struct pqph_ctx pqph_ctx;

/* Solver options (host struct).  Jacobi updates t <- t - r/D with the
 * orbital-energy denominators D = sum f_aa - sum f_ii over the particles and
 * holes of each excitation plus level_shift (Table IV: denominator
 * application), accelerated by DIIS (Sec. III) on the last diis_dim iterates
 * once iteration diis_start is reached (0 disables DIIS).  Convergence: 2-norm
 * of r over the packed unique slots <= tol.  Divergence: the norm exceeds
 * diverge_factor times the smallest norm seen, or 1e3 in absolute value.
 * With the environment variable PQPH_VERBOSE set to a nonzero value, every
 * solve prints one line per iteration (residual norm, elapsed time) to
 * stderr. */
typedef struct {
    int max_iter;          /* default 200                                */
    double tol;            /* default 1e-8                               */
    int diis_dim;          /* default 8, at most 16                      */
    int diis_start;        /* default 2                                  */
    double level_shift;    /* default 0                                  */
    double diverge_factor; /* default 1e4                                */
    int stall_window;      /* default 40: stop (NOT_CONVERGED) once the best
                              ||R|| has not halved over this many
                              iterations; 0 = never                      */
    int max_rank;          /* default 0 = every excitation of the model; r in
                              1..6 keeps only the excitations of at most r
                              holes (Sec. V: PH restricted to singles and
                              doubles, r = 2, or up to quadruples, r = 4):
                              the others have t = 0 and their residuals are
                              not solved for (left out of the norm and DIIS).
                              Not supported by pq_solve_batched.          */
    int solver;            /* default 0 = Jacobi/DIIS as above; 1 = inexact
                              Newton-Krylov (GMRES on J dx = -R,
                              preconditioned by D, J v by central
                              differences of R, backtracking on ||R||)
                              from t_inout; 2 = Jacobi/DIIS, then
                              Newton-Krylov from its iterate of smallest
                              ||R|| when it stalls, diverges or reaches
                              max_iter (Sec. IV.B: the iterations fail at
                              strong correlation).  The iteration count
                              reported is then residual evaluations.  In
                              pq_energy_grad it applies to the amplitude
                              solve; lambda uses Jacobi/DIIS.              */
    int spin_adapted;      /* default 0; 1 = closed-shell spin adaptation
                              (Sec. V: spin summation for closed shells):
                              the solver keeps one value per orbit of the
                              alpha/beta exchange of the packed slots
                              (t[partner] = sign * t, partner = the same
                              label set with alpha and beta exchanged on
                              every pair, sign = the reordering of the
                              exchanged generators), 2N + 16 C(N,2)
                              (+ 155 C(N,3) for PH) values instead of
                              3N + 29 C(N,2) (+ 303 C(N,3)): every solver
                              vector and DIIS history shrinks to about
                              half.  The residual runs on full packed
                              vectors unpacked from the reduced one; the PH
                              residual then evaluates only the orbit
                              representatives and copies their partners
                              with the sign.  Exact for the spin-free
                              integrals of this library: the solution is
                              the one of the full space; start amplitudes
                              are first projected onto the symmetric
                              subspace.  Reported norms are those of the
                              symmetrised full residual.  Not supported by
                              pq_solve_batched.                           */
} pqph_solve_opts;

/* Per-solve report (host struct). */
typedef struct {
    int iterations;        /* residual evaluations performed             */
    double rnorm;          /* final residual 2-norm                      */
    int status;            /* same code the call returned                */
    double solve_ms;       /* wall time of the solve on the stream       */
} pqph_solve_info;

/* Fill *opts with the defaults above. */
void pqph_default_opts(pqph_solve_opts* opts);

/* Create a context bound to a device and a HIP stream (hipStream_t passed as
 * void*; NULL means the default stream).  The context allocates nothing
 * until first use. */
pqph_status pqph_create(pqph_ctx** ctx, int device, void* hip_stream);
void pqph_destroy(pqph_ctx* ctx);
const char* pqph_last_error(const pqph_ctx* ctx);

/* Element counts of the packed layouts (host; no context needed). */
size_t pq_amp_len(int npair);
size_t ph_amp_len(int npair);
size_t pq_eri_len(int npair);
size_t ph_eri_len(int npair);

/* Integral transformation into pair blocks (Sec. III, RI/CD paragraph: the
 * two-electron integrals are formed from three-index factors, picking only
 * the elements needed).  For a zero-differential-overlap site Hamiltonian of
 * n = 2*npair sites with site-basis Fock matrix F (n x n), site interaction
 * matrix V (n x n) and paired MO coefficients C (n x n, columns
 * [o_0..o_{N-1}, v_0..v_{N-1}]):
 *     f   = C^T F C                                    (n x n, row-major)
 *     eri = packed (pq|rs) = sum_ij C_ip C_iq V_ij C_jr C_js
 *           for the label sets of at most k pairs (k = 2 or 3).
 * f_out holds n*n doubles, eri_out pq_eri_len / ph_eri_len doubles. */
pqph_status pqph_integrals(pqph_ctx* ctx, int npair, int k, const double* F,
                           const double* V, const double* C, double* f_out,
                           double* eri_out);

/* PQ residual r(t) = <mu| e^{-T} H_N e^{T} |0> for every packed slot (Sec. II,
 * Eq. (1) decomposition with k = 2).  t and r: pq_amp_len(npair) doubles;
 * eri: pq_eri_len(npair); h: (2N)^2.  Stream-ordered, no host sync.
 * npair in [1, 256]. */
pqph_status pq_residual(pqph_ctx* ctx, int npair, const double* h,
                        const double* eri, const double* t, double* r);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * residual as pq_residual, computed by the same kernels serially on the
 * context's stream, with its workspace taken from a static device array of
 * 48 MiB that each GPU holds from library load until the process ends (its
 * device address is looked up once per device in pqph_create).  No device
 * memory is allocated or freed and the stream is not synchronised; no
 * memset is issued either (every workspace value is written before it is
 * read).  The caller passes inputs and outputs as for pq_residual.  npair in
 * [1, 32]; a larger npair is PQPH_INVALID_ARG.  Every call on one GPU shares
 * that GPU's array and it keeps the last call's contents: calls that overlap
 * on one GPU (other streams, other contexts, other threads) race and must be
 * serialised by the caller. */
pqph_status pq_residual_noalloc(pqph_ctx* ctx, int npair, const double* h,
                                const double* eri, const double* t, double* r);

/* PQ correlation energy at amplitudes t (Eqs. (2)-(3)); energy is a host
 * pointer; the call synchronises the stream. */
pqph_status pq_energy(pqph_ctx* ctx, int npair, const double* h,
                      const double* eri, const double* t, double* energy);

/* PQ amplitude solve: Jacobi + DIIS from t_inout (zeros for the usual
 * start) until the residual norm is at most opts->tol.  On return t_inout
 * holds the last iterate, *energy (host) its correlation energy and *info
 * (host, may be NULL) the report.  opts may be NULL for the defaults. */
pqph_status pq_solve(pqph_ctx* ctx, int npair, const double* h,
                     const double* eri, const pqph_solve_opts* opts,
                     double* t_inout, double* energy, pqph_solve_info* info);

/* PH residual r(t) = <mu| e^{-T} H_N e^{T} |0> for every packed slot of the
 * three-pair model (Sec. II with k = 3: amplitudes and integrals on at most
 * three pairs).  t and r: ph_amp_len(npair) doubles; eri: ph_eri_len(npair);
 * h: (2N)^2.  Stream-ordered, no host sync after the first call.  The terms
 * are the derived PH term tables, read on the context's first PH call from
 * ph_terms.bin beside the library (or the file named by the environment
 * variable PQPH_PH_TERMS) and kept in device memory until pqph_destroy; a
 * missing or damaged file is PQPH_INVALID_ARG.  The kernels interpret the
 * tables in balanced work units (a host schedule built once per npair), so
 * the cost grows as C(N,3) N^3 times the term count: meant for small active
 * spaces (about 0.16 s at 8 pairs, 10 s at 16, 37 s at 20).  The context's workspace
 * grows to hold one partial sum per (label set, work unit): at most 60000
 * units per block size, so up to 60000 C(N,3) doubles.  npair in [1, 256];
 * a workspace that cannot be allocated is PQPH_OOM. */
pqph_status ph_residual(pqph_ctx* ctx, int npair, const double* h,
                        const double* eri, const double* t, double* r);

/* PH correlation energy <0| H_N e^T |0> at amplitudes t (Eqs. (2)-(3), with
 * the doubles and integrals of up to three pairs); energy is a host pointer;
 * the call synchronises the stream. */
pqph_status ph_energy(pqph_ctx* ctx, int npair, const double* h,
                      const double* eri, const double* t, double* energy);

/* PH amplitude solve: pq_solve's Jacobi + DIIS loop on ph_residual, with the
 * same options, outputs and status codes; t_inout holds ph_amp_len doubles. */
pqph_status ph_solve(pqph_ctx* ctx, int npair, const double* h,
                     const double* eri, const pqph_solve_opts* opts,
                     double* t_inout, double* energy, pqph_solve_info* info);

/* Diagnostic (per-phase tracing): one pq_residual with a HIP event recorded on
 * the context's stream after every kernel; phase_ms (host, nphase entries)
 * receives the elapsed time of each kernel in launch order and *nphase_out
 * their number (16 for npair >= 3: vertex1, vertex2, unpack_t2, spec_w,
 * spec_lam, dress, spec_xy (the materialised one-spectator sides; empty
 * unless that mode is in effect), gemm_s1, r2s2, r2c, spec_r1, r1s2,
 * r1s2_close, r1, r1c, final; 13 for npair = 2, without spec_r1, r1s2 and
 * r1s2_close; 4 for npair = 1: vertex1, r1, r1c, final).  The kernels run
 * serially on the context's stream here.  Synchronises the stream.  Fails
 * with INVALID_ARG if nphase is too small. */
pqph_status pq_residual_profile(pqph_ctx* ctx, int npair, const double* h,
                                const double* eri, const double* t, double* r,
                                double* phase_ms, int nphase, int* nphase_out);
/* Name of phase i of pq_residual_profile for npair >= 3 ("" if out of range;
 * the string is static). */
const char* pq_residual_phase_name(int i);

/* Autotuner (the analogue of the paper's benchmark-time choice between loop
 * and BLAS kernels, Sec. III): time the variants of the two-spectator
 * contraction for this npair on the given inputs (three residuals each, after
 * a warm-up; r receives the last residual) and keep the fastest for every
 * later call on this context.  *choice (host, may be NULL) = 1 (K-chunked
 * staging of the vertex) or 2 (vertex resident in LDS, npair <= 96).  The
 * one-spectator mode (pqph_set_s1_mode) is tuned jointly, over every pair of
 * choices; a non-default pair must be 3 % faster to be kept, so near-ties
 * keep the defaults.  Synchronises the stream.  Without tuning, variant 1 and the
 * size-based mode are used. */
pqph_status pqph_autotune(pqph_ctx* ctx, int npair, const double* h,
                          const double* eri, const double* t, double* r,
                          int* choice);

/* Force the two-spectator variant for npair on this context (0 = default,
 * 1, or 2 when npair <= 96); INVALID_ARG otherwise.  For tests and tuning. */
pqph_status pqph_set_variant(pqph_ctx* ctx, int npair, int variant);

/* Force how the one-spectator GEMM (Sec. II one-spectator terms, S_p(P,Q) =
 * sum_A X_x(P,A) Y_y(Q,A)) obtains its sides for npair on this context:
 * 0 = default (4, or as tuned by pqph_autotune),
 * 1 = each side formed
 * from its factors while staging, 2 = X and Y materialised first and read by
 * the GEMM, 3 = as 1 with the next chunk's loads overlapping the current
 * chunk's matrix-core steps (npair <= 128), 4 = as 2 with the next chunk's
 * loads overlapping the current chunk's matrix-core steps (bitwise the same
 * as 2).  All give the same residual up to rounding order.
 * INVALID_ARG for another mode.  For tests and tuning. */
pqph_status pqph_set_s1_mode(pqph_ctx* ctx, int npair, int mode);

/* The PQ model variant with two-pair intermediates (Sec. III: the paper
 * builds PQ with intermediates of up to three pairs and notes that truncating
 * them to two pairs, O(N^3), costs accuracy).  labels = 3 (the default) is
 * the exact projection; labels = 2 leaves out the two-spectator terms of the
 * two-pair outputs in which both spectators are linked to both output pairs
 * (the doubly-mixed terms), the only PQ terms whose contraction needs an
 * intermediate over three labels.  Applies to pq_residual, the solves, the
 * batched solve, pq_vjp and pq_energy_grad for npair on this context.
 * INVALID_ARG for other values. */
pqph_status pqph_set_pq_intermediates(pqph_ctx* ctx, int npair, int labels);

/* The choices in effect for npair on this context (host outputs, each may be
 * NULL): the two-spectator variant (1 or 2) and the one-spectator mode
 * (1-4). */
pqph_status pqph_tuning(pqph_ctx* ctx, int npair, int* s2_variant, int* s1_mode);

/* Diagnostic: the device's measured ceilings for roofline fractions, host
 * out[4] = { STREAM copy GB/s, STREAM triad GB/s (1 GiB arrays, counting the
 * bytes read and written), FP64 vector FMA TFLOP/s, FP64 matrix-core
 * (v_mfma_f64_16x16x4f64) TFLOP/s }.  Uses 3 GiB of the context's workspace;
 * synchronises the stream. */
pqph_status pqph_measure_ceilings(pqph_ctx* ctx, double* out);

/* Batched PQ solves (many Hamiltonians of uneven pair counts, solved
 * together; each chain runs its own Jacobi + DIIS exactly as pq_solve and
 * converges on its own).  Chain c has npair[c] pairs (host array) and reads
 * its Fock matrix at h + h_off[c], its packed integrals at eri + eri_off[c]
 * and its amplitudes at t_inout + t_off[c] (offsets in doubles, host arrays;
 * the caller packs the chains into three device buffers).  energies (host,
 * nbatch) receives each chain's correlation energy and infos (host, may be
 * NULL) each chain's report.  Returns OK if every chain converged, otherwise
 * the first failing chain's status; one bad chain does not stop the others.
 * Device memory: the residual workspace of the largest chain per stream (up
 * to 8 streams) plus, per chain, (4 + 2*diis_dim) amplitude vectors, the
 * chain's bare vertices (formed once per batch: 308 N^2 + 308 C(N,2) + 26 N
 * doubles, about 15 MB at N = 65) and about 4.3 KB of solver state.  By default the iterations run entirely
 * on the device: one iteration of the whole batch is captured into a HIP graph
 * and replayed, and the host only polls the chains' finished flags every few
 * replays (opts->stall_window must be below 257 here; opts->max_rank must
 * be 0).  With opts->solver = 2, every chain that ends NOT_CONVERGED or
 * DIVERGED is solved again afterwards, alone, by pq_solve with solver 2 from
 * zero amplitudes (its energy, report and amplitudes replaced); solver 1 is
 * not accepted here.  The t_inout values are
 * the starting amplitudes; iterates of converged chains stop changing.
 * Enqueued on the context's stream order (internal streams wait for it, and
 * it waits for them); the call returns after the results are on the host. */
pqph_status pq_solve_batched(pqph_ctx* ctx, int nbatch, const int* npair,
                             const int64_t* h_off, const int64_t* eri_off,
                             const int64_t* t_off, const double* h,
                             const double* eri, const pqph_solve_opts* opts,
                             double* t_inout, double* energies,
                             pqph_solve_info* infos);

/* Execution mode of pq_solve_batched on this context: 0 (default) = device-
 * resident iterations replayed from a HIP graph; 1 = host-driven lockstep
 * (three host synchronisations per iteration for the whole batch; kept for
 * comparison).  INVALID_ARG for other values. */
pqph_status pqph_set_batch_mode(pqph_ctx* ctx, int mode);

/* How pq_solve and the amplitude solve of pq_energy_grad / pq_densities
 * iterate with the Jacobi/DIIS solver (Sec. III) on this context: 1 (default)
 * = host-driven: one host synchronisation per iteration, the DIIS system
 * solved on the host; 0 = device-driven: the norm test, the convergence,
 * stall and divergence decisions and the DIIS coefficients are computed on
 * the device, and the host enqueues the next iteration before it reads the
 * state of the last one (a finished solve gates off the one iteration queued
 * beyond its end), so the GPU never waits for the host.  Both take the same
 * steps and tests; the DIIS coefficients may differ in the last bits.  Mode 0
 * falls back to host-driven when diis_dim > 16 or stall_window > 256.  PH
 * solves and the lambda equations are always host-driven.  INVALID_ARG for
 * other values. */
pqph_status pqph_set_solve_mode(pqph_ctx* ctx, int mode);

/* Transposed-residual contraction (the adjoint of pq_residual and pq_energy,
 * Sec. II: the de-excitation amplitudes lambda of the Lagrangian
 * L = E_c + lambda . R are truncated like t):
 *     tbar   = sum_mu lam_mu dR_mu/dt   + energy_weight dE_c/dt   (packed t layout)
 *     hbar   = sum_mu lam_mu dR_mu/dh   + energy_weight dE_c/dh   (2N x 2N, f read
 *              as a general matrix)
 *     eribar = the same with respect to each stored integral (packed layout).
 * hbar and eribar may both be NULL (then only tbar is formed).  t, lam: packed
 * amplitude vectors.  Stream-ordered, no host sync.  Accumulation uses FP64
 * atomics, so results may differ from run to run in the last bits. */
pqph_status pq_vjp(pqph_ctx* ctx, int npair, const double* h, const double* eri,
                   const double* t, const double* lam, double energy_weight,
                   double* tbar, double* hbar, double* eribar);

/* PQ energy and its gradient with respect to the Hamiltonian.  If t is NULL
 * the amplitudes are solved here from zero (opts); otherwise t must hold
 * converged amplitudes.  lambda then solves J^T lambda = -dE/dt (J = dR/dt) by
 * the same Jacobi + DIIS (opts), starting from lambda = t, and
 *     dE/dh = dE_c/dh + lambda . dR/dh,  dE/deri = dE_c/deri + lambda . dR/deri
 * (raw partials: dE = sum dE_dh . dh + sum dE_deri . deri over the stored
 * elements).  energy: host; dE_dh: 2N x 2N device; dE_deri: packed device;
 * lambda_out: device or NULL; info (host, may be NULL) reports the lambda
 * solve (iterations, residual norm) and the total time. */
pqph_status pq_energy_grad(pqph_ctx* ctx, int npair, const double* h,
                           const double* eri, const double* t,
                           const pqph_solve_opts* opts, double* energy,
                           double* dE_dh, double* dE_deri, double* lambda_out,
                           pqph_solve_info* info);

/* Unrelaxed one- and two-particle densities of the PQ Lagrangian and the
 * natural occupation numbers (Table IV caption: the densities are formed after
 * the lambda solve; Sec. IV.B and Fig. 7 report natural occupations).  Solves
 * (or takes) t and lambda exactly as pq_energy_grad, then
 *     gamma[p][q] = <E_pq> = 2 delta_pq [p < npair] + dE/dh[p][q]
 *                   (2N x 2N device, spin-summed, E_pq = sum_s p_s+ q_s; the
 *                   first npair orbitals are occupied in the reference; not
 *                   symmetric in general), its trace is the electron count 2N;
 *     Gamma = dE/deri, the two-body density conjugate to each stored integral
 *             (packed device, the integral layout);
 *     noons (host, 2N, may be NULL) = eigenvalues of (gamma + gamma^T)/2 in
 *             descending order, by cyclic Jacobi rotations on the host.
 * energy: host; info (host, may be NULL) as for pq_energy_grad.  Returns the
 * lambda solve's status; the densities are written for OK and NOT_CONVERGED.
 * Synchronises the stream. */
pqph_status pq_densities(pqph_ctx* ctx, int npair, const double* h,
                         const double* eri, const double* t,
                         const pqph_solve_opts* opts, double* energy,
                         double* gamma, double* Gamma, double* noons,
                         pqph_solve_info* info);

/* Orbital-energy denominators of the packed slots (length pq_amp_len or
 * ph_amp_len by k): D = sum of f_aa over particles - sum of f_ii over holes
 * + shift.  Exposed for callers that run their own update. */
pqph_status pqph_denominators(pqph_ctx* ctx, int npair, int k, const double* h,
                              double shift, double* D);

#ifdef __cplusplus
}
#endif

#endif /* PQPH_H */
