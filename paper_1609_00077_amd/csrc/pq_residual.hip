// PQ residual, energy and denominators on gfx950.
//
// R_mu = <mu| e^{-T} H_N e^{T} |0> for the two-pair truncated manifold (Sec. II,
// Eq. (1) and the k = 2 truncation of the integrals, Table I caption).  The
// terms come from the pair-site derivation in derive/ (constant tables in
// pq_tables.h); roles P, Q are output pairs and A, B spectators.  Kernels:
//   k_vertex1/2   Hamiltonian vertices h1[key][P], h2[key][P][Q] from f and the
//                 packed integrals (the pair-block integral subtensors)
//   k_unpack_t2   packed t -> t2[m][P][Q] for all ordered P != Q (mirror copy
//                 carries the reordering sign of the two pair operators)
//   k_spec        products of factors over ordered label pairs: the R2S1 sides
//                 X(P,A), Y(Q,A) and the dressed two-spectator vertex W(A,B)
//   k_gemm_s1     S_p(P,Q) = sum_A X_p(P,A) Y_p(Q,A)   (one spectator)
//   k_r1          one-pair outputs (0, 1, 2 spectators)
//   k_r2s2        sum_{A,B} L_a(P,Q,A) W(A,B) L_b(P,Q,B)  (two spectators)
//   k_r2          two-pair outputs: no-spectator terms + one-spectator epilogue
//                 + the two-spectator partial sums, written to the packed r
#include "pqph_internal.h"
#include "pq_tables.h"

#include <algorithm>
#include <cmath>

namespace {

constexpr int NP2 = 29;   // pattern pairs of a two-pair label set

struct View {
    const double* t1;   // [3][N] (first block of the packed t)
    const double* t2;   // [29][N][N]
    const double* h1;   // [PQ_H1_N][N]
    const double* h2;   // [PQ_H2_N][N][N]
    const double* S;    // [PQ_S1PAIRS_N][N][N]
    const double* W;    // [2 PQ_W_N][N][N] two-spectator vertices and their transposes
    const double* D;    // [PQ_DR_N][N][N] dressed vertices
    int N;
    long NN;
};

__device__ __forceinline__ int labr(int r, int L0, int L1, int L2, int L3) {
    return r == 0 ? L0 : (r == 1 ? L1 : (r == 2 ? L2 : L3));
}

__device__ __forceinline__ double fval(int code, int L0, int L1, int L2, int L3, const View& v) {
    const int kind = (code >> 28) & 15;
    const int a = labr((code >> 24) & 15, L0, L1, L2, L3);
    const int b = labr((code >> 20) & 15, L0, L1, L2, L3);
    const long idx = code & 0xFFFF;
    switch (kind) {
        case 1: return v.t1[idx * v.N + a];
        case 2: return v.t2[idx * v.NN + (long)a * v.N + b];
        case 3: return v.h1[idx * v.N + a];
        case 4: return v.h2[idx * v.NN + (long)a * v.N + b];
        case 5: return v.S[idx * v.NN + (long)L0 * v.N + L1];
        case 6: return v.W[idx * v.NN + (long)a * v.N + b];
        case 7: return v.D[idx * v.NN + (long)a * v.N + b];
        default: return 1.0;
    }
}

// sum of the terms of output m of an interpreted class
__device__ __forceinline__ double class_sum(const int* start, const double* coef, const int* fac,
                                            int m, int L0, int L1, int L2, int L3, const View& v) {
    double acc = 0.0;
    const int e = start[m + 1];
    for (int i = start[m]; i < e; ++i) {
        double x = coef[i];
        const int* f = fac + 5 * i;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
            const int c = f[j];
            if (c != 0) x *= fval(c, L0, L1, L2, L3, v);
        }
        acc += x;
    }
    return acc;
}


// ------------------------------------------------------------------ vertices
__global__ void k_vertex1(int N, const double* __restrict__ f, const double* __restrict__ eri,
                          double* __restrict__ h1, const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    const int P = blockIdx.x * blockDim.x + threadIdx.x;
    const int key = blockIdx.y;
    if (P >= N) return;
    const long n2 = 2L * N;
    double v = 0.0;
    for (int i = pq_h1_start[key]; i < pq_h1_start[key + 1]; ++i) {
        const double w = pq_h1_w[i];
        if (pq_h1_kind[i] == 0) {
            const int p = P + N * (pq_h1_a[i] & 1), q = P + N * (pq_h1_b[i] & 1);
            v += w * f[p * n2 + q];
        } else {
            v += w * eri[(long)pq_h1_a[i] * N + P];
        }
    }
    h1[(long)key * N + P] = v;
}

// h2[key][P][Q] for one key and a 32 x 32 tile of (P, Q) per workgroup, and
// its k-major copy h2K[key][pq] over the output pairs P < Q.  The values are
// formed with the lanes along the label whose packed integral index is
// contiguous, staged in LDS, and written row by row into h2 and, for tiles on
// or above the diagonal, pair by pair into h2K, so every store is a run of
// up to 32 consecutive doubles.
constexpr int V2_TILE = 32;
__global__ __launch_bounds__(256) void k_vertex2(int N, const double* __restrict__ f,
                                                 const double* __restrict__ eri, double* __restrict__ h2,
                                                 double* __restrict__ h2T, const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    __shared__ double tile[V2_TILE][V2_TILE + 1];
    const int nt = (N + V2_TILE - 1) / V2_TILE;
    const int tp = blockIdx.x / nt, tq = blockIdx.x % nt, key = blockIdx.y;
    const int P0 = tp * V2_TILE, Q0 = tq * V2_TILE;
    const long NN = (long)N * N, n2 = 2L * N, np2 = (long)N * (N - 1) / 2;
    const double* e2 = eri + 6L * N;
    const int i0 = pq_h2_start[key], i1 = pq_h2_start[key + 1];
    const bool upper = tp < tq;          // every P < Q: the packed index runs along P
    for (int e = threadIdx.x; e < V2_TILE * V2_TILE; e += blockDim.x) {
        const int a = e & (V2_TILE - 1), b = e / V2_TILE;
        const int pl = upper ? a : b, ql = upper ? b : a;
        const int P = P0 + pl, Q = Q0 + ql;
        double v = 0.0;
        if (P < N && Q < N && P != Q) {
            const int lo = min(P, Q), hi = max(P, Q);
            const long pidx = (long)hi * (hi - 1) / 2 + lo;
            for (int i = i0; i < i1; ++i) {
                const double w = pq_h2_w[i];
                if (pq_h2_kind[i] == 0) {
                    const int ka = pq_h2_a[i], kb = pq_h2_b[i];
                    const int p = ((ka >> 1) ? Q : P) + N * (ka & 1);
                    const int q = ((kb >> 1) ? Q : P) + N * (kb & 1);
                    v += w * f[p * n2 + q];
                } else {
                    const int u = P < Q ? pq_h2_a[i] : pq_h2_b[i];
                    v += w * e2[(long)u * np2 + pidx];
                }
            }
        }
        tile[pl][ql] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < V2_TILE * V2_TILE; e += blockDim.x) {
        const int pl = e / V2_TILE, ql = e & (V2_TILE - 1);
        const int P = P0 + pl, Q = Q0 + ql;
        if (P < N && Q < N) h2[(long)key * NN + (long)P * N + Q] = tile[pl][ql];
    }
    if (tp > tq) return;                 // no pair P < Q in this tile
    for (int e = threadIdx.x; e < V2_TILE * V2_TILE; e += blockDim.x) {
        const int pl = e & (V2_TILE - 1), ql = e / V2_TILE;
        const int P = P0 + pl, Q = Q0 + ql;
        if (P < Q && Q < N) h2T[(long)key * np2 + (long)Q * (Q - 1) / 2 + P] = tile[pl][ql];
    }
}

// ---------------------------------------------------------------- amplitudes
__global__ void k_unpack_t2(int N, const double* __restrict__ t, double* __restrict__ t2, const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    const int Q = blockIdx.x * blockDim.x + threadIdx.x;
    const int P = blockIdx.y, m = blockIdx.z;
    if (Q >= N) return;
    const long NN = (long)N * N, np2 = (long)N * (N - 1) / 2;
    const double* tp = t + 3L * N;
    double v = 0.0;
    if (P < Q)
        v = tp[(long)m * np2 + (long)Q * (Q - 1) / 2 + P];
    else if (P > Q)
        v = pq_swap2_sign[m] * tp[(long)pq_swap2[m] * np2 + (long)P * (P - 1) / 2 + Q];
    t2[(long)m * NN + (long)P * N + Q] = v;
}

// ---------------------------------------------------------- factor products
// spec tables: 0 X, 1 Y (one-spectator sides), 2 W (two-spectator vertices),
// 3 L (links), 4 lambda (one-sided links of the dressed vertices)
__device__ __forceinline__ const int* spec_start(int which) {
    return which == 0 ? pq_x_start
         : which == 1 ? pq_y_start
         : which == 2 ? pq_w_start
         : which == 3 ? pq_l_start
         : which == 4 ? pq_lam_start
                      : pq_r1f_start;
}
__device__ __forceinline__ const int* spec_fac(int which) {
    return which == 0 ? pq_x_fac
         : which == 1 ? pq_y_fac
         : which == 2 ? pq_w_fac
         : which == 3 ? pq_l_fac
         : which == 4 ? pq_lam_fac
                      : pq_r1f_fac;
}

// grid (ceil(N*N/256), number of specs): thread -> ordered label pair (L0, L1)
__global__ __launch_bounds__(256) void k_spec(int N, int which, View v, double* __restrict__ out,
                                              const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (e >= N * N) return;
    const int L0 = e / N, L1 = e - L0 * N;
    const int* st = spec_start(which);
    const int* fc = spec_fac(which);
    double x = 0.0;
    if (L0 != L1) {
        x = 1.0;
        for (int i = st[s]; i < st[s + 1]; ++i) x *= fval(fc[i], L0, L1, 0, 0, v);
    }
    out[(long)s * v.NN + (long)L0 * N + L1] = x;
    // two-spectator vertices are also used transposed (groups keyed by the B link)
    if (which == 2) out[(long)(PQ_W_N + s) * v.NN + (long)L1 * N + L0] = x;
}


__device__ __forceinline__ double spec_l(int s, int P, int Q, int A, const View& v) {
    double x = 1.0;
    for (int i = pq_l_start[s]; i < pq_l_start[s + 1]; ++i) x *= fval(pq_l_fac[i], P, Q, A, 0, v);
    return x;
}

// A link spec decoded once per use: prod_f t2[m_f][P or Q][spectator]
struct Link {
    int n;
    const double* base[3];   // row pointers t2[m_f][P or Q][.]
};

__device__ __forceinline__ void link_rows(int s, int P, int Q, const View& v, Link& L) {
    L.n = pq_ld_n[s];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const int m = pq_ld_m[3 * s + f];
        const int who = pq_ld_q[3 * s + f] ? Q : P;
        L.base[f] = v.t2 + (long)m * v.NN + (long)who * v.N;
    }
}

__device__ __forceinline__ double link_at(const Link& L, int A) {
    double x = 1.0;
    if (L.n > 0) x = L.base[0][A];
    if (L.n > 1) x *= L.base[1][A];
    if (L.n > 2) x *= L.base[2][A];
    return x;
}

// Link products of one spec s (NB factors, uniform over the workgroup) for a
// thread's four staged elements: rows with labels (P[j], Q[j]) at one
// spectator label A (clamped into range by the caller's masks: every load
// is in bounds).  All NB x 4 loads are issued together; the factors are
// multiplied in their listed order, as link_at does.
template <int NB>
__device__ __forceinline__ void link_vals4(int s, const int* P, const int* Q, int A, const View& v,
                                          double* out) {
    int fm[NB > 0 ? NB : 1];
    bool fq[NB > 0 ? NB : 1];
#pragma unroll
    for (int f = 0; f < NB; ++f) {
        fm[f] = pq_ld_m[3 * s + f];
        fq[f] = pq_ld_q[3 * s + f] != 0;
    }
    double l[4][NB > 0 ? NB : 1];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int f = 0; f < NB; ++f)
            l[j][f] = v.t2[(long)fm[f] * v.NN + (long)(fq[f] ? Q[j] : P[j]) * v.N + A];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double x = NB > 0 ? l[j][0] : 1.0;
#pragma unroll
        for (int f = 1; f < NB; ++f) x *= l[j][f];
        out[j] = x;
    }
}

__device__ __forceinline__ void link_vals4_any(int s, const int* P, const int* Q, int A, const View& v,
                                              double* out) {
    switch (pq_ld_n[s]) {
        case 0: link_vals4<0>(s, P, Q, A, v, out); break;
        case 1: link_vals4<1>(s, P, Q, A, v, out); break;
        case 2: link_vals4<2>(s, P, Q, A, v, out); break;
        default: link_vals4<3>(s, P, Q, A, v, out); break;
    }
}

// Link products of one spec s (NB factors) for one row (P, Q) at four
// spectator labels A[j] (in range): all loads issued together, factors
// multiplied in their listed order.
template <int NB>
__device__ __forceinline__ void link_row4(int s, int P, int Q, const int* A, const View& v, double* out) {
    const double* base[NB > 0 ? NB : 1];
#pragma unroll
    for (int f = 0; f < NB; ++f)
        base[f] = v.t2 + (long)pq_ld_m[3 * s + f] * v.NN + (long)(pq_ld_q[3 * s + f] ? Q : P) * v.N;
    double l[4][NB > 0 ? NB : 1];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int f = 0; f < NB; ++f) l[j][f] = base[f][A[j]];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double x = NB > 0 ? l[j][0] : 1.0;
#pragma unroll
        for (int f = 1; f < NB; ++f) x *= l[j][f];
        out[j] = x;
    }
}

__device__ __forceinline__ void link_row4_any(int s, int P, int Q, const int* A, const View& v, double* out) {
    switch (pq_ld_n[s]) {
        case 0: link_row4<0>(s, P, Q, A, v, out); break;
        case 1: link_row4<1>(s, P, Q, A, v, out); break;
        case 2: link_row4<2>(s, P, Q, A, v, out); break;
        default: link_row4<3>(s, P, Q, A, v, out); break;
    }
}

// ------------------------------------------------------------ one spectator

// S[p][pq] = S_p(P,Q) = sum_A X_x(P,A) Y_y(Q,A) for P < Q, on the FP64
// matrix cores (v_mfma_f64_16x16x4f64: A[i][k] at lane i+16k, B[k][j] at lane
// j+16k, D[(lane>>4)+4r][lane&15] in register r).  Workgroup: one pair p and
// up to S1_TPW upper-triangular 16x16 tiles of (P, Q) per wavefront; the rows
// of X_x and Y_y are staged through LDS in K-chunks of 16 (row pitch 17:
// conflict-free operand reads), so each operand element is fetched once per
// workgroup.  Each finished tile is transposed through LDS and written as
// 128-byte runs of consecutive pq (S is p-major: the lane-per-pair epilogue
// reads S_p for consecutive output pairs).  Zero diagonals of X and Y keep
// A != P, Q.  Workgroups are dealt out XCD by XCD, so consecutive pairs
// (numbered in (x, y) order, sharing X_x) run on one XCD's L2.
typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int S1_TPW = 4;                 // tiles per wavefront
constexpr int S1_TPG = 4 * S1_TPW;        // tiles per workgroup
constexpr int S1_PITCH = 17;

inline __device__ void tile_of(int t, int nt, int& tP, int& tQ) {
    tP = 0;
    while (t >= nt - tP) { t -= nt - tP; ++tP; }
    tQ = tP + t;
}

// The factors of one side spec, decoded once: factor f of the product at the
// ordered label pair (L0, L1) is p[f][L0 * sa[f] + L1 * sb[f]] (an N x N
// slice read as given or transposed, or a per-label vector), so a staging
// step issues all its loads at once instead of interpreting codes per element.
constexpr int SPEC_MAXF = 4;
struct SpecPtrs {
    const double* p[SPEC_MAXF];
    int sa[SPEC_MAXF], sb[SPEC_MAXF];
    int n;
};

__device__ __forceinline__ SpecPtrs spec_ptrs(const int* __restrict__ fc, int i0, int i1, const View& v) {
    SpecPtrs q;
    q.n = min(i1 - i0, SPEC_MAXF);
#pragma unroll
    for (int f = 0; f < SPEC_MAXF; ++f) {
        q.p[f] = v.t2;
        q.sa[f] = 0;
        q.sb[f] = 0;
        if (f < q.n) {
            const int code = fc[i0 + f];
            const int kind = (code >> 28) & 15, r0 = (code >> 24) & 15, r1 = (code >> 20) & 15;
            const long idx = code & 0xFFFF;
            if (kind == 1 || kind == 3) {       // per-label vectors t1, h1
                q.p[f] = (kind == 1 ? v.t1 : v.h1) + idx * v.N;
                q.sa[f] = r0 == 0;
                q.sb[f] = r0 == 1;
            } else {                            // N x N slices t2, h2, W, D
                q.p[f] = (kind == 2 ? v.t2 : kind == 4 ? v.h2 : kind == 6 ? v.W : v.D) + idx * v.NN;
                q.sa[f] = (r0 == 0 ? v.N : 0) + (r1 == 0 ? 1 : 0);
                q.sb[f] = (r0 == 1 ? v.N : 0) + (r1 == 1 ? 1 : 0);
            }
        }
    }
    return q;
}

__device__ __forceinline__ double spec_eval(const SpecPtrs& q, int L0, int L1) {
    double x = 1.0;
#pragma unroll
    for (int f = 0; f < SPEC_MAXF; ++f)
        if (f < q.n) x *= q.p[f][L0 * q.sa[f] + L1 * q.sb[f]];   // < 2^16: 32-bit offsets
    return x;
}

// Both sides of the one-spectator GEMM materialised in one launch (modes 2
// and 4, and the adjoint): grid (ceil(N*N / 512), PQ_X_N + PQ_Y_N), two
// consecutive elements per thread.  The factor list of a slice is decoded
// once (spec_ptrs) and its length, uniform over the block, selects a
// straight-line product, so all loads of a thread's two elements are in
// flight together.  Same product order as k_spec: bitwise the same sides.
__device__ __forceinline__ void spec_two(const SpecPtrs& q, int a0, int a1, int b0, int b1, double& xa,
                                         double& xb) {
    auto at = [&](int f, int L0, int L1) { return q.p[f][L0 * q.sa[f] + L1 * q.sb[f]]; };
    switch (q.n) {
        case 0:
            xa = xb = 1.0;
            break;
        case 1:
            xa = at(0, a0, a1);
            xb = at(0, b0, b1);
            break;
        case 2: {
            const double u0 = at(0, a0, a1), u1 = at(1, a0, a1);
            const double w0 = at(0, b0, b1), w1 = at(1, b0, b1);
            xa = u0 * u1;
            xb = w0 * w1;
            break;
        }
        case 3: {
            const double u0 = at(0, a0, a1), u1 = at(1, a0, a1), u2 = at(2, a0, a1);
            const double w0 = at(0, b0, b1), w1 = at(1, b0, b1), w2 = at(2, b0, b1);
            xa = (u0 * u1) * u2;
            xb = (w0 * w1) * w2;
            break;
        }
        default: {
            const double u0 = at(0, a0, a1), u1 = at(1, a0, a1), u2 = at(2, a0, a1), u3 = at(3, a0, a1);
            const double w0 = at(0, b0, b1), w1 = at(1, b0, b1), w2 = at(2, b0, b1), w3 = at(3, b0, b1);
            xa = ((u0 * u1) * u2) * u3;
            xb = ((w0 * w1) * w2) * w3;
            break;
        }
    }
}

__global__ __launch_bounds__(256) void k_spec_xy(int N, View v, double* __restrict__ X, double* __restrict__ Y,
                                                 const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    const int sl = blockIdx.y;
    const bool ys = sl >= PQ_X_N;
    const int sx = ys ? sl - PQ_X_N : sl;
    const SpecPtrs q = ys ? spec_ptrs(pq_y_fac, pq_y_start[sx], pq_y_start[sx + 1], v)
                          : spec_ptrs(pq_x_fac, pq_x_start[sx], pq_x_start[sx + 1], v);
    const int NN = N * N;
    const int e = 2 * (blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= NN) return;
    const int a0 = e / N, a1 = e - a0 * N;
    const bool two = e + 1 < NN;
    const int b0 = two ? (e + 1) / N : a0, b1 = two ? e + 1 - b0 * N : a1;
    double xa, xb;
    spec_two(q, a0, a1, b0, b1, xa, xb);
    double* out = (ys ? Y : X) + (long)sx * NN;
    out[e] = a0 != a1 ? xa : 0.0;                 // zero diagonal: A != P, Q
    if (two) out[e + 1] = b0 != b1 ? xb : 0.0;
}

// FUSED: the sides X_x(P,A) and Y_y(Q,A) are formed while staging, as the
// products of their factors (amplitudes, vertices, dressed vertices: arrays
// of at most a few hundred N x N slices that stay in the caches), instead of
// being read from materialised X and Y (about 1750 slices at 70 pairs)
// (five wavefronts per SIMD, as many workgroups as the LDS allows: at 96
// VGPRs a few values spill, which costs less than the lost occupancy)
template <bool FUSED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_gemm_s1(int N, View v, const double* __restrict__ X,
                                                 const double* __restrict__ Y,
                                                 double* __restrict__ SK, const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    extern __shared__ double sm[];
    const int nt = (N + 15) / 16, NR = nt * 16, ntile = nt * (nt + 1) / 2;
    const int ngrp = (ntile + S1_TPG - 1) / S1_TPG;
    const long nitem = (long)ngrp * PQ_S1PAIRS_N;
    const long per = gridDim.x / 8;
    const long w = (long)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (w >= nitem) return;
    const int p = (int)(w / ngrp), tg = (int)(w % ngrp);
    double* Xs = sm;                         // [NR][S1_PITCH]
    double* Ys = Xs + NR * S1_PITCH;         // [NR][S1_PITCH]
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: tile indices in SGPRs
    double* Ts = Ys + NR * S1_PITCH + wave * 16 * S1_PITCH;   // [16][S1_PITCH] per wavefront
    const long NN = (long)N * N;
    const int xi = pq_s1pairs[2 * p], yi = pq_s1pairs[2 * p + 1];
    const double* Xp = FUSED ? nullptr : X + (long)xi * NN;
    const double* Yp = FUSED ? nullptr : Y + (long)yi * NN;
    SpecPtrs xq, yq;
    if (FUSED) {
        xq = spec_ptrs(pq_x_fac, pq_x_start[xi], pq_x_start[xi + 1], v);
        yq = spec_ptrs(pq_y_fac, pq_y_start[yi], pq_y_start[yi + 1], v);
    }
    const int i = lane & 15, kq = lane >> 4;
    int tP[S1_TPW], tQ[S1_TPW];
    bool tv[S1_TPW];
#pragma unroll
    for (int u = 0; u < S1_TPW; ++u) {
        const int t = tg * S1_TPG + wave + 4 * u;
        tv[u] = t < ntile;
        tile_of(tv[u] ? t : 0, nt, tP[u], tQ[u]);
    }
    d4 D[S1_TPW];
#pragma unroll
    for (int u = 0; u < S1_TPW; ++u) D[u] = d4{0.0, 0.0, 0.0, 0.0};
    for (int kc = 0; kc < N; kc += 16) {
        __syncthreads();
        for (int e = tid; e < NR * 16; e += 256) {
            const int r = e >> 4, k = e & 15, A = kc + k;
            const bool in = r < N && A < N;
            if (FUSED) {
                const bool off = in && r != A;          // zero diagonals keep A != P, Q
                Xs[r * S1_PITCH + k] = off ? spec_eval(xq, r, A) : 0.0;
                Ys[r * S1_PITCH + k] = off ? spec_eval(yq, r, A) : 0.0;
            } else {
                Xs[r * S1_PITCH + k] = in ? Xp[(long)r * N + A] : 0.0;
                Ys[r * S1_PITCH + k] = in ? Yp[(long)r * N + A] : 0.0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < S1_TPW; ++u) {
            if (!tv[u]) continue;
            const double* xa = Xs + (tP[u] * 16 + i) * S1_PITCH + kq;
            const double* yb = Ys + (tQ[u] * 16 + i) * S1_PITCH + kq;
#pragma unroll
            for (int k4 = 0; k4 < 16; k4 += 4)
                D[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[k4], yb[k4], D[u], 0, 0, 0);
        }
    }
    const long np2 = (long)N * (N - 1) / 2;
    double* out = SK + (long)p * np2;
#pragma unroll
    for (int u = 0; u < S1_TPW; ++u) {
        if (!tv[u]) continue;
        // D[u][r] = S(P = tP*16 + kq + 4r, Q = tQ*16 + i): stage as Ts[Ql][Pl]
#pragma unroll
        for (int r = 0; r < 4; ++r) Ts[i * S1_PITCH + kq + 4 * r] = D[u][r];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int e = lane; e < 256; e += 64) {
            const int ql = e >> 4, pl = e & 15;
            const int P = tP[u] * 16 + pl, Q = tQ[u] * 16 + ql;
            if (P < Q && Q < N) out[(long)Q * (Q - 1) / 2 + P] = Ts[ql * S1_PITCH + pl];
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

// Mode 3 of the same contraction: the fused staging software-pipelined.  The
// raw factors of K-chunk k+1 are loaded into registers before the matrix-core
// steps of chunk k are issued, and multiplied into the other of two LDS
// buffers after them, so the loads overlap the MFMAs of the same wavefront;
// one barrier per chunk.  NT = row tiles (N <= 16 NT); thread element j of a
// chunk is e = tid + 256 j (row e/16, column e%16).
template <int NT>
__global__ __launch_bounds__(256) void k_gemm_s1p(int N, View v, double* __restrict__ SK,
                                                  const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    extern __shared__ double sm[];
    constexpr int NR = NT * 16, ntile = NT * (NT + 1) / 2;
    constexpr int ngrp = (ntile + S1_TPG - 1) / S1_TPG;
    const long nitem = (long)ngrp * PQ_S1PAIRS_N;
    const long per = gridDim.x / 8;
    const long w = (long)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (w >= nitem) return;
    const int p = (int)(w / ngrp), tg = (int)(w % ngrp);
    double* Xs = sm;                          // [2][NR][S1_PITCH]
    double* Ys = Xs + 2 * NR * S1_PITCH;      // [2][NR][S1_PITCH]
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: tile indices in SGPRs
    double* Ts = Ys + 2 * NR * S1_PITCH + wave * 16 * S1_PITCH;   // [16][S1_PITCH] per wavefront
    const int xi = pq_s1pairs[2 * p], yi = pq_s1pairs[2 * p + 1];
    const SpecPtrs xq = spec_ptrs(pq_x_fac, pq_x_start[xi], pq_x_start[xi + 1], v);
    const SpecPtrs yq = spec_ptrs(pq_y_fac, pq_y_start[yi], pq_y_start[yi + 1], v);
    const int i = lane & 15, kq = lane >> 4;
    int tP[S1_TPW], tQ[S1_TPW];
    bool tv[S1_TPW];
#pragma unroll
    for (int u = 0; u < S1_TPW; ++u) {
        const int t = tg * S1_TPG + wave + 4 * u;
        tv[u] = t < ntile;
        tile_of(tv[u] ? t : 0, NT, tP[u], tQ[u]);
    }
    d4 D[S1_TPW];
#pragma unroll
    for (int u = 0; u < S1_TPW; ++u) D[u] = d4{0.0, 0.0, 0.0, 0.0};
    // raw factors of this thread's NT elements of one chunk, both sides
    double fx[NT][SPEC_MAXF], fy[NT][SPEC_MAXF];
    auto load = [&](int kc) {
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int e = tid + 256 * j, r = e >> 4, A = kc + (e & 15);
            const bool off = r < N && A < N && r != A;     // zero diagonals keep A != P, Q
#pragma unroll
            for (int f = 0; f < SPEC_MAXF; ++f) {
                fx[j][f] = (off && f < xq.n) ? xq.p[f][r * xq.sa[f] + A * xq.sb[f]] : (off ? 1.0 : 0.0);
                fy[j][f] = (off && f < yq.n) ? yq.p[f][r * yq.sa[f] + A * yq.sb[f]] : (off ? 1.0 : 0.0);
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int e = tid + 256 * j, r = e >> 4, k = e & 15;
            double x = 1.0, y = 1.0;
#pragma unroll
            for (int f = 0; f < SPEC_MAXF; ++f) {
                x *= fx[j][f];
                y *= fy[j][f];
            }
            Xs[(buf * NR + r) * S1_PITCH + k] = x;
            Ys[(buf * NR + r) * S1_PITCH + k] = y;
        }
    };
    const int nch = (N + 15) / 16;
    load(0);
    store(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const int buf = c & 1;
        if (c + 1 < nch) load((c + 1) * 16);
#pragma unroll
        for (int u = 0; u < S1_TPW; ++u) {
            if (!tv[u]) continue;
            const double* xa = Xs + (buf * NR + tP[u] * 16 + i) * S1_PITCH + kq;
            const double* yb = Ys + (buf * NR + tQ[u] * 16 + i) * S1_PITCH + kq;
#pragma unroll
            for (int k4 = 0; k4 < 16; k4 += 4)
                D[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[k4], yb[k4], D[u], 0, 0, 0);
        }
        if (c + 1 < nch) store(buf ^ 1);
        __syncthreads();
    }
    const long np2 = (long)N * (N - 1) / 2;
    double* out = SK + (long)p * np2;
#pragma unroll
    for (int u = 0; u < S1_TPW; ++u) {
        if (!tv[u]) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) Ts[i * S1_PITCH + kq + 4 * r] = D[u][r];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int e = lane; e < 256; e += 64) {
            const int ql = e >> 4, pl = e & 15;
            const int P = tP[u] * 16 + pl, Q = tQ[u] * 16 + ql;
            if (P < Q && Q < N) out[(long)Q * (Q - 1) / 2 + P] = Ts[ql * S1_PITCH + pl];
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

// Mode 4: the materialised sides of mode 2, with the staging software-
// pipelined.  Each thread holds its share of the next K-chunk (NT slots of two
// consecutive columns, 16-byte loads when N is even) in registers: the loads
// are issued before the current chunk's matrix-core steps and written to the
// single LDS buffer after them, so their latency hides behind the MFMAs
// without a second buffer (occupancy stays that of mode 2).  Tiles, operand
// order and the epilogue are those of k_gemm_s1, so S is bitwise the same as
// in mode 2.  NT = row tiles (N <= 16 NT).
template <int NT, bool EVEN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NT <= 5 ? 5 : NT <= 8 ? 4 : NT <= 10 ? 3 : 2, 8))) void k_gemm_s1m(
    int N, const double* __restrict__ X, const double* __restrict__ Y, double* __restrict__ SK,
    const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    extern __shared__ double sm[];
    constexpr int NR = NT * 16, ntile = NT * (NT + 1) / 2;
    constexpr int ngrp = (ntile + S1_TPG - 1) / S1_TPG;
    constexpr int SE = NR * 8;                // two-column slots per side and chunk
    const long nitem = (long)ngrp * PQ_S1PAIRS_N;
    const long per = gridDim.x / 8;
    const long w = (long)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (w >= nitem) return;
    const int p = (int)(w / ngrp), tg = (int)(w % ngrp);
    double* Xs = sm;                          // [NR][S1_PITCH]
    double* Ys = Xs + NR * S1_PITCH;          // [NR][S1_PITCH]
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: tile indices in SGPRs
    double* Ts = Ys + NR * S1_PITCH + wave * 16 * S1_PITCH;   // [16][S1_PITCH] per wavefront
    const long NN = (long)N * N;
    const int xi = pq_s1pairs[2 * p], yi = pq_s1pairs[2 * p + 1];
    const double* Xp = X + (long)xi * NN;
    const double* Yp = Y + (long)yi * NN;
    const int i = lane & 15, kq = lane >> 4;
    int tP[S1_TPW], tQ[S1_TPW];
    bool tv[S1_TPW];
#pragma unroll
    for (int u = 0; u < S1_TPW; ++u) {
        const int t = tg * S1_TPG + wave + 4 * u;
        tv[u] = t < ntile;
        tile_of(tv[u] ? t : 0, NT, tP[u], tQ[u]);
    }
    d4 D[S1_TPW];
#pragma unroll
    for (int u = 0; u < S1_TPW; ++u) D[u] = d4{0.0, 0.0, 0.0, 0.0};
    // slot j of this thread: e = tid + 256 j < 2 SE (side = e >= SE), row
    // r = (e mod SE) / 8, columns A, A + 1 with A = kc + 2 (e mod 8)
    // every load is issued unconditionally at an in-bounds (clamped) address
    // and masked only when written to LDS, so a chunk's loads stay in flight
    // through the matrix-core steps
    double2 st[NT];
    auto load = [&](int kc) {
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int e = tid + 256 * j;
            const bool ys = e >= SE;
            const int idx = ys ? e - SE : e, r = idx >> 3, A = kc + 2 * (idx & 7);
            const double* base = ys ? Yp : Xp;
            if (EVEN) {              // A even, so A < N implies A + 1 < N; 16-byte aligned
                const bool in = r < N && A < N;
                st[j] = *(const double2*)(base + (in ? r * N + A : 0));
            } else {
                const bool in0 = r < N && A < N, in1 = r < N && A + 1 < N;
                st[j].x = base[in0 ? r * N + A : 0];
                st[j].y = base[in1 ? r * N + A + 1 : 0];
            }
        }
    };
    auto store = [&](int kc) {
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int e = tid + 256 * j;
            const bool ys = e >= SE;
            const int idx = ys ? e - SE : e, r = idx >> 3, k = 2 * (idx & 7), A = kc + k;
            double* dst = (ys ? Ys : Xs) + r * S1_PITCH + k;
            dst[0] = r < N && A < N ? st[j].x : 0.0;
            dst[1] = r < N && A + 1 < N ? st[j].y : 0.0;
        }
    };
    const int nch = (N + 15) / 16;
    load(0);
    for (int c = 0; c < nch; ++c) {
        __syncthreads();                      // the previous chunk's operands are consumed
        store(c * 16);
        __syncthreads();
        if (c + 1 < nch) load((c + 1) * 16);  // in flight during this chunk's MFMAs
#pragma unroll
        for (int u = 0; u < S1_TPW; ++u) {
            if (!tv[u]) continue;
            const double* xa = Xs + (tP[u] * 16 + i) * S1_PITCH + kq;
            const double* yb = Ys + (tQ[u] * 16 + i) * S1_PITCH + kq;
#pragma unroll
            for (int k4 = 0; k4 < 16; k4 += 4)
                D[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[k4], yb[k4], D[u], 0, 0, 0);
        }
    }
    const long np2 = (long)N * (N - 1) / 2;
    double* out = SK + (long)p * np2;
#pragma unroll
    for (int u = 0; u < S1_TPW; ++u) {
        if (!tv[u]) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) Ts[i * S1_PITCH + kq + 4 * r] = D[u][r];
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int e = lane; e < 256; e += 64) {
            const int ql = e >> 4, pl = e & 15;
            const int P = tP[u] * 16 + pl, Q = tQ[u] * 16 + ql;
            if (P < Q && Q < N) out[(long)Q * (Q - 1) / 2 + P] = Ts[ql * S1_PITCH + pl];
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

// Batched dense products C_g = A_g B_g^T of N x N row-major matrices on the
// FP64 matrix cores, with the staging and tiling of k_gemm_s1 (full square
// output, written directly: for fixed r the 16 lanes of a row hold 16
// consecutive columns).  which = 0: dressed vertices D_k = lambda_k W_k^T
// (lambda = 1 everywhere when its index is negative); which = 1: the one-pair
// two-spectator products M_g = G_g Mid_g = G_g (Mid_g^T)^T.
// Workgroup: one row block tP of C and the 4 column blocks tQ = 4 tq4 .. +3
// (one per wavefront); only those rows of A and B are staged per K-chunk.
__global__ __launch_bounds__(256) void k_bgemm(int N, int which, const double* __restrict__ Abase,
                                               const double* __restrict__ Bbase,
                                               double* __restrict__ Cbase, const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    __shared__ double As[16 * S1_PITCH];
    __shared__ double Bs[64 * S1_PITCH];
    const int nt = (N + 15) / 16;
    const int tP = blockIdx.x % nt, tq4 = blockIdx.x / nt, g = blockIdx.y;
    const long NN = (long)N * N;
    const int ai = which == 0 ? pq_dr_lam[g] : pq_r1g_gen[g];
    const int bi = which == 0 ? pq_dr_w[g] : pq_r1g_midT[g];
    const double* A = Abase + (long)(ai >= 0 ? ai : 0) * NN;
    const double* B = Bbase + (long)bi * NN;
    double* C = Cbase + (long)g * NN;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int i = lane & 15, kq = lane >> 4;
    const int tQ = tq4 * 4 + wave;
    d4 D = {0.0, 0.0, 0.0, 0.0};
    for (int kc = 0; kc < N; kc += 16) {
        __syncthreads();
        {
            const int r = tid >> 4, k = tid & 15, K = kc + k, row = tP * 16 + r;
            As[r * S1_PITCH + k] = (row < N && K < N) ? (ai >= 0 ? A[(long)row * N + K] : 1.0) : 0.0;
        }
        for (int e = tid; e < 64 * 16; e += 256) {
            const int r = e >> 4, k = e & 15, K = kc + k, row = tq4 * 64 + r;
            Bs[r * S1_PITCH + k] = (row < N && K < N) ? B[(long)row * N + K] : 0.0;
        }
        __syncthreads();
        if (tQ < nt) {
            const double* xa = As + i * S1_PITCH + kq;
            const double* yb = Bs + (wave * 16 + i) * S1_PITCH + kq;
#pragma unroll
            for (int k4 = 0; k4 < 16; k4 += 4)
                D = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[k4], yb[k4], D, 0, 0, 0);
        }
    }
    if (tQ < nt) {
        const int Q = tQ * 16 + i;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int P = tP * 16 + kq + 4 * r;
            if (P < N && Q < N) C[(long)P * N + Q] = D[r];
        }
    }
}

// closing of the one-pair two-spectator groups: for output pair P and group g,
// sum over closers c_i sum_j M_g(P,j) C_i(P,j), written per output pattern to
// the group's own partial chunk (fixed order, no atomics)
__global__ __launch_bounds__(64) void k_r1s2_close(int N, const double* __restrict__ F,
                                                   const double* __restrict__ M, double* __restrict__ part,
                                                   int chunk0, const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    // one wavefront per (P, g): lanes over j (contiguous rows), fixed-order shuffle reduction
    const int P = blockIdx.x, g = blockIdx.y, lane = threadIdx.x;
    const long NN = (long)N * N;
    const double* Mr = M + (long)g * NN + (long)P * N;
    double a[3] = {0.0, 0.0, 0.0};
    for (int i = pq_r1g_start[g]; i < pq_r1g_start[g + 1]; ++i) {
        const double* Cr = F + (long)pq_r1g_cl[i] * NN + (long)P * N;
        double s = 0.0;
        for (int j = lane; j < N; j += 64) s += Mr[j] * Cr[j];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        const int mu = pq_r1g_mu[i];
        const double x = pq_r1g_coef[i] * s;
        a[0] += mu == 0 ? x : 0.0;
        a[1] += mu == 1 ? x : 0.0;
        a[2] += mu == 2 ? x : 0.0;
    }
    if (lane < 3) part[((long)(chunk0 + g) * 3 + lane) * N + P] = lane == 0 ? a[0] : (lane == 1 ? a[1] : a[2]);
}

// ----------------------------------------------------------- one-pair outputs
// grid (N, nch): workgroup (P, ch) sums the chunk ch of the ordered spectator
// (two-spectator terms: k_bgemm and k_r1s2_close).
// no-spectator terms of the one-pair outputs, one thread per term, fixed-order
// block reduction (the one-spectator terms run in k_r1c, the two-spectator
// terms in k_bgemm and k_r1s2_close)
__global__ __launch_bounds__(64) void k_r1(int N, View v, double* __restrict__ part,
                                           const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    const int P = blockIdx.x, tid = threadIdx.x;
    double a[3] = {0.0, 0.0, 0.0};
    for (int i = tid; i < PQ_R1S0_NTERM; i += 64) {
        double x = pq_r1s0_coef[i];
        const int* f = pq_r1s0_fac + 5 * i;
#pragma unroll
        for (int j = 0; j < 5; ++j)
            if (f[j] != 0) x *= fval(f[j], P, 0, 0, 0, v);
        const int m = i < pq_r1s0_start[1] ? 0 : (i < pq_r1s0_start[2] ? 1 : 2);
        a[0] += m == 0 ? x : 0.0;
        a[1] += m == 1 ? x : 0.0;
        a[2] += m == 2 ? x : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
        for (int o = 32; o > 0; o >>= 1) a[k] += __shfl_xor(a[k], o);
    if (tid == 0) {
        part[0 * N + P] = a[0];
        part[1 * N + P] = a[1];
        part[2 * N + P] = a[2];
    }
}

// ------------------------------------------- one-pair outputs, two spectators
// Every term factorises as X(P,A) Z(A,B) Y(P,B) (products of factors on
// {P,A}, {A,B}, {P,B}); F holds all those products over ordered label pairs
// with zero diagonals (so A, B != P and A != B hold by construction), the
// Z products also transposed.
__global__ __launch_bounds__(256) void k_spec_r1(int N, View v, double* __restrict__ F,
                                                 const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (e >= N * N) return;
    const int L0 = e / N, L1 = e - L0 * N;
    double x = 0.0;
    if (L0 != L1) {
        x = 1.0;
        for (int i = pq_r1f_start[s]; i < pq_r1f_start[s + 1]; ++i)
            x *= fval(pq_r1f_fac[i], L0, L1, 0, 0, v);
    }
    F[(long)s * v.NN + (long)L0 * N + L1] = x;
    if (s >= PQ_R1F_Z0) F[(long)(PQ_R1F_N + s - PQ_R1F_Z0) * v.NN + (long)L1 * N + L0] = x;
}


// ----------------------------------------------------------- two spectators
// V(pq, B) = sum_A L_a(P,Q,A) W_w(A,B) is a dense GEMM over the spectator A
// whose left operand is generated on the fly (a Khatri-Rao product of the
// amplitudes linking P and Q to A); it runs on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64: A[i][k] at lane i+16k, B[k][j] at lane j+16k,
// D[(lane>>4)+4r][lane&15] in register r).  Each group (w, a) is then closed
// against the B-side links L_b(P,Q,B) and accumulated per output pattern.
// Workgroup: 64 output pairs (4 wavefronts x 16 rows) x all B; grid.y splits
// the groups, whose partial sums are combined in k_final.
constexpr int M2_ROWS = 64;
constexpr int M2_KC = 16;
// the staging loops give each of 256 threads four elements (rows tid/16 + 16 j, spectator tid % 16)
static_assert(M2_ROWS * M2_KC == 4 * 256 && M2_KC == 16, "two-spectator staging layout");
// The matrix-core kernels below ask for more resident wavefronts per SIMD
// (amdgpu_waves_per_eu) than their register use would give by default: the
// MFMA accumulators otherwise take AGPRs that halve the occupancy, and the
// latency of their staging loads is hidden by other wavefronts (measured:
// k_r2s2 20-37 % faster, k_r2s2_adjm 14 %, k_s1_adj up to 19 %, even where a
// few registers spill).

// Closing of a two-spectator group against one B-side link b of NB factors:
// s[r] = sum over this lane's columns B of V(row r, B) L_b(P, Q, B), for the
// wavefront's four rows of this lane.  The loads of a row are issued together
// (columns clamped in range, masked when added).  QM marks the factors read
// at Q (bit f): when the wavefront's 16 rows share Q (consecutive output
// pairs) their product is formed once per column for all four rows, and each
// row loads only its factors read at P.  Otherwise (QM = 0 call, or rows with
// different Q) every factor is loaded per row.
template <int NCB, int NB, int QM>
__device__ __forceinline__ void r2s2_close(int b, int N, const View& v, const int* rowP, const int* rowQ,
                                          int wave, int lane, const d4* D, double* s) {
    const double* base[NB > 0 ? NB : 1];
    double qp[NCB];
    if (QM) {
        const int Q0 = rowQ[wave * 16];
#pragma unroll
        for (int f = 0; f < NB; ++f)
            if (QM >> f & 1) base[f] = v.t2 + (long)pq_ld_m[3 * b + f] * v.NN + (long)Q0 * v.N;
        double lq[NCB][NB > 0 ? NB : 1];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int col = cb * 16 + (lane & 15);
            const int cc = col < N ? col : 0;
#pragma unroll
            for (int f = 0; f < NB; ++f)
                if (QM >> f & 1) lq[cb][f] = base[f][cc];
        }
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            double x = 1.0;
#pragma unroll
            for (int f = 0; f < NB; ++f)
                if (QM >> f & 1) x *= lq[cb][f];
            qp[cb] = x;
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        s[r] = 0.0;
        const int row = wave * 16 + (lane >> 4) + 4 * r;
        const int P = rowP[row], Q = rowQ[row];
        if (P < 0) continue;
#pragma unroll
        for (int f = 0; f < NB; ++f)
            if (!(QM >> f & 1))
                base[f] = v.t2 + (long)pq_ld_m[3 * b + f] * v.NN + (long)(pq_ld_q[3 * b + f] ? Q : P) * v.N;
        double l[NCB][NB > 0 ? NB : 1];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int col = cb * 16 + (lane & 15);
            const int cc = col < N ? col : 0;
#pragma unroll
            for (int f = 0; f < NB; ++f)
                if (!(QM >> f & 1)) l[cb][f] = base[f][cc];
        }
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int col = cb * 16 + (lane & 15);
            double x = QM ? qp[cb] : 1.0;
#pragma unroll
            for (int f = 0; f < NB; ++f)
                if (!(QM >> f & 1)) x *= l[cb][f];
            if (col < N && col != P && col != Q) s[r] += D[cb][r] * x;
        }
    }
}

// dispatch on the link's factor count and, for wavefronts whose rows share
// Q, on which factors are read at Q
template <int NCB>
__device__ __forceinline__ void r2s2_close_any(int b, int N, const View& v, const int* rowP, const int* rowQ,
                                              int wave, int lane, const d4* D, double* s, bool qsame) {
    const int nb = pq_ld_n[b];
    int qm = 0;
    if (qsame)
        for (int f = 0; f < nb; ++f) qm |= (pq_ld_q[3 * b + f] ? 1 : 0) << f;
    switch (nb * 8 + qm) {
        case 0: r2s2_close<NCB, 0, 0>(b, N, v, rowP, rowQ, wave, lane, D, s); break;
        case 8: r2s2_close<NCB, 1, 0>(b, N, v, rowP, rowQ, wave, lane, D, s); break;
        case 9: r2s2_close<NCB, 1, 1>(b, N, v, rowP, rowQ, wave, lane, D, s); break;
        case 16: r2s2_close<NCB, 2, 0>(b, N, v, rowP, rowQ, wave, lane, D, s); break;
        case 17: r2s2_close<NCB, 2, 1>(b, N, v, rowP, rowQ, wave, lane, D, s); break;
        case 18: r2s2_close<NCB, 2, 2>(b, N, v, rowP, rowQ, wave, lane, D, s); break;
        case 19: r2s2_close<NCB, 2, 3>(b, N, v, rowP, rowQ, wave, lane, D, s); break;
        case 24: r2s2_close<NCB, 3, 0>(b, N, v, rowP, rowQ, wave, lane, D, s); break;
        case 25: r2s2_close<NCB, 3, 1>(b, N, v, rowP, rowQ, wave, lane, D, s); break;
        case 26: r2s2_close<NCB, 3, 2>(b, N, v, rowP, rowQ, wave, lane, D, s); break;
        case 27: r2s2_close<NCB, 3, 3>(b, N, v, rowP, rowQ, wave, lane, D, s); break;
        case 28: r2s2_close<NCB, 3, 4>(b, N, v, rowP, rowQ, wave, lane, D, s); break;
        case 29: r2s2_close<NCB, 3, 5>(b, N, v, rowP, rowQ, wave, lane, D, s); break;
        case 30: r2s2_close<NCB, 3, 6>(b, N, v, rowP, rowQ, wave, lane, D, s); break;
        default: r2s2_close<NCB, 3, 7>(b, N, v, rowP, rowQ, wave, lane, D, s); break;
    }
}

template <int NCB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_r2s2(int N, View v, const double* __restrict__ W,
                                              int gchunk, double* __restrict__ part, const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    constexpr int NC = 16 * NCB;
    extern __shared__ double sm[];
    double* La = sm;                       // [M2_ROWS][M2_KC]
    double* Ws = La + M2_ROWS * M2_KC;     // [M2_KC][NC]
    double* acc = Ws + M2_KC * NC;         // [M2_ROWS][29]
    __shared__ int rowP[M2_ROWS], rowQ[M2_ROWS];
    const long np2 = (long)N * (N - 1) / 2;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const long ip0 = (long)blockIdx.x * M2_ROWS;
    if (tid < M2_ROWS) {
        int P = -1, Q = -1;
        if (ip0 + tid < np2) decode_pair(ip0 + tid, P, Q);
        rowP[tid] = P;
        rowQ[tid] = Q;
    }
    for (int i = tid; i < M2_ROWS * NP2; i += 256) acc[i] = 0.0;
    __syncthreads();
    // rows are consecutive output pairs (Q non-decreasing; missing rows last)
    const bool qsame = rowQ[wave * 16 + 15] >= 0 && rowQ[wave * 16] == rowQ[wave * 16 + 15];
    const int KP = (N + M2_KC - 1) / M2_KC * M2_KC;
    const int g0 = blockIdx.y * gchunk, g1 = min(PQ_G_N, g0 + gchunk);
    for (int g = g0; g < g1; ++g) {
        const int w = pq_g_w[g], a = pq_g_a[g];
        const double* Wg = W + (long)w * v.NN;
        d4 D[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) D[cb] = d4{0.0, 0.0, 0.0, 0.0};
        for (int kc = 0; kc < KP; kc += M2_KC) {
            if constexpr (NCB <= 6) {   // four elements: rows tid/16 + 16 j, one spectator A
                const int A = kc + (tid & 15);
                int Pj[4], Qj[4];
                bool ok[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = (tid >> 4) + 16 * j;
                    const int P = rowP[row], Q = rowQ[row];
                    ok[j] = P >= 0 && A < N && A != P && A != Q;
                    Pj[j] = P >= 0 ? P : 0;
                    Qj[j] = P >= 0 ? Q : 0;
                }
                double x[4];
                link_vals4_any(a, Pj, Qj, A < N ? A : 0, v, x);
#pragma unroll
                for (int j = 0; j < 4; ++j) La[tid + 256 * j] = ok[j] ? x[j] : 0.0;
            } else {      // wide rows: the accumulators leave no registers for batched loads
                for (int i = tid; i < M2_ROWS * M2_KC; i += 256) {
                    const int row = i / M2_KC, A = kc + i % M2_KC;
                    const int P = rowP[row], Q = rowQ[row];
                    double x = 0.0;
                    if (P >= 0 && A < N && A != P && A != Q) {
                        Link L;
                        link_rows(a, P, Q, v, L);
                        x = link_at(L, A);
                    }
                    La[i] = x;
                }
            }
            for (int i = tid; i < M2_KC * NC; i += 256) {
                const int A = kc + i / NC, col = i % NC;
                Ws[i] = (A < N && col < N) ? Wg[(long)A * N + col] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int k4 = 0; k4 < M2_KC; k4 += 4) {
                const double av = La[(wave * 16 + (lane & 15)) * M2_KC + k4 + (lane >> 4)];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    const double bv = Ws[(k4 + (lane >> 4)) * NC + cb * 16 + (lane & 15)];
                    D[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, D[cb], 0, 0, 0);
                }
            }
            __syncthreads();
        }
        for (int i = pq_g_start[g]; i < pq_g_start[g + 1]; ++i) {
            const int b = pq_g_b[i], m = pq_g_mu[i];
            double s[4];
            if constexpr (NCB <= 6) {
                // the link length is uniform: straight-line products whose loads
                // are all in flight together, row by row (measured: the closing
                // took half of this kernel with one round trip per product)
                r2s2_close_any<NCB>(b, N, v, rowP, rowQ, wave, lane, D, s, qsame);
            } else {      // wide rows: the registers of the straight-line form would spill
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    s[r] = 0.0;
                    const int row = wave * 16 + (lane >> 4) + 4 * r;
                    const int P = rowP[row], Q = rowQ[row];
                    if (P >= 0) {
                        Link L;
                        link_rows(b, P, Q, v, L);
#pragma unroll
                        for (int cb = 0; cb < NCB; ++cb) {
                            const int col = cb * 16 + (lane & 15);
                            if (col < N && col != P && col != Q) s[r] += D[cb][r] * link_at(L, col);
                        }
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                for (int o = 8; o > 0; o >>= 1) s[r] += __shfl_xor(s[r], o);
            if ((lane & 15) == 0) {
                const double c = pq_g_coef[i];
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[(wave * 16 + (lane >> 4) + 4 * r) * NP2 + m] += c * s[r];
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < M2_ROWS * NP2; i += 256) {
        const int row = i / NP2, m = i % NP2;
        const long ip = ip0 + row;
        if (ip < np2) part[((long)blockIdx.y * NP2 + m) * np2 + ip] = acc[i];
    }
}

// Same contraction with the whole vertex W_w resident in LDS (N <= 96): the
// groups are ordered by w, so W is staged once per vertex and each group needs
// two barriers (L_a fill, then the MFMA sweep over all A).
template <int NCB>
__global__ __launch_bounds__(256) void k_r2s2w(int N, View v, const double* __restrict__ W,
                                               int gchunk, double* __restrict__ part, const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    constexpr int NC = 16 * NCB;
    const int KP = (N + 3) / 4 * 4;
    extern __shared__ double sm[];
    double* Ws = sm;                       // [KP][NC]
    double* La = Ws + (size_t)KP * NC;     // [M2_ROWS][KP]
    double* acc = La + (size_t)M2_ROWS * KP;  // [M2_ROWS][29]
    __shared__ int rowP[M2_ROWS], rowQ[M2_ROWS];
    const long np2 = (long)N * (N - 1) / 2;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const long ip0 = (long)blockIdx.x * M2_ROWS;
    if (tid < M2_ROWS) {
        int P = -1, Q = -1;
        if (ip0 + tid < np2) decode_pair(ip0 + tid, P, Q);
        rowP[tid] = P;
        rowQ[tid] = Q;
    }
    for (int i = tid; i < M2_ROWS * NP2; i += 256) acc[i] = 0.0;
    const int g0 = blockIdx.y * gchunk, g1 = min(PQ_G_N, g0 + gchunk);
    int curw = -1;
    for (int g = g0; g < g1; ++g) {
        const int w = pq_g_w[g], a = pq_g_a[g];
        __syncthreads();
        if (w != curw) {
            const double* Wg = W + (long)w * v.NN;
            for (int i = tid; i < KP * NC; i += 256) {
                const int A = i / NC, col = i % NC;
                Ws[i] = (A < N && col < N) ? Wg[(long)A * N + col] : 0.0;
            }
            curw = w;
        }
        for (int i = tid; i < M2_ROWS * KP; i += 256) {
            const int row = i / KP, A = i % KP;
            const int P = rowP[row], Q = rowQ[row];
            double x = 0.0;
            if (P >= 0 && A < N && A != P && A != Q) {
                Link L;
                link_rows(a, P, Q, v, L);
                x = link_at(L, A);
            }
            La[i] = x;
        }
        __syncthreads();
        d4 D[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) D[cb] = d4{0.0, 0.0, 0.0, 0.0};
        const double* Lrow = La + (wave * 16 + (lane & 15)) * KP + (lane >> 4);
        const double* Wcol = Ws + (lane >> 4) * NC + (lane & 15);
        for (int k4 = 0; k4 < KP; k4 += 4) {
            const double av = Lrow[k4];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
                D[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Wcol[k4 * NC + cb * 16], D[cb], 0, 0, 0);
        }
        for (int i = pq_g_start[g]; i < pq_g_start[g + 1]; ++i) {
            const int b = pq_g_b[i], m = pq_g_mu[i];
            double s[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                s[r] = 0.0;
                const int row = wave * 16 + (lane >> 4) + 4 * r;
                const int P = rowP[row], Q = rowQ[row];
                if (P >= 0) {
                    Link L;
                    link_rows(b, P, Q, v, L);
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb) {
                        const int col = cb * 16 + (lane & 15);
                        if (col < N && col != P && col != Q) s[r] += D[cb][r] * link_at(L, col);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                for (int o = 8; o > 0; o >>= 1) s[r] += __shfl_xor(s[r], o);
            if ((lane & 15) == 0) {
                const double c = pq_g_coef[i];
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[(wave * 16 + (lane >> 4) + 4 * r) * NP2 + m] += c * s[r];
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < M2_ROWS * NP2; i += 256) {
        const int row = i / NP2, m = i % NP2;
        const long ip = ip0 + row;
        if (ip < np2) part[((long)blockIdx.y * NP2 + m) * np2 + ip] = acc[i];
    }
}

// ----------------------------------------------------------- two-pair outputs
// The no-spectator terms and the one-spectator epilogue of the two-pair
// outputs run in k_r2c (pq_lane.hip): straight-line generated code, one lane
// per output pair.

// packed r from the partial sums, in a fixed order (deterministic)
__global__ void k_final(int N, const double* __restrict__ p1, int nch1,
                        const double* __restrict__ p1s1, int nlane1,
                        const double* __restrict__ p2, const double* __restrict__ ps2, int nchunk,
                        double* __restrict__ R, const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    const long np2 = (long)N * (N - 1) / 2;
    const long n1 = 3L * N;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= n1 + NP2 * np2) return;
    double s = 0.0;
    if (gid < n1) {
        const int k = (int)(gid / N), P = (int)(gid % N);
#pragma unroll 8
        for (int c = 0; c < nch1; ++c) s += p1[((long)c * 3 + k) * N + P];
        for (int c = 0; c < nlane1; ++c) s += p1s1[((long)c * 3 + k) * N + P];
    } else {
        const long g2 = gid - n1;
        const int m = (int)(g2 / np2);
        const long ip = g2 - (long)m * np2;
#pragma unroll 8
        for (int k = pq_lane_m_slot_start[m]; k < pq_lane_m_slot_start[m + 1]; ++k)
            s += p2[(long)pq_lane_m_slots[k] * np2 + ip];
#pragma unroll 8
        for (int c = 0; c < nchunk; ++c) s += ps2[(long)c * NP2 * np2 + g2];
    }
    R[gid] = s;
}

// ------------------------------------------------------------------- energy
__global__ __launch_bounds__(256) void k_energy(int N, View v, double* __restrict__ partial) {
    const long NN = (long)N * N;
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (gid < NN) {
        const int P = (int)(gid / N), Q = (int)(gid % N);
        if (P == Q)
            e = class_sum(pq_e1_start, pq_e1_coef, pq_e1_fac, 0, P, 0, 0, 0, v);
        else
            e = 0.5 * class_sum(pq_e2_start, pq_e2_coef, pq_e2_fac, 0, P, Q, 0, 0, v);
    }
    __shared__ double red[256];
    red[threadIdx.x] = e;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_sum_fixed(const double* __restrict__ partial, int n, double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// ------------------------------------------------------------- denominators
__global__ void k_denom(int N, const double* __restrict__ f, double shift, double* __restrict__ D) {
    const long np2 = (long)N * (N - 1) / 2;
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long n1 = 3L * N;
    if (s >= n1 + NP2 * np2) return;
    const long n2 = 2L * N;
    auto foo = [&](int P) { return f[(long)P * n2 + P]; };
    auto fvv = [&](int P) { return f[(long)(N + P) * n2 + N + P]; };
    double d;
    if (s < n1) {
        const int k = (int)(s / N), P = (int)(s % N);
        d = pq_cnt1[2 * k + 1] * fvv(P) - pq_cnt1[2 * k] * foo(P);
    } else {
        const int m = (int)((s - n1) / np2);
        int P, Q;
        decode_pair((s - n1) % np2, P, Q);
        d = pq_cnt2[4 * m + 1] * fvv(P) - pq_cnt2[4 * m] * foo(P) + pq_cnt2[4 * m + 3] * fvv(Q) -
            pq_cnt2[4 * m + 2] * foo(Q);
    }
    D[s] = d + shift;
}


// =================================================================== adjoint
// Reverse mode of every kernel above: given weights lam on the residual
// outputs (and ew on the energy), accumulate
//   tbar = sum_mu lam_mu dR_mu/dt + ew dE/dt,   and optionally the same for
//   the Hamiltonian vertices, pulled back to f and the packed integrals.
// This is the transposed-residual contraction of the Lagrangian
// L = E + lam . R (Sec. II: lambda truncated like t; Table IV caption).
// Accumulation uses FP64 atomics (order-dependent in the last bits only).
struct AdjView {
    double* tb1;   // [3][N]
    double* tb2;   // [29][N][N]
    double* hb1;   // [PQ_H1_N][N]
    double* hb2;   // [PQ_H2_N][N][N]
    double* Wb;    // [2 PQ_W_N][N][N]
    double* Db;    // [PQ_DR_N][N][N]
    int N;
    long NN;
};

__device__ __forceinline__ void fadj(int code, int L0, int L1, int L2, int L3, const AdjView& a,
                                     double d) {
    const int kind = (code >> 28) & 15;
    const int x = labr((code >> 24) & 15, L0, L1, L2, L3);
    const int y = labr((code >> 20) & 15, L0, L1, L2, L3);
    const long idx = code & 0xFFFF;
    switch (kind) {
        case 1: atomicAdd(&a.tb1[idx * a.N + x], d); break;
        case 2: atomicAdd(&a.tb2[idx * a.NN + (long)x * a.N + y], d); break;
        case 3: atomicAdd(&a.hb1[idx * a.N + x], d); break;
        case 4: atomicAdd(&a.hb2[idx * a.NN + (long)x * a.N + y], d); break;
        case 6: atomicAdd(&a.Wb[idx * a.NN + (long)x * a.N + y], d); break;
        case 7: atomicAdd(&a.Db[idx * a.NN + (long)x * a.N + y], d); break;
        default: break;
    }
}

// adjoint of one interpreted term: d(term)/d(factor k) * w for every factor
__device__ __forceinline__ void term_adj(const int* f, double w, int L0, int L1, int L2, int L3,
                                         const View& v, const AdjView& a) {
    double fv[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) fv[j] = f[j] ? fval(f[j], L0, L1, L2, L3, v) : 1.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        if (!f[k]) continue;
        double d = w;
#pragma unroll
        for (int j = 0; j < 5; ++j)
            if (j != k) d *= fv[j];
        if (d != 0.0) fadj(f[k], L0, L1, L2, L3, a, d);
    }
}

__device__ __forceinline__ void class_adj(const int* start, const double* coef, const int* fac, int m,
                                          double w, int L0, int L1, int L2, int L3, const View& v,
                                          const AdjView& a) {
    if (w == 0.0) return;
    for (int i = start[m]; i < start[m + 1]; ++i) term_adj(fac + 5 * i, w * coef[i], L0, L1, L2, L3, v, a);
}

// one-pair outputs without spectators: weights lam1[k][P] (the one-spectator
// terms are k_r1c_adj's generated code)
__global__ __launch_bounds__(64) void k_r1_adj(int N, View v, const double* __restrict__ lam,
                                                AdjView a) {
    const int P = blockIdx.x, tid = threadIdx.x;
    const double l0 = lam[P], l1 = lam[N + P], l2 = lam[2 * N + P];
    if (tid == 0) {
        class_adj(pq_r1s0_start, pq_r1s0_coef, pq_r1s0_fac, 0, l0, P, 0, 0, 0, v, a);
        class_adj(pq_r1s0_start, pq_r1s0_coef, pq_r1s0_fac, 1, l1, P, 0, 0, 0, v, a);
        class_adj(pq_r1s0_start, pq_r1s0_coef, pq_r1s0_fac, 2, l2, P, 0, 0, 0, v, a);
    }
}

// adjoint of the factorised one-pair two-spectator terms (k_bgemm, k_r1s2_close): per group
// and tile of R1A_PB output pairs P, with M = G Mid recomputed,
//   Mbar(P,j) = sum_i c_i lam_{mu_i}(P) C_i(P,j),  Cbar_i(P,j) += c_i lam_{mu_i}(P) M(P,j),
//   Gbar = Mbar Mid^T,  Midbar += G^T Mbar   (into Fb, the adjoints of F)
constexpr int R1A_PB = 8;

__global__ __launch_bounds__(256) void k_r1s2_adj(int N, const double* __restrict__ F,
                                                  const double* __restrict__ lam,
                                                  double* __restrict__ Fb) {
    extern __shared__ double sm[];
    double* Gs = sm;                     // [R1A_PB][N]
    double* Mbs = Gs + R1A_PB * N;       // [R1A_PB][N]
    const int P0 = blockIdx.x * R1A_PB, g = blockIdx.y, tid = threadIdx.x;
    const long NN = (long)N * N;
    const int gen = pq_r1g_gen[g], mid = pq_r1g_mid[g];
    const double* G = F + (long)gen * NN;
    const double* Mid = F + (long)mid * NN;
    for (int e = tid; e < R1A_PB * N; e += blockDim.x) {
        const int p = e / N, k = e - p * N;
        Gs[e] = (P0 + p < N) ? G[(long)(P0 + p) * N + k] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < R1A_PB * N; e += blockDim.x) {
        const int p = e / N, j = e - p * N, P = P0 + p;
        double mb = 0.0;
        if (P < N) {
            double m = 0.0;
            for (int k = 0; k < N; ++k) m += Gs[p * N + k] * Mid[(long)k * N + j];
            for (int i = pq_r1g_start[g]; i < pq_r1g_start[g + 1]; ++i) {
                const int cl = pq_r1g_cl[i];
                const double w = pq_r1g_coef[i] * lam[(long)pq_r1g_mu[i] * N + P];
                mb += w * F[(long)cl * NN + (long)P * N + j];
                if (w * m != 0.0) atomicAdd(&Fb[(long)cl * NN + (long)P * N + j], w * m);
            }
        }
        Mbs[e] = mb;
    }
    __syncthreads();
    for (int e = tid; e < R1A_PB * N; e += blockDim.x) {
        const int p = e / N, k = e - p * N, P = P0 + p;
        if (P >= N) continue;
        double s = 0.0;
        for (int j = 0; j < N; ++j) s += Mbs[p * N + j] * Mid[(long)k * N + j];
        if (s != 0.0) atomicAdd(&Fb[(long)gen * NN + (long)P * N + k], s);
    }
    for (long e = tid; e < NN; e += blockDim.x) {
        const int k = (int)(e / N), j = (int)(e - (long)k * N);
        double s = 0.0;
#pragma unroll
        for (int p = 0; p < R1A_PB; ++p) s += Gs[p * N + k] * Mbs[p * N + j];
        if (s != 0.0) atomicAdd(&Fb[(long)mid * NN + e], s);
    }
}

// Fb_z(a,b) += Fb_{z transposed}(b,a) for the Z products of the one-pair class
__global__ void k_fold_r1z(int N, double* __restrict__ Fb) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const int a = blockIdx.y, z = blockIdx.z;
    if (b >= N) return;
    const long NN = (long)N * N;
    Fb[(long)(PQ_R1F_Z0 + z) * NN + (long)a * N + b] += Fb[(long)(PQ_R1F_N + z) * NN + (long)b * N + a];
}

__global__ void k_energy_adj(int N, View v, double ew, AdjView a) {
    const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (long)N * N) return;
    const int P = (int)(gid / N), Q = (int)(gid % N);
    if (P == Q)
        class_adj(pq_e1_start, pq_e1_coef, pq_e1_fac, 0, ew, P, 0, 0, 0, v, a);
    else
        class_adj(pq_e2_start, pq_e2_coef, pq_e2_fac, 0, 0.5 * ew, P, Q, 0, 0, v, a);
}

// One-spectator GEMM adjoint on the FP64 matrix cores, gathered per side:
//   SIDE 0: Xbar_x(P,A) += sum_{p = (x,y)} sum_{Q>P} Sbar_p(P,Q) Y_y(Q,A)
//   SIDE 1: Ybar_y(Q,A) += sum_{p = (x,y)} sum_{P<Q} Sbar_p(P,Q) X_x(P,A)
// Workgroup: one 64 x 64 tile (rows P or Q, columns A) and one segment of at
// most 32 pairs sharing x (SIDE 0) or y (SIDE 1); the segment's sum is
// added with one atomic per element.  Sbar is p-major (pq contiguous), so the
// staged rows of Sbar_p, for fixed Q and running P, are contiguous.
constexpr int S1A_T = 64, S1A_KC = 16, S1A_PITCH = S1A_KC + 1;

// The staging is software-pipelined over the flattened (pair, K-chunk)
// steps: each thread loads its four S-bar and four side elements of the next
// step into registers (at clamped, in-bounds addresses) before the current
// step's MFMAs and writes them, masked, to LDS after them.  Same staged values
// and MFMA order as the plain form: the sums are bitwise unchanged.
template <int SIDE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) void k_s1_adj(int N, const double* __restrict__ X,
                                                const double* __restrict__ Y,
                                                const double* __restrict__ Sb, double* __restrict__ out) {
    __shared__ double Us[S1A_T * S1A_PITCH];     // [row][k]: Sbar (SIDE 0) or Sbar^T (SIDE 1)
    __shared__ double Os[S1A_KC * S1A_T];        // [k][A]: Y_y or X_x rows
    const int nAt = (N + S1A_T - 1) / S1A_T;
    const int R0 = (blockIdx.x / nAt) * S1A_T, A0 = (blockIdx.x % nAt) * S1A_T;
    const int item = blockIdx.y;
    const long NN = (long)N * N, np2 = (long)N * (N - 1) / 2;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int i16 = lane & 15, kq = lane >> 4;
    const int j0 = SIDE == 0 ? pq_s1ax_p0[item] : pq_s1ay_i0[item];
    const int j1 = SIDE == 0 ? pq_s1ax_p0[item + 1] : pq_s1ay_i0[item + 1];
    const int p0 = SIDE == 0 ? j0 : pq_s1y_perm[j0];
    const int side = pq_s1pairs[2 * p0 + SIDE];          // x (SIDE 0) or y (SIDE 1)
    // K runs over Q > P (SIDE 0) or P < Q (SIDE 1): skip chunks that are all zero
    const int kbeg = SIDE == 0 ? R0 / S1A_KC * S1A_KC : 0;
    const int kend = SIDE == 0 ? N : min(N, R0 + S1A_T);
    const int nkc = (kend - kbeg + S1A_KC - 1) / S1A_KC;
    const int nstep = (j1 - j0) * nkc;
    d4 D[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) D[cb] = d4{0.0, 0.0, 0.0, 0.0};
    constexpr int NE = S1A_T * S1A_KC / 256;             // elements per thread and side
    double u[NE], o[NE];
    auto coords = [&](int i, int kc, int& row, int& k, int& P, int& Q) {
        const int e = tid + 256 * i;
        if (SIDE == 0) { row = e % S1A_T; k = e / S1A_T; }   // P fastest
        else { k = e % S1A_KC; row = e / S1A_KC; }            // P fastest
        const int R = R0 + row, K = kc + k;
        P = SIDE == 0 ? R : K;
        Q = SIDE == 0 ? K : R;
    };
    auto load = [&](int step) {
        const int j = j0 + step / nkc, kc = kbeg + (step % nkc) * S1A_KC;
        const int p = SIDE == 0 ? j : pq_s1y_perm[j];
        const double* Sp = Sb + (long)p * np2;
        const double* other = SIDE == 0 ? Y + (long)pq_s1pairs[2 * p + 1] * NN
                                        : X + (long)pq_s1pairs[2 * p] * NN;
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            int row, k, P, Q;
            coords(i, kc, row, k, P, Q);
            const bool in = P < Q && Q < N;
            u[i] = Sp[in ? (long)Q * (Q - 1) / 2 + P : 0];
            const int e = tid + 256 * i, kk = e / S1A_T, A = A0 + e % S1A_T, K = kc + kk;
            const bool ino = K < N && A < N;
            o[i] = other[ino ? (long)K * N + A : 0];
        }
    };
    auto store = [&](int step) {
        const int kc = kbeg + (step % nkc) * S1A_KC;
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            int row, k, P, Q;
            coords(i, kc, row, k, P, Q);
            Us[row * S1A_PITCH + k] = (P < Q && Q < N) ? u[i] : 0.0;
            const int e = tid + 256 * i, kk = e / S1A_T, A = A0 + e % S1A_T, K = kc + kk;
            Os[e] = (K < N && A < N) ? o[i] : 0.0;
        }
    };
    if (nstep > 0) load(0);
    for (int step = 0; step < nstep; ++step) {
        __syncthreads();                      // the previous step's operands are consumed
        store(step);
        __syncthreads();
        if (step + 1 < nstep) load(step + 1);     // in flight during this step's MFMAs
#pragma unroll
        for (int k4 = 0; k4 < S1A_KC; k4 += 4) {
            const double av = Us[(wave * 16 + i16) * S1A_PITCH + k4 + kq];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
                D[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Os[(k4 + kq) * S1A_T + cb * 16 + i16], D[cb],
                                                             0, 0, 0);
        }
    }
    double* op = out + (long)side * NN;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int R = R0 + wave * 16 + kq + 4 * r, A = A0 + cb * 16 + i16;
            if (R < N && A < N && R != A && D[cb][r] != 0.0) atomicAdd(&op[(long)R * N + A], D[cb][r]);
        }
}

// adjoint of the factor products X, Y, W
__global__ void k_spec_adj(int N, int which, View v, const double* __restrict__ sb, AdjView a) {
    const int L1 = blockIdx.x * blockDim.x + threadIdx.x;
    const int L0 = blockIdx.y, s = blockIdx.z;
    if (L1 >= N || L0 == L1) return;
    const double d0 = sb[(long)s * v.NN + (long)L0 * N + L1];
    if (d0 == 0.0) return;
    const int* st = spec_start(which);
    const int* fc = spec_fac(which);
    const int b = st[s], n = st[s + 1] - st[s];
    double fv[PQ_SPEC_MAXLEN];
    for (int j = 0; j < n; ++j) fv[j] = fval(fc[b + j], L0, L1, 0, 0, v);
    for (int k = 0; k < n; ++k) {
        double d = d0;
        for (int j = 0; j < n; ++j)
            if (j != k) d *= fv[j];
        fadj(fc[b + k], L0, L1, 0, 0, a, d);
    }
}

// adjoint of the dressed vertices D_k(s,A) = sum_B lambda(s,B) W(A,B):
//   lambda_bar(s,B) += sum_A Dbar(s,A) W(A,B),  W_bar(A,B) += sum_s Dbar(s,A) lambda(s,B)
// (grid.y runs over s for the first and over A for the second)
__global__ void k_dress_adj(int N, const double* __restrict__ lam, const double* __restrict__ W,
                            const double* __restrict__ Db, double* __restrict__ Lamb,
                            double* __restrict__ Wb) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y, k = blockIdx.z;
    if (B >= N) return;
    const long NN = (long)N * N;
    const int li = pq_dr_lam[k], we = pq_dr_w[k];
    const double* Dk = Db + (long)k * NN;
    if (li >= 0) {
        double x = 0.0;
        for (int A = 0; A < N; ++A) x += Dk[(long)r * N + A] * W[(long)we * NN + (long)A * N + B];
        if (x != 0.0) atomicAdd(&Lamb[(long)li * NN + (long)r * N + B], x);
    }
    double y = 0.0;
    for (int s2 = 0; s2 < N; ++s2)
        y += Dk[(long)s2 * N + r] * (li >= 0 ? lam[(long)li * NN + (long)s2 * N + B] : 1.0);
    if (y != 0.0) atomicAdd(&Wb[(long)we * NN + (long)r * N + B], y);
}

// Wbar_s(A,B) += Wbar_{nw+s}(B,A): the transposed vertices' adjoints folded back
__global__ void k_fold_wt(int N, double* __restrict__ Wb) {
    const int B = blockIdx.x * blockDim.x + threadIdx.x;
    const int A = blockIdx.y, s = blockIdx.z;
    if (B >= N) return;
    const long NN = (long)N * N;
    Wb[(long)s * NN + (long)A * N + B] += Wb[(long)(PQ_W_N + s) * NN + (long)B * N + A];
}

// link adjoint: scatter dL * d(prod)/d(factor) into t2bar
__device__ __forceinline__ void link_adj(int s, int P, int Q, int A, double dL, const View& v,
                                         const AdjView& a) {
    if (dL == 0.0) return;
    const int n = pq_ld_n[s];
    double fv[3];
    int who[3], mm[3];
    for (int f = 0; f < n; ++f) {
        mm[f] = pq_ld_m[3 * s + f];
        who[f] = pq_ld_q[3 * s + f] ? Q : P;
        fv[f] = v.t2[(long)mm[f] * v.NN + (long)who[f] * v.N + A];
    }
    for (int k = 0; k < n; ++k) {
        double d = dL;
        for (int j = 0; j < n; ++j)
            if (j != k) d *= fv[j];
        atomicAdd(&a.tb2[(long)mm[k] * a.NN + (long)who[k] * a.N + A], d);
    }
}

// Scatter the adjoint d[r] of link s at (P_r, Q_r, col) for the 4 rows r of
// this lane (rows wave*16 + kq + 4r of the matrix-core layout) into the
// amplitude adjoint: factor k receives d times the other factors.  When the
// wavefront's 16 rows share Q (consecutive output pairs), the Q-side factors
// are summed over the rows first (registers, then lanes 16 and 32 apart) and
// added with one atomic per column.  Control flow is wavefront-uniform.
__device__ __forceinline__ void link_adj4(int s, const int* Pr, const int* Qr, int col, const double* d,
                                          bool qsame, const View& v, const AdjView& a) {
    const int n = pq_ld_n[s];
    const int kq = (threadIdx.x & 63) >> 4;
    bool ok[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) ok[r] = Pr[r] >= 0 && col < v.N && col != Pr[r] && col != Qr[r] && d[r] != 0.0;
    double fv[3][4];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            fv[f][r] = 1.0;
            if (f < n && ok[r]) {
                const int who = pq_ld_q[3 * s + f] ? Qr[r] : Pr[r];
                fv[f][r] = v.t2[(long)pq_ld_m[3 * s + f] * v.NN + (long)who * v.N + col];
            }
        }
    }
    for (int k = 0; k < n; ++k) {
        const int m = pq_ld_m[3 * s + k];
        const bool isq = pq_ld_q[3 * s + k] != 0;
        double c[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            c[r] = ok[r] ? d[r] : 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j)
                if (j != k) c[r] *= fv[j][r];
        }
        if (isq && qsame) {
            double t = (c[0] + c[1]) + (c[2] + c[3]);
            t += __shfl_xor(t, 16);
            t += __shfl_xor(t, 32);
            if (kq == 0 && t != 0.0 && col < v.N) atomicAdd(&a.tb2[(long)m * a.NN + (long)Qr[0] * a.N + col], t);
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (c[r] != 0.0)
                    atomicAdd(&a.tb2[(long)m * a.NN + (long)(isq ? Qr[r] : Pr[r]) * a.N + col], c[r]);
        }
    }
}

// Two-spectator adjoint on the FP64 matrix cores, per block of 64 output
// pairs (4 wavefronts x 16 rows) and chunk of groups (w, a, {b_i}), with the
// forward kernel's staging:
//   V = L_a W                      (MFMA; L_a formed while staging)
//   Lbar_b_i = c_i lam_i V         (scattered into the amplitude adjoint)
//   Lbar_a = Vbar W^T,  Vbar = sum_i c_i lam_i L_b_i  (MFMA; Vbar formed while
//                                   staging, W^T read from the stored transposes)
// The vertex adjoint Wbar += L_a^T Vbar is k_wbar's.  Above 128 pairs the
// output columns (B of V, A of Lbar_a) are split over grid.z, which halves the
// accumulators (one more wavefront per SIMD) at the price of staging L_a and
// Vbar twice.
template <int NCB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_r2s2_adjm(int N, View v, const double* __restrict__ W,
                                                   const double* __restrict__ lam, int gchunk, AdjView a) {
    constexpr int NC = 16 * NCB;
    const int c0 = blockIdx.z * NC;        // this workgroup's output columns c0 .. c0 + NC - 1
    extern __shared__ double sm[];
    double* Ls = sm;                       // [M2_ROWS][M2_KC]: L_a, then Vbar
    double* Ws = Ls + M2_ROWS * M2_KC;     // [M2_KC][NC]: W, then W^T
    __shared__ int rowP[M2_ROWS], rowQ[M2_ROWS];
    __shared__ double lamr[M2_ROWS][NP2];
    const long np2 = (long)N * (N - 1) / 2;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int i16 = lane & 15, kq = lane >> 4;
    const long ip0 = (long)blockIdx.x * M2_ROWS;
    if (tid < M2_ROWS) {
        int P = -1, Q = -1;
        if (ip0 + tid < np2) decode_pair(ip0 + tid, P, Q);
        rowP[tid] = P;
        rowQ[tid] = Q;
    }
    for (int i = tid; i < M2_ROWS * NP2; i += 256) {
        const int r = i / NP2, m = i % NP2;
        lamr[r][m] = (ip0 + r < np2) ? lam[3L * N + (long)m * np2 + ip0 + r] : 0.0;
    }
    __syncthreads();
    int Pr[4], Qr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        Pr[r] = rowP[wave * 16 + kq + 4 * r];
        Qr[r] = rowQ[wave * 16 + kq + 4 * r];
    }
    // rows are consecutive output pairs (Q non-decreasing; missing rows last)
    const bool qsame = rowQ[wave * 16 + 15] >= 0 && rowQ[wave * 16] == rowQ[wave * 16 + 15];
    const int KP = (N + M2_KC - 1) / M2_KC * M2_KC;
    const int g0 = blockIdx.y * gchunk, g1 = min(PQ_G_N, g0 + gchunk);
    for (int g = g0; g < g1; ++g) {
        const int w = pq_g_w[g], sa = pq_g_a[g];
        const int wt = w < PQ_W_N ? w + PQ_W_N : w - PQ_W_N;
        const int ib0 = pq_g_start[g], ib1 = pq_g_start[g + 1];
        d4 D[NCB];
        // V = L_a W
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) D[cb] = d4{0.0, 0.0, 0.0, 0.0};
        for (int kc = 0; kc < KP; kc += M2_KC) {
            {   // the thread's four elements: rows tid/16 + 16 j, one spectator A
                const int A = kc + (tid & 15);
                int Pj[4], Qj[4];
                bool ok[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = (tid >> 4) + 16 * j;
                    const int P = rowP[row], Q = rowQ[row];
                    ok[j] = P >= 0 && A < N && A != P && A != Q;
                    Pj[j] = P >= 0 ? P : 0;
                    Qj[j] = P >= 0 ? Q : 0;
                }
                double x[4];
                link_vals4_any(sa, Pj, Qj, A < N ? A : 0, v, x);
#pragma unroll
                for (int j = 0; j < 4; ++j) Ls[tid + 256 * j] = ok[j] ? x[j] : 0.0;
            }
            const double* Wg = W + (long)w * v.NN;
            for (int i = tid; i < M2_KC * NC; i += 256) {
                const int A = kc + i / NC, col = c0 + i % NC;
                Ws[i] = (A < N && col < N) ? Wg[(long)A * N + col] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int k4 = 0; k4 < M2_KC; k4 += 4) {
                const double av = Ls[(wave * 16 + i16) * M2_KC + k4 + kq];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
                    D[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Ws[(k4 + kq) * NC + cb * 16 + i16], D[cb],
                                                                 0, 0, 0);
            }
            __syncthreads();
        }
        // Lbar_b_i = c_i lam_i V
        for (int ii = ib0; ii < ib1; ++ii) {
            const int b = pq_g_b[ii], mu = pq_g_mu[ii];
            const double c = pq_g_coef[ii];
            double wr[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) wr[r] = c * lamr[wave * 16 + kq + 4 * r][mu];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) {
                double d[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) d[r] = wr[r] * D[cb][r];
                link_adj4(b, Pr, Qr, c0 + cb * 16 + i16, d, qsame, v, a);
            }
        }
        // Lbar_a = Vbar W^T
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) D[cb] = d4{0.0, 0.0, 0.0, 0.0};
        for (int kc = 0; kc < KP; kc += M2_KC) {
            {   // Vbar for the thread's four elements, one B-side link at a time
                const int B = kc + (tid & 15);
                int Pj[4], Qj[4];
                bool ok[4];
                double x[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int row = (tid >> 4) + 16 * j;
                    const int P = rowP[row], Q = rowQ[row];
                    ok[j] = P >= 0 && B < N && B != P && B != Q;
                    Pj[j] = P >= 0 ? P : 0;
                    Qj[j] = P >= 0 ? Q : 0;
                    x[j] = 0.0;
                }
                for (int ii = ib0; ii < ib1; ++ii) {
                    double lv[4];
                    link_vals4_any(pq_g_b[ii], Pj, Qj, B < N ? B : 0, v, lv);
                    const double c = pq_g_coef[ii];
                    const int mu = pq_g_mu[ii];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const double wb = c * lamr[(tid >> 4) + 16 * j][mu];
                        if (wb != 0.0) x[j] += wb * lv[j];
                    }
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) Ls[tid + 256 * j] = ok[j] ? x[j] : 0.0;
            }
            const double* WTg = W + (long)wt * v.NN;     // W^T(B, A) = W(A, B)
            for (int i = tid; i < M2_KC * NC; i += 256) {
                const int B = kc + i / NC, A = c0 + i % NC;
                Ws[i] = (B < N && A < N) ? WTg[(long)B * N + A] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int k4 = 0; k4 < M2_KC; k4 += 4) {
                const double av = Ls[(wave * 16 + i16) * M2_KC + k4 + kq];
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb)
                    D[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Ws[(k4 + kq) * NC + cb * 16 + i16], D[cb],
                                                                 0, 0, 0);
            }
            __syncthreads();
        }
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            double d[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) d[r] = D[cb][r];
            link_adj4(sa, Pr, Qr, c0 + cb * 16 + i16, d, qsame, v, a);
        }
    }
}

// Vertex adjoint of the same groups, a contraction over the output pairs:
//   Wbar_w(A,B) += sum_{P<Q} L_a(P,Q,A) Vbar(P,Q,B),
//   Vbar(P,Q,B) = sum_i c_i lam(PQ, mu_i) L_b_i(P,Q,B)      (zero at A, B in {P,Q})
// on the FP64 matrix cores.  Workgroup: one 64 x 64 tile of (A,B), one group
// and one slice of the pairs; L_a and Vbar are formed per chunk of 16 pairs
// straight from the amplitudes and lambda (thread = (pair, 16 labels));
// wavefront w owns rows A = 16w.. of the tile.  The finished tile is added to
// Wbar with one atomic per element (a few per element over all slices).
constexpr int WB_T = 64, WB_KC = 16, WB_PITCH = WB_KC + 1;

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_wbar(int N, View v, const double* __restrict__ lam,
                                              long per, double* __restrict__ Wb) {
    __shared__ double Ls[WB_T * WB_PITCH];   // [A local][pair in chunk]
    __shared__ double Vs[WB_T * WB_PITCH];   // [B local][pair in chunk]
    const int nBt = (N + WB_T - 1) / WB_T;
    const int A0 = (blockIdx.x / nBt) * WB_T, B0 = (blockIdx.x % nBt) * WB_T;
    const int g = blockIdx.y;
    const long np2 = (long)N * (N - 1) / 2;
    const long k0 = (long)blockIdx.z * per, k1 = min(np2, k0 + per);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int i16 = lane & 15, kq = lane >> 4;
    const int kk = tid >> 4, l = tid & 15;     // staging: pair kk of the chunk, labels l + 16j
    const int a = pq_g_a[g], ib0 = pq_g_start[g], ib1 = pq_g_start[g + 1];
    d4 D[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) D[cb] = d4{0.0, 0.0, 0.0, 0.0};
    for (long kc = k0; kc < k1; kc += WB_KC) {
        const long ip = kc + kk;
        int P = -1, Q = -1;
        if (ip < k1) decode_pair(ip, P, Q);
        double la[4], vb[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) la[j] = vb[j] = 0.0;
        if (P >= 0) {      // straight-line link products, four labels at a time
            int Ac[4], Bc[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int A = A0 + l + 16 * j, B = B0 + l + 16 * j;
                Ac[j] = A < N ? A : 0;
                Bc[j] = B < N ? B : 0;
            }
            double x[4];
            link_row4_any(a, P, Q, Ac, v, x);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int A = A0 + l + 16 * j;
                if (A < N && A != P && A != Q) la[j] = x[j];
            }
            for (int i = ib0; i < ib1; ++i) {
                const double wb = pq_g_coef[i] * lam[3L * N + (long)pq_g_mu[i] * np2 + ip];
                if (wb == 0.0) continue;
                link_row4_any(pq_g_b[i], P, Q, Bc, v, x);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int B = B0 + l + 16 * j;
                    if (B < N && B != P && B != Q) vb[j] += wb * x[j];
                }
            }
        }
        __syncthreads();                      // previous chunk's operands consumed
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            Ls[(l + 16 * j) * WB_PITCH + kk] = la[j];
            Vs[(l + 16 * j) * WB_PITCH + kk] = vb[j];
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < WB_KC; k4 += 4) {
            const double av = Ls[(wave * 16 + i16) * WB_PITCH + k4 + kq];
#pragma unroll
            for (int cb = 0; cb < 4; ++cb)
                D[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Vs[(cb * 16 + i16) * WB_PITCH + k4 + kq],
                                                             D[cb], 0, 0, 0);
        }
    }
    double* out = Wb + (long)pq_g_w[g] * v.NN;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int A = A0 + wave * 16 + kq + 4 * r, B = B0 + cb * 16 + i16;
            if (A < N && B < N && A != B && D[cb][r] != 0.0) atomicAdd(&out[(long)A * N + B], D[cb][r]);
        }
}

// packed tbar from the adjoints of t1 and the mirrored t2
__global__ void k_pack_tbar(int N, const double* __restrict__ tb1, const double* __restrict__ tb2,
                            double* __restrict__ tbar) {
    const long np2 = (long)N * (N - 1) / 2;
    const long n1 = 3L * N;
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n1 + NP2 * np2) return;
    if (s < n1) {
        tbar[s] = tb1[s];
        return;
    }
    const int m = (int)((s - n1) / np2);
    int X, Y;
    decode_pair((s - n1) % np2, X, Y);
    const long NN = (long)N * N;
    tbar[s] = tb2[(long)m * NN + (long)X * N + Y] +
              pq_swap2_sign[m] * tb2[(long)pq_swap2[m] * NN + (long)Y * N + X];
}

// pull the vertex adjoints back to f (general matrix) and the packed integrals
__global__ void k_vertex1_adj(int N, const double* __restrict__ hb1, double* __restrict__ fb,
                              double* __restrict__ erib) {
    const int P = blockIdx.x * blockDim.x + threadIdx.x;
    const int key = blockIdx.y;
    if (P >= N) return;
    const double d = hb1[(long)key * N + P];
    if (d == 0.0) return;
    const long n2 = 2L * N;
    for (int i = pq_h1_start[key]; i < pq_h1_start[key + 1]; ++i) {
        const double w = pq_h1_w[i] * d;
        if (pq_h1_kind[i] == 0) {
            const int p = P + N * (pq_h1_a[i] & 1), q = P + N * (pq_h1_b[i] & 1);
            atomicAdd(&fb[p * n2 + q], w);
        } else {
            atomicAdd(&erib[(long)pq_h1_a[i] * N + P], w);
        }
    }
}

__global__ void k_vertex2_adj(int N, const double* __restrict__ hb2, double* __restrict__ fb,
                              double* __restrict__ erib) {
    const int Q = blockIdx.x * blockDim.x + threadIdx.x;
    const int P = blockIdx.y, key = blockIdx.z;
    if (Q >= N || P == Q) return;
    const long NN = (long)N * N, n2 = 2L * N;
    const double d = hb2[(long)key * NN + (long)P * N + Q];
    if (d == 0.0) return;
    const long np2 = (long)N * (N - 1) / 2;
    const int lo = min(P, Q), hi = max(P, Q);
    const long pidx = (long)hi * (hi - 1) / 2 + lo;
    for (int i = pq_h2_start[key]; i < pq_h2_start[key + 1]; ++i) {
        const double w = pq_h2_w[i] * d;
        if (pq_h2_kind[i] == 0) {
            const int a2 = pq_h2_a[i], b2 = pq_h2_b[i];
            const int p = ((a2 >> 1) ? Q : P) + N * (a2 & 1);
            const int q = ((b2 >> 1) ? Q : P) + N * (b2 & 1);
            atomicAdd(&fb[p * n2 + q], w);
        } else {
            const int u = P < Q ? pq_h2_a[i] : pq_h2_b[i];
            atomicAdd(&erib[6L * N + (long)u * np2 + pidx], w);
        }
    }
}

struct Carve {
    double *t2, *h1, *h2, *h2T, *X, *Y, *S, *W, *Lam, *D, *F1, *M1, *part, *p1, *p1s1, *p2, *epart, *scal;
    int nchunk, gchunk, nblkE, nch1;
};

inline int s2_rowtiles(int N) {
    const long np2 = (long)N * (N - 1) / 2;
    return (int)((np2 + M2_ROWS - 1) / M2_ROWS);
}

// 1-D grid of k_gemm_s1: all (pair, tile group) items, padded to a multiple of 8
inline unsigned gemm_s1_grid(int N) {
    const int nt = (N + 15) / 16, ntile = nt * (nt + 1) / 2;
    const long nitem = (long)((ntile + S1_TPG - 1) / S1_TPG) * PQ_S1PAIRS_N;
    return (unsigned)((nitem + 7) / 8 * 8);
}

inline size_t gemm_s1_lds(int N) {
    const int NR = (N + 15) / 16 * 16;
    return (size_t)(2 * NR * S1_PITCH + 4 * 16 * S1_PITCH) * sizeof(double);
}

// the pipelined form (mode 3): two LDS buffers per side, N <= 128
inline size_t gemm_s1p_lds(int N) {
    const int NR = (N + 15) / 16 * 16;
    return (size_t)(4 * NR * S1_PITCH + 4 * 16 * S1_PITCH) * sizeof(double);
}

inline unsigned bgemm_tile_groups(int N) {
    const int nt = (N + 15) / 16;
    return (unsigned)(nt * ((nt + 3) / 4));
}

// the mode-4 one-spectator GEMM (materialised sides, pipelined staging);
// false, launching nothing, when 16-byte row loads would be misaligned
bool launch_gemm_s1m(hipStream_t s, int N, const double* X, const double* Y, double* S, const int* gate) {
    if (!(N & 1) && ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) & 15) != 0) return false;
    const dim3 gg(gemm_s1_grid(N));
    const size_t lb = gemm_s1_lds(N);
#define PQ_S1M_LAUNCH(NT)                                                                             \
    do {                                                                                              \
        if (N & 1)                                                                                    \
            hipLaunchKernelGGL((k_gemm_s1m<NT, false>), gg, dim3(256), lb, s, N, X, Y, S, gate);      \
        else                                                                                          \
            hipLaunchKernelGGL((k_gemm_s1m<NT, true>), gg, dim3(256), lb, s, N, X, Y, S, gate);       \
    } while (0)
    switch ((N + 15) / 16) {
        case 1: PQ_S1M_LAUNCH(1); break;
        case 2: PQ_S1M_LAUNCH(2); break;
        case 3: PQ_S1M_LAUNCH(3); break;
        case 4: PQ_S1M_LAUNCH(4); break;
        case 5: PQ_S1M_LAUNCH(5); break;
        case 6: PQ_S1M_LAUNCH(6); break;
        case 7: PQ_S1M_LAUNCH(7); break;
        case 8: PQ_S1M_LAUNCH(8); break;
        case 9: PQ_S1M_LAUNCH(9); break;
        case 10: PQ_S1M_LAUNCH(10); break;
        case 11: PQ_S1M_LAUNCH(11); break;
        case 12: PQ_S1M_LAUNCH(12); break;
        case 13: PQ_S1M_LAUNCH(13); break;
        case 14: PQ_S1M_LAUNCH(14); break;
        case 15: PQ_S1M_LAUNCH(15); break;
        default: PQ_S1M_LAUNCH(16); break;
    }
#undef PQ_S1M_LAUNCH
    return true;
}

// allows the largest staging (npair 256) once per process
pqph_status gemm_s1_prepare(pqph_ctx* ctx) {
    static bool done = false;
    if (done) return PQPH_OK;
    hipError_t e = hipFuncSetAttribute((const void*)&k_gemm_s1<false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm_s1_lds(256));
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)&k_gemm_s1<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)gemm_s1_lds(256));
    const void* pipelined[] = {(const void*)&k_gemm_s1p<1>, (const void*)&k_gemm_s1p<2>,
                               (const void*)&k_gemm_s1p<3>, (const void*)&k_gemm_s1p<4>,
                               (const void*)&k_gemm_s1p<5>, (const void*)&k_gemm_s1p<6>,
                               (const void*)&k_gemm_s1p<7>, (const void*)&k_gemm_s1p<8>};
    for (int nt = 1; nt <= 8 && e == hipSuccess; ++nt)
        e = hipFuncSetAttribute(pipelined[nt - 1], hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)gemm_s1p_lds(nt * 16));
#define PQ_S1M_ATTR(NT)                                                                                    \
    if (e == hipSuccess)                                                                                   \
        e = hipFuncSetAttribute((const void*)&k_gemm_s1m<NT, true>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                (int)gemm_s1_lds(NT * 16));                                                \
    if (e == hipSuccess)                                                                                   \
        e = hipFuncSetAttribute((const void*)&k_gemm_s1m<NT, false>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                (int)gemm_s1_lds(NT * 16));
    PQ_S1M_ATTR(9) PQ_S1M_ATTR(10) PQ_S1M_ATTR(11) PQ_S1M_ATTR(12)
    PQ_S1M_ATTR(13) PQ_S1M_ATTR(14) PQ_S1M_ATTR(15) PQ_S1M_ATTR(16)
#undef PQ_S1M_ATTR
    if (e != hipSuccess)
        return pqph_fail(ctx, PQPH_DEVICE, std::string("LDS attribute: ") + hipGetErrorString(e));
    done = true;
    return PQPH_OK;
}


// partial-sum chunks of the one-pair outputs: one from k_r1, one per group from k_r1s2_close
inline int r1_chunks(int N) {
    if (N < 3) return 1;
    return 1 + PQ_R1G_N;   // k_r1, then one partial chunk per one-pair two-spectator group
}

inline size_t r1f_size(int N) {
    return (size_t)(PQ_R1F_N + PQ_R1F_N - PQ_R1F_Z0) * N * N;
}

inline void s2_chunks(int N, int& nchunk, int& gchunk) {
    const int rt = std::max(1, s2_rowtiles(N));
    nchunk = std::min(64, std::max(1, (1024 + rt - 1) / rt));
    gchunk = (PQ_G_N + nchunk - 1) / nchunk;
    nchunk = (PQ_G_N + gchunk - 1) / gchunk;
}

Carve carve(double* ws, int N) {
    const size_t NN = (size_t)N * N, np2 = (size_t)N * (N - 1) / 2;
    Carve c;
    size_t o = 0;
    auto take = [&](size_t n) { size_t at = o; o += n; return ws + at; };
    c.t2 = take(NP2 * NN);
    c.h1 = take((size_t)PQ_H1_N * N);
    c.h2 = take((size_t)PQ_H2_N * NN);
    c.h2T = take((size_t)PQ_H2_N * std::max(np2, (size_t)1));
    c.X = take((size_t)PQ_X_N * NN);                  // materialised sides (mode 2, adjoint)
    c.Y = take((size_t)PQ_Y_N * NN);
    c.S = take((size_t)PQ_S1PAIRS_N * std::max(np2, (size_t)1));
    c.W = take(2 * (size_t)PQ_W_N * NN);              // W and its transposes
    c.Lam = take((size_t)PQ_LAM_N * NN);
    c.D = take((size_t)PQ_DR_N * NN);
    c.F1 = take(r1f_size(N));
    c.M1 = take((size_t)PQ_R1G_N * NN);
    s2_chunks(N, c.nchunk, c.gchunk);
    c.part = take((size_t)c.nchunk * NP2 * std::max(np2, (size_t)1));
    c.nch1 = r1_chunks(N);
    c.p1 = take((size_t)c.nch1 * 3 * N);
    c.p1s1 = take((size_t)r1_lane_chunks() * 3 * N);
    c.p2 = take((size_t)PQ_LANE_NSLOT * std::max(np2, (size_t)1));
    c.nblkE = (int)((NN + 255) / 256);
    c.epart = take(c.nblkE);
    c.scal = take(8);
    return c;
}

size_t carve_size(int N) {
    const size_t NN = (size_t)N * N, np2 = (size_t)N * (N - 1) / 2;
    int nchunk, gchunk;
    s2_chunks(N, nchunk, gchunk);
    const size_t np2m = std::max(np2, (size_t)1);
    return NP2 * NN + (size_t)PQ_H1_N * N +
           ((size_t)PQ_H2_N + PQ_X_N + PQ_Y_N + 2 * PQ_W_N + PQ_LAM_N + PQ_DR_N) * NN +
           ((size_t)PQ_H2_N + PQ_S1PAIRS_N) * np2m + (size_t)nchunk * NP2 * np2m +
           (size_t)r1_chunks(N) * 3 * N + (size_t)PQ_LANE_NSLOT * np2m + (NN + 255) / 256 + 8 + r1f_size(N) +
           (size_t)PQ_R1G_N * NN + (size_t)r1_lane_chunks() * 3 * N;
}

View make_view(const double* t, const Carve& c, int N) {
    View v;
    v.t1 = t;
    v.t2 = c.t2;
    v.h1 = c.h1;
    v.h2 = c.h2;
    v.S = c.S;
    v.W = c.W;
    v.D = c.D;
    v.N = N;
    v.NN = (long)N * N;
    return v;
}

// the bare vertices h1, h2, h2K: functions of f and the integrals only
void launch_vertices(pqph_ctx* ctx, hipStream_t s, int N, const double* h, const double* eri,
                     const Carve& c, const int* gate) {
    const int tb = 64;
    const int gx = (N + tb - 1) / tb;
    hipLaunchKernelGGL(k_vertex1, dim3(gx, PQ_H1_N), dim3(tb), 0, s, N, h, eri, c.h1, gate);
    pqph_mark(ctx);
    if (N > 1) {
        const int nt = (N + V2_TILE - 1) / V2_TILE;
        hipLaunchKernelGGL(k_vertex2, dim3(nt * nt, PQ_H2_N), dim3(256), 0, s, N, h, eri, c.h2, c.h2T,
                           gate);
        pqph_mark(ctx);
    }
}

// vertices (unless the workspace already holds them for h and eri) and the
// mirrored two-pair amplitudes
pqph_status prepare(pqph_ctx* ctx, hipStream_t s, int N, const double* h, const double* eri,
                    const double* t, const Carve& c, const int* gate, bool vertices) {
    if (vertices) launch_vertices(ctx, s, N, h, eri, c, gate);
    if (N > 1) {
        const int tb = 64;
        const int gx = (N + tb - 1) / tb;
        hipLaunchKernelGGL(k_unpack_t2, dim3(gx, N, NP2), dim3(tb), 0, s, N, t, c.t2, gate);
        pqph_mark(ctx);
    }
    PQPH_HIP(ctx, hipGetLastError());
    return PQPH_OK;
}

}  // namespace

size_t pq_ws_doubles(int npair) { return carve_size(npair); }

pqph_status pq_residual_prepare(pqph_ctx* ctx) { return gemm_s1_prepare(ctx); }

pqph_status pq_vertices_ws(pqph_ctx* ctx, hipStream_t s, int N, const double* h,
                           const double* eri, double* ws) {
    launch_vertices(ctx, s, N, h, eri, carve(ws, N), nullptr);
    PQPH_HIP(ctx, hipGetLastError());
    return PQPH_OK;
}

// a private vertex block: h1 [PQ_H1_N][N], h2 [PQ_H2_N][N][N], h2K [PQ_H2_N][C(N,2)]
size_t pq_vertex_doubles(int N) {
    const size_t NN = (size_t)N * N, np2 = (size_t)N * (N - 1) / 2;
    return (size_t)PQ_H1_N * N + (size_t)PQ_H2_N * NN + (size_t)PQ_H2_N * std::max(np2, (size_t)1);
}

namespace {
void vertex_block(double* vtx, int N, Carve& c) {
    c.h1 = vtx;
    c.h2 = c.h1 + (size_t)PQ_H1_N * N;
    c.h2T = c.h2 + (size_t)PQ_H2_N * N * N;
}
}  // namespace

pqph_status pq_vertices_into(pqph_ctx* ctx, hipStream_t s, int N, const double* h,
                             const double* eri, double* vtx) {
    Carve c;
    vertex_block(vtx, N, c);
    launch_vertices(ctx, s, N, h, eri, c, nullptr);
    PQPH_HIP(ctx, hipGetLastError());
    return PQPH_OK;
}

pqph_status pq_residual_ws(pqph_ctx* ctx, hipStream_t s, int N, const double* h,
                           const double* eri, const double* t, double* r, double* ws,
                           const int* gate, int fork, bool vertices, const double* vtx) {
    Carve c = carve(ws, N);
    if (vtx) {               // read-only from here on
        vertex_block(const_cast<double*>(vtx), N, c);
        vertices = false;
    }
    pqph_status st = prepare(ctx, s, N, h, eri, t, c, gate, vertices);
    if (st) return st;
    View v = make_view(t, c, N);
    // the doubly-mixed two-spectator contraction (three-label intermediates)
    const bool mixed = pq_intermediates(ctx, N) == 3;
    const int tb = 64;
    const int gx = (N + tb - 1) / tb;
    const unsigned gsq = (unsigned)((N * N + 255) / 256);
    // Independent branches after the shared vertices and amplitudes: the
    // one-pair outputs (s2) and the dense two-spectator contraction (s1) run
    // beside the main chain (dressing, one-spectator GEMM, its epilogue); the
    // main stream joins both before the final sum.  Serial on s when a gate
    // is given (batched solves) or per-kernel times are taken.
    const bool forked = fork > 0 || (fork < 0 && !ctx->profiling && gate == nullptr && s == ctx->stream);
    hipStream_t s1 = s, s2 = s;
    if (forked) {
        if (pqph_status e_ = pqph_ensure_side(ctx)) return e_;
        s1 = ctx->side[0];
        s2 = ctx->side[1];
        PQPH_HIP(ctx, hipEventRecord(ctx->sev[0], s));
        PQPH_HIP(ctx, hipStreamWaitEvent(s2, ctx->sev[0], 0));
    }
    if (N > 1) {
        const long np2 = (long)N * (N - 1) / 2;
        hipLaunchKernelGGL(k_spec, dim3(gsq, PQ_W_N), dim3(256), 0, s, N, 2, v, c.W, gate);
        pqph_mark(ctx);
        hipLaunchKernelGGL(k_spec, dim3(gsq, PQ_LAM_N), dim3(256), 0, s, N, 4, v, c.Lam, gate);
        pqph_mark(ctx);
        if (forked) {
            PQPH_HIP(ctx, hipEventRecord(ctx->sev[1], s));
            PQPH_HIP(ctx, hipStreamWaitEvent(s1, ctx->sev[1], 0));
        }
        if (pqph_status e_ = gemm_s1_prepare(ctx)) return e_;
        hipLaunchKernelGGL(k_bgemm, dim3(bgemm_tile_groups(N), PQ_DR_N), dim3(256), 0, s, N, 0,
                           c.Lam, c.W, c.D, gate);
        pqph_mark(ctx);
        if (pqph_status e_ = gemm_s1_prepare(ctx)) return e_;
        const int s1m = pq_s1_mode(ctx, N);
        if (s1m == 2 || s1m == 4)     // materialised sides (an empty phase in the other modes)
            hipLaunchKernelGGL(k_spec_xy, dim3((N * N + 511) / 512, PQ_X_N + PQ_Y_N), dim3(256), 0, s, N, v,
                               c.X, c.Y, gate);
        pqph_mark(ctx);
        if (s1m == 3 && (N + 15) / 16 <= 8) {
            const dim3 gg(gemm_s1_grid(N));
            const size_t lb = gemm_s1p_lds(N);
            switch ((N + 15) / 16) {
                case 1: hipLaunchKernelGGL(k_gemm_s1p<1>, gg, dim3(256), lb, s, N, v, c.S, gate); break;
                case 2: hipLaunchKernelGGL(k_gemm_s1p<2>, gg, dim3(256), lb, s, N, v, c.S, gate); break;
                case 3: hipLaunchKernelGGL(k_gemm_s1p<3>, gg, dim3(256), lb, s, N, v, c.S, gate); break;
                case 4: hipLaunchKernelGGL(k_gemm_s1p<4>, gg, dim3(256), lb, s, N, v, c.S, gate); break;
                case 5: hipLaunchKernelGGL(k_gemm_s1p<5>, gg, dim3(256), lb, s, N, v, c.S, gate); break;
                case 6: hipLaunchKernelGGL(k_gemm_s1p<6>, gg, dim3(256), lb, s, N, v, c.S, gate); break;
                case 7: hipLaunchKernelGGL(k_gemm_s1p<7>, gg, dim3(256), lb, s, N, v, c.S, gate); break;
                default: hipLaunchKernelGGL(k_gemm_s1p<8>, gg, dim3(256), lb, s, N, v, c.S, gate); break;
            }
        } else if (s1m == 4 && launch_gemm_s1m(s, N, c.X, c.Y, c.S, gate)) {
            // (16-byte loads of even-N rows need 16-byte aligned sides; else mode 2 below)
        } else if (s1m == 2 || s1m == 4) {
            hipLaunchKernelGGL(k_gemm_s1<false>, dim3(gemm_s1_grid(N)), dim3(256), gemm_s1_lds(N), s, N, v,
                               c.X, c.Y, c.S, gate);
        } else {
            hipLaunchKernelGGL(k_gemm_s1<true>, dim3(gemm_s1_grid(N)), dim3(256), gemm_s1_lds(N), s, N, v,
                               nullptr, nullptr, c.S, gate);
        }
        pqph_mark(ctx);
        dim3 g2(s2_rowtiles(N), c.nchunk);
        const int ncb = (N + 15) / 16;
        const int variant = pq_s2_variant(ctx, N);
        if (!mixed) {
            // two-pair-intermediate model: the doubly-mixed terms are left out
        } else if (variant == 2 && ncb <= 6) {
            const int KP = (N + 3) / 4 * 4;
            auto ldsw = [&](int ncb_) {
                return (size_t)(KP * 16 * ncb_ + M2_ROWS * KP + M2_ROWS * NP2) * sizeof(double);
            };
#define PQ_S2W_LAUNCH(NB)                                                                       \
    do {                                                                                        \
        const size_t bytes = ldsw(NB);                                                          \
        if (bytes > 64 * 1024) {                                                                \
            hipError_t e_ = hipFuncSetAttribute((const void*)&k_r2s2w<NB>,                       \
                                                hipFuncAttributeMaxDynamicSharedMemorySize,     \
                                                (int)bytes);                                    \
            if (e_ != hipSuccess)                                                               \
                return pqph_fail(ctx, PQPH_DEVICE, std::string("LDS attribute: ") +             \
                                                       hipGetErrorString(e_));                  \
        }                                                                                       \
        hipLaunchKernelGGL(k_r2s2w<NB>, g2, dim3(256), bytes, s1, N, v, c.W, c.gchunk, c.part,  \
                           gate);                                                       \
    } while (0)
            if (ncb <= 1) PQ_S2W_LAUNCH(1);
            else if (ncb <= 2) PQ_S2W_LAUNCH(2);
            else if (ncb <= 3) PQ_S2W_LAUNCH(3);
            else if (ncb <= 4) PQ_S2W_LAUNCH(4);
            else if (ncb <= 5) PQ_S2W_LAUNCH(5);
            else PQ_S2W_LAUNCH(6);
#undef PQ_S2W_LAUNCH
        } else {
            auto lds = [](int ncb_) {
                return (size_t)(M2_ROWS * M2_KC + M2_KC * 16 * ncb_ + M2_ROWS * NP2) * sizeof(double);
            };
#define PQ_S2_LAUNCH(NB)                                                                       \
    hipLaunchKernelGGL(k_r2s2<NB>, g2, dim3(256), lds(NB), s1, N, v, c.W, c.gchunk, c.part, \
                       gate)
            if (ncb <= 1) PQ_S2_LAUNCH(1);
            else if (ncb <= 2) PQ_S2_LAUNCH(2);
            else if (ncb <= 3) PQ_S2_LAUNCH(3);
            else if (ncb <= 4) PQ_S2_LAUNCH(4);
            else if (ncb <= 5) PQ_S2_LAUNCH(5);
            else if (ncb <= 6) PQ_S2_LAUNCH(6);
            else if (ncb <= 8) PQ_S2_LAUNCH(8);
            else if (ncb <= 10) PQ_S2_LAUNCH(10);
            else if (ncb <= 13) PQ_S2_LAUNCH(13);
            else PQ_S2_LAUNCH(16);
#undef PQ_S2_LAUNCH
        }
        pqph_mark(ctx);
        if (forked) PQPH_HIP(ctx, hipEventRecord(ctx->sev[2], s1));
        launch_r2_lane(s, N, t, c.h1, c.h2T, c.S, c.p2, gate);
        pqph_mark(ctx);
    }
    if (N >= 3) {
        hipLaunchKernelGGL(k_spec_r1, dim3(gsq, PQ_R1F_N), dim3(256), 0, s2, N, v, c.F1, gate);
        pqph_mark(ctx);
        hipLaunchKernelGGL(k_bgemm, dim3(bgemm_tile_groups(N), PQ_R1G_N), dim3(256), 0, s2, N, 1,
                           c.F1, c.F1, c.M1, gate);
        pqph_mark(ctx);
        hipLaunchKernelGGL(k_r1s2_close, dim3(N, PQ_R1G_N), dim3(64), 0, s2, N, c.F1, c.M1, c.p1, 1,
                           gate);
        pqph_mark(ctx);
    }
    hipLaunchKernelGGL(k_r1, dim3(N), dim3(64), 0, s2, N, v, c.p1, gate);
    pqph_mark(ctx);
    launch_r1_lane(s2, N, t, c.t2, c.h1, c.h2, c.p1s1, gate);
    pqph_mark(ctx);
    if (forked) {
        PQPH_HIP(ctx, hipEventRecord(ctx->sev[3], s2));
        PQPH_HIP(ctx, hipStreamWaitEvent(s, ctx->sev[3], 0));
        if (N > 1) PQPH_HIP(ctx, hipStreamWaitEvent(s, ctx->sev[2], 0));
    }
    {
        const long ntot = 3L * N + (long)NP2 * N * (N - 1) / 2;
        hipLaunchKernelGGL(k_final, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, s, N, c.p1,
                           c.nch1, c.p1s1, r1_lane_chunks(), c.p2, c.part, (N > 1 && mixed) ? c.nchunk : 0, r,
                           gate);
    }

    pqph_mark(ctx);
    PQPH_HIP(ctx, hipGetLastError());
    return PQPH_OK;
}

pqph_status pq_energy_ws(pqph_ctx* ctx, hipStream_t s, int N, const double* h,
                         const double* eri, const double* t, double* dst, double* ws) {
    Carve c = carve(ws, N);
    pqph_status st = prepare(ctx, s, N, h, eri, t, c, nullptr, true);
    if (st) return st;
    View v = make_view(t, c, N);
    hipLaunchKernelGGL(k_energy, dim3(c.nblkE), dim3(256), 0, s, N, v, c.epart);
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, s, c.epart, c.nblkE, dst);
    PQPH_HIP(ctx, hipGetLastError());
    return PQPH_OK;
}

pqph_status pq_denominators_dev(pqph_ctx* ctx, hipStream_t s, int N, const double* h,
                                double shift, double* D) {
    const long n = (long)pq_amp_len(N);
    hipLaunchKernelGGL(k_denom, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N,
                       h, shift, D);
    PQPH_HIP(ctx, hipGetLastError());
    return PQPH_OK;
}


// ------------------------------------------------------------------ adjoint
size_t pq_adj_doubles(int N) {
    const size_t NN = (size_t)N * N, np2 = std::max((size_t)N * (N - 1) / 2, (size_t)1);
    return 3 * (size_t)N + NP2 * NN + (size_t)PQ_H1_N * N +
           ((size_t)PQ_H2_N + PQ_X_N + PQ_Y_N + 2 * PQ_W_N + PQ_DR_N + PQ_LAM_N) * NN +
           r1f_size(N) + (size_t)PQ_S1PAIRS_N * np2 + 8;
}

pqph_status pq_vjp_ws(pqph_ctx* ctx, hipStream_t s, int N, const double* h, const double* eri,
                      const double* t, const double* lam, double ew, double* tbar, double* hbar,
                      double* eribar, double* ws, double* aws, bool fwd_ready) {
    Carve c = carve(ws, N);
    if (!fwd_ready) {
        pqph_status st = prepare(ctx, s, N, h, eri, t, c, nullptr, true);
        if (st) return st;
    }
    View v = make_view(t, c, N);
    const size_t NN = (size_t)N * N, np2 = (size_t)N * (N - 1) / 2;
    AdjView a;
    a.N = N;
    a.NN = (long)NN;
    double* p = aws;
    a.tb1 = p; p += 3 * (size_t)N;
    a.tb2 = p; p += NP2 * NN;
    a.hb1 = p; p += (size_t)PQ_H1_N * N;
    a.hb2 = p; p += (size_t)PQ_H2_N * NN;
    double* Xb = p; p += (size_t)PQ_X_N * NN;
    double* Yb = p; p += (size_t)PQ_Y_N * NN;
    double* Wb = p; p += 2 * (size_t)PQ_W_N * NN;      // adjoints of W and of its transposes
    double* Db = p; p += (size_t)PQ_DR_N * NN;
    double* Lamb = p; p += (size_t)PQ_LAM_N * NN;
    double* F1b = p; p += r1f_size(N);
    a.Wb = Wb;
    a.Db = Db;
    double* Sb = p;
    // the one-spectator sides, materialised (their adjoints need them as operands)
    double* Xf = c.X;
    double* Yf = c.Y;
    const size_t nzero = (size_t)(Sb - aws);
    PQPH_HIP(ctx, hipMemsetAsync(aws, 0, nzero * sizeof(double), s));
    const int tb = 64, gx = (N + tb - 1) / tb;
    const unsigned gsq = (unsigned)((N * N + 255) / 256);
    if (N > 1) {
        if (!fwd_ready) {      // the forward intermediates the adjoint reads (functions of h, v, t)
            hipLaunchKernelGGL(k_spec, dim3(gsq, PQ_W_N), dim3(256), 0, s, N, 2, v, c.W, nullptr);
            hipLaunchKernelGGL(k_spec, dim3(gsq, PQ_LAM_N), dim3(256), 0, s, N, 4, v, c.Lam, nullptr);
            if (pqph_status e_ = gemm_s1_prepare(ctx)) return e_;
            hipLaunchKernelGGL(k_bgemm, dim3(bgemm_tile_groups(N), PQ_DR_N), dim3(256), 0, s, N, 0,
                               c.Lam, c.W, c.D, nullptr);
            hipLaunchKernelGGL(k_spec_xy, dim3((N * N + 511) / 512, PQ_X_N + PQ_Y_N), dim3(256), 0, s, N, v,
                               Xf, Yf, nullptr);
            if (!launch_gemm_s1m(s, N, Xf, Yf, c.S, nullptr))   // bitwise the S of mode 2
                hipLaunchKernelGGL(k_gemm_s1<false>, dim3(gemm_s1_grid(N)), dim3(256), gemm_s1_lds(N), s, N, v,
                                   Xf, Yf, c.S, nullptr);
        }
        launch_r2_lane_adj(s, N, t, c.h1, c.h2T, c.S, lam, a.tb1, a.tb2, a.hb1, a.hb2, Sb);
        if (pq_intermediates(ctx, N) == 3) {      // adjoint of the doubly-mixed terms
            const int rt2 = s2_rowtiles(N);
            const int nchunk = std::max(1, std::min(PQ_G_N, 2048 / std::max(rt2, 1)));
            const int gchunk = (PQ_G_N + nchunk - 1) / nchunk;
            auto ldsa = [](int ncb_) { return (size_t)(M2_ROWS * M2_KC + M2_KC * 16 * ncb_) * sizeof(double); };
            const int ncb = (N + 15) / 16;
            const int nsplit = ncb > 8 ? 2 : 1;          // column halves above 128 pairs
            const int nbh = (ncb + nsplit - 1) / nsplit;
            const dim3 ga(rt2, (PQ_G_N + gchunk - 1) / gchunk, nsplit);
#define PQ_S2A_LAUNCH(NB) \
    hipLaunchKernelGGL(k_r2s2_adjm<NB>, ga, dim3(256), ldsa(NB), s, N, v, c.W, lam, gchunk, a)
            switch (nbh) {
                case 1: PQ_S2A_LAUNCH(1); break;
                case 2: PQ_S2A_LAUNCH(2); break;
                case 3: PQ_S2A_LAUNCH(3); break;
                case 4: PQ_S2A_LAUNCH(4); break;
                case 5: PQ_S2A_LAUNCH(5); break;
                case 6: PQ_S2A_LAUNCH(6); break;
                case 7: PQ_S2A_LAUNCH(7); break;
                default: PQ_S2A_LAUNCH(8); break;
            }
#undef PQ_S2A_LAUNCH
            // vertex adjoint: about 2048 workgroups of (tile, group, pair slice)
            const int nt64 = (N + WB_T - 1) / WB_T;
            const long np2l = (long)N * (N - 1) / 2;
            const int nslice = (int)std::max(1L, std::min((np2l + WB_KC - 1) / WB_KC,
                                                          2048L / (nt64 * nt64 * PQ_G_N)));
            const long per = ((np2l + nslice - 1) / nslice + WB_KC - 1) / WB_KC * WB_KC;
            hipLaunchKernelGGL(k_wbar, dim3(nt64 * nt64, PQ_G_N, (unsigned)((np2l + per - 1) / per)),
                               dim3(256), 0, s, N, v, lam, per, Wb);
        }
        {
            const int nAt = (N + S1A_T - 1) / S1A_T;
            hipLaunchKernelGGL(k_s1_adj<0>, dim3(nAt * nAt, PQ_S1AX_N), dim3(256), 0, s, N, Xf, Yf, Sb, Xb);
            hipLaunchKernelGGL(k_s1_adj<1>, dim3(nAt * nAt, PQ_S1AY_N), dim3(256), 0, s, N, Xf, Yf, Sb, Yb);
        }
        hipLaunchKernelGGL(k_spec_adj, dim3(gx, N, PQ_X_N), dim3(tb), 0, s, N, 0, v, Xb, a);
        hipLaunchKernelGGL(k_spec_adj, dim3(gx, N, PQ_Y_N), dim3(tb), 0, s, N, 1, v, Yb, a);
        hipLaunchKernelGGL(k_dress_adj, dim3(gx, N, PQ_DR_N), dim3(tb), 0, s, N, c.Lam, c.W, Db, Lamb,
                           Wb);
        hipLaunchKernelGGL(k_spec_adj, dim3(gx, N, PQ_LAM_N), dim3(tb), 0, s, N, 4, v, Lamb, a);
        hipLaunchKernelGGL(k_fold_wt, dim3(gx, N, PQ_W_N), dim3(tb), 0, s, N, Wb);
        hipLaunchKernelGGL(k_spec_adj, dim3(gx, N, PQ_W_N), dim3(tb), 0, s, N, 2, v, Wb, a);
    }
    hipLaunchKernelGGL(k_r1_adj, dim3(N), dim3(64), 0, s, N, v, lam, a);
    launch_r1_lane_adj(s, N, t, c.t2, c.h1, c.h2, lam, a.tb1, a.tb2, a.hb1, a.hb2);
    if (N >= 3) {
        const unsigned gsq3 = (unsigned)((N * N + 255) / 256);
        if (!fwd_ready)
            hipLaunchKernelGGL(k_spec_r1, dim3(gsq3, PQ_R1F_N), dim3(256), 0, s, N, v, c.F1, nullptr);
        hipLaunchKernelGGL(k_r1s2_adj, dim3((N + R1A_PB - 1) / R1A_PB, PQ_R1G_N), dim3(256),
                           (size_t)2 * R1A_PB * N * sizeof(double), s, N, c.F1, lam, F1b);
        hipLaunchKernelGGL(k_fold_r1z, dim3(gx, N, PQ_R1F_N - PQ_R1F_Z0), dim3(tb), 0, s, N, F1b);
        hipLaunchKernelGGL(k_spec_adj, dim3(gx, N, PQ_R1F_N), dim3(tb), 0, s, N, 5, v, F1b, a);
    }
    if (ew != 0.0)
        hipLaunchKernelGGL(k_energy_adj, dim3((unsigned)((NN + 255) / 256)), dim3(256), 0, s, N, v, ew,
                           a);
    {
        const long ntot = 3L * N + (long)NP2 * (long)np2;
        hipLaunchKernelGGL(k_pack_tbar, dim3((unsigned)((ntot + 255) / 256)), dim3(256), 0, s, N,
                           a.tb1, a.tb2, tbar);
    }
    if (hbar || eribar) {
        if (!hbar || !eribar) return pqph_fail(ctx, PQPH_INVALID_ARG, "hbar and eribar go together");
        PQPH_HIP(ctx, hipMemsetAsync(hbar, 0, 4 * NN * sizeof(double), s));
        PQPH_HIP(ctx, hipMemsetAsync(eribar, 0, pq_eri_len(N) * sizeof(double), s));
        hipLaunchKernelGGL(k_vertex1_adj, dim3(gx, PQ_H1_N), dim3(tb), 0, s, N, a.hb1, hbar, eribar);
        if (N > 1)
            hipLaunchKernelGGL(k_vertex2_adj, dim3(gx, N, PQ_H2_N), dim3(tb), 0, s, N, a.hb2, hbar,
                               eribar);
    }
    PQPH_HIP(ctx, hipGetLastError());
    return PQPH_OK;
}
