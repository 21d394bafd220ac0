// No-spectator terms and one-spectator epilogue of the two-pair outputs
// (Sec. II residual, the terms whose factors all belong to the output pair
// (P, Q) itself), one lane per output pair.
//
// Every term is one streamed factor -- h1 of P or Q, h2 of the pair, or a
// one-spectator sum S_p of the pair, read from k-major arrays so that a
// wavefront's 64 consecutive pairs load 512 contiguous bytes -- times at most
// four amplitudes of the pair.  The amplitudes are held in registers and the
// terms are generated straight-line code (pq_lane_code.h, one function per
// chunk of terms), so a term costs a few multiplies and no table or LDS
// traffic.  A chunk serves a cluster of up to 8 outputs that share streamed
// sums S_p, so each S_p is loaded once per cluster rather than once per
// output.  Workgroup: 64 pairs x 4 chunks (one per wavefront); each chunk's
// sums go to its output slots part[slot][pq], combined per output in a fixed
// order.
#include "pqph_internal.h"
#include "pq_tables.h"
#include "pq_lane_code.h"

namespace {

__global__ __launch_bounds__(256) void k_r2c(int N, const double* __restrict__ t,
                                             const double* __restrict__ h1,
                                             const double* __restrict__ h2K,
                                             const double* __restrict__ SK,
                                             double* __restrict__ part, const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    const long np2 = (long)N * (N - 1) / 2;
    const long ip = (long)blockIdx.x * 64 + (threadIdx.x & 63);
    const int c = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (c >= PQ_LANE_NCHUNK) return;
    const long ipc = ip < np2 ? ip : np2 - 1;
    int P, Q;
    decode_pair(ipc, P, Q);
    double x[PQ_LANE_NLOC];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        x[i] = t[(long)i * N + P];
        x[3 + i] = t[(long)i * N + Q];
    }
#pragma unroll
    for (int i = PQ_LANE_T2; i < PQ_LANE_ONE; ++i) x[i] = t[3L * N + (long)(i - PQ_LANE_T2) * np2 + ipc];
    x[PQ_LANE_ONE] = 1.0;
    double acc[PQ_LANE_MAXOUT];
#pragma unroll
    for (int j = 0; j < PQ_LANE_MAXOUT; ++j) acc[j] = 0.0;
    PQ_LANE_SWITCH(c, x, acc, h1, h2K, SK, (long)N, np2, (long)P, (long)Q, ipc)
    const int s0 = pq_lane_ch_slot0[c], ns = pq_lane_ch_slot0[c + 1] - s0;
    if (ip < np2) {
#pragma unroll
        for (int j = 0; j < PQ_LANE_MAXOUT; ++j)
            if (j < ns) part[(long)(s0 + j) * np2 + ip] = acc[j];
    }
}

// One-pair outputs, one spectator: one workgroup per output pair P, one
// wavefront per chunk of terms, lanes over the spectator A (A = lane + 64 j).
// The staged amplitudes of P, A and (P, A) are in registers, the vertices
// h1(A) and h2(P, A) are streamed (contiguous over A), the terms are
// generated straight-line code.  Each wavefront reduces its lanes in a fixed
// shuffle order and writes part[chunk][k][P].
__global__ __launch_bounds__(256) void k_r1c(int N, const double* __restrict__ t,
                                             const double* __restrict__ t2,
                                             const double* __restrict__ h1,
                                             const double* __restrict__ h2,
                                             double* __restrict__ part, const int* __restrict__ gate) {
    if (gate && *gate == 0) return;   // chain finished (batched solves)
    const long NN = (long)N * N;
    const int P = blockIdx.x, c = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (c >= PQ_R1L_NCHUNK) return;
    double sum[3] = {0.0, 0.0, 0.0};
    for (int A = lane; A < N; A += 64) {
        if (A == P) continue;
        double x[36];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            x[i] = t[(long)i * N + P];
            x[3 + i] = t[(long)i * N + A];
        }
        const long e = (long)P * N + A;
#pragma unroll
        for (int m = 0; m < 29; ++m) x[6 + m] = t2[(long)m * NN + e];
        x[35] = 1.0;
        double acc[3] = {0.0, 0.0, 0.0};
        PQ_R1L_SWITCH(c, x, acc, h1, h2, (long)N, NN, (long)P, (long)A)
#pragma unroll
        for (int k = 0; k < 3; ++k) sum[k] += acc[k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
        for (int o = 32; o > 0; o >>= 1) sum[k] += __shfl_xor(sum[k], o);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) part[((long)c * 3 + k) * N + P] = sum[k];
    }
}

// Adjoint of the one-pair one-spectator terms: thread (P, A), lam-weighted
// generated code (r1_adj_code).  Targets only this thread touches -- the
// adjoints of t2(P,A) and of h2(P,A) -- are plain read-modify-writes (kernels
// on one stream run in order); those of the per-label vectors are atomics,
// the P ones after a wavefront reduction.
__global__ __launch_bounds__(64) void k_r1c_adj(int N, const double* __restrict__ t,
                                                const double* __restrict__ t2,
                                                const double* __restrict__ h1,
                                                const double* __restrict__ h2,
                                                const double* __restrict__ lam, double* __restrict__ tb1,
                                                double* __restrict__ tb2, double* __restrict__ hb1,
                                                double* __restrict__ hb2) {
    const long NN = (long)N * N;
    const int P = blockIdx.x, lane = threadIdx.x;
    const int A = blockIdx.y * 64 + lane;
    const bool ok = A < N && A != P;
    const int Ac = ok ? A : (P == 0 ? 1 : 0);          // a valid label for the idle lanes' loads
    double x[36], gx[36];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        x[i] = t[(long)i * N + P];
        x[3 + i] = t[(long)i * N + Ac];
    }
    const long e = (long)P * N + Ac;
#pragma unroll
    for (int m = 0; m < 29; ++m) x[6 + m] = t2[(long)m * NN + e];
    x[35] = 1.0;
#pragma unroll
    for (int i = 0; i < 36; ++i) gx[i] = 0.0;
    const double l[3] = {lam[P], lam[N + P], lam[2L * N + P]};
    if (ok) r1_adj_code(x, l, gx, h1, h2, hb1, hb2, (long)N, NN, (long)P, (long)A);
    if (ok) {
#pragma unroll
        for (int m = 0; m < 29; ++m)
            if (gx[6 + m] != 0.0) tb2[(long)m * NN + e] += gx[6 + m];
#pragma unroll
        for (int i = 0; i < 3; ++i)
            if (gx[3 + i] != 0.0) atomicAdd(&tb1[(long)i * N + A], gx[3 + i]);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double g = gx[i];
        for (int o = 32; o > 0; o >>= 1) g += __shfl_xor(g, o);
        if (lane == 0 && g != 0.0) atomicAdd(&tb1[(long)i * N + P], g);
    }
}

}  // namespace

void launch_r1_lane(hipStream_t s, int N, const double* t, const double* t2, const double* h1,
                    const double* h2, double* part, const int* gate) {
    hipLaunchKernelGGL(k_r1c, dim3(N), dim3(64 * PQ_R1L_NCHUNK), 0, s, N, t, t2, h1, h2, part, gate);
}

int r1_lane_chunks() { return PQ_R1L_NCHUNK; }

void launch_r1_lane_adj(hipStream_t s, int npair, const double* t, const double* t2, const double* h1,
                        const double* h2, const double* lam, double* tb1, double* tb2, double* hb1,
                        double* hb2) {
    if (npair < 2) return;
    hipLaunchKernelGGL(k_r1c_adj, dim3(npair, (npair + 63) / 64), dim3(64), 0, s, npair, t, t2, h1, h2, lam,
                       tb1, tb2, hb1, hb2);
}

void launch_r2_lane(hipStream_t s, int N, const double* t, const double* h1, const double* h2K,
                    const double* SK, double* part, const int* gate) {
    const long np2 = (long)N * (N - 1) / 2;
    hipLaunchKernelGGL(k_r2c, dim3((unsigned)((np2 + 63) / 64), (PQ_LANE_NCHUNK + 3) / 4), dim3(256), 0, s,
                       N, t, h1, h2K, SK, part, gate);
}
