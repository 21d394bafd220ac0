// Adjoint of the two-pair outputs' no- and one-spectator terms (the terms of
// k_r2c, Sec. II residual), one lane per output pair.
//
// The terms are generated straight-line code (pq_lane_adj_code.h) grouped by
// streamed factor over all outputs: each streamed factor -- h1 of P or Q, h2
// of the pair, a one-spectator sum S_p of the pair -- lives in exactly one
// chunk, whose lane computes its whole adjoint (lam-weighted sum over the
// terms that use it) and writes it once: Sbar_p and h2bar(P,Q) are owned by
// the lane (plain stores), the per-label h1 adjoints are atomics.  The
// adjoints of the pair's 35 staged amplitudes are summed over the four
// chunks of a workgroup in LDS, then added to the amplitude adjoints with
// one atomic per (pair, amplitude).
#include "pqph_internal.h"
#include "pq_tables.h"
#include "pq_lane_adj_code.h"

namespace {

__global__ __launch_bounds__(256) void k_r2c_adj(int N, const double* __restrict__ t,
                                                 const double* __restrict__ h1,
                                                 const double* __restrict__ h2K,
                                                 const double* __restrict__ SK,
                                                 const double* __restrict__ lam, double* __restrict__ tb1,
                                                 double* __restrict__ tb2, double* __restrict__ hb1,
                                                 double* __restrict__ hb2, double* __restrict__ SbK) {
    __shared__ double red[64][PQ_LANE_ONE + 1];
    const long np2 = (long)N * (N - 1) / 2, NN = (long)N * N;
    const int lane = threadIdx.x & 63;
    const long ip = (long)blockIdx.x * 64 + lane;
    const int c = blockIdx.y * 4 + (threadIdx.x >> 6);
    for (int i = threadIdx.x; i < 64 * (PQ_LANE_ONE + 1); i += 256) (&red[0][0])[i] = 0.0;
    __syncthreads();
    const bool ok = ip < np2 && c < PQ_LANEA_NCHUNK;
    int P = 0, Q = 1;
    if (ip < np2) decode_pair(ip, P, Q);
    if (ok) {
        double x[PQ_LANE_NLOC], gx[PQ_LANE_NLOC];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            x[i] = t[(long)i * N + P];
            x[3 + i] = t[(long)i * N + Q];
        }
#pragma unroll
        for (int i = PQ_LANE_T2; i < PQ_LANE_ONE; ++i) x[i] = t[3L * N + (long)(i - PQ_LANE_T2) * np2 + ip];
        x[PQ_LANE_ONE] = 1.0;
#pragma unroll
        for (int i = 0; i < PQ_LANE_NLOC; ++i) gx[i] = 0.0;
        PQ_LANEA_SWITCH(c, x, gx, lam, h1, h2K, SK, hb1, hb2, SbK, (long)N, NN, np2, (long)P, (long)Q, ip)
#pragma unroll
        for (int i = 0; i < PQ_LANE_ONE; ++i)
            if (gx[i] != 0.0) atomicAdd(&red[lane][i], gx[i]);
    }
    __syncthreads();
    if (ip >= np2) return;
    for (int i = threadIdx.x >> 6; i < PQ_LANE_ONE; i += 4) {
        const double g = red[lane][i];
        if (g == 0.0) continue;
        if (i < 3) atomicAdd(&tb1[(long)i * N + P], g);
        else if (i < PQ_LANE_T2) atomicAdd(&tb1[(long)(i - 3) * N + Q], g);
        else atomicAdd(&tb2[(long)(i - PQ_LANE_T2) * NN + (long)P * N + Q], g);
    }
}

}  // namespace

void launch_r2_lane_adj(hipStream_t s, int npair, const double* t, const double* h1, const double* h2K,
                        const double* SK, const double* lam, double* tb1, double* tb2, double* hb1,
                        double* hb2, double* SbK) {
    const long np2 = (long)npair * (npair - 1) / 2;
    if (np2 < 1) return;
    hipLaunchKernelGGL(k_r2c_adj, dim3((unsigned)((np2 + 63) / 64), (PQ_LANEA_NCHUNK + 3) / 4), dim3(256), 0,
                       s, npair, t, h1, h2K, SK, lam, tb1, tb2, hb1, hb2, SbK);
}
