// Integral transformation into pair blocks (Sec. III, RI/CD paragraph).
//
// For a zero-differential-overlap site Hamiltonian the three-index factor of
// the pair (p, q) is X[i][pq] = C[i][p] C[i][q] on site i and the metric is the
// site interaction matrix V, so (pq|rs) = sum_ij X[i][pq] V[i][j] X[j][rs].
// Y = V X is a dense FP64 GEMM; each stored integral of the packed pair-block
// layout is then one column dot product sum_i X[i][pq] Y[i][rs], so only the
// integrals of label sets of at most k pairs are ever formed.
#include "pqph_internal.h"
#include "pq_tables.h"

#include <algorithm>

namespace {

constexpr int TS = 16;

// C = op(A) * B with op(A) = A or A^T; A is (m x k) or (k x m), B is (k x n)
__global__ __launch_bounds__(256) void k_gemm(int m, int n, int kdim, bool transA,
                                              const double* __restrict__ A, int lda,
                                              const double* __restrict__ B, int ldb,
                                              double* __restrict__ C, int ldc) {
    __shared__ double As[TS][TS + 1];
    __shared__ double Bs[TS][TS + 1];
    const int ty = threadIdx.x / TS, tx = threadIdx.x % TS;
    const int row = blockIdx.y * TS + ty, col = blockIdx.x * TS + tx;
    double acc = 0.0;
    for (int k0 = 0; k0 < kdim; k0 += TS) {
        const int ka = k0 + tx;
        double a = 0.0;
        if (row < m && ka < kdim) a = transA ? A[(size_t)ka * lda + row] : A[(size_t)row * lda + ka];
        As[ty][tx] = a;
        const int kb = k0 + ty;
        Bs[ty][tx] = (kb < kdim && col < n) ? B[(size_t)kb * ldb + col] : 0.0;
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TS; ++kk) acc += As[ty][kk] * Bs[kk][tx];
        __syncthreads();
    }
    if (row < m && col < n) C[(size_t)row * ldc + col] = acc;
}

// X[i][pq] = C[i][p] C[i][q], pq = p(p+1)/2 + q, p >= q
__global__ void k_pair_factor(int n, const double* __restrict__ C, double* __restrict__ X) {
    const size_t npq = (size_t)n * (n + 1) / 2;
    const int i = blockIdx.y;
    for (size_t pq = (size_t)blockIdx.x * blockDim.x + threadIdx.x; pq < npq;
         pq += (size_t)gridDim.x * blockDim.x) {
        int p = (int)((sqrt(8.0 * (double)pq + 1.0) - 1.0) * 0.5);
        while ((size_t)p * (p + 1) / 2 > pq) --p;
        while ((size_t)(p + 1) * (p + 2) / 2 <= pq) ++p;
        const int q = (int)(pq - (size_t)p * (p + 1) / 2);
        X[(size_t)i * npq + pq] = C[(size_t)i * n + p] * C[(size_t)i * n + q];
    }
}

__device__ __forceinline__ size_t compound(int p, int q) {
    if (p < q) { int t = p; p = q; q = t; }
    return (size_t)p * (p + 1) / 2 + q;
}

__device__ void decode_set(int size, long si, int* lab) {
    if (size == 1) {
        lab[0] = (int)si;
        return;
    }
    if (size == 2) {
        int q = (int)((1.0 + sqrt(1.0 + 8.0 * (double)si)) * 0.5);
        while ((long)q * (q - 1) / 2 > si) --q;
        while ((long)(q + 1) * q / 2 <= si) ++q;
        lab[1] = q;
        lab[0] = (int)(si - (long)q * (q - 1) / 2);
        return;
    }
    int r = 2;
    while ((long)(r + 1) * r * (r - 1) / 6 <= si) ++r;
    long rest = si - (long)r * (r - 1) * (r - 2) / 6;
    int q = 1;
    while ((long)(q + 1) * q / 2 <= rest) ++q;
    lab[2] = r;
    lab[1] = q;
    lab[0] = (int)(rest - (long)q * (q - 1) / 2);
}

__global__ void k_pack_eri(int N, int k, const double* __restrict__ X, const double* __restrict__ Y,
                           double* __restrict__ out) {
    const int n = 2 * N;
    const size_t npq = (size_t)n * (n + 1) / 2;
    const long n1 = 6L * N, n2 = 43L * N * (N - 1) / 2;
    const long n3 = (k >= 3) ? 84L * N * (N - 1) * (N - 2) / 6 : 0;
    const long total = n1 + n2 + n3;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        int size;
        long off, nsets;
        const int* quads;
        if (e < n1) {
            size = 1; off = 0; nsets = N; quads = pqph_quads1;
        } else if (e < n1 + n2) {
            size = 2; off = n1; nsets = (long)N * (N - 1) / 2; quads = pqph_quads2;
        } else {
            size = 3; off = n1 + n2; nsets = (long)N * (N - 1) * (N - 2) / 6; quads = pqph_quads3;
        }
        const long u = (e - off) / nsets, si = (e - off) % nsets;
        int lab[3];
        decode_set(size, si, lab);
        int g[4];
        for (int x = 0; x < 4; ++x) {
            const int loc = quads[4 * u + x];
            g[x] = lab[loc >> 1] + N * (loc & 1);
        }
        const size_t pq = compound(g[0], g[1]), rs = compound(g[2], g[3]);
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += X[(size_t)i * npq + pq] * Y[(size_t)i * npq + rs];
        out[e] = s;
    }
}

}  // namespace

extern "C" pqph_status pqph_integrals(pqph_ctx* ctx, int npair, int k, const double* F,
                                      const double* V, const double* C, double* f_out,
                                      double* eri_out) {
    if (!ctx) return pqph_fail(nullptr, PQPH_INVALID_ARG, "null context");
    if (npair < 1 || npair > 4096 || (k != 2 && k != 3))
        return pqph_fail(ctx, PQPH_INVALID_ARG, "npair must be >= 1 and k 2 or 3");
    if (!F || !V || !C || !f_out || !eri_out) return pqph_fail(ctx, PQPH_INVALID_ARG, "null array");
    PQPH_HIP(ctx, hipSetDevice(ctx->device));
    const int n = 2 * npair;
    const size_t npq = (size_t)n * (n + 1) / 2;
    const size_t need = (size_t)n * n + 2 * (size_t)n * npq;
    pqph_status st = pqph_ensure_ws(ctx, need * sizeof(double));
    if (st) return st;
    double* T = ctx->ws;
    double* X = T + (size_t)n * n;
    double* Y = X + (size_t)n * npq;
    hipStream_t s = ctx->stream;
    const dim3 b(256);
    // f = C^T (F C)
    hipLaunchKernelGGL(k_gemm, dim3((n + TS - 1) / TS, (n + TS - 1) / TS), b, 0, s, n, n, n, false,
                       F, n, C, n, T, n);
    hipLaunchKernelGGL(k_gemm, dim3((n + TS - 1) / TS, (n + TS - 1) / TS), b, 0, s, n, n, n, true,
                       C, n, T, n, f_out, n);
    // X, then Y = V X
    const int gx = (int)std::min<size_t>(4096, (npq + 255) / 256);
    hipLaunchKernelGGL(k_pair_factor, dim3(gx, n), b, 0, s, n, C, X);
    hipLaunchKernelGGL(k_gemm, dim3((unsigned)((npq + TS - 1) / TS), (n + TS - 1) / TS), b, 0, s, n,
                       (int)npq, n, false, V, n, X, (int)npq, Y, (int)npq);
    const size_t total = (k == 2) ? pq_eri_len(npair) : ph_eri_len(npair);
    hipLaunchKernelGGL(k_pack_eri, dim3((unsigned)std::min<size_t>(8192, (total + 255) / 256)), b, 0,
                       s, npair, k, X, Y, eri_out);
    PQPH_HIP(ctx, hipGetLastError());
    return PQPH_OK;
}
