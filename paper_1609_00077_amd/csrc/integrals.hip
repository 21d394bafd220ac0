// Integral transformation into pair blocks (Sec. III, RI/CD paragraph).
//
// For a zero-differential-overlap site Hamiltonian the three-index factor of
// the orbital pair (p, q) is X[pq][i] = C[i][p] C[i][q] on site i and the
// metric is the site interaction matrix V, so (pq|rs) = sum_ij X[pq][i] V[i][j]
// X[rs][j].  Y[rs][i] = sum_j V[i][j] X[rs][j] (npq x n times n x n) is the one
// dense contraction and runs on the FP64 matrix cores (v_mfma_f64_16x16x4f64),
// as does f = C^T F C.  Both factors are kept pair-major (one contiguous
// row of n site values per orbital pair), so each stored integral is a dot
// product of two contiguous rows; one workgroup per label set stages the rows of its orbital pairs in
// LDS and forms exactly the integrals of that set, so only the integrals of
// label sets of at most k pairs are ever formed.
#include "pqph_internal.h"
#include "pq_tables.h"

#include <algorithm>

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int GT = 64;        // output tile (GT x GT) per workgroup
constexpr int GK = 32;        // K chunk staged in LDS
constexpr int GP = GK + 1;    // LDS row pitch (doubles)

// C[m][n] = sum_k A(m, k) B(n, k) with A(m, k) = A[m*sam + k*sak] and
// B(n, k) = B[n*sbn + k*sbk]: any of C = A B, A^T B, A B^T through the
// strides.  256 threads = 4 wavefronts, each owning a 32 x 32 quarter of the
// 64 x 64 tile as 2 x 2 blocks of 16 x 16 MFMA accumulators.  MFMA operand
// layout: lane l supplies A(i, k) and B(j, k) with i, j = l & 15 and
// k = l >> 4; accumulator register r holds C((l >> 4) + 4r, l & 15).
// Workgroups are dealt out XCD by XCD (workgroup b runs on XCD b mod 8), so
// tiles sharing rows of A sit on one XCD and share its L2.
__global__ __launch_bounds__(256) void k_dgemm_nt(int M, int Nn, int K, const double* __restrict__ A,
                                                  long sam, long sak, const double* __restrict__ B,
                                                  long sbn, long sbk, double* __restrict__ C, long ldc,
                                                  int ntn, int ntiles) {
    __shared__ double As[GT * GP];
    __shared__ double Bs[GT * GP];
    const int per = (ntiles + 7) / 8;
    const int tile = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
    if (tile >= ntiles) return;
    const int m0 = (tile / ntn) * GT, n0 = (tile % ntn) * GT;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    d4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += GK) {
        __syncthreads();
        // consecutive threads read consecutive addresses: along k when the k
        // stride is 1, along the rows otherwise
        for (int e = tid; e < GT * GK; e += 256) {
            const int r = sak == 1 ? e / GK : e % GT, k = sak == 1 ? e % GK : e / GT;
            const int m = m0 + r, kk = k0 + k;
            As[r * GP + k] = (m < M && kk < K) ? A[m * sam + kk * sak] : 0.0;
        }
        for (int e = tid; e < GT * GK; e += 256) {
            const int r = sbk == 1 ? e / GK : e % GT, k = sbk == 1 ? e % GK : e / GT;
            const int n = n0 + r, kk = k0 + k;
            Bs[r * GP + k] = (n < Nn && kk < K) ? B[n * sbn + kk * sbk] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k4 = 0; k4 < GK; k4 += 4) {
            const double a0 = As[(wm + li) * GP + k4 + lk], a1 = As[(wm + 16 + li) * GP + k4 + lk];
            const double b0 = Bs[(wn + li) * GP + k4 + lk], b1 = Bs[(wn + 16 + li) * GP + k4 + lk];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * a + lk + 4 * r, n = n0 + wn + 16 * b + li;
                if (m < M && n < Nn) C[(long)m * ldc + n] = acc[a][b][r];
            }
}

// CT = C^T (n x n), 32 x 32 tiles through LDS: coalesced reads and writes
__global__ __launch_bounds__(256) void k_transpose(int n, const double* __restrict__ C,
                                                   double* __restrict__ CT) {
    __shared__ double tl[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8)
        if (by + r < n && bx + tx < n) tl[r][tx] = C[(long)(by + r) * n + bx + tx];
    __syncthreads();
    for (int r = ty; r < 32; r += 8)
        if (bx + r < n && by + tx < n) CT[(long)(bx + r) * n + by + tx] = tl[tx][r];
}

// X[pq][i] = C[i][p] C[i][q] = CT[p][i] CT[q][i], pq = p(p+1)/2 + q, p >= q:
// one workgroup per orbital pair (grid-stride), threads over the sites, so
// reads and writes are contiguous
__global__ void k_pair_factor(int n, const double* __restrict__ CT, double* __restrict__ X) {
    const long npq = (long)n * (n + 1) / 2;
    for (long pq = blockIdx.x; pq < npq; pq += gridDim.x) {
        int p = (int)((sqrt(8.0 * (double)pq + 1.0) - 1.0) * 0.5);
        while ((long)p * (p + 1) / 2 > pq) --p;
        while ((long)(p + 1) * (p + 2) / 2 <= pq) ++p;
        const int q = (int)(pq - (long)p * (p + 1) / 2);
        const double* cp = CT + (long)p * n;
        const double* cq = CT + (long)q * n;
        for (int i = threadIdx.x; i < n; i += blockDim.x) X[pq * n + i] = cp[i] * cq[i];
    }
}

__device__ __forceinline__ long compound(int p, int q) {
    if (p < q) { int t = p; p = q; q = t; }
    return (long)p * (p + 1) / 2 + q;
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

// One workgroup per label set of `size` pairs (set index blockIdx.x, label
// sets in packed order): the X and Y rows of every orbital pair of the set's
// 2*size orbitals are staged in LDS (3, 10 or 21 pairs), then each wavefront
// forms stored integrals of the set, one per round, as a fixed-order dot over
// the sites (lanes strided over i, shuffle reduction).
__global__ __launch_bounds__(256) void k_pack_sets(int N, int size, long nsets, long off,
                                                   const double* __restrict__ X,
                                                   const double* __restrict__ Y, double* __restrict__ out) {
    extern __shared__ double lds[];
    const int n = 2 * N;
    const int norb = 2 * size, npl = norb * (norb + 1) / 2;
    const int nq = size == 1 ? 6 : (size == 2 ? 43 : 84);
    const int* quads = size == 1 ? pqph_quads1 : (size == 2 ? pqph_quads2 : pqph_quads3);
    const long si = blockIdx.x;
    int lab[3];
    decode_set(size, si, lab);
    double* Xs = lds;
    double* Ys = lds + (long)npl * n;
    __shared__ long grow[21];
    if (threadIdx.x < npl) {
        const int a = threadIdx.x;
        int p = 0;
        while ((p + 1) * (p + 2) / 2 <= a) ++p;
        const int q = a - p * (p + 1) / 2;
        grow[a] = compound(lab[p >> 1] + N * (p & 1), lab[q >> 1] + N * (q & 1)) * n;
    }
    __syncthreads();
    // one flat loop over (row, site): every thread keeps several loads in flight
    for (int e = threadIdx.x; e < npl * n; e += blockDim.x) {
        const int a = e / n, i = e - a * n;
        Xs[e] = X[grow[a] + i];
        Ys[e] = Y[grow[a] + i];
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int u = wave; u < nq; u += 4) {
        const int p = quads[4 * u], q = quads[4 * u + 1], r = quads[4 * u + 2], s = quads[4 * u + 3];
        const int a = (p >= q) ? p * (p + 1) / 2 + q : q * (q + 1) / 2 + p;
        const int b = (r >= s) ? r * (r + 1) / 2 + s : s * (s + 1) / 2 + r;
        const double* xr = Xs + (long)a * n;
        const double* yr = Ys + (long)b * n;
        double acc = 0.0;
        for (int i = lane; i < n; i += 64) acc += xr[i] * yr[i];
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (lane == 0) out[off + (long)u * nsets + si] = acc;
    }
}

size_t pack_lds_bytes(int N, int size) {
    const int norb = 2 * size, npl = norb * (norb + 1) / 2;
    return (size_t)2 * npl * 2 * N * sizeof(double);
}

void launch_dgemm_nt(hipStream_t s, int M, int Nn, int K, const double* A, long sam, long sak,
                     const double* B, long sbn, long sbk, double* C, long ldc) {
    const int ntm = (M + GT - 1) / GT, ntn = (Nn + GT - 1) / GT, ntiles = ntm * ntn;
    const int grid = 8 * ((ntiles + 7) / 8);
    hipLaunchKernelGGL(k_dgemm_nt, dim3(grid), dim3(256), 0, s, M, Nn, K, A, sam, sak, B, sbn, sbk, C,
                       ldc, ntn, ntiles);
}

}  // namespace

extern "C" pqph_status pqph_integrals(pqph_ctx* ctx, int npair, int k, const double* F,
                                      const double* V, const double* C, double* f_out,
                                      double* eri_out) {
    if (!ctx) return pqph_fail(nullptr, PQPH_INVALID_ARG, "null context");
    if (k != 2 && k != 3) return pqph_fail(ctx, PQPH_INVALID_ARG, "k must be 2 (PQ) or 3 (PH)");
    // the staged rows of one label set must fit in LDS (160 KB per CU)
    const int nmax = k == 2 ? 256 : 240;
    if (npair < 1 || npair > nmax)
        return pqph_fail(ctx, PQPH_INVALID_ARG,
                         std::string("npair must be in [1, ") + std::to_string(nmax) + "] for k = " +
                             std::to_string(k));
    if (!F || !V || !C || !f_out || !eri_out) return pqph_fail(ctx, PQPH_INVALID_ARG, "null array");
    PQPH_HIP(ctx, hipSetDevice(ctx->device));
    const int n = 2 * npair;
    const long npq = (long)n * (n + 1) / 2;
    const size_t need = 2 * (size_t)n * n + 2 * (size_t)n * npq;
    pqph_status st = pqph_ensure_ws(ctx, need * sizeof(double));
    if (st) return st;
    static bool lds_set = false;
    if (!lds_set) {
        const hipError_t e = hipFuncSetAttribute((const void*)&k_pack_sets,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)pack_lds_bytes(240, 3));
        if (e != hipSuccess)
            return pqph_fail(ctx, PQPH_DEVICE, std::string("LDS attribute: ") + hipGetErrorString(e));
        lds_set = true;
    }
    double* CT = ctx->ws;
    double* TT = CT + (size_t)n * n;
    double* X = TT + (size_t)n * n;
    double* Y = X + (size_t)n * npq;
    hipStream_t s = ctx->stream;
    hipLaunchKernelGGL(k_transpose, dim3((n + 31) / 32, (n + 31) / 32), dim3(256), 0, s, n, C, CT);
    // f = C^T F C with every operand read along its rows:
    // TT[p][a] = sum_b CT[p][b] F[a][b], f[p][q] = sum_a CT[p][a] TT[q][a]
    launch_dgemm_nt(s, n, n, n, CT, n, 1, F, n, 1, TT, n);
    launch_dgemm_nt(s, n, n, n, CT, n, 1, TT, n, 1, f_out, n);
    // X (pair-major), then Y[rs][i] = sum_j V[i][j] X[rs][j]
    hipLaunchKernelGGL(k_pair_factor, dim3((unsigned)std::min<long>(npq, 65535)), dim3(128), 0, s, n,
                       CT, X);
    launch_dgemm_nt(s, (int)npq, n, n, X, n, 1, V, n, 1, Y, n);
    long off = 0;
    for (int size = 1; size <= std::min(k, npair); ++size) {
        long nsets = npair;
        if (size == 2) nsets = (long)npair * (npair - 1) / 2;
        if (size == 3) nsets = (long)npair * (npair - 1) * (npair - 2) / 6;
        hipLaunchKernelGGL(k_pack_sets, dim3((unsigned)nsets), dim3(256), pack_lds_bytes(npair, size), s,
                           npair, size, nsets, off, X, Y, eri_out);
        off += (size == 1 ? 6 : (size == 2 ? 43 : 84)) * nsets;
    }
    PQPH_HIP(ctx, hipGetLastError());
    return PQPH_OK;
}
