// Streaming kernels of the Jacobi/DIIS solver (Table IV: denominator
// application; Sec. III: DIIS), shared by the single and batched solves.
#include "pqph_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace {
// ------------------------------------------------------------ vector kernels
__global__ void k_dot_partial(const double* __restrict__ a, const double* __restrict__ b, size_t n,
                              double* __restrict__ partial) {
    __shared__ double red[256];
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        s += a[i] * b[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// out[j] = sum of partial[j*nblk .. (j+1)*nblk)
__global__ void k_sum_rows(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) s += partial[(size_t)j * nblk + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = red[0];
}

// e = -r/D ; tn = t + e ; also ||r||^2 partials are computed separately
__global__ void k_jacobi(const double* __restrict__ t, const double* __restrict__ r,
                         const double* __restrict__ D, size_t n, double* __restrict__ tn,
                         double* __restrict__ e) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const double d = -r[i] / D[i];
        e[i] = d;
        tn[i] = t[i] + d;
    }
}

// One Jacobi/DIIS step in one pass: e = -r/D into the new history slot
// eh[slot], tn = t + e, and the block partials of ||r||^2 (row 0) and of
// e . eh[j] for the m history vectors (rows 1..m; the new slot from the
// register value): wavefront sums, then the four wavefronts in a fixed order.
__global__ __launch_bounds__(256) void k_step(const double* __restrict__ t, const double* __restrict__ r,
                                              const double* __restrict__ D, size_t n, double* __restrict__ tn,
                                              double* __restrict__ eh, int m, int slot,
                                              double* __restrict__ partial) {
    double sr = 0.0, sg[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) sg[j] = 0.0;
    double* es = eh + (size_t)slot * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const double ri = r[i];
        const double d = -ri / D[i];
        es[i] = d;
        tn[i] = t[i] + d;
        sr += ri * ri;
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (j < m) sg[j] += (j == slot ? d : eh[(size_t)j * n + i]) * d;
    }
    __shared__ double red[4][17];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 17; ++j) {
        if (j <= m) {
            double v = j == 0 ? sr : sg[j > 0 ? j - 1 : 0];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
            if (lane == 0) red[wv][j] = v;
        }
    }
    __syncthreads();
    const int j = threadIdx.x;
    if (j <= m) partial[(size_t)j * gridDim.x + blockIdx.x] = (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
}

// t = sum_i c[i] * hist[slot_i]
__global__ void k_combine(const double* __restrict__ hist, const double* __restrict__ c, int m,
                          size_t n, double* __restrict__ t) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += c[j] * hist[(size_t)j * n + i];
        t[i] = s;
    }
}

// t = sum_j c.v[j] hist[j], the coefficients passed by value (m <= 16)
struct Coef16 {
    double v[16];
};
__global__ void k_combine_v(const double* __restrict__ hist, Coef16 c, int m, size_t n,
                            double* __restrict__ t) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += c.v[j] * hist[(size_t)j * n + i];
        t[i] = s;
    }
}

// several dot products against one vector: out[j] partials for a[j] . b
__global__ void k_dots_partial(const double* __restrict__ A, int m, const double* __restrict__ b,
                               size_t n, int nblk, double* __restrict__ partial) {
    __shared__ double red[256];
    const int j = blockIdx.y;
    double s = 0.0;
    const double* a = A + (size_t)j * n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        s += a[i] * b[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t)j * nblk + blockIdx.x] = red[0];
}


// Solve the (m+1) x (m+1) DIIS system with partial pivoting; false if singular.
bool diis_solve_impl(const std::vector<double>& B, int m, std::vector<double>& c) {
    const int n = m + 1;
    std::vector<double> A((size_t)n * (n + 1));
    double scale = 0.0;
    for (int i = 0; i < m; ++i) scale = std::max(scale, std::fabs(B[(size_t)i * 16 + i]));
    if (!(scale > 0.0)) return false;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) {
            double v;
            if (i < m && j < m) v = B[(size_t)i * 16 + j] / scale;
            else if (i == m && j == m) v = 0.0;
            else v = -1.0;
            A[(size_t)i * (n + 1) + j] = v;
        }
        A[(size_t)i * (n + 1) + n] = (i == m) ? -1.0 : 0.0;
    }
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int i = col + 1; i < n; ++i)
            if (std::fabs(A[(size_t)i * (n + 1) + col]) > std::fabs(A[(size_t)piv * (n + 1) + col]))
                piv = i;
        if (std::fabs(A[(size_t)piv * (n + 1) + col]) < 1e-300) return false;
        if (piv != col)
            for (int j = 0; j <= n; ++j)
                std::swap(A[(size_t)piv * (n + 1) + j], A[(size_t)col * (n + 1) + j]);
        for (int i = 0; i < n; ++i) {
            if (i == col) continue;
            const double fct = A[(size_t)i * (n + 1) + col] / A[(size_t)col * (n + 1) + col];
            for (int j = col; j <= n; ++j) A[(size_t)i * (n + 1) + j] -= fct * A[(size_t)col * (n + 1) + j];
        }
    }
    c.assign(m, 0.0);
    for (int i = 0; i < m; ++i) c[i] = A[(size_t)i * (n + 1) + n] / A[(size_t)i * (n + 1) + i];
    for (double x : c)
        if (!std::isfinite(x)) return false;
    return true;
}

__global__ void k_absmin_partial(const double* __restrict__ a, size_t n, double* __restrict__ partial) {
    __shared__ double red[256];
    double s = INFINITY;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        s = fmin(s, fabs(a[i]));
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + k]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_min_rows(const double* __restrict__ partial, int nblk, double* __restrict__ out) {
    __shared__ double red[256];
    double s = INFINITY;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) s = fmin(s, partial[i]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + k]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}
}  // namespace

void launch_absmin(hipStream_t s, const double* a, size_t n, double* part, int nblk, double* out) {
    hipLaunchKernelGGL(k_absmin_partial, dim3(nblk), dim3(256), 0, s, a, n, part);
    hipLaunchKernelGGL(k_min_rows, dim3(1), dim3(256), 0, s, part, nblk, out);
}

int stream_blocks(size_t n) { return (int)std::min<size_t>(1024, (n + 255) / 256); }

bool diis_solve(const std::vector<double>& B, int m, std::vector<double>& c) {
    return diis_solve_impl(B, m, c);
}

void launch_norm2(hipStream_t s, const double* r, size_t n, double* part, int nblk, double* out) {
    hipLaunchKernelGGL(k_dot_partial, dim3(nblk), dim3(256), 0, s, r, r, n, part);
    hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, s, part, nblk, out);
}

void launch_jacobi(hipStream_t s, const double* t, const double* r, const double* D, size_t n,
                   double* tn, double* e) {
    hipLaunchKernelGGL(k_jacobi, dim3(stream_blocks(n)), dim3(256), 0, s, t, r, D, n, tn, e);
}

void launch_gram(hipStream_t s, const double* eh, int m, const double* enew, size_t n, double* part,
                 int nblk, double* out) {
    hipLaunchKernelGGL(k_dots_partial, dim3(nblk, m), dim3(256), 0, s, eh, m, enew, n, nblk, part);
    hipLaunchKernelGGL(k_sum_rows, dim3(m), dim3(256), 0, s, part, nblk, out);
}

void launch_step(hipStream_t s, const double* t, const double* r, const double* D, size_t n, double* tn,
                 double* eh, int m, int slot, double* part, int nblk, double* out) {
    hipLaunchKernelGGL(k_step, dim3(nblk), dim3(256), 0, s, t, r, D, n, tn, eh, m, slot, part);
    hipLaunchKernelGGL(k_sum_rows, dim3(m + 1), dim3(256), 0, s, part, nblk, out);
}

void launch_combine(hipStream_t s, const double* th, const double* c, int m, size_t n, double* t) {
    hipLaunchKernelGGL(k_combine, dim3(stream_blocks(n)), dim3(256), 0, s, th, c, m, n, t);
}

void launch_combine_host(hipStream_t s, const double* th, const double* c, int m, size_t n, double* t) {
    Coef16 cv;
    for (int j = 0; j < 16; ++j) cv.v[j] = j < m ? c[j] : 0.0;
    hipLaunchKernelGGL(k_combine_v, dim3(stream_blocks(n)), dim3(256), 0, s, th, cv, m, n, t);
}

// gamma_pp += 2 for the occupied orbitals p < npair: the reference part of
// the one-particle density (the correlation part is dE/df)
__global__ void k_add_reference_occupation(double* __restrict__ gamma, int npair) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < npair) gamma[(size_t)p * 2 * npair + p] += 2.0;
}

void launch_add_reference_occupation(hipStream_t s, double* gamma, int npair) {
    hipLaunchKernelGGL(k_add_reference_occupation, dim3((npair + 255) / 256), dim3(256), 0, s, gamma,
                       npair);
}

// f = diag(-1 on the occupied orbitals p < npair, 0 elsewhere): with it the
// denominator kernels give D = (number of holes) = the excitation rank
__global__ void k_rank_fock(double* __restrict__ f, int npair) {
    const long n = 2L * npair;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * n) return;
    const long p = i / n, q = i % n;
    f[i] = (p == q && p < npair) ? -1.0 : 0.0;
}

// r[s] = 0 where rank[s] > max_rank (excitations outside the kept ranks)
__global__ void k_rank_mask(double* __restrict__ r, const double* __restrict__ rank, int max_rank,
                            size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        if (rank[i] > max_rank + 0.5) r[i] = 0.0;
}

void launch_rank_fock(hipStream_t s, double* f, int npair) {
    const long n2 = 4L * npair * npair;
    hipLaunchKernelGGL(k_rank_fock, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s, f, npair);
}

void launch_rank_mask(hipStream_t s, double* r, const double* rank, int max_rank, size_t n) {
    const unsigned g = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_rank_mask, dim3(g), dim3(256), 0, s, r, rank, max_rank, n);
}

// out = a x + b y (y may be null), optionally with y divided elementwise by D
__global__ void k_axpby(double* __restrict__ out, double a, const double* __restrict__ x, double b,
                        const double* __restrict__ y, const double* __restrict__ D, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double v = a * x[i];
        if (y) v += b * (D ? y[i] / D[i] : y[i]);
        out[i] = v;
    }
}

// y -= sum_j c[j] V[j] (c in device memory, m vectors of length n)
__global__ void k_sub_combine(double* __restrict__ y, const double* __restrict__ V,
                              const double* __restrict__ c, int m, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < m; ++j) s += c[j] * V[(size_t)j * n + i];
        y[i] -= s;
    }
}

void launch_axpby(hipStream_t s, double* out, double a, const double* x, double b, const double* y,
                  const double* D, size_t n) {
    hipLaunchKernelGGL(k_axpby, dim3(stream_blocks(n)), dim3(256), 0, s, out, a, x, b, y, D, n);
}

void launch_sub_combine(hipStream_t s, double* y, const double* V, const double* c, int m, size_t n) {
    hipLaunchKernelGGL(k_sub_combine, dim3(stream_blocks(n)), dim3(256), 0, s, y, V, c, m, n);
}

// ------------------------------------------------ device-driven single solve
// The iteration of jacobi_diis with its decisions on the device (Sec. III:
// Jacobi steps with DIIS extrapolation).  The state sits in device memory
// behind SolveHead; a solve that has ended reads active == 0 and every later
// kernel returns at once, so iterations enqueued beyond the end do nothing.
namespace {

struct DevSolve {
    SolveHead h;
    double B[16 * 16];              // Gram matrix of the stored error vectors
    double coef[16];                // DIIS coefficients of the last extrapolation
    double ring[kSolveRing];        // smallest norm up to iteration i, at (i - 1) % kSolveRing
};

// sum of v over one wavefront, valid in lane 0 (fixed order)
__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__global__ void k_ds_init(DevSolve* __restrict__ ds) {
    if (threadIdx.x != 0) return;
    SolveHead& h = ds->h;
    h.active = 1;
    h.iters = h.next = h.stored = h.use = h.last = h.stalled = h.improved = h.pad = 0;
    h.status = PQPH_NOT_CONVERGED;
    h.rn = h.rmin = INFINITY;
    for (int i = 0; i < 16 * 16; ++i) ds->B[i] = 0.0;
    for (int i = 0; i < 16; ++i) ds->coef[i] = 0.0;
}

// One pass: e = -r/D, th[next] = x + e, eh[next] = e, and the block partials
// of ||r||^2 and e . eh[j] (j < m; the new slot from the register value).
// Wavefront sums, then the four wavefronts in a fixed order.
__global__ __launch_bounds__(256) void k_ds_step(const DevSolve* __restrict__ ds,
                                                 const double* __restrict__ x,
                                                 const double* __restrict__ r,
                                                 const double* __restrict__ D, size_t n,
                                                 double* __restrict__ th, double* __restrict__ eh,
                                                 int m, double* __restrict__ partial) {
    if (!ds->h.active) return;
    const int slot = ds->h.next;
    double* es = eh + (size_t)slot * n;
    double* xs = th + (size_t)slot * n;
    double sr = 0.0, sg[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) sg[j] = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const double ri = r[i];
        const double d = -ri / D[i];
        es[i] = d;
        xs[i] = x[i] + d;
        sr += ri * ri;
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (j < m) sg[j] += (j == slot ? d : eh[(size_t)j * n + i]) * d;
    }
    __shared__ double red[4][17];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < 17; ++j) {
        if (j <= m) {
            const double v = wave_sum(j == 0 ? sr : sg[j > 0 ? j - 1 : 0]);
            if (lane == 0) red[wv][j] = v;
        }
    }
    __syncthreads();
    const int j = threadIdx.x;
    if (j <= m) partial[(size_t)j * gridDim.x + blockIdx.x] = (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
}

// One workgroup of 256: row sums of the partials (all loads issued before
// the sums; nblk <= 1024), then (thread 0, on a register copy of the state
// loaded up front) the tests of the host loop in its order -- non-finite,
// converged, stalled, diverged, iteration limit -- and, while the solve goes
// on, the history bookkeeping and the Gram row; then the DIIS coefficients
// by the whole workgroup.
__global__ __launch_bounds__(256) void k_ds_decide(DevSolve* __restrict__ ds,
                                                   const double* __restrict__ partial, int nblk,
                                                   DevSolveOpts o) {
    SolveHead hd = ds->h;
    if (!hd.active) return;    // the same copy in every thread; thread 0 writes after the barrier
    __shared__ double red[4][17];
    __shared__ double Bs[16 * 16];   // the Gram matrix, updated here and read by the DIIS solve
    __shared__ int nk;         // DIIS vectors to extrapolate with, 0 = none
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    Bs[tid] = ds->B[tid];
    const int it = hd.iters + 1;
    const bool stall_test = o.stall_window > 0 && it > o.stall_window;
    const double old_min = stall_test ? ds->ring[(it - 1 - o.stall_window) % kSolveRing] : 0.0;
    double v[17];
#pragma unroll
    for (int j = 0; j < 17; ++j) {
        v[j] = 0.0;
        if (j <= o.m) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = tid + q * 256;
                if (i < nblk) v[j] += partial[(size_t)j * nblk + i];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 17; ++j) {
        if (j <= o.m) {
            const double x = wave_sum(v[j]);
            if (lane == 0) red[wv][j] = x;
        }
    }
    __syncthreads();
    if (tid == 0) {
        nk = 0;
        auto row = [&](int j) { return (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]); };
        hd.iters = it;
        const double rn = sqrt(row(0));
        hd.rn = rn;
        hd.improved = 0;
        int stt = 1;   // 1 = go on
        if (!isfinite(rn)) {
            stt = PQPH_NONFINITE;
        } else {
            hd.improved = rn < hd.rmin;
            hd.rmin = fmin(hd.rmin, rn);
            ds->ring[(it - 1) % kSolveRing] = hd.rmin;
            if (rn <= o.tol) {
                stt = PQPH_OK;
            } else if (stall_test && hd.rmin > 0.5 * old_min) {
                stt = PQPH_NOT_CONVERGED;
                hd.stalled = 1;
            } else if (rn > 1e3 || rn > o.diverge_factor * hd.rmin) {
                stt = PQPH_DIVERGED;
            } else if (it >= o.max_iter) {
                stt = PQPH_NOT_CONVERGED;
            }
        }
        if (stt != 1) {
            hd.status = stt;
            hd.active = 0;
        } else {
            const int slot = hd.next;
            hd.last = slot;
            hd.next = (slot + 1) % o.m;
            hd.use = 0;
            if (o.diis_on) {
                hd.stored = min(hd.stored + 1, o.m);
                for (int j = 0; j < o.m; ++j) {
                    const double g = row(1 + j);
                    ds->B[slot * 16 + j] = g;
                    ds->B[j * 16 + slot] = g;
                    Bs[slot * 16 + j] = g;
                    Bs[j * 16 + slot] = g;
                }
                if (it >= o.diis_start && hd.stored >= 2) nk = hd.stored;
            }
        }
        if (nk == 0) ds->h = hd;
    }
    __syncthreads();
    const int k = nk;
    if (k == 0) return;
    const bool ok = diis_coefficients(Bs, k, ds->coef);
    if (tid != 0) return;
    if (ok) hd.use = 1;
    ds->h = hd;
}

// Also copies the state to mirror (pinned host memory) from one thread: the
// write to host memory overlaps the other workgroups' work.
__global__ void k_ds_update(const DevSolve* __restrict__ ds, const double* __restrict__ th,
                            size_t n, double* __restrict__ x, double* __restrict__ best,
                            SolveHead* __restrict__ mirror) {
    if (mirror && blockIdx.x == 0 && threadIdx.x == 0) *mirror = ds->h;
    const bool active = ds->h.active != 0;
    const bool keep = best != nullptr && ds->h.improved != 0;
    if (!active && !keep) return;
    const bool use = ds->h.use != 0;
    const int k = ds->h.stored;
    const double* last = th + (size_t)ds->h.last * n;
    double c[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) c[j] = ds->coef[j];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        if (keep) best[i] = x[i];
        if (!active) continue;
        if (use) {
            double v = 0.0;
            for (int j = 0; j < k; ++j) v += c[j] * th[(size_t)j * n + i];
            x[i] = v;
        } else {
            x[i] = last[i];
        }
    }
}

}  // namespace

size_t dev_solve_doubles() { return (sizeof(DevSolve) + sizeof(double) - 1) / sizeof(double); }

void launch_dsolve_init(hipStream_t s, double* state) {
    hipLaunchKernelGGL(k_ds_init, dim3(1), dim3(64), 0, s, reinterpret_cast<DevSolve*>(state));
}

void launch_dsolve_step(hipStream_t s, const double* state, const double* x, const double* r,
                        const double* D, size_t n, double* th, double* eh, int m, double* part,
                        int nblk) {
    hipLaunchKernelGGL(k_ds_step, dim3(nblk), dim3(256), 0, s, reinterpret_cast<const DevSolve*>(state),
                       x, r, D, n, th, eh, m, part);
}

void launch_dsolve_decide(hipStream_t s, double* state, const double* part, int nblk,
                          const DevSolveOpts& o) {
    hipLaunchKernelGGL(k_ds_decide, dim3(1), dim3(256), 0, s, reinterpret_cast<DevSolve*>(state), part,
                       nblk, o);
}

void launch_dsolve_update(hipStream_t s, const double* state, const double* th, size_t n,
                          double* x, double* best, SolveHead* mirror) {
    hipLaunchKernelGGL(k_ds_update, dim3(stream_blocks(n)), dim3(256), 0, s,
                       reinterpret_cast<const DevSolve*>(state), th, n, x, best, mirror);
}
