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
// register value).  Same grid-stride order and tree reductions as
// k_dot_partial / k_dots_partial, so the sums are the same.
__global__ void k_step(const double* __restrict__ t, const double* __restrict__ r,
                       const double* __restrict__ D, size_t n, double* __restrict__ tn,
                       double* __restrict__ eh, int m, int slot, double* __restrict__ partial) {
    __shared__ double red[256];
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
    for (int row = 0; row <= m; ++row) {
        red[threadIdx.x] = row == 0 ? sr : sg[row - 1];
        __syncthreads();
        for (int k = 128; k > 0; k >>= 1) {
            if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(size_t)row * gridDim.x + blockIdx.x] = red[0];
        __syncthreads();
    }
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
