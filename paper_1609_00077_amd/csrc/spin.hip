// Closed-shell spin adaptation of the packed amplitude space (Sec. V: spin
// summation for closed shells roughly halves the amplitude storage).
//
// With a spin-free Hamiltonian and the closed-shell reference, exchanging
// alpha and beta on every pair maps an excitation g_{P0}^{e0} g_{P1}^{e1} ...
// to g_{P0}^{e0'} g_{P1}^{e1'} ... (e' = e with bits 0<->1 and 2<->3
// exchanged) times a sign: each g^{e'} is the product of the exchanged
// generators taken in the order of e, reordered to ascending bits.  The
// solution and the residual at any spin-symmetric point keep
// t[partner] = sign * t.  The orbits of this involution are the unit of the
// reduced space: one value per orbit, x = sqrt(w) t[rep] with w = 2 for an
// exchanged pair of slots and w = 1 for a slot that is its own partner, so
// that Euclidean norms and inner products of reduced vectors equal those of
// the full symmetric vectors and the Jacobi/DIIS and Newton-Krylov
// iterations run unchanged in the smaller space.
//
// The exchange keeps the label set, so it acts on the pattern index m of a
// slot only: the orbit tables below list, per label-set size, the orbits of
// the pattern tuples (representative = the smaller index).  The reduced
// layout mirrors the packed one, orbit-major within each size block.
#include "pqph_internal.h"

namespace {

constexpr int kMaxPat = 303;

struct SpinOrbits {
    int npat[4];            // pattern tuples per label-set size (index 1..3)
    int norb[4];            // orbits per size
    int rep[4][kMaxPat];    // representative pattern index of orbit o
    int par[4][kMaxPat];    // its partner (== rep for a self-partnered orbit)
    int sgn[4][kMaxPat];    // t[par] = sgn * t[rep]
};

constexpr int charge_a(int e) { return ((e >> 2) & 1) - (e & 1); }
constexpr int charge_b(int e) { return ((e >> 3) & 1) - ((e >> 1) & 1); }
constexpr int exchange(int e) {
    return ((e & 1) << 1) | ((e >> 1) & 1) | ((e & 4) << 1) | ((e >> 1) & 4);
}
// sign of sorting the exchanged generators (in the order of e) ascending
constexpr int exchange_sign(int e) {
    int b[4] = {0, 0, 0, 0};
    int c = 0;
    for (int i = 0; i < 4; ++i)
        if (e >> i & 1) b[c++] = i ^ 1;
    int inv = 0;
    for (int i = 0; i < c; ++i)
        for (int j = i + 1; j < c; ++j)
            if (b[i] > b[j]) ++inv;
    return inv % 2 ? -1 : 1;
}

// tuple of L patterns in 1..15 (first label most significant) -> code
constexpr int tuple_code(const int* e, int L) {
    int c = 0;
    for (int i = 0; i < L; ++i) c = c * 16 + e[i];
    return c;
}

constexpr SpinOrbits build_spin_orbits() {
    SpinOrbits o{};
    for (int L = 1; L <= 3; ++L) {
        int index[4096] = {};       // code -> pattern index + 1 (0 = not a tuple)
        int codes[kMaxPat] = {};
        int m = 0;
        const int total = L == 1 ? 15 : L == 2 ? 225 : 3375;
        for (int t = 0; t < total; ++t) {          // lexicographic over (e0, e1, e2)
            int e[3] = {0, 0, 0};
            int r = t;
            for (int i = L - 1; i >= 0; --i) {
                e[i] = 1 + r % 15;
                r /= 15;
            }
            int ca = 0, cb = 0;
            for (int i = 0; i < L; ++i) {
                ca += charge_a(e[i]);
                cb += charge_b(e[i]);
            }
            if (ca != 0 || cb != 0) continue;
            codes[m] = tuple_code(e, L);
            index[codes[m]] = m + 1;
            ++m;
        }
        o.npat[L] = m;
        int q = 0;
        for (int a = 0; a < m; ++a) {
            int e[3] = {0, 0, 0}, f[3] = {0, 0, 0};
            int c = codes[a], sg = 1;
            for (int i = L - 1; i >= 0; --i) {
                e[i] = c % 16;
                c /= 16;
            }
            for (int i = 0; i < L; ++i) {
                f[i] = exchange(e[i]);
                sg *= exchange_sign(e[i]);
            }
            const int b = index[tuple_code(f, L)] - 1;
            if (b < a) continue;                     // listed with its representative
            o.rep[L][q] = a;
            o.par[L][q] = b;
            o.sgn[L][q] = sg;
            ++q;
        }
        o.norb[L] = q;
    }
    return o;
}

constexpr SpinOrbits kOrbits = build_spin_orbits();

constexpr bool self_orbits_symmetric() {
    for (int L = 1; L <= 3; ++L)
        for (int q = 0; q < kOrbits.norb[L]; ++q)
            if (kOrbits.rep[L][q] == kOrbits.par[L][q] && kOrbits.sgn[L][q] != 1) return false;
    return true;
}
static_assert(kOrbits.npat[1] == 3 && kOrbits.npat[2] == 29 && kOrbits.npat[3] == 303,
              "pattern tuple counts of the packed layout");
// a self-partnered slot with sign -1 would be forced to zero; none exists
static_assert(self_orbits_symmetric(), "self-partnered slots keep their sign");

__device__ const SpinOrbits d_orbits = kOrbits;

size_t choose(int n, int k) {
    if (k < 0 || k > n) return 0;
    size_t c = 1;
    for (int i = 0; i < k; ++i) c = c * (size_t)(n - i) / (size_t)(i + 1);
    return c;
}

struct SpinGeom {
    size_t nsets[4];    // C(N, L)
    size_t off[4];      // full block offsets
    size_t roff[4];     // reduced block offsets; roff[k+1] = reduced length
};

SpinGeom geometry(int npair, int k) {
    SpinGeom g{};
    size_t a = 0, b = 0;
    for (int L = 1; L <= 3; ++L) {
        g.nsets[L] = L <= k ? choose(npair, L) : 0;
        g.off[L] = a;
        g.roff[L] = b;
        a += g.nsets[L] * kOrbits.npat[L];
        b += g.nsets[L] * kOrbits.norb[L];
    }
    g.roff[0] = b;      // total reduced length
    return g;
}

__device__ inline void locate(const SpinGeom& g, size_t j, int& L, size_t& o, size_t& set) {
    L = j >= g.roff[3] ? 3 : j >= g.roff[2] ? 2 : 1;
    const size_t r = j - g.roff[L];
    o = r / g.nsets[L];
    set = r - o * g.nsets[L];
}

// mode 0: x_j = sqrt(w) * (v[rep] + sgn v[par]) / w  (orthogonal projection
// onto the symmetric subspace, in reduced coordinates);
// mode 1: x_j = v[rep] (denominators, ranks: equal on both slots)
__global__ __launch_bounds__(256) void k_spin_pack(const double* __restrict__ v, double* __restrict__ x,
                                                   SpinGeom g, int mode) {
    const size_t nr = g.roff[0];
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < nr;
         j += (size_t)gridDim.x * blockDim.x) {
        int L;
        size_t o, set;
        locate(g, j, L, o, set);
        const int a = d_orbits.rep[L][o], b = d_orbits.par[L][o];
        const double va = v[g.off[L] + (size_t)a * g.nsets[L] + set];
        if (mode == 1 || a == b) {
            x[j] = va;
        } else {
            const double vb = v[g.off[L] + (size_t)b * g.nsets[L] + set];
            x[j] = (va + d_orbits.sgn[L][o] * vb) * M_SQRT1_2;
        }
    }
}

// v[rep] = x_j / sqrt(w), v[par] = sgn v[rep]: every full slot written once
__global__ __launch_bounds__(256) void k_spin_unpack(const double* __restrict__ x, double* __restrict__ v,
                                                     SpinGeom g) {
    const size_t nr = g.roff[0];
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < nr;
         j += (size_t)gridDim.x * blockDim.x) {
        int L;
        size_t o, set;
        locate(g, j, L, o, set);
        const int a = d_orbits.rep[L][o], b = d_orbits.par[L][o];
        const size_t pa = g.off[L] + (size_t)a * g.nsets[L] + set;
        if (a == b) {
            v[pa] = x[j];
        } else {
            const double y = x[j] * M_SQRT1_2;
            v[pa] = y;
            v[g.off[L] + (size_t)b * g.nsets[L] + set] = d_orbits.sgn[L][o] * y;
        }
    }
}

}  // namespace

size_t spin_len(int npair, int k) { return geometry(npair, k).roff[0]; }

void launch_spin_pack(hipStream_t s, const double* v, double* x, int npair, int k, int mode) {
    const SpinGeom g = geometry(npair, k);
    const int grid = stream_blocks(g.roff[0]);
    if (grid == 0) return;
    hipLaunchKernelGGL(k_spin_pack, dim3(grid), dim3(256), 0, s, v, x, g, mode);
}

void launch_spin_unpack(hipStream_t s, const double* x, double* v, int npair, int k) {
    const SpinGeom g = geometry(npair, k);
    const int grid = stream_blocks(g.roff[0]);
    if (grid == 0) return;
    hipLaunchKernelGGL(k_spin_unpack, dim3(grid), dim3(256), 0, s, x, v, g);
}

void spin_pattern_reps(int n, int* rep, int* sgn) {
    for (int q = 0; q < kOrbits.norb[n]; ++q) {
        const int a = kOrbits.rep[n][q], b = kOrbits.par[n][q];
        rep[a] = a;
        sgn[a] = 1;
        rep[b] = a;
        sgn[b] = kOrbits.sgn[n][q];
    }
}
