// PH residual, energy and denominators (k = 3: excitations and integrals on
// at most three pairs, Sec. II; Table I caption keeps integral subtensors up
// to rank 3).  The residual is r_mu = <mu| e^{-T} H_3 e^{T} |0> over the packed
// one-, two- and three-label blocks; every connected term of an output block
// touches at most three spectator pairs, all of them through the Hamiltonian.
//
// The derived terms (one table per output block size and spectator count,
// grouped by output pattern) are read from a binary file written by the
// package's PH table generator and kept in device memory per context.  One
// workgroup owns one output slot: its threads run over (term, ordered
// spectator tuple) pairs, evaluate the Hamiltonian symbol sum and the amplitude factors
// from the packed arrays, and the sums are combined in a fixed order, so
// results are deterministic.  This is a generic interpreter: its cost grows as
// C(N,3) x N^3 x terms, far from a factorised kernel.
#include <dlfcn.h>
#include <zlib.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "pqph_internal.h"

namespace {

constexpr int kPhMagic = 0x31485450;
constexpr int kPhzMagic = 0x315A4850;      // zlib-compressed container of the above
constexpr int kMaxClass = 16;

struct PhClass {
    int nout, nspec, nterm, off, npat, soff;
};

struct PhArgs {
    int nclass;
    PhClass cls[kMaxClass];
    const int* starts;      // per class npat + 1 term offsets (relative to off)
    long nterm;
    const unsigned short* th;     // per term: Hamiltonian term
    const unsigned char* tcw;     // per term: index into cw_dict
    const unsigned short* ts;     // 4 x nterm (slot-major): indices into slot_dict
    const int* cw_dict;           // (nf << 16) | (coef + 32768)
    const int* slot_dict;         // amplitude slot codes
    const int* hstart;      // nh + 1
    const double* sym_w;
    const int* sym_code;
    const int* pat2m;       // 16 + 256 + 4096
    const int* m2pat;       // 3 + 29 + 303
    const int* canon;       // 3 + 29 + 303: canonical pattern, role order, sign
    const int* quad;        // 3 x 1296
};

// Index arithmetic in 32 bits: with npair <= 256 every packed position fits
// (ph_amp_len(256) = 837 M, ph_eri_len(256) = 233 M, N (N-1) (N-2) <= 16.6 M),
// and 32-bit multiplies are a fraction of the 64-bit ones in this interpreted
// hot loop.  Offsets into the per-unit partial sums stay 64-bit.
__device__ __forceinline__ int ncomb(int N, int k) {
    if (k == 1) return N;
    if (k == 2) return N * (N - 1) / 2;
    return N * (N - 1) * (N - 2) / 6;
}

// index of an ascending label set in the packed layout
__device__ __forceinline__ int set_index(const int* l, int n) {
    if (n == 1) return l[0];
    if (n == 2) return l[1] * (l[1] - 1) / 2 + l[0];
    return l[2] * (l[2] - 1) * (l[2] - 2) / 6 + l[1] * (l[1] - 1) / 2 + l[0];
}

__device__ __forceinline__ int amp_off(int N, int n) {
    return n == 1 ? 0 : n == 2 ? 3 * N : 3 * N + 29 * ncomb(N, 2);
}

__device__ __forceinline__ int eri_off(int N, int n) {
    return n == 1 ? 0 : n == 2 ? 6 * N : 6 * N + 43 * ncomb(N, 2);
}

// The labels of a term's roles packed 8 bits each (labels < 256): reading
// role r is one shift, where an indexed local array costs a chain of selects.
struct Labs {
    unsigned long long w;
    __device__ __forceinline__ int operator[](int r) const { return (int)((w >> (8 * r)) & 255); }
};

// packed position of one amplitude factor: the labels of its roles, put in
// ascending order (swapping two odd patterns flips the sign); -1 for no
// factor (code 0) or a pattern tuple the layout does not store
__device__ __forceinline__ int amp_pos(const PhArgs& a, const Labs& lab, int code, int N,
                                        double& sg) {
    const int n = code & 3;
    int l[3], p[3];
    for (int i = 0; i < 3; ++i) {
        l[i] = i < n ? lab[(code >> (2 + 3 * i)) & 7] : 0;
        p[i] = i < n ? (code >> (11 + 4 * i)) & 15 : 0;
    }
    sg = 1.0;
    auto sw = [&](int i) {
        if (l[i] > l[i + 1]) {
            if ((__popc(p[i]) & 1) && (__popc(p[i + 1]) & 1)) sg = -sg;
            int x = l[i]; l[i] = l[i + 1]; l[i + 1] = x;
            x = p[i]; p[i] = p[i + 1]; p[i + 1] = x;
        }
    };
    if (n == 2) sw(0);
    if (n == 3) { sw(0); sw(1); sw(0); }
    if (n == 0) return -1;
    const int base = n == 1 ? 0 : n == 2 ? 16 : 272;
    const int m = a.pat2m[base + (p[0] | p[1] << 4 | p[2] << 8)];
    if (m < 0) return -1;
    return amp_off(N, n) + m * ncomb(N, n) + set_index(l, n);
}

// Hamiltonian factor: sum of weighted f and chemists' (pq|rs) symbols, local
// orbital x = 2 * role + type read at label lab[role]
__device__ __forceinline__ double hval(const PhArgs& a, const Labs& lab, int hidx, int N,
                                       const double* __restrict__ f,
                                       const double* __restrict__ eri) {
    double v = 0.0;
    const int n2 = 2 * N;
    for (int j = a.hstart[hidx]; j < a.hstart[hidx + 1]; ++j) {
        const int c = a.sym_code[j];
        int x[4];
        for (int i = 0; i < 4; ++i) x[i] = (c >> (4 + 4 * i)) & 15;
        if ((c & 15) == 0) {
            const int o0 = lab[x[0] >> 1] + N * (x[0] & 1), o1 = lab[x[1] >> 1] + N * (x[1] & 1);
            v += a.sym_w[j] * f[o0 * n2 + o1];
            continue;
        }
        int s[4], ns = 0;
        for (int i = 0; i < 4; ++i) {
            const int L = lab[x[i] >> 1];
            bool seen = false;
            for (int k = 0; k < ns; ++k) seen |= s[k] == L;
            if (!seen) s[ns++] = L;
        }
        if (ns > 3) continue;
        for (int i = 1; i < ns; ++i)      // insertion sort, at most three labels
            for (int k = i; k > 0 && s[k - 1] > s[k]; --k) {
                const int y = s[k]; s[k] = s[k - 1]; s[k - 1] = y;
            }
        int loc[4];
        for (int i = 0; i < 4; ++i) {
            const int L = lab[x[i] >> 1];
            const int rk = L == s[0] ? 0 : L == s[1] ? 1 : 2;
            loc[i] = 2 * rk + (x[i] & 1);
        }
        const int u = a.quad[(ns - 1) * 1296 + ((loc[0] * 6 + loc[1]) * 6 + loc[2]) * 6 + loc[3]];
        if (u < 0) continue;
        v += a.sym_w[j] * eri[eri_off(N, ns) + u * ncomb(N, ns) + set_index(s, ns)];
    }
    return v;
}

// j-th label (ascending) outside the ascending set L of size n
__device__ __forceinline__ int outside(int j, const int* L, int n) {
    for (int i = 0; i < n; ++i)
        if (j >= L[i]) ++j;
    return j;
}

// labels of an output slot's roles and of one ordered spectator tuple (number
// perm of n_o (n_o - 1) ...); output role i sits at label Lr[i], L is the
// same set in ascending order
__device__ __forceinline__ Labs role_labels(int N, const int* Lr, const int* L, int nout,
                                            int nspec, int perm) {
    unsigned long long w = 0;
    for (int i = 0; i < nout; ++i) w |= (unsigned long long)Lr[i] << (8 * i);
    const int no = N - nout;
    int j[3] = {0, 0, 0};
    for (int i = 0; i < nspec; ++i) {
        j[i] = (int)(perm % (no - i));
        perm /= (no - i);
    }
    // position among the outside labels, skipping those already taken
    if (nspec >= 2 && j[1] >= j[0]) ++j[1];
    if (nspec == 3) {
        const int lo = j[0] < j[1] ? j[0] : j[1], hi = j[0] < j[1] ? j[1] : j[0];
        if (j[2] >= lo) ++j[2];
        if (j[2] >= hi) ++j[2];
    }
    for (int i = 0; i < nspec; ++i) w |= (unsigned long long)outside(j[i], L, nout) << (8 * (nout + i));
    return Labs{w};
}

// the terms q0 .. q1-1 at one label assignment; consecutive terms of one
// Hamiltonian term (the tables keep them together) reuse its value
__device__ __forceinline__ double chunk_value(const PhArgs& a, int N, const Labs& lab, int q0,
                                              int q1, const double* __restrict__ f,
                                              const double* __restrict__ eri,
                                              const double* __restrict__ t) {
    double sum = 0.0, hv = 0.0;
    int hprev = -1;
    for (int q = q0; q < q1; ++q) {
        const int h = a.th[q];
        if (h != hprev) {
            hv = hval(a, lab, h, N, f, eri);
            hprev = h;
        }
        if (hv == 0.0) continue;
        const int cw = a.cw_dict[a.tcw[q]];
        const int nf = cw >> 16;
        // the factors are independent: all their loads can be in flight at once
        int code[4];
        const int nt = (int)a.nterm;      // < 2^31 (the file's term count is 32-bit)
        for (int i = 0; i < 4; ++i) code[i] = i < nf ? a.slot_dict[a.ts[i * nt + q]] : 0;
        int pos[4];
        double sg[4];
        for (int i = 0; i < 4; ++i) pos[i] = amp_pos(a, lab, code[i], N, sg[i]);
        double v = hv * (double)((cw & 0xffff) - 32768);
        for (int i = 0; i < 4; ++i)
            if (i < nf) v *= pos[i] >= 0 ? sg[i] * t[pos[i]] : 0.0;
        sum += v;
    }
    return sum;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ long nperm(int no, int nspec) {
    long p = 1;
    for (int i = 0; i < nspec; ++i) p *= (no - i);
    return p;
}

// 1 / nspec!: the terms are summed over ordered spectator tuples
__device__ __forceinline__ double inv_fact(int n) { return n == 2 ? 0.5 : n == 3 ? 1.0 / 6.0 : 1.0; }

// ascending labels of set number si among the label sets of size n
__device__ __forceinline__ void decode_set(long si, int n, int* L) {
    if (n == 1) {
        L[0] = (int)si;
        return;
    }
    if (n == 3) {
        int R = 2;
        while ((long)(R + 1) * R * (R - 1) / 6 <= si) ++R;
        L[2] = R;
        si -= (long)R * (R - 1) * (R - 2) / 6;
    }
    int Q = 1;
    while ((long)(Q + 1) * Q / 2 <= si) ++Q;
    L[1] = Q;
    L[0] = (int)(si - (long)Q * (Q - 1) / 2);
}

// decode a packed slot into (block size, pattern number, ascending labels)
__device__ __forceinline__ void decode_slot(long s, int N, int& n, int& m, int* L) {
    const long c2 = ncomb(N, 2), c3 = ncomb(N, 3);
    long si;
    if (s < 3L * N) {
        n = 1; m = (int)(s / N); L[0] = (int)(s % N);
        return;
    }
    s -= 3L * N;
    if (s < 29 * c2) {
        n = 2; m = (int)(s / c2); si = s % c2;
    } else {
        s -= 29 * c2;
        n = 3; m = (int)(s / c3); si = s % c3;
        int R = 2;
        while ((long)(R + 1) * R * (R - 1) / 6 <= si) ++R;
        L[2] = R;
        si -= (long)R * (R - 1) * (R - 2) / 6;
    }
    int Q = 1;
    while ((long)(Q + 1) * Q / 2 <= si) ++Q;
    L[1] = Q;
    L[0] = (int)(si - (long)Q * (Q - 1) / 2);
}

// The residual runs as balanced work units.  A unit is a range of one
// class's work items for one output pattern m of block size n; items are
// (chunk of PH_CHUNK consecutive terms, ordered spectator tuple), spectator
// tuple fastest, so the lanes of a wave walk the same terms at different
// spectators.  k_ph_part runs one workgroup per (label set, unit) and writes
// the unit's sum; k_ph_gather adds a slot's units in their fixed order (the
// result is deterministic).  Splitting matters: the term count of the
// three-pair output patterns ranges over a factor of 20.
constexpr int PH_WAVES = 8;
constexpr int PH_BLOCK = 64 * PH_WAVES;
constexpr int PH_CHUNK = 16;

struct PhUnits {
    const int* m;          // per unit: output pattern
    const int* cls;        // class
    const long* i0;        // item range
    const long* i1;
};

__global__ __launch_bounds__(PH_BLOCK) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_ph_part(int N, int n, PhArgs a, PhUnits u,
                                                      const double* __restrict__ f,
                                                      const double* __restrict__ eri,
                                                      const double* __restrict__ t,
                                                      double* __restrict__ part) {
    __shared__ double red[PH_WAVES];
    const long si = blockIdx.x, nsets = gridDim.x;
    const int un = blockIdx.y, tid = threadIdx.x, lane = tid & 63;
    int L[3] = {0, 0, 0};
    decode_set(si, n, L);
    const int m = u.m[un];
    // terms are stored for the canonical reordering of the output tuple: its
    // role i sits at label L[p_i]
    const int cn = a.canon[(n == 1 ? 0 : n == 2 ? 3 : 32) + m];
    const int mc = cn & 511;
    int Lr[3];
    for (int i = 0; i < 3; ++i) Lr[i] = L[(cn >> (9 + 2 * i)) & 3];
    const PhClass& k = a.cls[u.cls[un]];
    const int* st = a.starts + k.soff;
    const int t0 = k.off + st[mc], t1 = k.off + st[mc + 1];
    const int np = (int)nperm(N - n, k.nspec);
    const long i0 = u.i0[un], i1 = u.i1[un];
    const int dq = PH_BLOCK / np, dp = PH_BLOCK % np;
    int ch = (int)((i0 + tid) / np);
    int p = (int)((i0 + tid) % np);
    double acc = 0.0;
    for (long i = i0 + tid; i < i1; i += PH_BLOCK) {
        const Labs lab = role_labels(N, Lr, L, n, k.nspec, p);
        const int q0 = t0 + ch * PH_CHUNK;
        acc += chunk_value(a, N, lab, q0, q0 + PH_CHUNK < t1 ? q0 + PH_CHUNK : t1, f, eri, t);
        ch += dq;
        p += dp;
        if (p >= np) {
            p -= np;
            ++ch;
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double sum = 0.0;
        for (int w = 0; w < PH_WAVES; ++w) sum += red[w];
        part[(long)un * nsets + si] = inv_fact(k.nspec) * sum;
    }
}

// r(slot) = sign * (sum of the slot's unit sums, in unit order)
// spin (may be null): per pattern of the 1/2/3-label blocks (offsets 0, 3,
// 32), rep | negative << 16 -- a slot whose pattern is not its orbit's
// representative takes the representative's value (same labels) with the sign
__global__ void k_ph_gather(int N, long namp, PhArgs a, const int* __restrict__ ustart,
                            const double* __restrict__ part1, const double* __restrict__ part2,
                            const double* __restrict__ part3, const int* __restrict__ spin,
                            double* __restrict__ r) {
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= namp) return;
    int n, m, L[3];
    decode_slot(s, N, n, m, L);
    const int base = n == 1 ? 0 : n == 2 ? 3 : 32;
    bool flip = false;
    if (spin) {
        const int w = spin[base + m];
        m = w & 0xffff;
        flip = (w >> 16) & 1;
    }
    const long nsets = ncomb(N, n), si = set_index(L, n);
    const int* us = ustart + (n == 1 ? 0 : n == 2 ? 4 : 34);
    const double* part = n == 1 ? part1 : n == 2 ? part2 : part3;
    double sum = 0.0;
    for (int un = us[m]; un < us[m + 1]; ++un) sum += part[(long)un * nsets + si];
    const int cn = a.canon[base + m];
    if ((cn >> 15) & 1) sum = -sum;
    r[s] = flip ? -sum : sum;
}

// E_c = <0| H_3 e^T |0>: the energy classes (no output labels) over ordered
// tuples of 1..3 labels, block partials then one fixed-order sum
__global__ __launch_bounds__(256) void k_ph_energy(int N, PhArgs a, const double* __restrict__ f,
                                                   const double* __restrict__ eri,
                                                   const double* __restrict__ t,
                                                   double* __restrict__ part) {
    __shared__ double red[256];
    const long g = (long)blockIdx.x * blockDim.x + threadIdx.x, G = (long)gridDim.x * blockDim.x;
    const int L[1] = {0};
    double acc = 0.0;
    for (int c = 0; c < a.nclass; ++c) {
        const PhClass& k = a.cls[c];
        if (k.nout != 0 || k.nspec > N) continue;
        const long np = nperm(N, k.nspec), tot = (long)k.nterm * np;
        double s = 0.0;
        for (long i = g; i < tot; i += G) {
            const long q = i / np;
            const Labs lab = role_labels(N, L, L, 0, k.nspec, (int)(i - q * np));
            s += chunk_value(a, N, lab, k.off + (int)q, k.off + (int)q + 1, f, eri, t);
        }
        acc += inv_fact(k.nspec) * s;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_ph_sum(int n, const double* __restrict__ part, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    out[0] = s;
}

// D_mu = sum of f_aa over its particles - sum of f_ii over its holes (+ shift)
__global__ void k_ph_denom(int N, long namp, PhArgs a, const double* __restrict__ f, double shift,
                           double* __restrict__ D) {
    const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= namp) return;
    int n, m, L[3] = {0, 0, 0};
    decode_slot(s, N, n, m, L);
    const int pat = a.m2pat[(n == 1 ? 0 : n == 2 ? 3 : 32) + m];
    const long n2 = 2L * N;
    double d = 0.0;
    for (int i = 0; i < n; ++i) {
        const int e = (pat >> (4 * i)) & 15;
        d += __popc(e & 12) * f[(long)(N + L[i]) * n2 + N + L[i]] - __popc(e & 3) * f[(long)L[i] * n2 + L[i]];
    }
    D[s] = d + shift;
}

}  // namespace

// ------------------------------------------------------------ table loading
// work units of one pair count: per block size n, a list of (pattern m,
// class, item range), grouped by m (ustart: 4 + 30 + 304 offsets)
struct PhSched {
    void* dev = nullptr;
    PhUnits units[4] = {};
    const int* ustart = nullptr;
    const int* spin = nullptr;    // pattern -> representative map (spin-symmetric schedules)
    int nunit[4] = {};
    size_t part_off[4] = {};      // partial sums of size n start here (doubles)
    size_t part_doubles = 0;
};

struct PhTables {
    PhArgs args{};
    void* dev = nullptr;
    int nh = 0;
    std::vector<int> starts_h, canon_h;     // host copies for scheduling
    std::vector<PhSched*> sched = std::vector<PhSched*>(257, nullptr);
    std::vector<PhSched*> sched_sym = std::vector<PhSched*>(257, nullptr);   // representatives only
};

namespace {

std::string ph_terms_path() {
    const char* env = getenv("PQPH_PH_TERMS");
    if (env && *env) return env;
    Dl_info info{};
    if (dladdr((void*)&ph_amp_len, &info) && info.dli_fname) {
        std::string p(info.dli_fname);
        const size_t k = p.rfind('/');
        return (k == std::string::npos ? std::string(".") : p.substr(0, k)) + "/ph_terms.bin";
    }
    return "ph_terms.bin";
}

struct Reader {
    const std::vector<char>& b;
    size_t pos = 0;
    bool ok = true;
    template <class T>
    const T* take(size_t n) {
        if (!ok || pos + n * sizeof(T) > b.size()) {
            ok = false;
            return nullptr;
        }
        const T* p = reinterpret_cast<const T*>(b.data() + pos);
        pos += n * sizeof(T);
        return p;
    }
};

// every index the kernels follow is checked here, so that a damaged file is an
// error and never an out-of-bounds device read
pqph_status ph_parse(pqph_ctx* ctx, const std::vector<char>& buf, PhTables& tb,
                     std::vector<char>& blob, size_t off[13]) {
    Reader rd{buf};
    const int* hdr = rd.take<int>(8);
    if (!hdr || hdr[0] != kPhMagic || hdr[1] != 3)
        return pqph_fail(ctx, PQPH_INVALID_ARG, "PH term tables: bad header");
    const int nclass = hdr[2], nh = hdr[3], nsym = hdr[4], nterm = hdr[5], ncw = hdr[6],
              nslot = hdr[7];
    if (nclass < 1 || nclass > kMaxClass || nh < 1 || nh > 65536 || nsym < 1 || nterm < 1 ||
        ncw < 1 || ncw > 256 || nslot < 1 || nslot > 65536)
        return pqph_fail(ctx, PQPH_INVALID_ARG, "PH term tables: bad sizes");
    std::vector<int> starts;
    PhArgs& a = tb.args;
    a.nclass = nclass;
    a.nterm = nterm;
    for (int c = 0; c < nclass; ++c) {
        const int* ch = rd.take<int>(5);
        if (!ch) return pqph_fail(ctx, PQPH_INVALID_ARG, "PH term tables: truncated");
        PhClass k{ch[0], ch[1], ch[2], ch[3], ch[4], (int)starts.size()};
        const int want = k.nout == 0 ? 1 : k.nout == 1 ? 3 : k.nout == 2 ? 29 : 303;
        if (k.nout < 0 || k.nout > 3 || k.nspec < 0 || k.nspec > 3 || k.nout + k.nspec > 6 ||
            (k.nout == 0 && k.nspec == 0) || k.npat != want || k.nterm < 0 || k.off < 0 ||
            (long)k.off + k.nterm > nterm)
            return pqph_fail(ctx, PQPH_INVALID_ARG, "PH term tables: bad class header");
        const int* st = rd.take<int>(k.npat + 1);
        if (!st || st[0] != 0 || st[k.npat] != k.nterm)
            return pqph_fail(ctx, PQPH_INVALID_ARG, "PH term tables: bad class offsets");
        for (int i = 0; i < k.npat; ++i)
            if (st[i + 1] < st[i]) return pqph_fail(ctx, PQPH_INVALID_ARG, "PH term tables: bad class offsets");
        starts.insert(starts.end(), st, st + k.npat + 1);
        a.cls[c] = k;
    }
    auto pad = [](size_t b) { return (b + 3) / 4 * 4; };
    const int* cw_dict = rd.take<int>(ncw);
    const int* slot_dict = rd.take<int>(nslot);
    const char* th = rd.take<char>(pad((size_t)nterm * 2));
    const char* tcw = rd.take<char>(pad((size_t)nterm));
    const char* ts = rd.take<char>(pad((size_t)nterm * 8));
    const int* hstart = rd.take<int>(nh + 1);
    const double* sym_w = rd.take<double>(nsym);
    const int* sym_code = rd.take<int>(nsym);
    const int* pat2m = rd.take<int>(16 + 256 + 4096);
    const int* m2pat = rd.take<int>(3 + 29 + 303);
    const int* canon = rd.take<int>(3 + 29 + 303);
    const int* quad = rd.take<int>(3 * 1296);
    if (!rd.ok || rd.pos != buf.size())
        return pqph_fail(ctx, PQPH_INVALID_ARG, "PH term tables: truncated or oversized file");
    auto bad = [&](const char* what) {
        return pqph_fail(ctx, PQPH_INVALID_ARG, std::string("PH term tables: bad ") + what);
    };
    if (hstart[0] != 0 || hstart[nh] != nsym) return bad("symbol offsets");
    for (int i = 0; i < nh; ++i)
        if (hstart[i + 1] < hstart[i]) return bad("symbol offsets");
    for (int j = 0; j < nsym; ++j) {
        const int c = sym_code[j];
        if ((c & 15) > 1 || (c >> 20) != 0) return bad("symbol code");
    }
    // pattern numbers and integral indices stay inside their block of the
    // packed layouts (3 / 29 / 303 patterns, 6 / 43 / 84 integrals per set)
    for (int i = 0; i < 16 + 256 + 4096; ++i) {
        const int np = i < 16 ? 3 : i < 272 ? 29 : 303;
        if (pat2m[i] < -1 || pat2m[i] >= np) return bad("pattern map");
    }
    for (int i = 0; i < 3 * 1296; ++i) {
        const int nq = i < 1296 ? 6 : i < 2592 ? 43 : 84;
        if (quad[i] < -1 || quad[i] >= nq) return bad("integral map");
    }
    for (int i = 0; i < 3 + 29 + 303; ++i) {
        if (m2pat[i] < 0 || m2pat[i] >= 4096) return bad("pattern list");
        const int n = i < 3 ? 1 : i < 32 ? 2 : 3, np = n == 1 ? 3 : n == 2 ? 29 : 303;
        const int c = canon[i];
        if (c < 0 || (c >> 16) != 0 || (c & 511) >= np) return bad("canonical map");
        int seen = 0;
        for (int u = 0; u < n; ++u) seen |= 1 << ((c >> (9 + 2 * u)) & 3);
        for (int u = n; u < 3; ++u)
            if ((c >> (9 + 2 * u)) & 3) return bad("canonical map");
        if (seen != (1 << n) - 1) return bad("canonical map");
    }
    for (int i = 0; i < ncw; ++i)
        if (cw_dict[i] < 0 || (cw_dict[i] >> 16) > 4) return bad("coefficient word");
    if (slot_dict[0] != 0) return bad("slot dictionary");
    for (int i = 1; i < nslot; ++i)
        if ((slot_dict[i] & 3) < 1 || (slot_dict[i] >> 23) != 0) return bad("slot dictionary");
    // every index of every term stays in its table, its roles below its
    // class's role count (so lab[] reads are initialised), and every
    // Hamiltonian symbol names roles of the term
    const unsigned short* h16 = reinterpret_cast<const unsigned short*>(th);
    const unsigned char* c8 = reinterpret_cast<const unsigned char*>(tcw);
    const unsigned short* s16 = reinterpret_cast<const unsigned short*>(ts);
    std::vector<int> hrole(nh, 0);     // 1 + largest role a Hamiltonian term reads
    for (int h = 0; h < nh; ++h)
        for (int j = hstart[h]; j < hstart[h + 1]; ++j)
            for (int i = 0; i < 4; ++i) {
                const int r = ((sym_code[j] >> (4 + 4 * i)) & 15) >> 1;
                if (r + 1 > hrole[h]) hrole[h] = r + 1;
            }
    std::vector<int> srole(nslot, 0);
    for (int i = 1; i < nslot; ++i)
        for (int u = 0; u < (slot_dict[i] & 3); ++u) {
            const int r = (slot_dict[i] >> (2 + 3 * u)) & 7;
            if (r + 1 > srole[i]) srole[i] = r + 1;
        }
    for (int c = 0; c < nclass; ++c) {
        const PhClass& k = a.cls[c];
        const int nrole = k.nout + k.nspec;
        for (long q = k.off; q < (long)k.off + k.nterm; ++q) {
            if (h16[q] >= nh || hrole[h16[q]] > nrole || c8[q] >= ncw) return bad("term");
            const int nf = cw_dict[c8[q]] >> 16;
            for (int i = 0; i < nf; ++i) {
                const int si = s16[(size_t)i * nterm + q];
                if (si < 1 || si >= nslot || srole[si] > nrole) return bad("amplitude factor");
            }
        }
    }
    // one device block (8-byte aligned segments): starts, cw_dict, slot_dict,
    // h, cw, slots, hstart, sym_code, pat2m, m2pat, canon, quad, sym_w
    const size_t sz[13] = {starts.size() * 4, (size_t)ncw * 4, (size_t)nslot * 4,
                           (size_t)nterm * 2, (size_t)nterm, (size_t)nterm * 8,
                           (size_t)(nh + 1) * 4, (size_t)nsym * 4, (16 + 256 + 4096) * 4,
                           (3 + 29 + 303) * 4, (3 + 29 + 303) * 4, 3 * 1296 * 4,
                           (size_t)nsym * 8};
    const void* src[13] = {starts.data(), cw_dict, slot_dict, th, tcw, ts, hstart, sym_code,
                           pat2m, m2pat, canon, quad, sym_w};
    size_t p = 0;
    blob.clear();
    for (int i = 0; i < 13; ++i) {
        off[i] = p;
        blob.insert(blob.end(), (const char*)src[i], (const char*)src[i] + sz[i]);
        p += sz[i];
        while (p % 8) {
            blob.push_back(0);
            ++p;
        }
    }
    tb.nh = nh;
    tb.starts_h = starts;
    tb.canon_h.assign(canon, canon + 3 + 29 + 303);
    return PQPH_OK;
}

}  // namespace

pqph_status ph_tables_load(pqph_ctx* ctx) {
    if (ctx->ph) return PQPH_OK;
    const std::string path = ph_terms_path();
    FILE* fp = fopen(path.c_str(), "rb");
    if (!fp) return pqph_fail(ctx, PQPH_INVALID_ARG, "PH term tables not found at " + path);
    std::vector<char> buf;
    char chunk[1 << 16];
    size_t got;
    while ((got = fread(chunk, 1, sizeof(chunk), fp)) > 0) buf.insert(buf.end(), chunk, chunk + got);
    fclose(fp);
    if (buf.size() >= 12 && *reinterpret_cast<const int*>(buf.data()) == kPhzMagic) {
        long long raw = 0;
        memcpy(&raw, buf.data() + 4, 8);
        if (raw <= 0 || raw > (1LL << 34))
            return pqph_fail(ctx, PQPH_INVALID_ARG, "PH term tables: bad compressed size");
        std::vector<char> out((size_t)raw);
        uLongf got_len = (uLongf)raw;
        if (uncompress(reinterpret_cast<Bytef*>(out.data()), &got_len,
                       reinterpret_cast<const Bytef*>(buf.data() + 12), (uLong)(buf.size() - 12)) != Z_OK ||
            (long long)got_len != raw)
            return pqph_fail(ctx, PQPH_INVALID_ARG, "PH term tables: corrupt compressed file");
        buf.swap(out);
    }
    PhTables* tb = new PhTables();
    std::vector<char> blob;
    size_t off[13];
    pqph_status st = ph_parse(ctx, buf, *tb, blob, off);
    if (st) {
        delete tb;
        return st;
    }
    if (hipMalloc(&tb->dev, blob.size()) != hipSuccess) {
        delete tb;
        return pqph_fail(ctx, PQPH_OOM, "PH term tables: device allocation failed");
    }
    if (hipMemcpy(tb->dev, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(tb->dev);
        delete tb;
        return pqph_fail(ctx, PQPH_DEVICE, "PH term tables: upload failed");
    }
    const char* d = static_cast<const char*>(tb->dev);
    PhArgs& a = tb->args;
    a.starts = reinterpret_cast<const int*>(d + off[0]);
    a.cw_dict = reinterpret_cast<const int*>(d + off[1]);
    a.slot_dict = reinterpret_cast<const int*>(d + off[2]);
    a.th = reinterpret_cast<const unsigned short*>(d + off[3]);
    a.tcw = reinterpret_cast<const unsigned char*>(d + off[4]);
    a.ts = reinterpret_cast<const unsigned short*>(d + off[5]);
    a.hstart = reinterpret_cast<const int*>(d + off[6]);
    a.sym_code = reinterpret_cast<const int*>(d + off[7]);
    a.pat2m = reinterpret_cast<const int*>(d + off[8]);
    a.m2pat = reinterpret_cast<const int*>(d + off[9]);
    a.canon = reinterpret_cast<const int*>(d + off[10]);
    a.quad = reinterpret_cast<const int*>(d + off[11]);
    a.sym_w = reinterpret_cast<const double*>(d + off[12]);
    ctx->ph = tb;
    return PQPH_OK;
}

void ph_tables_free(pqph_ctx* ctx) {
    if (!ctx->ph) return;
    for (auto* list : {&ctx->ph->sched, &ctx->ph->sched_sym})
        for (PhSched* sc : *list)
            if (sc) {
                if (sc->dev) (void)hipFree(sc->dev);
                delete sc;
            }
    if (ctx->ph->dev) (void)hipFree(ctx->ph->dev);
    delete ctx->ph;
    ctx->ph = nullptr;
}

namespace {

long host_nperm(int no, int k) {
    long p = 1;
    for (int i = 0; i < k; ++i) p *= no - i;
    return p;
}

long host_ncomb(int N, int k) {
    return k == 1 ? N : k == 2 ? (long)N * (N - 1) / 2 : (long)N * (N - 1) * (N - 2) / 6;
}

// units of at most U items, U chosen so that no block size has more than
// 60000 units (the grid's second dimension); sym: units only for the output
// patterns that represent their alpha/beta exchange orbit, and the pattern map
// the gather uses for the others
pqph_status ph_schedule(pqph_ctx* ctx, int N, PhSched*& out, bool sym = false) {
    PhTables& tb = *ctx->ph;
    std::vector<PhSched*>& cache = sym ? tb.sched_sym : tb.sched;
    if ((out = cache[N])) return PQPH_OK;
    int srep[3 + 29 + 303], ssgn[3 + 29 + 303];
    spin_pattern_reps(1, srep, ssgn);
    spin_pattern_reps(2, srep + 3, ssgn + 3);
    spin_pattern_reps(3, srep + 32, ssgn + 32);
    const PhArgs& a = tb.args;
    auto items = [&](int n, int m, int c) -> long {
        const PhClass& k = a.cls[c];
        if (k.nout != n || k.nspec > N - n) return 0;
        const int mc = tb.canon_h[(n == 1 ? 0 : n == 2 ? 3 : 32) + m] & 511;
        const long nt = tb.starts_h[k.soff + mc + 1] - tb.starts_h[k.soff + mc];
        return (nt + PH_CHUNK - 1) / PH_CHUNK * host_nperm(N - n, k.nspec);
    };
    long U = 4096;
    for (int n = 1; n <= 3 && n <= N; ++n) {
        const int npat = n == 1 ? 3 : n == 2 ? 29 : 303;
        long tot = 0;
        for (int m = 0; m < npat; ++m)
            for (int c = 0; c < a.nclass; ++c) tot += items(n, m, c);
        // units of size n <= tot / U + (patterns x classes)
        U = std::max(U, tot / (60000 - npat * kMaxClass) + 1);
    }
    std::vector<int> um, uc, ustart;
    std::vector<long> ui0, ui1;
    PhSched* sc = new PhSched();
    size_t first[4] = {};
    for (int n = 1; n <= 3; ++n) {
        const int npat = n == 1 ? 3 : n == 2 ? 29 : 303;
        first[n] = um.size();
        int cnt = 0;
        const int base = n == 1 ? 0 : n == 2 ? 3 : 32;
        for (int m = 0; m < npat; ++m) {
            ustart.push_back(cnt);
            if (n > N || (sym && srep[base + m] != m)) continue;
            for (int c = 0; c < a.nclass; ++c) {
                const long it = items(n, m, c);
                for (long i0 = 0; i0 < it; i0 += U) {
                    um.push_back(m);
                    uc.push_back(c);
                    ui0.push_back(i0);
                    ui1.push_back(std::min(i0 + U, it));
                    ++cnt;
                }
            }
        }
        ustart.push_back(cnt);
        sc->nunit[n] = cnt;
        sc->part_off[n] = sc->part_doubles;
        if (n <= N) sc->part_doubles += (size_t)cnt * host_ncomb(N, n);
    }
    const size_t nu = um.size();
    const size_t bytes = nu * 24 + ustart.size() * 4 + (3 + 29 + 303) * 4 + 64;
    if (hipMalloc(&sc->dev, bytes) != hipSuccess) {
        delete sc;
        return pqph_fail(ctx, PQPH_OOM, "PH schedule: device allocation failed");
    }
    std::vector<char> blob(bytes, 0);
    char* p = blob.data();
    const size_t o_i0 = 0, o_i1 = nu * 8, o_m = nu * 16, o_c = nu * 20, o_us = nu * 24;
    memcpy(p + o_i0, ui0.data(), nu * 8);
    memcpy(p + o_i1, ui1.data(), nu * 8);
    memcpy(p + o_m, um.data(), nu * 4);
    memcpy(p + o_c, uc.data(), nu * 4);
    memcpy(p + o_us, ustart.data(), ustart.size() * 4);
    const size_t o_sp = o_us + ustart.size() * 4;
    int* spin = reinterpret_cast<int*>(p + o_sp);
    for (int i = 0; i < 3 + 29 + 303; ++i) spin[i] = srep[i] | (ssgn[i] < 0 ? 1 << 16 : 0);
    if (hipMemcpy(sc->dev, blob.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(sc->dev);
        delete sc;
        return pqph_fail(ctx, PQPH_DEVICE, "PH schedule: upload failed");
    }
    const char* d = static_cast<const char*>(sc->dev);
    for (int n = 1; n <= 3; ++n) {
        sc->units[n].i0 = reinterpret_cast<const long*>(d + o_i0) + first[n];
        sc->units[n].i1 = reinterpret_cast<const long*>(d + o_i1) + first[n];
        sc->units[n].m = reinterpret_cast<const int*>(d + o_m) + first[n];
        sc->units[n].cls = reinterpret_cast<const int*>(d + o_c) + first[n];
    }
    sc->ustart = reinterpret_cast<const int*>(d + o_us);
    sc->spin = sym ? reinterpret_cast<const int*>(d + o_sp) : nullptr;
    cache[N] = out = sc;
    return PQPH_OK;
}

}  // namespace

pqph_status ph_residual_ws_doubles(pqph_ctx* ctx, int N, size_t* out) {
    pqph_status st = ph_tables_load(ctx);
    if (st) return st;
    PhSched* sc = nullptr;
    if ((st = ph_schedule(ctx, N, sc))) return st;
    *out = sc->part_doubles;
    return PQPH_OK;
}

pqph_status ph_residual_dev(pqph_ctx* ctx, hipStream_t s, int N, const double* h,
                            const double* eri, const double* t, double* r, double* ws, bool spin_sym) {
    pqph_status st = ph_tables_load(ctx);
    if (st) return st;
    PhSched* sc = nullptr;
    if ((st = ph_schedule(ctx, N, sc, spin_sym))) return st;
    for (int n = 1; n <= 3 && n <= N; ++n) {
        if (sc->nunit[n] == 0) continue;
        hipLaunchKernelGGL(k_ph_part, dim3((unsigned)host_ncomb(N, n), (unsigned)sc->nunit[n]),
                           dim3(PH_BLOCK), 0, s, N, n, ctx->ph->args, sc->units[n], h, eri, t,
                           ws + sc->part_off[n]);
        PQPH_HIP(ctx, hipGetLastError());
    }
    const long namp = (long)ph_amp_len(N);
    hipLaunchKernelGGL(k_ph_gather, dim3((unsigned)((namp + 255) / 256)), dim3(256), 0, s, N, namp,
                       ctx->ph->args, sc->ustart, ws + sc->part_off[1], ws + sc->part_off[2],
                       ws + sc->part_off[3], sc->spin, r);
    PQPH_HIP(ctx, hipGetLastError());
    return PQPH_OK;
}

size_t ph_energy_ws_doubles() { return 1024 + 8; }

pqph_status ph_energy_dev(pqph_ctx* ctx, hipStream_t s, int N, const double* h, const double* eri,
                          const double* t, double* out, double* ws) {
    pqph_status st = ph_tables_load(ctx);
    if (st) return st;
    const int G = 1024;
    hipLaunchKernelGGL(k_ph_energy, dim3(G), dim3(256), 0, s, N, ctx->ph->args, h, eri, t, ws);
    PQPH_HIP(ctx, hipGetLastError());
    hipLaunchKernelGGL(k_ph_sum, dim3(1), dim3(64), 0, s, G, ws, out);
    PQPH_HIP(ctx, hipGetLastError());
    return PQPH_OK;
}

pqph_status ph_denominators_dev(pqph_ctx* ctx, hipStream_t s, int N, const double* h, double shift,
                                double* D) {
    pqph_status st = ph_tables_load(ctx);
    if (st) return st;
    const long namp = (long)ph_amp_len(N);
    hipLaunchKernelGGL(k_ph_denom, dim3((unsigned)((namp + 255) / 256)), dim3(256), 0, s, N, namp,
                       ctx->ph->args, h, shift, D);
    PQPH_HIP(ctx, hipGetLastError());
    return PQPH_OK;
}
