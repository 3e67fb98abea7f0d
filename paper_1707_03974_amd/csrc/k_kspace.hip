// Translation-symmetric Hubbard sectors in momentum space (Sec. IV.A).
//
// On an L1 x L2 periodic cluster the Fourier transformed Hamiltonian is Eq. (4):
// the band energies eps_k are diagonal and the interaction (U/N) scatters an
// up electron k -> k+q and a down electron k' -> k'-q, so the total momentum K
// of a basis state is conserved and each K is a sector of about 1/N of the
// real-space dimension.  Orbital i carries the momentum
// (2 pi/L1 (i mod L1), 2 pi/L2 (i div L1)); a momentum is named by its orbital.
//
// Ranking follows the k-space maps of Sec. IV.A:
//   Ck[i][m][k]  strings of m electrons on orbitals 0..i-1 with momentum k
//                (Eq. 5; the orbital added to an i-orbital string is i-1),
//   Ct[i][m][k]  = sum_kd Ck[i][m][k - kd] Ck[N][n_dn][kd] (Eq. 7),
//   single-spin forward map: idx = sum over set bits i (m-th electron, running
//                momentum k including k_i) of Ck[i][m][k] (Eq. 6),
//   spin-full forward map: the down string's own rank plus, for each set up
//                bit, Ct[i][m][k] with the running momentum started at the down
//                string's momentum,
//   and the two backward maps that undo them bit by bit from the top.
// A sector is therefore ordered by the up string, then the down string: the
// vector is a ragged matrix X[up string][down rank within momentum K - K_up],
// and row u starts at the spin-full forward map of (u, lowest down string).
//
// H.v (gather form, H_K real symmetric): for target (u', d') and each q != 0,
// the sources are u = u' with one up electron p -> p - q and d = d' with one
// down electron p' -> p' + q, amplitude (U/N) s_up s_dn, each s = (-1)^(same
// spin electrons strictly between the two orbitals) (the operator order of
// Sec. II.A; the up and down pairs carry no sign across each other).  The sum
// factorises per q: Z_q = sum_moves s_up X[u] (whole source rows, read
// contiguously), then y[u', d'] += sum_{d} s_dn Z_q[d] from a down-move table
// that the k-space forward map fills once per sector.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "pdz_internal.h"
#include "perfect_hash.h"

namespace pdz {

struct KSpace {
    int L1 = 0, L2 = 0, N = 0, K = 0, nmax = 0;
    std::vector<double> eps;
    std::vector<uint8_t> kadd;      // N x N: orbital index of k_a + k_b
    std::vector<uint32_t> Ck;       // (N+1) x (nmax+1) x N
    std::vector<uint64_t> Ct;       // (N+1) x (n_up+1) x N
    std::vector<uint32_t> Ld;       // N: down strings per momentum
    std::vector<uint64_t> dn_off;   // N+1: first down string of each momentum
    std::vector<uint64_t> tb_off;   // N x N: first entry of the down-move table of (target momentum, q)
    std::vector<uint32_t> Lp;       // N: table pitch of each momentum (its down strings, padded so that
                                    // a thread's run of consecutive strings is one aligned load)
    std::vector<uint64_t> cnt_off;  // N+1: first count of each momentum
    uint64_t D_up = 0, D_dn = 0, nrows = 0, entries = 0;
    uint64_t staged = 0;            // source-row elements one H.v stages: sum over rows and q of moves x row length
    uint32_t Lmax = 0;
    int slots = 0;                  // most down moves of one string for one q
    uint8_t* d_kadd = nullptr;
    uint32_t* d_Ck = nullptr;
    uint64_t* d_Ct = nullptr;
    uint32_t* d_Ld = nullptr;
    uint64_t* d_dn_off = nullptr;
    uint64_t* d_tb_off = nullptr;
    double* d_eps = nullptr;
    uint32_t* d_dn_str = nullptr;   // D_dn: down strings, grouped by momentum, ascending within
    double* d_eps_dn = nullptr;     // D_dn: band energy of each down string
    uint32_t* d_Lp = nullptr;
    uint64_t* d_cnt_off = nullptr;
    uint8_t* d_dcnt = nullptr;      // down moves of (string, q): [momentum][q][rank], pitch Lp, 0 past Ld
    void* d_dtab = nullptr;         // entries: source rank | sign in the top bit (16 bits when every
                                    // momentum has < 2^15 down strings, else 32), slot major per
                                    // (momentum, q) with pitch Lp
    bool dtab16 = false;
    int uslots = 0;                 // most up moves of one string for one q
    uint64_t* d_upm = nullptr;      // D_up x (N-1) x uslots: source row start | sign << 63 of each up
                                    // move, in electron order, ~0 past the last
    uint32_t* d_up_str = nullptr;   // D_up: every up string, ascending (backward map of Sec. III)
    uint64_t* d_row_off = nullptr;  // D_up: start of the row of each up string
    uint8_t* d_row_kd = nullptr;    // D_up: momentum K - K_up of the row's down strings
    double* d_eps_up = nullptr;     // D_up: band energy of each up string
    uint32_t* d_rows = nullptr;     // nrows: non-empty rows ordered by down momentum
};

namespace {

constexpr int kKBlock = 256;
constexpr int kKMaxZ = 32 * kKBlock;   // longest row (down strings of one momentum) the H.v kernel takes

struct KArgs {
    const uint8_t* kadd;
    const uint32_t* Ck;
    const uint64_t* Ct;
    const uint32_t* Ld;
    const uint64_t* dn_off;
    const uint64_t* tb_off;
    const double* eps;
    const uint32_t* dn_str;
    const double* eps_dn;
    const uint32_t* Lp;
    const uint64_t* cnt_off;
    const uint8_t* dcnt;
    const void* dtab;
    const uint64_t* upm;
    const uint32_t* up_str;
    const uint64_t* row_off;
    const uint8_t* row_kd;
    const double* eps_up;
    const uint32_t* rows;
    uint64_t nrows, D_up, D_dn, D;
    int N, n_up, n_dn, nmax, K, uslots, slots;
    uint32_t Lmax;
    double u_n;      // U / N
    double diag_u;   // (U / N) n_up n_dn: the q = 0 part of the interaction
};

__device__ __forceinline__ uint32_t ck(const KArgs& a, int i, int m, int k) {
    return a.Ck[((size_t)i * (a.nmax + 1) + m) * a.N + k];
}
__device__ __forceinline__ uint64_t ct(const KArgs& a, int i, int m, int k) {
    return a.Ct[((size_t)i * (a.n_up + 1) + m) * a.N + k];
}

// orbital index of k_a - k_b
__device__ __forceinline__ int ksub(const uint8_t* kadd, int N, int a, int b) {
    // -k_b is the orbital c with kadd[b][c] = 0; the table row of b is searched once per call
    int nb = 0;
    for (int c = 0; c < N; ++c)
        if (kadd[b * N + c] == 0) nb = c;
    return kadd[a * N + nb];
}

// Single-spin k-space forward map: rank among the strings of its momentum; *k_out = that momentum.
__device__ __forceinline__ uint32_t forward_map_k(const KArgs& a, const uint8_t* kadd, uint32_t phi, int* k_out) {
    uint32_t idx = 0;
    int m = 0, k = 0;
    while (phi) {
        const int i = __builtin_ctz(phi);
        phi &= phi - 1u;
        ++m;
        k = kadd[k * a.N + i];
        idx += ck(a, i, m, k);
    }
    *k_out = k;
    return idx;
}

// Single-spin k-space backward map: the string of rank p among the n-electron strings of momentum k.
// Returns false when p is out of range.
__device__ __forceinline__ bool backward_map_k(const KArgs& a, const uint8_t* kadd, uint64_t p, int n, int k,
                                               uint32_t* phi_out) {
    uint32_t phi = 0;
    int m = n;
    for (int i = a.N - 1; i >= 0 && m > 0; --i) {
        const uint32_t c = ck(a, i, m, k);
        if (p >= c) {
            phi |= 1u << i;
            p -= c;
            --m;
            k = ksub(kadd, a.N, k, i);
        }
    }
    *phi_out = phi;
    return m == 0 && p == 0 && k == 0;
}

// Up part of the spin-full forward map: start of the row of up string phi
// whose down strings carry momentum kd.
__device__ __forceinline__ uint64_t row_offset(const KArgs& a, const uint8_t* kadd, uint32_t phi, int kd) {
    uint64_t o = 0;
    int m = 0, k = kd;
    while (phi) {
        const int i = __builtin_ctz(phi);
        phi &= phi - 1u;
        ++m;
        k = kadd[k * a.N + i];
        o += ct(a, i, m, k);
    }
    return o;
}

__device__ __forceinline__ double band_sum(const double* eps, uint32_t phi) {
    double e = 0.0;
    while (phi) {
        e += eps[__builtin_ctz(phi)];
        phi &= phi - 1u;
    }
    return e;
}

// parity of the electrons of phi strictly between orbitals i and j (i != j)
__device__ __forceinline__ bool odd_between(uint32_t phi, int i, int j) {
    const int lo = i < j ? i : j, hi = i < j ? j : i;
    const uint32_t below_hi = (hi >= 32) ? 0xFFFFFFFFu : ((1u << hi) - 1u);
    const uint32_t upto_lo = (lo >= 31) ? 0xFFFFFFFFu : ((2u << lo) - 1u);
    return (__builtin_popcount(phi & below_hi & ~upto_lo) & 1) != 0;
}

__device__ __forceinline__ void stage_kadd(uint8_t* s, const uint8_t* g, int N) {
    for (int i = threadIdx.x; i < N * N; i += blockDim.x) s[i] = g[i];
    __syncthreads();
}

// Down strings of every momentum (backward map per rank) and their band energies.
__global__ __launch_bounds__(kKBlock) void k_kdn_states(const KArgs a, uint32_t* dn_str, double* eps_dn,
                                                         uint32_t* err) {
    __shared__ uint8_t skadd[kMaxSites * kMaxSites];
    stage_kadd(skadd, a.kadd, a.N);
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < a.D_dn; j += (uint64_t)gridDim.x * blockDim.x) {
        int kd = 0;
        while (kd + 1 < a.N && a.dn_off[kd + 1] <= j) ++kd;
        uint32_t phi = 0;
        if (!backward_map_k(a, skadd, j - a.dn_off[kd], a.n_dn, kd, &phi)) atomicOr(err, kErrTable);
        dn_str[j] = phi;
        eps_dn[j] = band_sum(a.eps, phi);
    }
}

// Down-move table: for target string d' (momentum kd) and q != 0, every
// electron p' (ascending) with p' + q empty gives the source string
// d' - p' + (p' + q) of momentum kd + q; its rank comes from the forward map.
template <typename TE>
__global__ __launch_bounds__(kKBlock) void k_kdn_moves(const KArgs a, int slots, uint8_t* dcnt, TE* dtab,
                                                        uint32_t* err) {
    constexpr TE neg = (TE)((TE)1 << (8 * sizeof(TE) - 1));
    __shared__ uint8_t skadd[kMaxSites * kMaxSites];
    stage_kadd(skadd, a.kadd, a.N);
    const uint64_t total = a.D_dn * (uint64_t)a.N;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t j = t / a.N;
        const int q = (int)(t % a.N);
        int kd = 0;
        while (kd + 1 < a.N && a.dn_off[kd + 1] <= j) ++kd;
        const uint64_t dp = j - a.dn_off[kd];
        const uint64_t L = a.Lp[kd];   // pitch
        const uint64_t cidx = a.cnt_off[kd] + (uint64_t)q * L + dp;
        if (q == 0) {
            dcnt[cidx] = 0;
            continue;
        }
        const uint32_t phi = a.dn_str[j];
        const int kds = skadd[kd * a.N + q];
        const uint64_t tb = a.tb_off[kd * a.N + q];
        int s = 0;
        for (uint32_t bits = phi; bits; bits &= bits - 1u) {
            const int p = __builtin_ctz(bits);
            const int pp = skadd[p * a.N + q];
            if ((phi >> pp) & 1u) continue;
            const uint32_t src = phi ^ (1u << p) ^ (1u << pp);
            int ks = 0;
            const uint32_t d = forward_map_k(a, skadd, src, &ks);
            if (ks != kds || d >= a.Ld[kds] || d >= (uint32_t)neg || s >= slots) {
                atomicOr(err, kErrTable);
                continue;
            }
            dtab[tb + (uint64_t)s * L + dp] = (TE)(d | (odd_between(phi, p, pp) ? neg : (TE)0));
            ++s;
        }
        dcnt[cidx] = (uint8_t)s;
    }
}

// Every up string (plain backward map), its row momentum, row start (spin-full
// forward map) and band energy.
__global__ __launch_bounds__(kKBlock) void k_krows(const KArgs a, const uint32_t* binom, uint32_t* up_str,
                                                    uint64_t* row_off, uint8_t* row_kd, double* eps_up) {
    __shared__ uint32_t sC[kBinomStride * kBinomStride];
    __shared__ uint8_t skadd[kMaxSites * kMaxSites];
    stage_binom(sC, binom);
    stage_kadd(skadd, a.kadd, a.N);
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < a.D_up; r += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t phi = backward_map((uint32_t)r, a.n_up, a.N, sC);
        int ku = 0;
        for (uint32_t b = phi; b; b &= b - 1u) ku = skadd[ku * a.N + __builtin_ctz(b)];
        const int kd = ksub(skadd, a.N, a.K, ku);
        up_str[r] = phi;
        row_kd[r] = (uint8_t)kd;
        row_off[r] = row_offset(a, skadd, phi, kd);
        eps_up[r] = band_sum(a.eps, phi);
    }
}

// Up-move table: for up string r (row momentum kd) and q != 0, every electron
// p (ascending) with p - q empty gives the source up string r - p + (p - q),
// whose row (down momentum kd + q) starts at the spin-full forward map of it.
__global__ __launch_bounds__(kKBlock) void k_kup_moves(const KArgs a, uint64_t* upm) {
    __shared__ uint8_t skadd[kMaxSites * kMaxSites];
    stage_kadd(skadd, a.kadd, a.N);
    const uint64_t nq = (uint64_t)(a.N - 1);
    const uint64_t total = a.D_up * nq;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = t / nq;
        const int q = (int)(t % nq) + 1;
        const uint32_t phi = a.up_str[r];
        const int kds = skadd[a.row_kd[r] * a.N + q];
        uint64_t* out = upm + t * a.uslots;
        int s = 0;
        for (uint32_t bits = phi; bits && s < a.uslots; bits &= bits - 1u) {
            const int p = __builtin_ctz(bits);
            const int pm = ksub(skadd, a.N, p, q);
            if ((phi >> pm) & 1u) continue;
            const uint32_t src = phi ^ (1u << p) ^ (1u << pm);
            out[s++] = row_offset(a, skadd, src, kds) | (odd_between(phi, p, pm) ? (1ull << 63) : 0ull);
        }
        for (; s < a.uslots; ++s) out[s] = ~0ull;
    }
}

// Spin-full forward map of (up, dn) pairs; pairs outside the sector get ~0 and an error bit.
__global__ __launch_bounds__(kKBlock) void k_krank(const KArgs a, const uint32_t* up, const uint32_t* dn,
                                                    uint64_t count, uint64_t* idx, uint32_t* err) {
    __shared__ uint8_t skadd[kMaxSites * kMaxSites];
    stage_kadd(skadd, a.kadd, a.N);
    const uint32_t mask = a.N >= 32 ? 0xFFFFFFFFu : ((1u << a.N) - 1u);
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t u = up[t], d = dn[t];
        bool bad = (u & ~mask) || (d & ~mask) || __builtin_popcount(u) != a.n_up || __builtin_popcount(d) != a.n_dn;
        uint64_t r = ~0ull;
        if (!bad) {
            int kd = 0;
            const uint32_t rd = forward_map_k(a, skadd, d, &kd);
            int k = kd;
            for (uint32_t b = u; b; b &= b - 1u) k = skadd[k * a.N + __builtin_ctz(b)];
            if (k != a.K) bad = true;
            else r = row_offset(a, skadd, u, kd) + rd;
        }
        if (bad) atomicOr(err, kErrRankInput);
        idx[t] = r;
    }
}

// Spin-full backward map.
__global__ __launch_bounds__(kKBlock) void k_kunrank(const KArgs a, const uint64_t* idx, uint64_t count, uint32_t* up,
                                                      uint32_t* dn, uint32_t* err) {
    __shared__ uint8_t skadd[kMaxSites * kMaxSites];
    stage_kadd(skadd, a.kadd, a.N);
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t p = idx[t];
        uint32_t u = 0, d = 0;
        bool good = p < a.D;
        if (good) {
            int m = a.n_up, k = a.K;
            for (int i = a.N - 1; i >= 0 && m > 0; --i) {
                const uint64_t c = ct(a, i, m, k);
                if (p >= c) {
                    u |= 1u << i;
                    p -= c;
                    --m;
                    k = ksub(skadd, a.N, k, i);
                }
            }
            good = m == 0 && backward_map_k(a, skadd, p, a.n_dn, k, &d);
        }
        if (!good) {
            atomicOr(err, kErrUnrankInput);
            u = d = 0xFFFFFFFFu;
        }
        up[t] = u;
        dn[t] = d;
    }
}

// H.v of Eq. (4) on one total-momentum sector.  One work group per target up
// string (row); E elements of the row per thread.  Rows are taken in the
// order of their down momentum, a contiguous range per XCD (work group b runs
// on XCD b mod 8), so the down-move tables a range needs stay in that XCD's L2.
// Per momentum transfer q: Z_q = sum over the row's up moves of +-(source row)
// is staged in LDS (contiguous row reads), then every element gathers its
// down moves from Z_q.  Z is double buffered: the staging of the next q and
// the gathers of this one share a phase, one barrier per q.
constexpr uint64_t kMoveNone = ~0ull;
constexpr uint64_t kMoveNeg = 1ull << 63;

__host__ __device__ constexpr size_t hvk_z_bytes(uint32_t Lmax, size_t es) { return ((size_t)Lmax * es + 15) & ~(size_t)15; }

// A thread takes E consecutive elements of a row, read and written as one
// vector where all E lie inside the row (16-byte pieces; memory rows start at
// any element, so memory pieces are element aligned).
template <typename T, int E>
__device__ __forceinline__ void kvec_load(const T* p, T (&o)[E]) {
    constexpr int C = (E * (int)sizeof(T) >= 16) ? 16 / (int)sizeof(T) : E;
    if constexpr (C == 1) {
#pragma unroll
        for (int i = 0; i < E; ++i) o[i] = p[i];
    } else {
        typedef T ct __attribute__((ext_vector_type(C), aligned(sizeof(T))));
#pragma unroll
        for (int c = 0; c < E; c += C) {
            const ct t = *reinterpret_cast<const ct*>(p + c);
#pragma unroll
            for (int i = 0; i < C; ++i) o[c + i] = t[i];
        }
    }
}
template <typename T, int E>
__device__ __forceinline__ void kvec_store(T* p, const T (&v)[E]) {
    constexpr int C = (E * (int)sizeof(T) >= 16) ? 16 / (int)sizeof(T) : E;
    if constexpr (C == 1) {
#pragma unroll
        for (int i = 0; i < E; ++i) p[i] = v[i];
    } else {
        typedef T ct __attribute__((ext_vector_type(C), aligned(sizeof(T))));
#pragma unroll
        for (int c = 0; c < E; c += C) {
            ct t;
#pragma unroll
            for (int i = 0; i < C; ++i) t[i] = v[c + i];
            *reinterpret_cast<ct*>(p + c) = t;
        }
    }
}
// E values at p, aligned to E values (table rows, whose pitch is a multiple of
// E, and the LDS rows Z)
template <typename V, int E>
__device__ __forceinline__ void kvec_store_aligned(V* p, const V (&v)[E]) {
    constexpr int C = (E * (int)sizeof(V) >= 16) ? 16 / (int)sizeof(V) : E;
    if constexpr (C == 1) {
        p[0] = v[0];
    } else {
        typedef V ct __attribute__((ext_vector_type(C)));
#pragma unroll
        for (int c = 0; c < E; c += C) {
            ct t;
#pragma unroll
            for (int i = 0; i < C; ++i) t[i] = v[c + i];
            *reinterpret_cast<ct*>(p + c) = t;
        }
    }
}
template <typename V, int E>
__device__ __forceinline__ void kvec_load_aligned(const V* p, V (&o)[E]) {
    constexpr int C = (E * (int)sizeof(V) >= 16) ? 16 / (int)sizeof(V) : E;
    if constexpr (C == 1) {
        o[0] = p[0];
    } else {
        typedef V ct __attribute__((ext_vector_type(C)));
#pragma unroll
        for (int c = 0; c < E; c += C) {
            const ct t = *reinterpret_cast<const ct*>(p + c);
#pragma unroll
            for (int i = 0; i < C; ++i) o[c + i] = t[i];
        }
    }
}

// Element mapping of a thread's E elements: FP32, E consecutive elements
// (vector loads and stores, measured faster); FP64, elements tid + e * kKBlock
// (the vector form measured slower there).  Either way each element sums the
// same terms in the same order.
template <typename T>
constexpr bool hvk_consecutive() { return sizeof(T) == 4; }

// Z_b[d] = sum over the nv up moves mv[0..nv) of +-(source row)[d], summed in
// move order.  Several moves at a time: the loads of a thread are independent.
template <typename T, int E>
__device__ __forceinline__ void hvk_stage(const T* __restrict__ x, const uint64_t* mv, int nv, uint32_t Ls, T* Zb) {
    if constexpr (!hvk_consecutive<T>()) {
        T z[E];
#pragma unroll
        for (int e = 0; e < E; ++e) z[e] = (T)0;
        int m = 0;
        for (; m + 1 < nv; m += 2) {
            const uint64_t e0 = mv[m], e1 = mv[m + 1];
            const T* r0 = x + (e0 & ~kMoveNeg);
            const T* r1 = x + (e1 & ~kMoveNeg);
            T v0[E], v1[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const uint32_t d = threadIdx.x + e * kKBlock;
                v0[e] = d < Ls ? r0[d] : (T)0;
                v1[e] = d < Ls ? r1[d] : (T)0;
            }
#pragma unroll
            for (int e = 0; e < E; ++e) {
                z[e] += (e0 & kMoveNeg) ? -v0[e] : v0[e];
                z[e] += (e1 & kMoveNeg) ? -v1[e] : v1[e];
            }
        }
        if (m < nv) {
            const uint64_t e0 = mv[m];
            const T* r0 = x + (e0 & ~kMoveNeg);
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const uint32_t d = threadIdx.x + e * kKBlock;
                const T v = d < Ls ? r0[d] : (T)0;
                z[e] += (e0 & kMoveNeg) ? -v : v;
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t d = threadIdx.x + e * kKBlock;
            if (d < Ls) Zb[d] = z[e];
        }
        return;
    }
    const uint32_t d0 = E * threadIdx.x;
    if (d0 >= Ls) return;
    const bool full = d0 + E <= Ls;
    T z[E];
#pragma unroll
    for (int e = 0; e < E; ++e) z[e] = (T)0;
    auto row = [&](uint64_t m, T (&v)[E]) {
        const T* r = x + (m & ~kMoveNeg) + d0;
        if (full) {
            kvec_load<T, E>(r, v);
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = d0 + e < Ls ? r[e] : (T)0;
        }
    };
    int m = 0;
    for (; m + 3 < nv; m += 4) {
        const uint64_t e0 = mv[m], e1 = mv[m + 1], e2 = mv[m + 2], e3 = mv[m + 3];
        T v0[E], v1[E], v2[E], v3[E];
        row(e0, v0);
        row(e1, v1);
        row(e2, v2);
        row(e3, v3);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            z[e] += (e0 & kMoveNeg) ? -v0[e] : v0[e];
            z[e] += (e1 & kMoveNeg) ? -v1[e] : v1[e];
            z[e] += (e2 & kMoveNeg) ? -v2[e] : v2[e];
            z[e] += (e3 & kMoveNeg) ? -v3[e] : v3[e];
        }
    }
    for (; m < nv; ++m) {
        const uint64_t e0 = mv[m];
        T v0[E];
        row(e0, v0);
#pragma unroll
        for (int e = 0; e < E; ++e) z[e] += (e0 & kMoveNeg) ? -v0[e] : v0[e];
    }
    if (full) {
        kvec_store_aligned<T, E>(Zb + d0, z);
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (d0 + e < Ls) Zb[d0 + e] = z[e];
    }
}

// acc[e] += sum over the down moves of element E tid + e of +-Z[source]: the
// counts of the thread's E elements (one load; zero past the row), then the
// table entries four slots at a time (one load per slot), then the LDS reads
// in slot order.  cnt and the slot rows have pitch Lp.
template <typename T, int E, typename TE>
__device__ __forceinline__ void hvk_gather(const TE* __restrict__ dtab, const uint8_t* __restrict__ cnt, uint64_t tb,
                                           uint32_t Lp, uint32_t L, int slots, const T* Z, T* acc) {
    constexpr TE neg = (TE)((TE)1 << (8 * sizeof(TE) - 1));
    constexpr int SB = 4;
    if constexpr (!hvk_consecutive<T>()) {   // element tid + e * kKBlock: counts first, then four slots at a time
        int c[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t dp = threadIdx.x + e * kKBlock;
            c[e] = dp < L ? (int)cnt[dp] : 0;
        }
        for (int s0 = 0; s0 < slots; s0 += SB) {
            TE ent[SB][E];
#pragma unroll
            for (int j = 0; j < SB; ++j)
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const uint32_t dp = threadIdx.x + e * kKBlock;
                    ent[j][e] = (s0 + j < c[e]) ? dtab[tb + (uint64_t)(s0 + j) * Lp + dp] : (TE)0;
                }
#pragma unroll
            for (int j = 0; j < SB; ++j)
#pragma unroll
                for (int e = 0; e < E; ++e)
                    if (s0 + j < c[e]) {
                        const T v = Z[ent[j][e] & (TE)~neg];
                        acc[e] += (ent[j][e] & neg) ? -v : v;
                    }
        }
        return;
    }
    const uint32_t d0 = E * threadIdx.x;
    if (d0 >= L) return;
    uint8_t c8[E];
    kvec_load_aligned<uint8_t, E>(cnt + d0, c8);
    int c[E];
    int cmax = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        c[e] = c8[e];
        cmax = c[e] > cmax ? c[e] : cmax;
    }
    for (int s0 = 0; s0 < slots; s0 += SB) {
        TE ent[SB][E];
#pragma unroll
        for (int j = 0; j < SB; ++j) {
            if (s0 + j < cmax) {
                kvec_load_aligned<TE, E>(dtab + tb + (uint64_t)(s0 + j) * Lp + d0, ent[j]);
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) ent[j][e] = (TE)0;
            }
        }
#pragma unroll
        for (int j = 0; j < SB; ++j)
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (s0 + j < c[e]) {
                    const T v = Z[ent[j][e] & (TE)~neg];
                    acc[e] += (ent[j][e] & neg) ? -v : v;
                }
    }
}

template <typename T, int E, typename TE>
__global__ __launch_bounds__(kKBlock) void k_hvk(const KArgs a, const T* __restrict__ x, T* __restrict__ y,
                                                  const int* skip) {
    if (skip && *skip) return;
    extern __shared__ __align__(16) unsigned char kdyn[];
    const size_t zb = hvk_z_bytes(a.Lmax, sizeof(T));
    T* Zbuf[2] = {reinterpret_cast<T*>(kdyn), reinterpret_cast<T*>(kdyn + zb)};
    uint64_t* smv = reinterpret_cast<uint64_t*>(kdyn + 2 * zb);   // (N-1) x uslots up moves of this row
    __shared__ uint8_t skadd[kMaxSites * kMaxSites];
    __shared__ int snv[kMaxSites];                                 // valid up moves per q
    const uint64_t per = (a.nrows + 7) / 8;
    const uint64_t row = (uint64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (row >= a.nrows) return;
    const uint32_t r = a.rows[row];
    const int nmv = (a.N - 1) * a.uslots;
    for (int i = threadIdx.x; i < nmv; i += kKBlock) smv[i] = a.upm[(uint64_t)r * nmv + i];
    stage_kadd(skadd, a.kadd, a.N);   // its barrier also publishes smv
    const int kd = a.row_kd[r];
    if (threadIdx.x >= 1 && threadIdx.x < a.N) {   // moves of q = threadIdx.x, 0 when its source rows are empty
        const int q = threadIdx.x;
        int n = 0;
        if (a.Ld[skadd[kd * a.N + q]] > 0)
            while (n < a.uslots && smv[(q - 1) * a.uslots + n] != kMoveNone) ++n;
        snv[q] = n;
    }
    __syncthreads();
    const TE* __restrict__ dtab = static_cast<const TE*>(a.dtab);
    const uint32_t L = a.Ld[kd], Lp = a.Lp[kd];
    const uint64_t off = a.row_off[r];
    const uint64_t dbase = a.dn_off[kd];
    const int tid = threadIdx.x;
    T acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = (T)0;
    auto next_q = [&](int q0) {   // next q >= q0 with at least one up move into non-empty rows (uniform)
        int q = q0;
        while (q < a.N && snv[q] == 0) ++q;
        return q;
    };
    int q = next_q(1);
    if (q < a.N) hvk_stage<T, E>(x, smv + (q - 1) * a.uslots, snv[q], a.Ld[skadd[kd * a.N + q]], Zbuf[0]);
    __syncthreads();
    int b = 0;
    while (q < a.N) {
        const int qn = next_q(q + 1);
        if (qn < a.N) hvk_stage<T, E>(x, smv + (qn - 1) * a.uslots, snv[qn], a.Ld[skadd[kd * a.N + qn]], Zbuf[b ^ 1]);
        hvk_gather<T, E, TE>(dtab, a.dcnt + a.cnt_off[kd] + (uint64_t)q * Lp, a.tb_off[kd * a.N + q], Lp, L,
                             a.slots, Zbuf[b], acc);
        __syncthreads();
        q = qn;
        b ^= 1;
    }
    const double eu = a.eps_up[r] + a.diag_u;
    if constexpr (!hvk_consecutive<T>()) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t dp = tid + e * kKBlock;
            if (dp < L) {
                const T dg = (T)(eu + a.eps_dn[dbase + dp]);
                y[off + dp] = dg * x[off + dp] + (T)a.u_n * acc[e];
            }
        }
        return;
    }
    const uint32_t d0 = E * (uint32_t)tid;
    if (d0 + E <= L) {
        T xv[E], yv[E];
        kvec_load<T, E>(x + off + d0, xv);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const T dg = (T)(eu + a.eps_dn[dbase + d0 + e]);
            yv[e] = dg * xv[e] + (T)a.u_n * acc[e];
        }
        kvec_store<T, E>(y + off + d0, yv);
    } else {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const uint32_t dp = d0 + e;
            if (dp < L) {
                const T dg = (T)(eu + a.eps_dn[dbase + dp]);
                y[off + dp] = dg * x[off + dp] + (T)a.u_n * acc[e];
            }
        }
    }
}

size_t hvk_lds_bytes(uint32_t Lmax, size_t es, int N, int uslots) {
    return 2 * hvk_z_bytes(Lmax, es) + (size_t)(N > 1 ? N - 1 : 0) * uslots * 8;
}

template <typename T, int E>
pdz_status set_hvk_lds() {
    const int bytes = (int)hvk_lds_bytes(kKMaxZ, sizeof(T), kMaxSites, kMaxSites);
    PDZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hvk<T, E, uint16_t>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    PDZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hvk<T, E, uint32_t>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    return ok();
}

int hvk_elems(uint32_t Lmax) {
    int e = 1;
    while ((uint64_t)e * kKBlock < Lmax) e *= 2;
    return e;
}

template <typename T, int E>
void launch_hvk_e(const KArgs& a, bool t16, const T* x, T* y, hipStream_t s, const int* skip, size_t lds) {
    const uint64_t per = (a.nrows + 7) / 8;
    if (t16)
        hipLaunchKernelGGL((k_hvk<T, E, uint16_t>), dim3((unsigned)(8 * per)), dim3(kKBlock), lds, s, a, x, y, skip);
    else
        hipLaunchKernelGGL((k_hvk<T, E, uint32_t>), dim3((unsigned)(8 * per)), dim3(kKBlock), lds, s, a, x, y, skip);
}

KArgs kargs(const pdz_problem_s* p) {
    const KSpace* ks = p->ks;
    KArgs a;
    a.kadd = ks->d_kadd;
    a.Ck = ks->d_Ck;
    a.Ct = ks->d_Ct;
    a.Ld = ks->d_Ld;
    a.dn_off = ks->d_dn_off;
    a.tb_off = ks->d_tb_off;
    a.eps = ks->d_eps;
    a.dn_str = ks->d_dn_str;
    a.eps_dn = ks->d_eps_dn;
    a.dcnt = ks->d_dcnt;
    a.Lp = ks->d_Lp;
    a.cnt_off = ks->d_cnt_off;
    a.dtab = ks->d_dtab;
    a.upm = ks->d_upm;
    a.uslots = ks->uslots;
    a.slots = ks->slots;
    a.Lmax = ks->Lmax;
    a.up_str = ks->d_up_str;
    a.row_off = ks->d_row_off;
    a.row_kd = ks->d_row_kd;
    a.eps_up = ks->d_eps_up;
    a.rows = ks->d_rows;
    a.nrows = ks->nrows;
    a.D_up = ks->D_up;
    a.D_dn = ks->D_dn;
    a.D = p->D;
    a.N = ks->N;
    a.n_up = p->n_up;
    a.n_dn = p->n_dn;
    a.nmax = ks->nmax;
    a.K = ks->K;
    a.u_n = p->U / ks->N;
    a.diag_u = p->U / ks->N * p->n_up * p->n_dn;
    return a;
}

unsigned grid_for(uint64_t n, unsigned cu) {
    uint64_t g = (n + kKBlock - 1) / kKBlock;
    const uint64_t gmax = (uint64_t)cu * 16;
    if (g > gmax) g = gmax;
    return (unsigned)(g < 1 ? 1 : g);
}

template <typename T>
pdz_status run_hvk(const pdz_problem_s* p, const T* x, T* y, hipStream_t s, const int* skip) {
    const KArgs a = kargs(p);
    if (a.nrows == 0) return ok();
    const size_t lds = hvk_lds_bytes(p->ks->Lmax, sizeof(T), p->ks->N, p->ks->uslots);
    const bool t16 = p->ks->dtab16;
    switch (hvk_elems(p->ks->Lmax)) {
        case 1: launch_hvk_e<T, 1>(a, t16, x, y, s, skip, lds); break;
        case 2: launch_hvk_e<T, 2>(a, t16, x, y, s, skip, lds); break;
        case 4: launch_hvk_e<T, 4>(a, t16, x, y, s, skip, lds); break;
        case 8: launch_hvk_e<T, 8>(a, t16, x, y, s, skip, lds); break;
        case 16: launch_hvk_e<T, 16>(a, t16, x, y, s, skip, lds); break;
        case 32: launch_hvk_e<T, 32>(a, t16, x, y, s, skip, lds); break;
        default: return fail(PDZ_ERANGE, "momentum sector row longer than the kernel supports");
    }
    PDZ_HIP(hipGetLastError());
    return ok();
}

template <typename V>
pdz_status upload(V** dst, const std::vector<V>& src) {
    PDZ_HIP(hipMalloc(dst, std::max<size_t>(1, src.size()) * sizeof(V)));
    if (!src.empty()) PDZ_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice));
    return ok();
}

template <typename V>
pdz_status alloc(V** dst, uint64_t n) {
    PDZ_HIP(hipMalloc(dst, std::max<uint64_t>(1, n) * sizeof(V)));
    return ok();
}

}  // namespace

void kspace_free(KSpace* ks) {
    if (!ks) return;
    void* ptrs[] = {ks->d_kadd,   ks->d_Ck,      ks->d_Ct,     ks->d_Ld,      ks->d_dn_off, ks->d_tb_off,
                    ks->d_Lp,     ks->d_cnt_off, ks->d_eps,    ks->d_dn_str,  ks->d_eps_dn, ks->d_dcnt,
                    ks->d_dtab,   ks->d_up_str,  ks->d_row_off, ks->d_row_kd, ks->d_eps_up, ks->d_rows,
                    ks->d_upm};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    delete ks;
}

pdz_status kspace_prepare() {
    pdz_status st = ok();
#define KP(T, E) \
    if (st == PDZ_OK) st = set_hvk_lds<T, E>();
    KP(double, 1) KP(double, 2) KP(double, 4) KP(double, 8) KP(double, 16) KP(double, 32)
    KP(float, 1) KP(float, 2) KP(float, 4) KP(float, 8) KP(float, 16) KP(float, 32)
#undef KP
    return st;
}

pdz_status launch_hvk(const pdz_problem_s* p, pdz_dtype dt, const void* x, void* y, hipStream_t s, const int* skip) {
    if (dt == PDZ_F64)
        return run_hvk<double>(p, static_cast<const double*>(x), static_cast<double*>(y), s, skip);
    return run_hvk<float>(p, static_cast<const float*>(x), static_cast<float*>(y), s, skip);
}

// Host set-up of a momentum sector: counting tables, then the device builds
// the string lists, the down-move table and the row table, and the host
// checks that the spin-full forward map lays the rows end to end.
pdz_status kspace_build(pdz_problem_s* p, int L1, int L2, const double* eps, int K, uint32_t* err) {
    KSpace* ks = new KSpace();
    p->ks = ks;
    const int N = L1 * L2;
    ks->L1 = L1;
    ks->L2 = L2;
    ks->N = N;
    ks->K = K;
    ks->nmax = std::max(p->n_up, p->n_dn);
    ks->eps.assign(eps, eps + N);
    ks->kadd.resize((size_t)N * N);
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b)
            ks->kadd[(size_t)a * N + b] =
                (uint8_t)((a % L1 + b % L1) % L1 + L1 * ((a / L1 + b / L1) % L2));
    auto kneg = [&](int b) { return (L1 - b % L1) % L1 + L1 * ((L2 - b / L1) % L2); };
    auto kadd = [&](int a, int b) { return (int)ks->kadd[(size_t)a * N + b]; };
    const int nm = ks->nmax;
    // Eq. (5): C[i][m][k] = C[i-1][m][k] + C[i-1][m-1][k - k_{i-1}], C[0][0][k] = [k = 0]
    std::vector<uint64_t> C((size_t)(N + 1) * (nm + 1) * N, 0);
    auto Cix = [&](int i, int m, int k) { return ((size_t)i * (nm + 1) + m) * N + k; };
    C[Cix(0, 0, 0)] = 1;
    for (int i = 1; i <= N; ++i)
        for (int m = 0; m <= nm; ++m)
            for (int k = 0; k < N; ++k)
                C[Cix(i, m, k)] = C[Cix(i - 1, m, k)] + (m > 0 ? C[Cix(i - 1, m - 1, kadd(k, kneg(i - 1)))] : 0);
    ks->Ck.resize(C.size());
    for (size_t t = 0; t < C.size(); ++t) {
        if (C[t] > 0xFFFFFFFFull) return fail(PDZ_ERANGE, "momentum count exceeds 32 bits");
        ks->Ck[t] = (uint32_t)C[t];
    }
    // Eq. (7): Ct[i][m][k] = sum_kd C[i][m][k - kd] C[N][n_dn][kd]
    const int nu = p->n_up, nd = p->n_dn;
    ks->Ct.assign((size_t)(N + 1) * (nu + 1) * N, 0);
    for (int i = 0; i <= N; ++i)
        for (int m = 0; m <= nu; ++m)
            for (int k = 0; k < N; ++k) {
                uint64_t sum = 0;
                for (int kd = 0; kd < N; ++kd) sum += C[Cix(i, m, kadd(k, kneg(kd)))] * C[Cix(N, nd, kd)];
                ks->Ct[((size_t)i * (nu + 1) + m) * N + k] = sum;
            }
    ks->Ld.resize(N);
    ks->dn_off.assign(N + 1, 0);
    for (int k = 0; k < N; ++k) {
        ks->Ld[k] = (uint32_t)C[Cix(N, nd, k)];
        ks->dn_off[k + 1] = ks->dn_off[k] + ks->Ld[k];
        ks->Lmax = std::max(ks->Lmax, ks->Ld[k]);
    }
    ks->D_dn = ks->dn_off[N];
    ks->D_up = binom(N, nu);
    uint64_t D = 0;
    for (int ku = 0; ku < N; ++ku) D += C[Cix(N, nu, ku)] * ks->Ld[kadd(K, kneg(ku))];
    if (D == 0) return fail(PDZ_ERANGE, "the momentum sector is empty");
    if (ks->D_up > 0xFFFFFFFFull) return fail(PDZ_ERANGE, "too many up strings");
    if (ks->Lmax > (uint32_t)kKMaxZ) return fail(PDZ_ERANGE, "a momentum sector's down strings exceed the H.v kernel's row limit");
    p->D = D;
    ks->slots = std::min(nd, N - nd);
    ks->uslots = std::min(nu, N - nu);
    ks->dtab16 = ks->Lmax < 32768u;
    // pitch: a multiple of 8 and of the run of consecutive strings one H.v thread takes
    const uint32_t pa = (uint32_t)std::max(8, hvk_elems(ks->Lmax));
    ks->Lp.resize(N);
    ks->cnt_off.assign(N + 1, 0);
    for (int k = 0; k < N; ++k) {
        ks->Lp[k] = (ks->Ld[k] + pa - 1) / pa * pa;
        ks->cnt_off[k + 1] = ks->cnt_off[k] + (uint64_t)N * ks->Lp[k];
    }
    ks->tb_off.assign((size_t)N * N, 0);
    uint64_t e = 0;
    for (int k = 0; k < N; ++k)
        for (int q = 0; q < N; ++q) {
            ks->tb_off[(size_t)k * N + q] = e;
            if (q != 0) e += (uint64_t)ks->Lp[k] * ks->slots;
        }
    ks->entries = e;

    DeviceCtx* ctx = nullptr;
    pdz_status st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    if ((st = upload(&ks->d_kadd, ks->kadd)) != PDZ_OK) return st;
    if ((st = upload(&ks->d_Ck, ks->Ck)) != PDZ_OK) return st;
    if ((st = upload(&ks->d_Ct, ks->Ct)) != PDZ_OK) return st;
    if ((st = upload(&ks->d_Ld, ks->Ld)) != PDZ_OK) return st;
    if ((st = upload(&ks->d_dn_off, ks->dn_off)) != PDZ_OK) return st;
    if ((st = upload(&ks->d_tb_off, ks->tb_off)) != PDZ_OK) return st;
    if ((st = upload(&ks->d_Lp, ks->Lp)) != PDZ_OK) return st;
    if ((st = upload(&ks->d_cnt_off, ks->cnt_off)) != PDZ_OK) return st;
    if ((st = upload(&ks->d_eps, ks->eps)) != PDZ_OK) return st;
    if ((st = alloc(&ks->d_dn_str, ks->D_dn)) != PDZ_OK) return st;
    if ((st = alloc(&ks->d_eps_dn, ks->D_dn)) != PDZ_OK) return st;
    if ((st = alloc(&ks->d_dcnt, ks->cnt_off[N])) != PDZ_OK) return st;
    PDZ_HIP(hipMemset(ks->d_dcnt, 0, ks->cnt_off[N]));   // padding past Ld: no moves
    if (ks->dtab16) {
        uint16_t* t = nullptr;
        if ((st = alloc(&t, ks->entries)) != PDZ_OK) return st;
        ks->d_dtab = t;
    } else {
        uint32_t* t = nullptr;
        if ((st = alloc(&t, ks->entries)) != PDZ_OK) return st;
        ks->d_dtab = t;
    }
    PDZ_HIP(hipMemset(ks->d_dtab, 0, ks->entries * (ks->dtab16 ? 2 : 4)));
    if ((st = alloc(&ks->d_upm, ks->D_up * (uint64_t)(N > 1 ? N - 1 : 0) * ks->uslots)) != PDZ_OK) return st;
    if ((st = alloc(&ks->d_up_str, ks->D_up)) != PDZ_OK) return st;
    if ((st = alloc(&ks->d_row_off, ks->D_up)) != PDZ_OK) return st;
    if ((st = alloc(&ks->d_row_kd, ks->D_up)) != PDZ_OK) return st;
    if ((st = alloc(&ks->d_eps_up, ks->D_up)) != PDZ_OK) return st;

    const KArgs a = kargs(p);
    const unsigned cu = (unsigned)ctx->cu_count;
    hipLaunchKernelGGL(k_kdn_states, dim3(grid_for(ks->D_dn, cu)), dim3(kKBlock), 0, nullptr, a, ks->d_dn_str,
                       ks->d_eps_dn, err);
    PDZ_HIP(hipGetLastError());
    if (ks->dtab16)
        hipLaunchKernelGGL(k_kdn_moves<uint16_t>, dim3(grid_for(ks->D_dn * N, cu)), dim3(kKBlock), 0, nullptr, a,
                           ks->slots, ks->d_dcnt, static_cast<uint16_t*>(ks->d_dtab), err);
    else
        hipLaunchKernelGGL(k_kdn_moves<uint32_t>, dim3(grid_for(ks->D_dn * N, cu)), dim3(kKBlock), 0, nullptr, a,
                           ks->slots, ks->d_dcnt, static_cast<uint32_t*>(ks->d_dtab), err);
    PDZ_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_krows, dim3(grid_for(ks->D_up, cu)), dim3(kKBlock), 0, nullptr, a, ctx->binom, ks->d_up_str,
                       ks->d_row_off, ks->d_row_kd, ks->d_eps_up);
    PDZ_HIP(hipGetLastError());
    if (N > 1 && ks->uslots > 0) {
        hipLaunchKernelGGL(k_kup_moves, dim3(grid_for(ks->D_up * (uint64_t)(N - 1), cu)), dim3(kKBlock), 0, nullptr, a,
                           ks->d_upm);
        PDZ_HIP(hipGetLastError());
    }
    PDZ_HIP(hipDeviceSynchronize());
    uint32_t word = 0;
    PDZ_HIP(hipMemcpy(&word, err, sizeof(word), hipMemcpyDeviceToHost));
    if (word & kErrTable) return fail(PDZ_EDEVICE, "momentum table build: a k-space map left its range");

    // rows laid end to end by the spin-full forward map; non-empty rows by down momentum
    std::vector<uint64_t> off(ks->D_up);
    std::vector<uint8_t> rkd(ks->D_up);
    std::vector<uint32_t> ups(ks->D_up);
    std::vector<uint8_t> cnt(ks->cnt_off[N]);
    PDZ_HIP(hipMemcpy(off.data(), ks->d_row_off, off.size() * 8, hipMemcpyDeviceToHost));
    PDZ_HIP(hipMemcpy(rkd.data(), ks->d_row_kd, rkd.size(), hipMemcpyDeviceToHost));
    PDZ_HIP(hipMemcpy(ups.data(), ks->d_up_str, ups.size() * 4, hipMemcpyDeviceToHost));
    PDZ_HIP(hipMemcpy(cnt.data(), ks->d_dcnt, cnt.size(), hipMemcpyDeviceToHost));
    uint64_t run = 0;
    std::vector<std::vector<uint32_t>> by_kd(N);
    for (uint64_t r = 0; r < ks->D_up; ++r) {
        if (off[r] != run) return fail(PDZ_EDEVICE, "spin-full forward map does not lay the rows end to end");
        run += ks->Ld[rkd[r]];
        if (ks->Ld[rkd[r]] > 0) by_kd[rkd[r]].push_back((uint32_t)r);
    }
    if (run != D) return fail(PDZ_EDEVICE, "row lengths do not add up to the sector dimension");
    std::vector<uint32_t> rows;
    for (int k = 0; k < N; ++k) rows.insert(rows.end(), by_kd[k].begin(), by_kd[k].end());
    ks->nrows = rows.size();
    if ((st = upload(&ks->d_rows, rows)) != PDZ_OK) return st;
    // structural nonzeros: D diagonal entries plus, per row and q, up moves x down moves
    std::vector<uint64_t> mdn((size_t)N * N, 0);   // [momentum][q]: down moves summed over the strings
    for (int k = 0; k < N; ++k)
        for (int q = 1; q < N; ++q) {
            uint64_t sum = 0;
            const uint8_t* c = cnt.data() + ks->cnt_off[k] + (uint64_t)q * ks->Lp[k];
            for (uint32_t d = 0; d < ks->Ld[k]; ++d) sum += c[d];
            mdn[(size_t)k * N + q] = sum;
        }
    uint64_t nnz = D;
    for (uint64_t r = 0; r < ks->D_up; ++r) {
        const uint32_t phi = ups[r];
        for (int q = 1; q < N; ++q) {
            uint64_t mu = 0;
            for (uint32_t b = phi; b; b &= b - 1u) {
                const int pbit = __builtin_ctz(b);
                if (!((phi >> kadd(pbit, kneg(q))) & 1u)) ++mu;
            }
            nnz += mu * mdn[(size_t)rkd[r] * N + q];
            if (ks->Ld[rkd[r]] > 0) ks->staged += mu * ks->Ld[kadd(rkd[r], q)];
        }
    }
    p->nnz = nnz;
    return ok();
}

}  // namespace pdz

using namespace pdz;

extern "C" {

pdz_status pdz_kspace_band(int32_t L1, int32_t L2, const pdz_bond* bonds, int32_t n_bonds, double* eps) {
    if (!eps || (n_bonds > 0 && !bonds)) return fail(PDZ_EINVAL, "NULL argument");
    if (L1 < 1 || L2 < 1 || L1 * L2 > kMaxSites) return fail(PDZ_ERANGE, "L1 * L2 must be in [1, 32]");
    if (n_bonds < 0) return fail(PDZ_EINVAL, "n_bonds < 0");
    const int N = L1 * L2;
    std::vector<double> t((size_t)N * N, 0.0);   // symmetric hopping matrix, repeated bonds add
    for (int b = 0; b < n_bonds; ++b) {
        const pdz_bond& bd = bonds[b];
        if (bd.i < 0 || bd.i >= N || bd.j < 0 || bd.j >= N || bd.i == bd.j || !std::isfinite(bd.t))
            return fail(PDZ_EINVAL, "bond " + std::to_string(b) + " is invalid");
        t[(size_t)bd.i * N + bd.j] += bd.t;
        t[(size_t)bd.j * N + bd.i] += bd.t;
    }
    auto shift = [&](int s, int dx, int dy) { return (s % L1 + dx) % L1 + L1 * ((s / L1 + dy) % L2); };
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            for (int dir = 0; dir < 2; ++dir) {
                const int a = shift(i, dir == 0, dir == 1), b = shift(j, dir == 0, dir == 1);
                if (std::fabs(t[(size_t)a * N + b] - t[(size_t)i * N + j]) > 1e-12 * (1.0 + std::fabs(t[(size_t)i * N + j])))
                    return fail(PDZ_EINVAL, "bond list is not invariant under the lattice translations");
            }
    // eps_k = -(1/N) sum_{i != j} t_ij cos(k . (r_j - r_i)), every bond counted in both directions
    const double two_pi = 6.283185307179586476925286766559;
    for (int k = 0; k < N; ++k) {
        const int k1 = k % L1, k2 = k / L1;
        double e = 0.0;
        for (int b = 0; b < n_bonds; ++b) {
            const int dx = bonds[b].j % L1 - bonds[b].i % L1, dy = bonds[b].j / L1 - bonds[b].i / L1;
            e -= 2.0 * bonds[b].t * std::cos(two_pi * ((double)k1 * dx / L1 + (double)k2 * dy / L2));
        }
        eps[k] = e / N;
    }
    return ok();
}

pdz_status pdz_kspace_problem_create(int32_t L1, int32_t L2, const double* eps, double U, int32_t n_up,
                                     int32_t n_dn, int32_t K, pdz_problem* out) {
    if (!out || !eps) return fail(PDZ_EINVAL, "NULL argument");
    *out = nullptr;
    if (L1 < 1 || L2 < 1 || L1 * L2 > kMaxSites) return fail(PDZ_ERANGE, "L1 * L2 must be in [1, 32]");
    const int N = L1 * L2;
    if (n_up < 0 || n_up > N || n_dn < 0 || n_dn > N) return fail(PDZ_EINVAL, "n_up and n_dn must be in [0, N]");
    if (K < 0 || K >= N) return fail(PDZ_EINVAL, "K must be an orbital index in [0, N)");
    if (!std::isfinite(U)) return fail(PDZ_EINVAL, "U is not finite");
    for (int k = 0; k < N; ++k)
        if (!std::isfinite(eps[k])) return fail(PDZ_EINVAL, "eps is not finite");
    DeviceCtx* ctx = nullptr;
    pdz_status st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    pdz_problem_s* p = new pdz_problem_s();
    p->device = ctx->device;
    p->N = N;
    p->n_up = n_up;
    p->n_dn = n_dn;
    p->U = U;
    p->hv_path = 2;
    st = kspace_build(p, L1, L2, eps, K, ctx->err);
    if (st != PDZ_OK) {
        const std::string msg = pdz_last_error();
        pdz_problem_destroy(p);
        return fail(st, msg);
    }
    p->up.D = p->ks->D_up;
    p->dn.D = p->ks->D_dn;
    *out = p;
    return ok();
}

pdz_status pdz_kspace_rank(pdz_problem p, const uint32_t* up, const uint32_t* dn, uint64_t count, uint64_t* idx,
                           void* stream) {
    if (!p || !p->ks) return fail(PDZ_EINVAL, "not a momentum-space problem");
    if (count > 0 && (!up || !dn || !idx)) return fail(PDZ_EINVAL, "NULL array");
    if (count == 0) return ok();
    DeviceCtx* ctx = nullptr;
    pdz_status st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    hipLaunchKernelGGL(k_krank, dim3(grid_for(count, (unsigned)ctx->cu_count)), dim3(kKBlock), 0, (hipStream_t)stream,
                       kargs(p), up, dn, count, idx, ctx->err);
    PDZ_HIP(hipGetLastError());
    return ok();
}

pdz_status pdz_kspace_unrank(pdz_problem p, const uint64_t* idx, uint64_t count, uint32_t* up, uint32_t* dn,
                             void* stream) {
    if (!p || !p->ks) return fail(PDZ_EINVAL, "not a momentum-space problem");
    if (count > 0 && (!up || !dn || !idx)) return fail(PDZ_EINVAL, "NULL array");
    if (count == 0) return ok();
    DeviceCtx* ctx = nullptr;
    pdz_status st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    hipLaunchKernelGGL(k_kunrank, dim3(grid_for(count, (unsigned)ctx->cu_count)), dim3(kKBlock), 0,
                       (hipStream_t)stream, kargs(p), idx, count, up, dn, ctx->err);
    PDZ_HIP(hipGetLastError());
    return ok();
}

pdz_status pdz_kspace_info(pdz_problem p, int32_t* L1, int32_t* L2, int32_t* K, uint32_t* row_max, uint64_t* rows,
                           uint64_t* staged) {
    if (!p || !p->ks) return fail(PDZ_EINVAL, "not a momentum-space problem");
    if (L1) *L1 = p->ks->L1;
    if (L2) *L2 = p->ks->L2;
    if (K) *K = p->ks->K;
    if (row_max) *row_max = p->ks->Lmax;
    if (rows) *rows = p->ks->nrows;
    if (staged) *staged = p->ks->staged;
    return ok();
}

}  // extern "C"
