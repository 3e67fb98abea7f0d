// Inversion-parity subspaces (Sec. IV.B).
//
// F maps site i to N-1-i in every creation operator (a chain reversed; on an
// Lx x Ly cluster numbered s = x + Lx*y, the point inversion through its
// centre).  On a basis state it reverses both strings and multiplies by the
// sign of restoring the operator order of Sec. II.A, which for n electrons of
// one spin is (-1)^(n(n-1)/2): sigma = (-1)^(n_up(n_up-1)/2 + n_dn(n_dn-1)/2)
// for the whole sector.  With mirror-symmetric bonds F commutes with H and
// each sector splits into P = +1 and P = -1.
//
// Ranking by the decision tree of Sec. IV.B, per string: at depth d the pair
// (bit N-1-d, bit d) is class A (0,1), B (0,0) or C (1,1); (1,0) marks the
// mirror image of an A string.  An A string ends the walk with the plain
// forward map of its inner bits; B adds the count of the A node, C that of the
// A and B nodes (the counts C_{i-2}^{m-1} and S_{i-2}^m of the paper's
// recursion S_i^m = C_{i-2}^{m-1} + S_{i-2}^m + S_{i-2}^{m-2}).  A string whose
// pairs are all B or C is a palindrome.  Representatives: A strings and
// palindromes; their tree index is that forward map.
//
// Two spins: the up string decides the representative, the down string when
// the up string is a palindrome.  Rows are the up representatives in tree
// order; a non-palindromic row holds every down string in mirror pairs (each
// down representative in tree order followed by its mirror image), then the
// down palindromes: the mirror of a column is its neighbour and pairs start at
// even columns; a
// palindromic row holds the down representatives in tree order (down
// palindromes only when sigma = P).  Basis vector of a representative r:
// (|r> + P F|r>)/sqrt(2), or |r> when F|r> = P|r>.
//
// H.v (gather form, H_P real symmetric): for a target t and each term of H
// (diagonal, every hop of either spin, from the real-space hop tables) with
// source s, y_t += w_t w_s H[t, s] x[rep(s)], with w_t = sqrt(2) for a pair
// state and 1 for a self-mapped one, w_s = 1/sqrt(2) (pair state; times
// P sigma when s is the image of its representative) or 1 (self-mapped).
// rep(s) comes from per-string tables: class, mirror rank, row, column.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>
#include <type_traits>
#include <vector>

#include "pdz_internal.h"
#include "perfect_hash.h"

namespace pdz {

struct ParSpace {
    int P = 1, sigma = 1;
    uint64_t nrows = 0, Lp = 0, n_dn_reps = 0;
    uint8_t* d_ucls = nullptr;     // D_up: 0 A representative, 1 mirror image, 2 palindrome
    uint32_t* d_uinv = nullptr;    // D_up: rank of the mirrored string
    uint32_t* d_utree = nullptr;   // D_up: tree index (of the string, or of its mirror for an image)
    uint32_t* d_urow = nullptr;    // D_up: row of the representative of the string's orbit
    uint8_t* d_dcls = nullptr;
    uint32_t* d_dinv = nullptr;
    uint32_t* d_dtree = nullptr;
    uint32_t* d_dcol = nullptr;    // D_dn: column in a palindromic row (representatives), ~0 when excluded
    uint32_t* d_dlist = nullptr;   // Lp: down rank of each column of a palindromic row
    uint32_t* d_dcolf = nullptr;   // D_dn: column of each down string in a full row
    uint32_t* d_dlistf = nullptr;  // D_dn: down rank of each column of a full row
    uint32_t* d_fmir = nullptr;    // D_dn: column of the mirror of a full row's column
    uint8_t* d_fcnt = nullptr;     // D_dn: down hops of a full row's column
    uint32_t* d_fell = nullptr;    // max_hops x D_dn: those hops as target column | amplitude index << 24
    uint32_t* d_fell2 = nullptr;   // ceil(max_hops / 2) x D_dn: the same hops as 16-bit pairs (column |
                                   // amplitude << pshift), hop 2i in the low half; null when they do not fit
    int pshift = 0;
    bool wide_table = false;       // PDZ_PARITY_WIDE_TABLE=1: keep the 32-bit table (its test)
    uint64_t* d_fup = nullptr;     // n_full x max_hops: up hops of each full row, source row start |
                                   // class << 40 | amplitude index << 48, ~0 past the last
    int fup_stride = 0;
    uint64_t npair2 = 0;           // columns of a full row taken by mirror pairs (the rest: palindromes)
    bool force_gather = false;     // PDZ_PARITY_GATHER=1: full rows by the one-pass gather kernel (its test)
    int up_lpr = 64;               // up pass lanes per row (slab width / up_cols); PDZ_PARITY_UP_LANES = 16, 32, 64
    uint32_t* d_row_rank = nullptr;   // nrows: up rank of each row
    uint64_t* d_row_off = nullptr;    // nrows + 1
    uint8_t* d_row_pal = nullptr;     // nrows
    uint32_t* d_rows_full = nullptr;  // rows of non-palindromic up strings (every down string)
    uint32_t* d_rows_pal = nullptr;   // rows of palindromic up strings
    uint64_t n_full = 0, n_pal = 0;
    uint32_t* d_S = nullptr;          // (N+1) x (nmax+1): representatives (palindromes included), Sec. IV.B
    // Scheduled down pass of the full rows (two-pass form): the gather
    // schedule of the column hop table (fcnt, fell), the down string of each
    // column, and the rows in groups of consecutive full rows that follow
    // each other in memory, at most 1 (index 0, FP64) or 3 (index 1, FP32)
    // rows a group.  No schedule (rows shorter than 1024 or longer than a
    // plane, more than two hop magnitudes): the looped down pass.
    DownSchedule fsched;
    uint32_t* d_col_dn = nullptr;
    uint64_t* d_goff[2] = {nullptr, nullptr};
    uint8_t* d_gnr[2] = {nullptr, nullptr};
    uint32_t* d_grp_up[2] = {nullptr, nullptr};
    uint64_t ngroups[2] = {0, 0};
    bool force_loop = false;          // PDZ_PARITY_LOOPED_DOWN=1: the looped down pass (its test)
};

namespace {

constexpr int kPBlock = 256;
constexpr uint8_t kClsA = 0, kClsImage = 1, kClsPal = 2;
constexpr uint32_t kNoCol = 0xFFFFFFFFu;
constexpr int kPHopNB = 8;   // hops of an element whose lookups are in flight together

__device__ __forceinline__ uint32_t mirror(uint32_t phi, int N) {
    return N >= 32 ? __builtin_bitreverse32(phi) : (__builtin_bitreverse32(phi) >> (32 - N));
}

__device__ __forceinline__ uint8_t classify(uint32_t phi, int N) {
    for (int d = 0; d < N / 2; ++d) {
        const uint32_t hi = (phi >> (N - 1 - d)) & 1u, lo = (phi >> d) & 1u;
        if (hi != lo) return lo ? kClsA : kClsImage;
    }
    return kClsPal;
}

// Tree index of a representative string (A or palindrome): the decision-tree forward map.
__device__ __forceinline__ uint32_t forward_map_inversion(uint32_t phi, int n, int N, const uint32_t* sC,
                                                          const uint32_t* S, int smax) {
    uint32_t idx = 0;
    int m = n, i = N;
    for (int d = 0; d < N / 2; ++d) {
        const uint32_t hi = (phi >> (N - 1 - d)) & 1u, lo = (phi >> d) & 1u;
        const uint32_t a_cnt = (m >= 1 && i >= 2) ? sC[(i - 2) * kBinomStride + (m - 1)] : 0u;
        if (hi == 0u && lo == 1u) {
            const int w = i - 2;
            const uint32_t inner = w > 0 ? ((phi >> (d + 1)) & ((w >= 32) ? 0xFFFFFFFFu : ((1u << w) - 1u))) : 0u;
            return idx + forward_map(inner, sC);
        }
        if (hi == 0u) {
            idx += a_cnt;
        } else {
            idx += a_cnt + S[(i - 2) * (smax + 1) + m];
            m -= 2;
        }
        i -= 2;
    }
    return idx;
}

// Per string of one spin sector: class, mirror rank, tree index.
__global__ __launch_bounds__(kPBlock) void k_pinfo(const uint32_t* binom, const uint32_t* S, int smax, int N, int n,
                                                    const uint32_t* states, uint64_t D, uint8_t* cls, uint32_t* inv,
                                                    uint32_t* tree) {
    __shared__ uint32_t sC[kBinomStride * kBinomStride];
    stage_binom(sC, binom);
    for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < D; r += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t phi = states[r];
        const uint32_t rev = mirror(phi, N);
        const uint8_t c = classify(phi, N);
        cls[r] = c;
        inv[r] = forward_map(rev, sC);
        tree[r] = forward_map_inversion(c == kClsImage ? rev : phi, n, N, sC, S, smax);
    }
}

struct PArgs {
    const uint32_t* up_states;
    const uint32_t* dn_states;
    const uint8_t* up_cnt;
    const uint32_t* up_ell;
    const uint8_t* dn_cnt;
    const uint32_t* dn_ell;
    uint64_t Dup, Ddn;
    const uint8_t* ucls;
    const uint32_t* urow;
    const uint8_t* dcls;
    const uint32_t* dinv;
    const uint32_t* dcol;
    const uint32_t* dlist;
    const uint32_t* dcolf;
    const uint32_t* dlistf;
    const uint32_t* fmir;
    const uint8_t* fcnt;
    const uint32_t* fell;
    const uint32_t* fell2;
    int pshift;
    const uint64_t* fup;
    int fup_stride;
    uint64_t npair2;
    const uint32_t* row_rank;
    const uint64_t* row_off;
    const uint8_t* row_pal;
    const uint32_t* uinv;
    const uint32_t* rows;   // the rows a launch covers
    uint64_t nrows, nlist, Lp;
    double U;
    double ps;      // P * sigma
    int pal_in;     // self-mapped states belong to this parity (sigma == P)
};

// *out = sum of v over a work group of kPBlock threads, in a fixed order
// (every thread of the group calls it).
__device__ __forceinline__ void block_sum_store(double v, double* out) {
    __shared__ double red[kPBlock / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kPBlock / 64; ++w) t += red[w];
        *out = t;
    }
}

// Rows of palindromic up strings (few): one work group per row, threads over
// its columns (down representatives).
// With dotp set, work group b writes dotp[b] = its elements' sum of x y.
template <typename T>
__global__ __launch_bounds__(kPBlock) void k_hvp(const PArgs a, const T* __restrict__ coef, const T* __restrict__ x,
                                                  T* __restrict__ y, const int* skip, double* dotp) {
    if (skip && *skip) return;
    const T r2 = (T)1.4142135623730950488, ir2 = (T)0.70710678118654752440, ps = (T)a.ps;
    // work group b: row b / chunks, columns (b % chunks) * kPBlock + thread
    const uint64_t chunks = (a.Lp + kPBlock - 1) / kPBlock;
    double dsum = 0.0;
    for (uint64_t b = blockIdx.x; b < a.nlist * chunks; b += gridDim.x) {
        const uint64_t k = a.rows[b / chunks];
        const uint32_t ru = a.row_rank[k];
        const uint64_t off = a.row_off[k];
        const uint64_t len = a.row_off[k + 1] - off;
        const uint32_t phu = a.up_states[ru];
        const int nup_h = a.up_cnt[ru];
        const uint64_t c = (b % chunks) * kPBlock + threadIdx.x;
        if (c < len) {
            const uint32_t rd = a.dlist[c];
            const T wt = a.dcls[rd] == kClsPal ? (T)1 : r2;
            const T xc = x[off + c];
            T acc = (T)(a.U * __builtin_popcount(phu & a.dn_states[rd])) * xc;
            const int ndh = a.dn_cnt[rd];
            // hops in order, kPHopNB at a time: each level of a batch's lookups
            // (entries, classes, columns, operands) is loaded before the next
            int h = 0;
            for (; h + kPHopNB <= ndh; h += kPHopNB) {   // the up string stays: a column of this row
                uint32_t rd2[kPHopNB], col[kPHopNB];
                uint8_t cl[kPHopNB];
                T cf[kPHopNB], xv[kPHopNB];
#pragma unroll
                for (int j = 0; j < kPHopNB; ++j) {
                    const uint32_t e = a.dn_ell[(uint64_t)(h + j) * a.Ddn + rd];
                    rd2[j] = e & kTargetMask;
                    cf[j] = coef[e >> kTargetBits];
                }
#pragma unroll
                for (int j = 0; j < kPHopNB; ++j) cl[j] = a.dcls[rd2[j]];
#pragma unroll
                for (int j = 0; j < kPHopNB; ++j) col[j] = a.dcol[cl[j] == kClsImage ? a.dinv[rd2[j]] : rd2[j]];
#pragma unroll
                for (int j = 0; j < kPHopNB; ++j)   // excluded palindromes have no column
                    xv[j] = (cl[j] != kClsPal || a.pal_in) ? x[off + col[j]] : (T)0;
#pragma unroll
                for (int j = 0; j < kPHopNB; ++j) {
                    if (cl[j] == kClsA)
                        acc += wt * ir2 * cf[j] * xv[j];
                    else if (cl[j] == kClsImage)
                        acc += wt * ir2 * ps * cf[j] * xv[j];
                    else if (a.pal_in)
                        acc += wt * cf[j] * xv[j];
                }
            }
            for (; h < ndh; ++h) {
                const uint32_t e = a.dn_ell[(uint64_t)h * a.Ddn + rd];
                const uint32_t rd2 = e & kTargetMask;
                const T cf = coef[e >> kTargetBits];
                const uint8_t cl = a.dcls[rd2];
                if (cl == kClsA)
                    acc += wt * ir2 * cf * x[off + a.dcol[rd2]];
                else if (cl == kClsImage)
                    acc += wt * ir2 * ps * cf * x[off + a.dcol[a.dinv[rd2]]];
                else if (a.pal_in)
                    acc += wt * cf * x[off + a.dcol[rd2]];
            }
            // one hop never leaves a palindrome a palindrome: a full row
            const uint32_t cA = a.dcolf[rd], cI = a.dcolf[a.dinv[rd]];
            h = 0;
            for (; h + kPHopNB <= nup_h; h += kPHopNB) {
                uint32_t ru2[kPHopNB];
                uint64_t off2[kPHopNB];
                bool isA[kPHopNB];
                T cf[kPHopNB], xv[kPHopNB];
#pragma unroll
                for (int j = 0; j < kPHopNB; ++j) {
                    const uint32_t e = a.up_ell[(uint64_t)(h + j) * a.Dup + ru];
                    ru2[j] = e & kTargetMask;
                    cf[j] = coef[e >> kTargetBits];
                }
#pragma unroll
                for (int j = 0; j < kPHopNB; ++j) {
                    off2[j] = a.row_off[a.urow[ru2[j]]];
                    isA[j] = a.ucls[ru2[j]] == kClsA;
                }
#pragma unroll
                for (int j = 0; j < kPHopNB; ++j) xv[j] = x[off2[j] + (isA[j] ? cA : cI)];
#pragma unroll
                for (int j = 0; j < kPHopNB; ++j) {
                    if (isA[j])
                        acc += wt * ir2 * cf[j] * xv[j];
                    else
                        acc += wt * ir2 * ps * cf[j] * xv[j];
                }
            }
            for (; h < nup_h; ++h) {
                const uint32_t e = a.up_ell[(uint64_t)h * a.Dup + ru];
                const uint32_t ru2 = e & kTargetMask;
                const T cf = coef[e >> kTargetBits];
                const uint64_t off2 = a.row_off[a.urow[ru2]];
                if (a.ucls[ru2] == kClsA)
                    acc += wt * ir2 * cf * x[off2 + cA];
                else
                    acc += wt * ir2 * ps * cf * x[off2 + cI];
            }
            y[off + c] = acc;
            dsum += (double)xc * (double)acc;
        }
    }
    if (dotp) block_sum_store(dsum, dotp + blockIdx.x);
}

// Rows of non-palindromic up strings in one pass, for rows too long for the
// LDS of the two-pass form or with more up hops than a wave holds: one work
// group per row, threads over its columns.  Down hops stay in the row
// (column-space hop table); an up hop reads the source row at the same column
// (representative) or at the mirror column, its neighbour (image).
template <typename T>
__global__ __launch_bounds__(kPBlock) void k_hvp_full(const PArgs a, const T* __restrict__ coef,
                                                       const T* __restrict__ x, T* __restrict__ y, const int* skip) {
    if (skip && *skip) return;
    const T r2 = (T)1.4142135623730950488, ir2 = (T)0.70710678118654752440, ps = (T)a.ps;
    const uint32_t Dd = (uint32_t)a.Ddn;
    for (uint64_t kk = blockIdx.x; kk < a.nlist; kk += gridDim.x) {
        const uint64_t k = a.rows[kk];
        const uint32_t ru = a.row_rank[k];
        const uint64_t off = a.row_off[k];
        const uint32_t phu = a.up_states[ru];
        const int nup_h = a.up_cnt[ru];
        for (uint32_t c = threadIdx.x; c < Dd; c += kPBlock) {
            const uint32_t rd = a.dlistf[c];
            T acc = (T)(a.U * __builtin_popcount(phu & a.dn_states[rd])) * x[off + c];
            const int ndh = a.fcnt[c];
            for (int h = 0; h < ndh; ++h) {
                const uint32_t e = a.fell[(uint64_t)h * Dd + c];
                acc += coef[e >> kTargetBits] * x[off + (e & kTargetMask)];
            }
            for (int h = 0; h < nup_h; ++h) {
                const uint32_t e = a.up_ell[(uint64_t)h * a.Dup + ru];
                const uint32_t ru2 = e & kTargetMask;
                const T cf = coef[e >> kTargetBits];
                const uint8_t cl = a.ucls[ru2];
                const uint64_t off2 = a.row_off[a.urow[ru2]];
                if (cl == kClsA) {
                    acc += r2 * ir2 * cf * x[off2 + c];
                } else if (cl == kClsImage) {
                    acc += r2 * ir2 * ps * cf * x[off2 + a.fmir[c]];
                } else {   // palindromic source up string: its row holds representatives only
                    const uint8_t dc = a.dcls[rd];
                    if (dc == kClsA)
                        acc += r2 * ir2 * cf * x[off2 + a.dcol[rd]];
                    else if (dc == kClsImage)
                        acc += r2 * ir2 * ps * cf * x[off2 + a.dcol[a.dinv[rd]]];
                    else if (a.pal_in)
                        acc += r2 * cf * x[off2 + a.dcol[rd]];
                }
            }
            y[off + c] = acc;
        }
    }
}

// LDS budget of the two-pass form: one staged row per work group of 1024 threads.
constexpr int kPLdsBlock = 1024;
constexpr size_t kPRowLds = 150 * 1024;

// Two-pass form for full rows.  Down pass: the row staged in LDS, diagonal and
// down hops, y written.  Up pass: work groups of kPUpBlock threads over (rows,
// slab of LPR lanes x up_cols columns); slabs are dealt out XCD by XCD (work
// group b runs on XCD b mod 8) and each XCD walks its slabs one at a time over
// every row, so the slab (all rows at those columns) stays in that XCD's L2
// while 34 rows read it.  Each row's up hops come from one precomputed 64-bit
// entry (source row start, class, amplitude), palindromic sources last;
// a work group decodes its rows' entries into LDS once.
constexpr int kPUpBlock = 256;
constexpr int kPUpNB = 8;   // hop loads in flight per lane
constexpr int kPFupMax = 64;   // up hops per row the two-pass form takes
constexpr uint64_t kFupNone = ~0ull;

// Lanczos recurrence carried by a pass (the whole H q_k is in y):
// q_{k+1} = sc_k y - alpha_k sc_k q_k - beta_k sc_{k-1} q_{k-1}, written over
// q2 = q_{k-1} (and to slot k + 1 of keep when set), with one |q_{k+1}|^2
// partial per work group in norm.
template <typename T>
struct PFuse {
    const T* q1 = nullptr;
    T* q2 = nullptr;
    T* keep = nullptr;
    uint64_t keep_ld = 0;
    int keep_cap = 0;
    const double* alpha = nullptr;
    const double* beta = nullptr;
    const double* sc = nullptr;
    const int* kidx = nullptr;
    double* norm = nullptr;
};

// The recurrence's coefficients at step *kidx and the keep slot it fills.
template <typename T>
__device__ __forceinline__ void pfuse_coefs(const PFuse<T>& f, double* fa, double* fb, double* fc, T** keep) {
    const int k = *f.kidx;
    *fa = f.sc[k];
    *fb = f.alpha[k] * f.sc[k];
    *fc = k > 0 ? f.beta[k] * f.sc[k - 1] : 0.0;
    *keep = f.keep && k + 1 < f.keep_cap ? f.keep + (uint64_t)(k + 1) * f.keep_ld : nullptr;
}

// *out = sum of v over a work group of kPLdsBlock threads, in a fixed order.
__device__ __forceinline__ void block_sum_store_wide(double v, double* out) {
    __shared__ double red[kPLdsBlock / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kPLdsBlock / 64; ++w) t += red[w];
        *out = t;
    }
}

// PACKED: the table as 16-bit pairs (half the bytes and loads per hop).
// FUSE: the rows staged are q_{k+1}, formed here from y (the whole H q_k,
// then overwritten by the down part of H q_{k+1}) and f; x is unused.
template <typename T, bool PACKED, bool FUSE>
__global__ __launch_bounds__(kPLdsBlock) void k_hvp_down(const PArgs a, const T* __restrict__ coef,
                                                          const T* __restrict__ x, T* __restrict__ y,
                                                          const int* skip, const PFuse<T> f) {
    if (skip && *skip) return;
    extern __shared__ __align__(16) unsigned char pdyn[];
    T* R = reinterpret_cast<T*>(pdyn);
    __shared__ T s_coef[kMaxCoef];
    for (int i = threadIdx.x; i < kMaxCoef; i += kPLdsBlock) s_coef[i] = coef[i];
    const uint32_t Dd = (uint32_t)a.Ddn;
    double fa = 0.0, fb = 0.0, fc = 0.0, nsum = 0.0;
    T* fkeep = nullptr;
    if constexpr (FUSE) pfuse_coefs(f, &fa, &fb, &fc, &fkeep);
    for (uint64_t kk = blockIdx.x; kk < a.nlist; kk += gridDim.x) {
        const uint64_t k = a.rows[kk];
        const uint64_t off = a.row_off[k];
        const uint32_t phu = a.up_states[a.row_rank[k]];
        __syncthreads();
        if constexpr (FUSE) {
            // four elements per thread at a time: every operand load of the
            // batch is issued before its stores (q2 is both read and written)
            for (uint32_t c0 = threadIdx.x; c0 < Dd; c0 += 4 * kPLdsBlock) {
                T vy[4], v1[4], v2[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t c = c0 + j * kPLdsBlock;
                    if (c < Dd) {   // streamed past L2, which keeps the hop table
                        vy[j] = __builtin_nontemporal_load(y + off + c);
                        v1[j] = __builtin_nontemporal_load(f.q1 + off + c);
                        v2[j] = __builtin_nontemporal_load(f.q2 + off + c);
                    }
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint32_t c = c0 + j * kPLdsBlock;
                    if (c < Dd) {
                        const T v = lanczos_recurrence<T>(vy[j], (T)0, v1[j], v2[j], fa, fb, fc);
                        __builtin_nontemporal_store(v, f.q2 + off + c);
                        if (fkeep) __builtin_nontemporal_store(v, fkeep + off + c);
                        nsum += (double)v * (double)v;
                        R[c] = v;
                    }
                }
            }
        } else {
            for (uint32_t c = threadIdx.x; c < Dd; c += kPLdsBlock) R[c] = __builtin_nontemporal_load(x + off + c);
        }
        __syncthreads();
        // each column: its down string and hop count (prefetched one column
        // ahead), then its table entries NB at a time, then their LDS reads.
        // NB = 16 in FP64, whose row takes the whole LDS budget (one work group
        // per CU); in FP32 two work groups share a CU, which needs the 8 waves
        // per SIMD that NB = 8 keeps.
        constexpr int NB = sizeof(T) == 8 ? 16 : 8;
        uint32_t c = threadIdx.x;
        uint32_t phd = c < Dd ? a.dn_states[a.dlistf[c]] : 0u;
        int ndh = c < Dd ? a.fcnt[c] : 0;
        for (; c < Dd; c += kPLdsBlock) {
            const uint32_t cn = c + kPLdsBlock;
            const uint32_t phd_n = cn < Dd ? a.dn_states[a.dlistf[cn]] : 0u;
            const int ndh_n = cn < Dd ? a.fcnt[cn] : 0;
            T acc = (T)(a.U * __builtin_popcount(phu & phd)) * R[c];
            if constexpr (PACKED) {
                const uint32_t tm = (1u << a.pshift) - 1u;
                for (int h0 = 0; h0 < ndh; h0 += NB) {   // NB hops = NB / 2 words
                    uint32_t w[NB / 2];
#pragma unroll
                    for (int j = 0; j < NB / 2; ++j)
                        w[j] = h0 + 2 * j < ndh ? a.fell2[(uint64_t)(h0 / 2 + j) * Dd + c] : 0u;
#pragma unroll
                    for (int j = 0; j < NB / 2; ++j) {
                        const uint32_t e0 = w[j] & 0xFFFFu, e1 = w[j] >> 16;
                        if (h0 + 2 * j < ndh) acc += s_coef[e0 >> a.pshift] * R[e0 & tm];
                        if (h0 + 2 * j + 1 < ndh) acc += s_coef[e1 >> a.pshift] * R[e1 & tm];
                    }
                }
            } else {
                for (int h0 = 0; h0 < ndh; h0 += NB) {
                    uint32_t e[NB];
#pragma unroll
                    for (int j = 0; j < NB; ++j) e[j] = h0 + j < ndh ? a.fell[(uint64_t)(h0 + j) * Dd + c] : 0u;
#pragma unroll
                    for (int j = 0; j < NB; ++j)
                        if (h0 + j < ndh) acc += s_coef[e[j] >> kTargetBits] * R[e[j] & kTargetMask];
                }
            }
            __builtin_nontemporal_store(acc, y + off + c);
            phd = phd_n;
            ndh = ndh_n;
        }
    }
    if constexpr (FUSE) block_sum_store_wide(nsum, f.norm + blockIdx.x);
}

// The recurrence on the palindromic rows (FUSE companion of k_hvp_down, which
// covers the full rows): norm partials at f.norm[norm_off + work group].
template <typename T>
__global__ __launch_bounds__(kPBlock) void k_pform(const PArgs a, T* __restrict__ y, const int* skip,
                                                    const PFuse<T> f, int norm_off) {
    if (skip && *skip) return;
    double fa, fb, fc, nsum = 0.0;
    T* fkeep;
    pfuse_coefs(f, &fa, &fb, &fc, &fkeep);
    const uint64_t n = a.nlist * a.Lp;   // row kk of the list, column c < Lp (past the row's length: none)
    for (uint64_t i = (uint64_t)blockIdx.x * kPBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kPBlock) {
        const uint64_t k = a.rows[i / a.Lp], c = i % a.Lp;
        const uint64_t off = a.row_off[k];
        if (c >= a.row_off[k + 1] - off) continue;
        const uint64_t e = off + c;
        const T v = lanczos_recurrence<T>(y[e], (T)0, f.q1[e], f.q2[e], fa, fb, fc);
        f.q2[e] = v;
        if (fkeep) fkeep[e] = v;
        nsum += (double)v * (double)v;
    }
    block_sum_store(nsum, f.norm + norm_off + blockIdx.x);
}

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

// Columns per thread: two mirror pairs in FP32 (one 16-byte load), one pair in FP64.
template <typename T> constexpr int up_cols() { return sizeof(T) == 4 ? 4 : 2; }

// Each lane takes up_cols consecutive columns starting at a multiple of
// up_cols.  When they all lie in the head of the row (mirror pairs), the
// source's columns are read as one block and an image source swaps each
// pair; lanes on the palindrome tail (or straddling it) read single columns
// with the mirror column from the table.  Hops from palindromic source rows
// (listed last) read the columns of the representatives.  With dotp set,
// work group b writes dotp[b] = its share of x . y over the finished rows.
template <typename T, int LPR>
__global__ __launch_bounds__(kPUpBlock) void k_hvp_up(const PArgs a, const T* __restrict__ coef,
                                                      const T* __restrict__ x, T* __restrict__ y, const int* skip,
                                                      uint64_t nslab, int vec_ok, double* dotp) {
    if (skip && *skip) return;
    using V2 = typename Vec2<T>::type;
    constexpr int CPT = up_cols<T>();
    constexpr int ROWS = kPUpBlock / LPR;
    static_assert(kPUpBlock % LPR == 0 && LPR <= 64, "lanes per row");
    static_assert(kPUpBlock == kPBlock, "block_sum_store takes kPBlock threads");
    extern __shared__ __align__(16) unsigned char pup[];
    const int stride = a.fup_stride;
    uint64_t* s_e = reinterpret_cast<uint64_t*>(pup);   // ROWS x stride entries
    T* s_f = reinterpret_cast<T*>(s_e + ROWS * stride);   // their factors
    __shared__ int s_n[ROWS], s_nh[ROWS];                 // hops from A / image sources, all hops
    const T r2 = (T)1.4142135623730950488, ir2 = (T)0.70710678118654752440, ps = (T)a.ps;
    const uint64_t groups = (a.nlist + ROWS - 1) / ROWS;   // work groups per slab
    const uint64_t per_xcd = (nslab + 7) / 8;              // slabs per XCD
    const uint64_t xcd = blockIdx.x % 8, j = blockIdx.x / 8;
    const uint64_t slab = (j / groups) * 8 + xcd;          // slab-major within the XCD
    if (j / groups >= per_xcd || slab >= nslab) {          // whole work group
        if (dotp && threadIdx.x == 0) dotp[blockIdx.x] = 0.0;
        return;
    }
    const uint64_t kk0 = (j % groups) * ROWS;
    if (threadIdx.x < ROWS) s_n[threadIdx.x] = s_nh[threadIdx.x] = 0;
    __syncthreads();
    for (int t = threadIdx.x; t < ROWS * stride; t += kPUpBlock) {
        const int r = t / stride, h = t - r * stride;
        const uint64_t e = kk0 + r < a.nlist ? a.fup[(kk0 + r) * stride + h] : kFupNone;
        T f = (T)0;
        if (e != kFupNone) {
            const uint8_t cl = (uint8_t)((e >> 40) & 3u);
            const T cf = coef[(e >> 48) & 0xFFu];
            f = cl == kClsPal ? cf : (cl == kClsA ? r2 * ir2 : r2 * ir2 * ps) * cf;
            atomicMax(&s_nh[r], h + 1);
            if (cl != kClsPal) atomicMax(&s_n[r], h + 1);
        }
        s_e[t] = e;
        s_f[t] = f;
    }
    __syncthreads();
    const int r = threadIdx.x / LPR, lane = threadIdx.x % LPR;
    const uint64_t kk = kk0 + r;
    const uint32_t Dd = (uint32_t)a.Ddn;
    const uint32_t c0 = (uint32_t)(slab * (CPT * LPR) + CPT * lane);
    // returns this thread's share of x . y (its columns of the finished row)
    auto row_part = [&]() -> double {
        const int nv = c0 + CPT <= Dd ? CPT : (int)(Dd - c0);
        const bool pair = c0 + CPT <= (uint32_t)a.npair2;   // all CPT columns are mirror pairs
        const uint64_t off = a.row_off[a.rows[kk]];
        const uint64_t* er = s_e + r * stride;
        const T* fr = s_f + r * stride;
        const int n_np = s_n[r], nh = s_nh[r];
        T acc[CPT];
#pragma unroll
        for (int t = 0; t < CPT; ++t) acc[t] = (T)0;
        if (pair) {
            // an image source contributes the other member of each pair: its
            // products go to accI, whose columns are swapped once at the end
            T accI[CPT];
#pragma unroll
            for (int t = 0; t < CPT; ++t) accI[t] = (T)0;
            // hops in batches of kPUpNB, then of kPUpNB/2, ..., 1 while they
            // fit: one load per hop, the batch's entries first, then its loads
            int h = 0;
            auto batch = [&](auto bc) {
                constexpr int B = decltype(bc)::value;
                T v[B][CPT], fa[B], fi[B];
                uint64_t e[B];
#pragma unroll
                for (int q = 0; q < B; ++q) {
                    e[q] = er[h + q];
                    const T f = fr[h + q];
                    const bool img = ((e[q] >> 40) & 3u) == kClsImage;
                    fa[q] = img ? (T)0 : f;
                    fi[q] = img ? f : (T)0;
                }
#pragma unroll
                for (int q = 0; q < B; ++q) {
                    const T* src = x + (e[q] & 0xFFFFFFFFFFull) + c0;   // one wide load (any alignment)
#pragma unroll
                    for (int t = 0; t < CPT; ++t) v[q][t] = src[t];
                }
#pragma unroll
                for (int q = 0; q < B; ++q)
#pragma unroll
                    for (int t = 0; t < CPT; ++t) {
                        acc[t] += fa[q] * v[q][t];
                        accI[t] += fi[q] * v[q][t];
                    }
                h += B;
            };
            static_assert(kPUpNB == 8, "tail batches below");
            while (h + kPUpNB <= n_np) batch(std::integral_constant<int, kPUpNB>{});
            if (h + 4 <= n_np) batch(std::integral_constant<int, 4>{});
            if (h + 2 <= n_np) batch(std::integral_constant<int, 2>{});
            if (h + 1 <= n_np) batch(std::integral_constant<int, 1>{});
#pragma unroll
            for (int t = 0; t < CPT; ++t) acc[t] += accI[t ^ 1];
        } else {
            for (int h = 0; h < n_np; ++h) {
                const uint64_t e = er[h];
                const T f = fr[h];
                const uint64_t off2 = e & 0xFFFFFFFFFFull;
                const bool img = ((e >> 40) & 3u) == kClsImage;
#pragma unroll
                for (int t = 0; t < CPT; ++t)
                    if (t < nv) acc[t] += f * x[off2 + (img ? a.fmir[c0 + t] : c0 + t)];
            }
        }
        if (n_np < nh) {   // rare: a palindromic source row holds representatives only
            uint32_t pcol[CPT];
            T pfac[CPT];
#pragma unroll
            for (int t = 0; t < CPT; ++t) {
                pcol[t] = 0u;
                pfac[t] = (T)0;
                if (t >= nv) continue;
                const uint32_t rd = a.dlistf[c0 + t];
                const uint8_t dc = a.dcls[rd];
                if (dc == kClsA) {
                    pcol[t] = a.dcol[rd];
                    pfac[t] = r2 * ir2;
                } else if (dc == kClsImage) {
                    pcol[t] = a.dcol[a.dinv[rd]];
                    pfac[t] = r2 * ir2 * ps;
                } else if (a.pal_in) {
                    pcol[t] = a.dcol[rd];
                    pfac[t] = r2;
                }
            }
            for (int h = n_np; h < nh; ++h) {
                const uint64_t off2 = er[h] & 0xFFFFFFFFFFull;
                const T cf = fr[h];
#pragma unroll
                for (int t = 0; t < CPT; ++t)
                    if (pfac[t] != (T)0) acc[t] += (pfac[t] * cf) * x[off2 + pcol[t]];
            }
        }
        T* yr = y + off + c0;
        T yv[CPT];
        if (vec_ok && nv == CPT && ((off + c0) % CPT) == 0u) {
            if constexpr (CPT == 4) {
                float4 q4 = *reinterpret_cast<const float4*>(yr);
                q4.x += acc[0];
                q4.y += acc[1];
                q4.z += acc[2];
                q4.w += acc[3];
                *reinterpret_cast<float4*>(yr) = q4;
                yv[0] = q4.x;
                yv[1] = q4.y;
                yv[2] = q4.z;
                yv[3] = q4.w;
            } else {
                V2 q2 = *reinterpret_cast<const V2*>(yr);
                q2.x += acc[0];
                q2.y += acc[1];
                *reinterpret_cast<V2*>(yr) = q2;
                yv[0] = q2.x;
                yv[1] = q2.y;
            }
        } else {
#pragma unroll
            for (int t = 0; t < CPT; ++t)
                if (t < nv) {
                    yv[t] = yr[t] + acc[t];
                    yr[t] = yv[t];
                }
        }
        double ds = 0.0;
        if (dotp) {
            const T* xr = x + off + c0;
#pragma unroll
            for (int t = 0; t < CPT; ++t)
                if (t < nv) ds += (double)xr[t] * (double)yv[t];
        }
        return ds;
    };
    const double ds = kk < a.nlist && c0 < Dd ? row_part() : 0.0;
    if (dotp) block_sum_store(ds, dotp + blockIdx.x);
}

// Full-row down-hop table in column space.
__global__ __launch_bounds__(kPBlock) void k_pcolhops(const PArgs a, int max_hops, uint8_t* fcnt, uint32_t* fell) {
    for (uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; c < a.Ddn; c += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t rd = a.dlistf[c];
        const int n = a.dn_cnt[rd];
        fcnt[c] = (uint8_t)n;
        for (int h = 0; h < n && h < max_hops; ++h) {
            const uint32_t e = a.dn_ell[(uint64_t)h * a.Ddn + rd];
            fell[(uint64_t)h * a.Ddn + c] = a.dcolf[e & kTargetMask] | (e & ~kTargetMask);
        }
    }
}

// Index of basis states (up, dn) given as strings; states outside the basis get ~0 and an error bit.
__global__ __launch_bounds__(kPBlock) void k_prank(const PArgs a, const uint32_t* binom, const uint32_t* S, int smax,
                                                    int N, int n_up, int n_dn, const uint32_t* up, const uint32_t* dn,
                                                    uint64_t count, uint64_t* idx, uint32_t* err) {
    __shared__ uint32_t sC[kBinomStride * kBinomStride];
    stage_binom(sC, binom);
    const uint32_t mask = N >= 32 ? 0xFFFFFFFFu : ((1u << N) - 1u);
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t u = up[t], d = dn[t];
        uint64_t r = ~0ull;
        bool bad = (u & ~mask) || (d & ~mask) || __builtin_popcount(u) != n_up || __builtin_popcount(d) != n_dn;
        if (!bad) {
            const uint8_t cu = classify(u, N);
            if (cu == kClsImage) {
                bad = true;
            } else {
                const uint32_t row = forward_map_inversion(u, n_up, N, sC, S, smax);
                const uint32_t rd = forward_map(d, sC);
                if (cu == kClsA) {
                    r = a.row_off[row] + a.dcolf[rd];
                } else {
                    const uint32_t col = a.dcol[rd];
                    if (classify(d, N) == kClsImage || col == kNoCol) bad = true;
                    else r = a.row_off[row] + col;
                }
            }
        }
        if (bad) {
            atomicOr(err, kErrRankInput);
            r = ~0ull;
        }
        idx[t] = r;
    }
}

// Basis state of each index: the row by binary search over the row starts.
__global__ __launch_bounds__(kPBlock) void k_punrank(const PArgs a, const uint64_t* idx, uint64_t count, uint32_t* up,
                                                      uint32_t* dn, uint32_t* err) {
    const uint64_t D = a.row_off[a.nrows];
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t p = idx[t];
        if (p >= D) {
            atomicOr(err, kErrUnrankInput);
            up[t] = dn[t] = 0xFFFFFFFFu;
            continue;
        }
        uint64_t lo = 0, hi = a.nrows;   // last row with row_off <= p
        while (hi - lo > 1) {
            const uint64_t mid = (lo + hi) / 2;
            if (a.row_off[mid] <= p) lo = mid; else hi = mid;
        }
        const uint64_t c = p - a.row_off[lo];
        const uint32_t rd = a.row_pal[lo] ? a.dlist[c] : a.dlistf[c];
        up[t] = a.up_states[a.row_rank[lo]];
        dn[t] = a.dn_states[rd];
    }
}

template <typename V>
pdz_status dalloc(V** dst, uint64_t n) {
    PDZ_HIP(hipMalloc(dst, std::max<uint64_t>(1, n) * sizeof(V)));
    return ok();
}

template <typename V>
pdz_status dupload(V** dst, const std::vector<V>& src) {
    PDZ_HIP(hipMalloc(dst, std::max<size_t>(1, src.size()) * sizeof(V)));
    if (!src.empty()) PDZ_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice));
    return ok();
}

PArgs pargs(const pdz_problem_s* p) {
    const ParSpace* q = p->par;
    PArgs a;
    a.up_states = p->up.states;
    a.dn_states = p->dn.states;
    a.up_cnt = p->up.count;
    a.up_ell = p->up.ell;
    a.dn_cnt = p->dn.count;
    a.dn_ell = p->dn.ell;
    a.Dup = p->up.D;
    a.Ddn = p->dn.D;
    a.ucls = q->d_ucls;
    a.urow = q->d_urow;
    a.dcls = q->d_dcls;
    a.dinv = q->d_dinv;
    a.dcol = q->d_dcol;
    a.dlist = q->d_dlist;
    a.dcolf = q->d_dcolf;
    a.dlistf = q->d_dlistf;
    a.fmir = q->d_fmir;
    a.fcnt = q->d_fcnt;
    a.fell = q->d_fell;
    a.fell2 = q->d_fell2;
    a.pshift = q->pshift;
    a.fup = q->d_fup;
    a.fup_stride = q->fup_stride;
    a.npair2 = q->npair2;
    a.row_rank = q->d_row_rank;
    a.row_off = q->d_row_off;
    a.row_pal = q->d_row_pal;
    a.uinv = q->d_uinv;
    a.rows = nullptr;
    a.nlist = 0;
    a.nrows = q->nrows;
    a.Lp = q->Lp;
    a.U = p->U;
    a.ps = (double)(q->P * q->sigma);
    a.pal_in = q->sigma == q->P;
    return a;
}

unsigned pgrid(uint64_t n, unsigned cu) {
    uint64_t g = (n + kPBlock - 1) / kPBlock;
    const uint64_t gmax = (uint64_t)cu * 16;
    if (g > gmax) g = gmax;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

void parity_free(ParSpace* q) {
    if (!q) return;
    void* ptrs[] = {q->d_ucls, q->d_uinv, q->d_utree, q->d_urow, q->d_dcls, q->d_dinv, q->d_dtree, q->d_dcol,
                    q->d_dlist, q->d_row_rank, q->d_row_off, q->d_row_pal, q->d_S, q->d_rows_full, q->d_rows_pal,
                    q->d_dcolf, q->d_dlistf, q->d_fmir, q->d_fcnt, q->d_fell, q->d_fell2, q->d_fup};
    for (void* v : ptrs)
        if (v) (void)hipFree(v);
    void* gptrs[] = {q->d_col_dn, q->d_goff[0], q->d_goff[1], q->d_gnr[0], q->d_gnr[1], q->d_grp_up[0], q->d_grp_up[1]};
    for (void* v : gptrs)
        if (v) (void)hipFree(v);
    free_down_schedule(&q->fsched);
    delete q;
}

namespace {

// Launch geometry of one H.v: whether the full rows take the two-pass form,
// the up pass's slabs and grid, and the palindromic-row grid.
struct PGeom {
    bool two_pass = false;
    uint64_t nslab = 0, g_up = 0, g_pal = 0;
    size_t ulds = 0;
};

PGeom pgeom(const ParSpace* q, uint64_t Ddn, size_t es) {
    PGeom m;
    if (q->n_full > 0) {
        m.two_pass = !q->force_gather && Ddn * es <= kPRowLds && q->d_fup && q->fup_stride <= kPFupMax;
        if (m.two_pass) {
            const uint64_t rows = kPUpBlock / q->up_lpr;
            const uint64_t span = (uint64_t)(es == 4 ? 4 : 2) * q->up_lpr;   // up_cols: columns of a slab
            m.nslab = (Ddn + span - 1) / span;
            m.g_up = 8 * ((m.nslab + 7) / 8) * ((q->n_full + rows - 1) / rows);
            m.ulds = (size_t)rows * q->fup_stride * (sizeof(uint64_t) + es);
        }
    }
    if (q->n_pal > 0)
        m.g_pal = std::min<uint64_t>(std::max<uint64_t>(q->n_pal * ((q->Lp + kPBlock - 1) / kPBlock), 1), 1ull << 20);
    return m;
}

// Work groups of the fused down pass (|q_{k+1}|^2 partials: these plus
// kPFormGrid for the palindromic rows).
constexpr uint64_t kPFuseGrid = 2048;
constexpr uint64_t kPFormGrid = 256;

// The scheduled down pass's row groups for element size es, or none (the
// looped down pass runs).
bool sched_groups_of(const pdz_problem_s* p, size_t es, SchedGroups* g) {
    const ParSpace* q = p->par;
    if (q->force_loop || !q->fsched.words) return false;
    const int i = es == 8 ? 0 : 1;
    if (!q->d_goff[i]) return false;
    g->sched = &q->fsched;
    g->D_dn = p->dn.D;
    g->U = p->U;
    g->grp_up = q->d_grp_up[i];
    g->col_dn = q->d_col_dn;
    g->goff = q->d_goff[i];
    g->gnr = q->d_gnr[i];
    g->ngroups = q->ngroups[i];
    g->R = es == 8 ? 1 : 3;
    return true;
}

// Work groups of the fused down pass over the full rows (one |q_{k+1}|^2
// partial each).
uint64_t full_fuse_grid(const pdz_problem_s* p, size_t es) {
    const ParSpace* q = p->par;
    if (q->n_full == 0) return 0;
    SchedGroups g;
    if (sched_groups_of(p, es, &g)) return sched_groups_grid(g);
    return std::min<uint64_t>(q->n_full, kPFuseGrid);
}

// passes: kPassDown launches the down pass (with the recurrence when f is
// set: then x is unused and the palindromic rows' q_{k+1} is formed too),
// kPassUp the up pass and the palindromic rows; both: the whole H.v.
// dotp (optional, two-pass form only, with the up part): one partial sum of
// x . y per work group of the up pass, then per work group of the
// palindromic rows.
template <typename T>
pdz_status run_hvp(const pdz_problem_s* p, const T* coef, const T* x, T* y, hipStream_t s, const int* skip,
                   double* dotp, unsigned passes, const PFuse<T>* f) {
    const ParSpace* q = p->par;
    PArgs a = pargs(p);
    const PGeom m = pgeom(q, a.Ddn, sizeof(T));
    static_assert(up_cols<float>() == 4 && up_cols<double>() == 2, "slab width in pgeom");
    const bool down = passes & kPassDown, up = passes & kPassUp;
    if ((dotp || f || passes != (kPassDown | kPassUp)) && q->n_full > 0 && !m.two_pass)
        return fail(PDZ_EINVAL, "separate passes, x . y partials and the fused recurrence need the two-pass parity H.v");
    if (f && (!down || up)) return fail(PDZ_EINVAL, "the fused recurrence rides on the down pass alone");
    if (q->n_full > 0) {
        a.rows = q->d_rows_full;
        a.nlist = q->n_full;
        const unsigned grid = (unsigned)std::min<uint64_t>(q->n_full, f ? kPFuseGrid : (1ull << 20));
        if (m.two_pass) {
            const size_t lds = (size_t)a.Ddn * sizeof(T);
            const PFuse<T> f0 = f ? *f : PFuse<T>();
            SchedGroups sg;
            if (down && sched_groups_of(p, sizeof(T), &sg)) {
                HvSplit hs;
                if (f) {
                    hs.fq1 = f->q1;
                    hs.fq2 = f->q2;
                    hs.fkeep = f->keep;
                    hs.fkeep_ld = f->keep_ld;
                    hs.fkeep_cap = f->keep_cap;
                    hs.falpha = f->alpha;
                    hs.fbeta = f->beta;
                    hs.fsc = f->sc;
                    hs.fkidx = f->kidx;
                    hs.fnorm = f->norm;
                }
                const pdz_status st =
                    launch_sched_groups(sg, sizeof(T) == 8 ? PDZ_F64 : PDZ_F32, x, y, s, skip, f ? &hs : nullptr);
                if (st != PDZ_OK) return st;
            } else if (down) {
                if (f && q->d_fell2)
                    hipLaunchKernelGGL((k_hvp_down<T, true, true>), dim3(grid), dim3(kPLdsBlock), lds, s, a, coef, x, y,
                                       skip, f0);
                else if (f)
                    hipLaunchKernelGGL((k_hvp_down<T, false, true>), dim3(grid), dim3(kPLdsBlock), lds, s, a, coef, x,
                                       y, skip, f0);
                else if (q->d_fell2)
                    hipLaunchKernelGGL((k_hvp_down<T, true, false>), dim3(grid), dim3(kPLdsBlock), lds, s, a, coef, x,
                                       y, skip, f0);
                else
                    hipLaunchKernelGGL((k_hvp_down<T, false, false>), dim3(grid), dim3(kPLdsBlock), lds, s, a, coef, x,
                                       y, skip, f0);
            }
            if (up) {
                if (m.g_up >= (1ull << 31)) return fail(PDZ_ERANGE, "parity up pass grid too large");
                const size_t al = up_cols<T>() * sizeof(T);
                const int vec_ok =
                    reinterpret_cast<uintptr_t>(x) % al == 0 && reinterpret_cast<uintptr_t>(y) % al == 0;
                const dim3 ug((unsigned)m.g_up);
                if (q->up_lpr == 16)
                    hipLaunchKernelGGL((k_hvp_up<T, 16>), ug, dim3(kPUpBlock), m.ulds, s, a, coef, x, y, skip, m.nslab,
                                       vec_ok, dotp);
                else if (q->up_lpr == 32)
                    hipLaunchKernelGGL((k_hvp_up<T, 32>), ug, dim3(kPUpBlock), m.ulds, s, a, coef, x, y, skip, m.nslab,
                                       vec_ok, dotp);
                else
                    hipLaunchKernelGGL((k_hvp_up<T, 64>), ug, dim3(kPUpBlock), m.ulds, s, a, coef, x, y, skip, m.nslab,
                                       vec_ok, dotp);
            }
        } else
            hipLaunchKernelGGL(k_hvp_full<T>, dim3(grid), dim3(kPBlock), 0, s, a, coef, x, y, skip);
    }
    if (q->n_pal > 0) {
        a.rows = q->d_rows_pal;
        a.nlist = q->n_pal;
        if (f)
            hipLaunchKernelGGL(k_pform<T>, dim3((unsigned)kPFormGrid), dim3(kPBlock), 0, s, a, y, skip, *f,
                               (int)full_fuse_grid(p, sizeof(T)));
        if (up)
            hipLaunchKernelGGL(k_hvp<T>, dim3((unsigned)m.g_pal), dim3(kPBlock), 0, s, a, coef, x, y, skip,
                               dotp ? dotp + m.g_up : nullptr);
    }
    PDZ_HIP(hipGetLastError());
    return ok();
}

}  // namespace

pdz_status parity_prepare() {
    const void* downs[] = {
        reinterpret_cast<const void*>(&k_hvp_down<double, false, false>),
        reinterpret_cast<const void*>(&k_hvp_down<float, false, false>),
        reinterpret_cast<const void*>(&k_hvp_down<double, true, false>),
        reinterpret_cast<const void*>(&k_hvp_down<float, true, false>),
        reinterpret_cast<const void*>(&k_hvp_down<double, false, true>),
        reinterpret_cast<const void*>(&k_hvp_down<float, false, true>),
        reinterpret_cast<const void*>(&k_hvp_down<double, true, true>),
        reinterpret_cast<const void*>(&k_hvp_down<float, true, true>)};
    for (const void* k : downs)
        PDZ_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPRowLds));
    return ok();
}

pdz_status launch_hvp(const pdz_problem_s* p, pdz_dtype dt, const void* x, void* y, hipStream_t s, const int* skip,
                      double* dotp) {
    const unsigned both = kPassDown | kPassUp;
    if (dt == PDZ_F64)
        return run_hvp<double>(p, p->d_coef64, static_cast<const double*>(x), static_cast<double*>(y), s, skip, dotp,
                               both, nullptr);
    return run_hvp<float>(p, p->d_coef32, static_cast<const float*>(x), static_cast<float*>(y), s, skip, dotp, both,
                          nullptr);
}

namespace {
template <typename T>
PFuse<T> pfuse_of(const HvSplit* sp) {
    PFuse<T> f;
    f.q1 = static_cast<const T*>(sp->fq1);
    f.q2 = static_cast<T*>(sp->fq2);
    f.keep = static_cast<T*>(sp->fkeep);
    f.keep_ld = sp->fkeep_ld;
    f.keep_cap = sp->fkeep_cap;
    f.alpha = sp->falpha;
    f.beta = sp->fbeta;
    f.sc = sp->fsc;
    f.kidx = sp->fkidx;
    f.norm = sp->fnorm;
    return f;
}
}  // namespace

pdz_status launch_hvp_split(const pdz_problem_s* p, pdz_dtype dt, const void* x, void* y, hipStream_t s,
                            const int* skip, unsigned passes, const HvSplit* sp) {
    if (sp && (sp->z || sp->dotp_dn || sp->fz))
        return fail(PDZ_EINVAL, "a parity H.v keeps its parts in y: no z, down-pass dots or fz");
    if (sp && sp->dotp_up && !(passes & kPassUp)) return fail(PDZ_EINVAL, "x . y partials come with the up part");
    if (sp && sp->fq2 && !sp->fnorm) return fail(PDZ_EINVAL, "the fused recurrence needs fnorm");
    double* dotp = sp ? sp->dotp_up : nullptr;
    const bool fuse = sp && sp->fq2;
    if (dt == PDZ_F64) {
        const PFuse<double> f = fuse ? pfuse_of<double>(sp) : PFuse<double>();
        return run_hvp<double>(p, p->d_coef64, static_cast<const double*>(x), static_cast<double*>(y), s, skip, dotp,
                               passes, fuse ? &f : nullptr);
    }
    const PFuse<float> f = fuse ? pfuse_of<float>(sp) : PFuse<float>();
    return run_hvp<float>(p, p->d_coef32, static_cast<const float*>(x), static_cast<float*>(y), s, skip, dotp, passes,
                          fuse ? &f : nullptr);
}

int parity_fused_norms(const pdz_problem_s* p, pdz_dtype dt) {
    if (!p->par) return 0;
    const ParSpace* q = p->par;
    const PGeom m = pgeom(q, p->dn.D, dt == PDZ_F64 ? 8 : 4);
    if (q->n_full > 0 && !m.two_pass) return 0;
    return (int)(full_fuse_grid(p, dt == PDZ_F64 ? 8 : 4) + (q->n_pal > 0 ? kPFormGrid : 0));
}

bool parity_sched_down(const pdz_problem_s* p, pdz_dtype dt) {
    if (!p->par) return false;
    const ParSpace* q = p->par;
    const size_t es = dt == PDZ_F64 ? 8 : 4;
    SchedGroups g;
    return q->n_full > 0 && pgeom(q, p->dn.D, es).two_pass && sched_groups_of(p, es, &g);
}

int parity_dot_count(const pdz_problem_s* p, pdz_dtype dt) {
    if (!p->par) return 0;
    const PGeom m = pgeom(p->par, p->dn.D, dt == PDZ_F64 ? 8 : 4);
    if (p->par->n_full > 0 && !m.two_pass) return 0;
    const uint64_t n = m.g_up + m.g_pal;
    return n < (1ull << 30) ? (int)n : 0;
}

// Parity tables on top of a real-space problem with sector hop tables.
pdz_status parity_build(pdz_problem_s* p, int P) {
    ParSpace* q = new ParSpace();
    p->par = q;
    const int N = p->N, nu = p->n_up, nd = p->n_dn;
    q->P = P;
    {
        const char* env = std::getenv("PDZ_PARITY_GATHER");
        q->force_gather = env && env[0] == '1';
        const char* wide = std::getenv("PDZ_PARITY_WIDE_TABLE");
        q->wide_table = wide && wide[0] == '1';
        const char* loop = std::getenv("PDZ_PARITY_LOOPED_DOWN");
        q->force_loop = loop && loop[0] == '1';
        const char* lanes = std::getenv("PDZ_PARITY_UP_LANES");
        if (lanes) {
            const std::string v(lanes);
            if (v != "16" && v != "32" && v != "64")
                return fail(PDZ_EINVAL, "PDZ_PARITY_UP_LANES must be 16, 32 or 64");
            q->up_lpr = std::stoi(v);
        }
    }
    q->sigma = (((nu * (nu - 1) / 2) + (nd * (nd - 1) / 2)) % 2) ? -1 : 1;
    const int smax = std::max(nu, nd);
    // S_i^m = C_{i-2}^{m-1} + S_{i-2}^m + S_{i-2}^{m-2}, S_0^0 = 1, S_1^0 = S_1^1 = 1
    std::vector<uint64_t> S((size_t)(N + 1) * (smax + 1), 0);
    auto Sx = [&](int i, int m) -> uint64_t& { return S[(size_t)i * (smax + 1) + m]; };
    for (int i = 0; i <= N; ++i)
        for (int m = 0; m <= smax; ++m) {
            if (i == 0) Sx(i, m) = m == 0;
            else if (i == 1) Sx(i, m) = m <= 1;
            else Sx(i, m) = (m >= 1 ? binom(i - 2, m - 1) : 0) + Sx(i - 2, m) + (m >= 2 ? Sx(i - 2, m - 2) : 0);
        }
    std::vector<uint32_t> S32(S.size());
    for (size_t t = 0; t < S.size(); ++t) S32[t] = (uint32_t)S[t];
    DeviceCtx* ctx = nullptr;
    pdz_status st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    const uint64_t Du = p->up.D, Dd = p->dn.D;
    if ((st = dupload(&q->d_S, S32)) != PDZ_OK) return st;
    if ((st = dalloc(&q->d_ucls, Du)) != PDZ_OK) return st;
    if ((st = dalloc(&q->d_uinv, Du)) != PDZ_OK) return st;
    if ((st = dalloc(&q->d_utree, Du)) != PDZ_OK) return st;
    if ((st = dalloc(&q->d_dcls, Dd)) != PDZ_OK) return st;
    if ((st = dalloc(&q->d_dinv, Dd)) != PDZ_OK) return st;
    if ((st = dalloc(&q->d_dtree, Dd)) != PDZ_OK) return st;
    const unsigned cu = (unsigned)ctx->cu_count;
    hipLaunchKernelGGL(k_pinfo, dim3(pgrid(Du, cu)), dim3(kPBlock), 0, nullptr, ctx->binom, q->d_S, smax, N, nu,
                       p->up.states, Du, q->d_ucls, q->d_uinv, q->d_utree);
    hipLaunchKernelGGL(k_pinfo, dim3(pgrid(Dd, cu)), dim3(kPBlock), 0, nullptr, ctx->binom, q->d_S, smax, N, nd,
                       p->dn.states, Dd, q->d_dcls, q->d_dinv, q->d_dtree);
    PDZ_HIP(hipGetLastError());
    PDZ_HIP(hipDeviceSynchronize());
    std::vector<uint8_t> ucls(Du), dcls(Dd);
    std::vector<uint32_t> utree(Du), uinv(Du), dtree(Dd);
    PDZ_HIP(hipMemcpy(ucls.data(), q->d_ucls, Du, hipMemcpyDeviceToHost));
    PDZ_HIP(hipMemcpy(utree.data(), q->d_utree, Du * 4, hipMemcpyDeviceToHost));
    PDZ_HIP(hipMemcpy(uinv.data(), q->d_uinv, Du * 4, hipMemcpyDeviceToHost));
    PDZ_HIP(hipMemcpy(dcls.data(), q->d_dcls, Dd, hipMemcpyDeviceToHost));
    PDZ_HIP(hipMemcpy(dtree.data(), q->d_dtree, Dd * 4, hipMemcpyDeviceToHost));
    // rows: up representatives by tree index (must be a permutation of [0, reps))
    const uint64_t ureps = Sx(N, nu);
    std::vector<uint32_t> row_rank(ureps, 0xFFFFFFFFu);
    for (uint64_t r = 0; r < Du; ++r) {
        if (ucls[r] == kClsImage) continue;
        if (utree[r] >= ureps || row_rank[utree[r]] != 0xFFFFFFFFu)
            return fail(PDZ_EDEVICE, "decision-tree forward map is not a bijection onto the up representatives");
        row_rank[utree[r]] = (uint32_t)r;
    }
    // down columns of a palindromic row: down representatives in tree order, palindromes only if sigma == P
    const uint64_t dreps = Sx(N, nd);
    std::vector<uint32_t> dby_tree(dreps, 0xFFFFFFFFu);
    for (uint64_t r = 0; r < Dd; ++r) {
        if (dcls[r] == kClsImage) continue;
        if (dtree[r] >= dreps || dby_tree[dtree[r]] != 0xFFFFFFFFu)
            return fail(PDZ_EDEVICE, "decision-tree forward map is not a bijection onto the down representatives");
        dby_tree[dtree[r]] = (uint32_t)r;
    }
    std::vector<uint32_t> dcol(Dd, kNoCol), dlist;
    for (uint64_t k = 0; k < dreps; ++k) {
        const uint32_t r = dby_tree[k];
        if (dcls[r] == kClsPal && q->sigma != P) continue;
        dcol[r] = (uint32_t)dlist.size();
        dlist.push_back(r);
    }
    q->Lp = dlist.size();
    std::vector<uint32_t> dinv(Dd);
    PDZ_HIP(hipMemcpy(dinv.data(), q->d_dinv, Dd * 4, hipMemcpyDeviceToHost));
    std::vector<uint32_t> dlistf, dcolf(Dd, kNoCol), fmir(Dd);
    for (uint64_t k = 0; k < dreps; ++k) {   // each representative, then its mirror
        const uint32_t r = dby_tree[k];
        if (dcls[r] != kClsA) continue;
        dlistf.push_back(r);
        dlistf.push_back(dinv[r]);
    }
    q->npair2 = dlistf.size();                 // the pairs fill the even-aligned head of a full row
    for (uint64_t k = 0; k < dreps; ++k)       // then the palindromes
        if (dcls[dby_tree[k]] == kClsPal) dlistf.push_back(dby_tree[k]);
    if (dlistf.size() != Dd) return fail(PDZ_EDEVICE, "mirror pairs do not cover the down sector");
    for (uint64_t c = 0; c < Dd; ++c) {
        if (dcolf[dlistf[c]] != kNoCol) return fail(PDZ_EDEVICE, "a down string appears twice in a full row");
        dcolf[dlistf[c]] = (uint32_t)c;
    }
    for (uint64_t c = 0; c < Dd; ++c) fmir[c] = dcolf[dinv[dlistf[c]]];
    std::vector<uint64_t> row_off(ureps + 1, 0);
    std::vector<uint8_t> row_pal(ureps);
    for (uint64_t k = 0; k < ureps; ++k) {
        row_pal[k] = ucls[row_rank[k]] == kClsPal;
        row_off[k + 1] = row_off[k] + (row_pal[k] ? q->Lp : Dd);
    }
    std::vector<uint32_t> urow(Du);
    for (uint64_t r = 0; r < Du; ++r) urow[r] = ucls[r] == kClsImage ? utree[uinv[r]] : utree[r];
    for (uint64_t r = 0; r < Du; ++r)
        if (ucls[r] == kClsImage && (ucls[uinv[r]] != kClsA || utree[r] != utree[uinv[r]]))
            return fail(PDZ_EDEVICE, "mirror of an image string is not its representative");
    q->nrows = ureps;
    p->D = row_off[ureps];
    if (p->D == 0) return fail(PDZ_ERANGE, "the parity subspace is empty");
    if ((st = dupload(&q->d_row_rank, row_rank)) != PDZ_OK) return st;
    if ((st = dupload(&q->d_row_off, row_off)) != PDZ_OK) return st;
    if ((st = dupload(&q->d_row_pal, row_pal)) != PDZ_OK) return st;
    if ((st = dupload(&q->d_urow, urow)) != PDZ_OK) return st;
    if ((st = dupload(&q->d_dcol, dcol)) != PDZ_OK) return st;
    if ((st = dupload(&q->d_dlist, dlist)) != PDZ_OK) return st;
    if ((st = dupload(&q->d_dlistf, dlistf)) != PDZ_OK) return st;
    if ((st = dupload(&q->d_dcolf, dcolf)) != PDZ_OK) return st;
    if ((st = dupload(&q->d_fmir, fmir)) != PDZ_OK) return st;
    const int mh = p->dn.max_hops > 0 ? p->dn.max_hops : 1;
    if ((st = dalloc(&q->d_fcnt, Dd)) != PDZ_OK) return st;
    if ((st = dalloc(&q->d_fell, (uint64_t)mh * Dd)) != PDZ_OK) return st;
    {
        const PArgs pa = pargs(p);
        hipLaunchKernelGGL(k_pcolhops, dim3(pgrid(Dd, cu)), dim3(kPBlock), 0, nullptr, pa, mh, q->d_fcnt, q->d_fell);
        PDZ_HIP(hipGetLastError());
        PDZ_HIP(hipDeviceSynchronize());
    }
    if (!q->wide_table && p->dn.max_hops > 0) {   // 16-bit pairs when column and amplitude index fit
        std::vector<uint8_t> fcnt(Dd);
        std::vector<uint32_t> fell((size_t)mh * Dd);
        PDZ_HIP(hipMemcpy(fcnt.data(), q->d_fcnt, Dd, hipMemcpyDeviceToHost));
        PDZ_HIP(hipMemcpy(fell.data(), q->d_fell, fell.size() * 4, hipMemcpyDeviceToHost));
        uint32_t cmax = 0;
        for (uint64_t c = 0; c < Dd; ++c)
            for (int h = 0; h < fcnt[c]; ++h) cmax = std::max(cmax, fell[(size_t)h * Dd + c] >> kTargetBits);
        int cbits = 0;
        while ((1u << cbits) <= cmax) ++cbits;
        const int tbits = 16 - cbits;
        if (tbits > 0 && Dd <= (1ull << tbits)) {
            const int mh2 = (mh + 1) / 2;
            std::vector<uint32_t> fell2((size_t)mh2 * Dd, 0u);
            for (uint64_t c = 0; c < Dd; ++c)
                for (int h = 0; h < fcnt[c]; ++h) {
                    const uint32_t e = fell[(size_t)h * Dd + c];
                    const uint32_t e16 = (e & kTargetMask) | ((e >> kTargetBits) << tbits);
                    fell2[(size_t)(h / 2) * Dd + c] |= e16 << (16 * (h % 2));
                }
            q->pshift = tbits;
            if ((st = dupload(&q->d_fell2, fell2)) != PDZ_OK) return st;
        }
    }
    std::vector<uint32_t> rows_full, rows_pal;
    for (uint64_t k = 0; k < ureps; ++k) (row_pal[k] ? rows_pal : rows_full).push_back((uint32_t)k);
    q->n_full = rows_full.size();
    q->n_pal = rows_pal.size();
    if ((st = dupload(&q->d_rows_full, rows_full)) != PDZ_OK) return st;
    {   // up hops of every full row as single entries
        const int mhu = p->up.max_hops;
        std::vector<uint8_t> ucnt_h(Du);
        std::vector<uint32_t> uell_h((size_t)std::max(mhu, 1) * Du);
        PDZ_HIP(hipMemcpy(ucnt_h.data(), p->up.count, Du, hipMemcpyDeviceToHost));
        if (mhu > 0) PDZ_HIP(hipMemcpy(uell_h.data(), p->up.ell, (size_t)mhu * Du * 4, hipMemcpyDeviceToHost));
        const int stride = std::max(mhu, 1);
        std::vector<uint64_t> fup((size_t)rows_full.size() * stride, kFupNone);
        bool fits = row_off[ureps] < (1ull << 40);
        for (size_t kk = 0; kk < rows_full.size() && fits; ++kk) {
            const uint32_t ru = row_rank[rows_full[kk]];
            int h2 = 0;
            for (int pass = 0; pass < 2; ++pass)   // A and image sources first, palindromic ones last
                for (int h = 0; h < ucnt_h[ru]; ++h) {
                    const uint32_t e = uell_h[(size_t)h * Du + ru];
                    const uint32_t ru2 = e & kTargetMask;
                    if ((ucls[ru2] == kClsPal) != (pass == 1)) continue;
                    fup[kk * stride + h2++] =
                        row_off[urow[ru2]] | ((uint64_t)ucls[ru2] << 40) | ((uint64_t)(e >> kTargetBits) << 48);
                }
        }
        if (fits) {
            q->fup_stride = stride;
            if ((st = dupload(&q->d_fup, fup)) != PDZ_OK) return st;
        }
    }
    if ((st = dupload(&q->d_rows_pal, rows_pal)) != PDZ_OK) return st;
    if (!q->force_loop && q->n_full > 0 && p->dn.max_hops > 0) {
        // the scheduled down pass: the column hop table's gather schedule
        // (none when it does not apply), then the row groups
        SectorTables cv;
        cv.D = Dd;
        cv.max_hops = mh;
        cv.count = q->d_fcnt;
        cv.ell = q->d_fell;
        if ((st = build_down_schedule(cv, p->coef_host, &q->fsched, nullptr)) != PDZ_OK) return st;
    }
    if (q->fsched.words) {
        std::vector<uint32_t> ust(Du), dst(Dd), col_dn(Dd);
        PDZ_HIP(hipMemcpy(ust.data(), p->up.states, Du * 4, hipMemcpyDeviceToHost));
        PDZ_HIP(hipMemcpy(dst.data(), p->dn.states, Dd * 4, hipMemcpyDeviceToHost));
        for (uint64_t c = 0; c < Dd; ++c) col_dn[c] = dst[dlistf[c]];
        if ((st = dupload(&q->d_col_dn, col_dn)) != PDZ_OK) return st;
        for (int i = 0; i < 2; ++i) {
            const uint32_t R = i == 0 ? 1u : 3u;
            std::vector<uint64_t> goff;
            std::vector<uint8_t> gnr;
            std::vector<uint32_t> gup;
            for (uint32_t k : rows_full) {
                const bool join = !gnr.empty() && gnr.back() < R && row_off[k] == goff.back() + gnr.back() * Dd;
                if (!join) {
                    goff.push_back(row_off[k]);
                    gnr.push_back(0);
                    gup.resize(gup.size() + R, 0u);
                }
                gup[(gnr.size() - 1) * R + gnr.back()] = ust[row_rank[k]];
                ++gnr.back();
            }
            q->ngroups[i] = gnr.size();
            if ((st = dupload(&q->d_goff[i], goff)) != PDZ_OK) return st;
            if ((st = dupload(&q->d_gnr[i], gnr)) != PDZ_OK) return st;
            if ((st = dupload(&q->d_grp_up[i], gup)) != PDZ_OK) return st;
        }
    }
    // structural nonzeros: per element its diagonal plus every hop whose source has a component here
    std::vector<uint8_t> ucnt(Du), dcnt(Dd);
    PDZ_HIP(hipMemcpy(ucnt.data(), p->up.count, Du, hipMemcpyDeviceToHost));
    PDZ_HIP(hipMemcpy(dcnt.data(), p->dn.count, Dd, hipMemcpyDeviceToHost));
    uint64_t dsum = 0, dsum_pal = 0;
    for (uint64_t r = 0; r < Dd; ++r) dsum += dcnt[r];
    for (uint32_t r : dlist) dsum_pal += dcnt[r];
    uint64_t nnz = p->D;
    for (uint64_t k = 0; k < ureps; ++k) {
        const uint32_t ru = row_rank[k];
        if (row_pal[k]) nnz += dsum_pal + (uint64_t)ucnt[ru] * q->Lp;
        else nnz += dsum + (uint64_t)ucnt[ru] * Dd;
    }
    p->nnz = nnz;   // counts hops onto excluded self-mapped states as well (an upper bound by at most those)
    return ok();
}

}  // namespace pdz

using namespace pdz;

extern "C" {

pdz_status pdz_parity_problem_create(int32_t n_sites, const pdz_bond* bonds, int32_t n_bonds, double U, int32_t n_up,
                                     int32_t n_dn, int32_t parity, pdz_problem* out) {
    if (!out) return fail(PDZ_EINVAL, "out is NULL");
    *out = nullptr;
    if (parity != 1 && parity != -1) return fail(PDZ_EINVAL, "parity must be +1 or -1");
    if (n_sites < 1 || n_sites > kMaxSites) return fail(PDZ_ERANGE, "n_sites must be in [1, 32]");
    if (n_bonds < 0 || (n_bonds > 0 && !bonds)) return fail(PDZ_EINVAL, "bad bond list");
    {   // mirror symmetry of the bonds: (i, j, t) -> (N-1-i, N-1-j, t), repeated pairs summed
        std::vector<double> t((size_t)n_sites * n_sites, 0.0);
        for (int b = 0; b < n_bonds; ++b) {
            const pdz_bond& bd = bonds[b];
            if (bd.i < 0 || bd.i >= n_sites || bd.j < 0 || bd.j >= n_sites || bd.i == bd.j || !std::isfinite(bd.t))
                return fail(PDZ_EINVAL, "bond " + std::to_string(b) + " is invalid");
            t[(size_t)bd.i * n_sites + bd.j] += bd.t;
            t[(size_t)bd.j * n_sites + bd.i] += bd.t;
        }
        for (int i = 0; i < n_sites; ++i)
            for (int j = 0; j < n_sites; ++j) {
                const double a = t[(size_t)i * n_sites + j];
                const double b = t[(size_t)(n_sites - 1 - i) * n_sites + (n_sites - 1 - j)];
                if (std::fabs(a - b) > 1e-12 * (1.0 + std::fabs(a)))
                    return fail(PDZ_EINVAL, "bonds are not symmetric under site i -> N-1-i");
            }
    }
    pdz_problem p = nullptr;
    pdz_status st = pdz_problem_create(n_sites, bonds, n_bonds, U, n_up, n_dn, &p);
    if (st != PDZ_OK) return st;
    if (p->hv_path != 0) {
        pdz_problem_destroy(p);
        return fail(PDZ_ERANGE, "parity subspaces need the sector hop tables (sectors below 2^24 strings)");
    }
    st = parity_build(p, parity);
    if (st != PDZ_OK) {
        const std::string msg = pdz_last_error();
        pdz_problem_destroy(p);
        return fail(st, msg);
    }
    p->hv_path = 3;
    *out = p;
    return ok();
}

pdz_status pdz_parity_rank(pdz_problem p, const uint32_t* up, const uint32_t* dn, uint64_t count, uint64_t* idx,
                           void* stream) {
    if (!p || !p->par) return fail(PDZ_EINVAL, "not a parity problem");
    if (count > 0 && (!up || !dn || !idx)) return fail(PDZ_EINVAL, "NULL array");
    if (count == 0) return ok();
    DeviceCtx* ctx = nullptr;
    pdz_status st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    hipLaunchKernelGGL(k_prank, dim3(pgrid(count, (unsigned)ctx->cu_count)), dim3(kPBlock), 0, (hipStream_t)stream,
                       pargs(p), ctx->binom, p->par->d_S, std::max(p->n_up, p->n_dn), p->N, p->n_up, p->n_dn, up, dn,
                       count, idx, ctx->err);
    PDZ_HIP(hipGetLastError());
    return ok();
}

pdz_status pdz_parity_unrank(pdz_problem p, const uint64_t* idx, uint64_t count, uint32_t* up, uint32_t* dn,
                             void* stream) {
    if (!p || !p->par) return fail(PDZ_EINVAL, "not a parity problem");
    if (count > 0 && (!up || !dn || !idx)) return fail(PDZ_EINVAL, "NULL array");
    if (count == 0) return ok();
    DeviceCtx* ctx = nullptr;
    pdz_status st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    hipLaunchKernelGGL(k_punrank, dim3(pgrid(count, (unsigned)ctx->cu_count)), dim3(kPBlock), 0, (hipStream_t)stream,
                       pargs(p), idx, count, up, dn, ctx->err);
    PDZ_HIP(hipGetLastError());
    return ok();
}

}  // extern "C"
