// y = H x for the Hubbard Hamiltonian (Eq. 1), matrix-free.
//
// Vector layout: X[i_up][i_dn], index i_up * D_dn + i_dn (composite index of
// Sec. III).  With this layout
//     y[u,d] = U popc(phi_up(u) & phi_dn(d)) x[u,d]
//            + sum_{dn hops d->d'} a(d,d') x[u,d']      (gathers inside row u)
//            + sum_{up hops u->u'} a(u,u') x[u',d]      (rows of X, coalesced)
// where a = -t_b * sign.  Each hop target index comes from the forward map
// (perfect hash), evaluated once per sector state when the problem is created
// (hop tables, k_hash.hip), or per element on the fallback path below.
//
// Two passes with opposite locality:
//  1. down pass (k_hv_down_*): rows of x are staged in LDS and each thread
//     gathers the down-hop targets of its column from LDS; writes
//     diag + down term to y.
//  2. up pass (k_hv_up): a column chunk of x stays L2-resident while the work
//     groups of one XCD stream every row's up hops over it as coalesced row
//     segments; adds the up term to y in place.
// Every output element is summed by one thread in a fixed order (diagonal,
// down hops in bond order, up hops in bond order): no atomics, bitwise
// reproducible, and the same order as the fallback path.
#include <type_traits>

#include "pdz_internal.h"

namespace pdz {

namespace {

constexpr int kWideBlock = 1024;   // down pass, long rows
constexpr int kNarrowBlock = 256;  // down pass, short rows
constexpr int kUpBlock = 256;      // up pass
constexpr int kFlyBlock = 256;
constexpr size_t kLdsBytes = 160 * 1024;
constexpr size_t kDynLds = kLdsBytes - 1024;   // kernels also hold a few static words

template <typename T, typename E>
struct DownArgs {
    uint64_t D_up, D_dn;
    uint64_t pitch;   // elements from one row of x, y (and the recurrence vectors) to the next: D_dn, or
                      // more with zeros past column D_dn that the pass keeps zero
    T U;
    const uint32_t* up_states;
    const uint32_t* dn_states;
    const uint8_t* dn_count;
    const E* dn_ell;
    uint32_t tmask;   // target mask of an entry
    int cshift;       // amplitude index = entry >> cshift
    uint32_t ell_bytes;   // size of dn_ell (16-bit tables; 0 otherwise)
    const T* coef;
    int ncoef;
    int rows;         // rows staged per group
    int add_y;        // scheduled pass: 1 adds its part to y (written by the up pass), 0 writes y
    double* dotp;     // NULL, or one partial sum of x . y (this pass's output) per work group
    const int* skip;
    // Row groups other than R consecutive rows of the D_up x pitch matrix
    // (scheduled pass only; the full rows of a parity subspace): group g has
    // gnr[g] rows of pitch elements from element goff[g]; up_states then holds
    // the up string of row r of group g at g * R + r, and dn_states the down
    // string of each column (the GRP kernels; the others ignore these).
    const uint64_t* goff;
    const uint8_t* gnr;
    uint64_t ngroups;
    // Fused Lanczos recurrence (FUSE kernels only): the staged rows are
    // q_{k+1} = sc[k] (y + fz) - alpha[k] sc[k] fq1 - beta[k] sc[k-1] fq2 (row groups: y alone),
    // formed element by element from the previous step's down part (y, then
    // overwritten by this pass's output), its up part fz, q_k (fq1) and
    // q_{k-1} (fq2, overwritten by q_{k+1}; also copied to slot k + 1 of fkeep
    // when that is set), with k = *fkidx.  fnorm: one partial |q_{k+1}|^2 per
    // work group.
    const T* fz;
    const T* fq1;
    T* fq2;
    T* fkeep;
    uint64_t fkeep_ld;
    int fkeep_cap;
    const double* falpha;
    const double* fbeta;
    const double* fsc;
    const int* fkidx;
    double* fnorm;
};

template <typename T, typename E>
struct UpArgs {
    uint64_t D_up, D_dn;
    uint64_t pitch;   // row pitch of x and y, as in DownArgs
    const uint8_t* up_count;
    const E* up_ell;
    uint32_t tmask;
    int cshift;
    const T* coef;
    int ncoef;
    uint32_t n_chunks;    // column chunks of width CW
    uint32_t row_tiles;   // row tiles of ROWS_PER_TILE rows
    int max_hops;         // hop slots per row in the table
    int map;              // block -> tile order (up_tile)
    int add_y;            // 1: out = y + up term (y from the down pass); 0: out = up term
    double* dotp;         // NULL, or one partial sum of x . out per work group
    const int* skip;
};

// Hop slot h of sector state s: 32-bit tables are slot major, 16-bit tables
// keep slot pairs together (k_hash.hip).
template <typename E>
__device__ __forceinline__ uint32_t hop_entry(const E* ell, uint32_t h, uint64_t s, uint64_t D) {
    if (sizeof(E) == 2) return ell[(((uint64_t)(h >> 1) * D + s) << 1) + (h & 1u)];
    return ell[(uint64_t)h * D + s];
}

// VEC consecutive elements at element alignment (the ISA's multi-dword loads
// need only 4-byte alignment).
template <typename T, int VEC>
__device__ __forceinline__ void vec_load(const T* p, T (&out)[VEC]) {
    if constexpr (VEC == 1) {
        out[0] = p[0];
    } else {
        typedef T vt __attribute__((ext_vector_type(VEC), aligned(sizeof(T))));
        const vt t = *reinterpret_cast<const vt*>(p);
#pragma unroll
        for (int i = 0; i < VEC; ++i) out[i] = t[i];
    }
}

template <typename T, int VEC>
__device__ __forceinline__ void vec_store(T* p, const T (&in)[VEC]) {
    if constexpr (VEC == 1) {
        p[0] = in[0];
    } else {
        typedef T vt __attribute__((ext_vector_type(VEC), aligned(sizeof(T))));
        vt t;
#pragma unroll
        for (int i = 0; i < VEC; ++i) t[i] = in[i];
        *reinterpret_cast<vt*>(p) = t;
    }
}

template <typename T>
__device__ __forceinline__ void load_coef(T* sc, const T* __restrict__ g, int n) {
    for (int k = threadIdx.x; k < n; k += blockDim.x) sc[k] = g[k];
}

// Sum of one double per thread over the work group (fixed order) into
// *out by thread 0; BLOCK threads, a multiple of 64.
template <int BLOCK>
__device__ __forceinline__ void block_dot_store(double v, double* out) {
    __shared__ double wsum[BLOCK / 64];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < BLOCK / 64; ++i) t += wsum[i];
        *out = t;
    }
}

// Two sums at once (fixed order) into *out1, *out2 by thread 0.
template <int BLOCK>
__device__ __forceinline__ void block_dot_store2(double v1, double* out1, double v2, double* out2) {
    __shared__ double wsum2[2][BLOCK / 64];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        v1 += __shfl_xor(v1, m);
        v2 += __shfl_xor(v2, m);
    }
    if ((threadIdx.x & 63) == 0) {
        wsum2[0][threadIdx.x >> 6] = v1;
        wsum2[1][threadIdx.x >> 6] = v2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t1 = 0.0, t2 = 0.0;
        for (int i = 0; i < BLOCK / 64; ++i) {
            t1 += wsum2[0][i];
            t2 += wsum2[1][i];
        }
        *out1 = t1;
        *out2 = t2;
    }
}

// ---------------------------------------------------------------- down pass

// Long rows: R (1 to 3) consecutive rows staged interleaved as
// lds[d * R + r]; each thread owns columns d and accumulates R outputs, so one
// table entry and one LDS gather serve R rows.  The rows of the next group are
// loaded into registers (up to PER per thread) while the current group computes.
// Four hops from two slot-pair words: acc[r] += c_h * row_r[target_h], in
// slot order.
template <typename T, int R>
__device__ __forceinline__ void hops4(T (&acc)[R], const T* coef, const T* rows, uint32_t w0, uint32_t w1,
                                      uint32_t tmask, int cshift) {
    const uint32_t e0 = w0 & 0xFFFFu, e1 = w0 >> 16, e2 = w1 & 0xFFFFu, e3 = w1 >> 16;
    const T c0 = coef[e0 >> cshift], c1 = coef[e1 >> cshift], c2 = coef[e2 >> cshift], c3 = coef[e3 >> cshift];
    const T* s0 = rows + (size_t)(e0 & tmask) * R;
    const T* s1 = rows + (size_t)(e1 & tmask) * R;
    const T* s2 = rows + (size_t)(e2 & tmask) * R;
    const T* s3 = rows + (size_t)(e3 & tmask) * R;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        acc[r] += c0 * s0[r];
        acc[r] += c1 * s1[r];
        acc[r] += c2 * s2[r];
        acc[r] += c3 * s3[r];
    }
}

// The last n (1 to 3) hops of a column; slots past n read entry 0.
template <typename T, int R>
__device__ __forceinline__ void hops_tail(T (&acc)[R], const T* coef, const T* rows, uint32_t w0, uint32_t w1, int n,
                                          uint32_t tmask, int cshift) {
    const uint32_t e0 = w0 & 0xFFFFu;
    const uint32_t e1 = n > 1 ? w0 >> 16 : 0u;
    const uint32_t e2 = n > 2 ? w1 & 0xFFFFu : 0u;
    const T c0 = coef[e0 >> cshift], c1 = coef[e1 >> cshift], c2 = coef[e2 >> cshift];
    const T* s0 = rows + (size_t)(e0 & tmask) * R;
    const T* s1 = rows + (size_t)(e1 & tmask) * R;
    const T* s2 = rows + (size_t)(e2 & tmask) * R;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        acc[r] += c0 * s0[r];
        if (n > 1) acc[r] += c1 * s1[r];
        if (n > 2) acc[r] += c2 * s2[r];
    }
}

// Row of flat index k in a group of R rows of Dn elements each.
template <int R>
__device__ __forceinline__ uint32_t row_of(uint32_t k, uint32_t Dn) {
    if (R == 1) return 0u;
    if (R == 2) return k >= Dn ? 1u : 0u;
    return k >= 2 * Dn ? 2u : (k >= Dn ? 1u : 0u);
}

template <typename T, typename E, int R, int MAXH, bool FUSE = false>
__global__ __launch_bounds__(kWideBlock) void k_hv_down_wide(const DownArgs<T, E> a, const T* __restrict__ x,
                                                             T* __restrict__ y) {
    if (a.skip && *a.skip) return;
    static_assert(!FUSE || MAXH == 0, "the fused recurrence rides on the looped table reads");
    extern __shared__ __align__(16) unsigned char smem[];
    T* coef = reinterpret_cast<T*>(smem);
    T* rows = coef + kMaxCoef;
    load_coef(coef, a.coef, a.ncoef);
    const uint64_t D_up = a.D_up, D_dn = a.D_dn;
    const uint32_t Dn = (uint32_t)D_dn;
    const uint64_t pitch = a.pitch;   // a group's rows are R * pitch consecutive elements
    const uint32_t Pn = (uint32_t)pitch;
    const uint64_t ngroups = (D_up + R - 1) / R;
    // raw buffer over the 16-bit table (dword 3: the gfx9 untyped 32-bit format)
    const __amdgpu_buffer_rsrc_t ell_rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<E*>(a.dn_ell), (short)0, (int)a.ell_bytes, 0x00020000);
    static_assert(R >= 1 && R <= 3, "rows per group");
    // elements per thread loaded ahead for the next group: the fused form holds
    // four raw operands per element until the group is staged
    constexpr int PER = FUSE ? (sizeof(T) == 8 ? 6 : 12)
                             : (R >= 2 ? (sizeof(T) == 8 ? 8 : 12) : (sizeof(T) == 8 ? 16 : 24));
    T pre[PER];
    T pz[FUSE ? PER : 1], p1[FUSE ? PER : 1], p2[FUSE ? PER : 1];   // FUSE: fz, fq1, fq2 (pre holds y)
    double dsum = 0.0;   // x . y over this work group's elements (when a.dotp is set)
    double nsum = 0.0;   // |q_{k+1}|^2 over this work group's elements (FUSE)
    double fa = 0.0, fb = 0.0, fc = 0.0;
    T* fkeep = nullptr;
    if constexpr (FUSE) {
        const int k = *a.fkidx;
        fa = a.fsc[k];
        fb = a.falpha[k] * a.fsc[k];
        fc = k > 0 ? a.fbeta[k] * a.fsc[k - 1] : 0.0;
        if (a.fkeep && k + 1 < a.fkeep_cap) fkeep = a.fkeep + (uint64_t)(k + 1) * a.fkeep_ld;
    }
    // element k of the rows that start at element `off`: x, or q_{k+1} formed
    // (and stored) here
    auto stage_elem = [&](uint64_t off, uint32_t k) -> T {
        if constexpr (FUSE) {
            const T v = lanczos_recurrence<T>(y[off + k], a.fz[off + k], a.fq1[off + k], a.fq2[off + k], fa, fb, fc);
            a.fq2[off + k] = v;
            if (fkeep) fkeep[off + k] = v;
            nsum += (double)v * (double)v;
            return v;
        } else {
            return __builtin_nontemporal_load(x + off + k);
        }
    };
    auto fetch = [&](uint64_t g) {
        const uint64_t u0 = g * R;
        const uint64_t nelem = ((D_up - u0) < (uint64_t)R ? (D_up - u0) : (uint64_t)R) * pitch;
        if constexpr (FUSE) {
            // raw operands only: the recurrence is formed when the group is staged,
            // so these loads stay in flight while the current group computes
            const uint64_t off = u0 * pitch;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const uint64_t k = threadIdx.x + (uint64_t)i * kWideBlock;
                if (k < nelem) {
                    pre[i] = y[off + k];
                    pz[i] = a.fz[off + k];
                    p1[i] = a.fq1[off + k];
                    p2[i] = a.fq2[off + k];
                }
            }
        } else {
            const T* base = x + u0 * pitch;
#pragma unroll
            for (int i = 0; i < PER; ++i) {
                const uint64_t k = threadIdx.x + (uint64_t)i * kWideBlock;
                pre[i] = (k < nelem) ? __builtin_nontemporal_load(base + k) : (T)0;
            }
        }
    };
    if (blockIdx.x < ngroups) fetch(blockIdx.x);
    for (uint64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const uint64_t u0 = g * R;
        const int nr = (int)((D_up - u0) < (uint64_t)R ? (D_up - u0) : (uint64_t)R);
        __syncthreads();
        const uint64_t nelem_g = (uint64_t)nr * pitch;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const uint32_t k = threadIdx.x + (uint32_t)i * kWideBlock;
            if (k < (uint32_t)R * Pn) {
                const uint32_t r = row_of<R>(k, Pn);
                T v = pre[i];
                if constexpr (FUSE) {
                    v = (T)0;
                    if (k < nelem_g) {
                        const uint64_t e = u0 * pitch + k;
                        v = lanczos_recurrence<T>(pre[i], pz[i], p1[i], p2[i], fa, fb, fc);
                        a.fq2[e] = v;
                        if (fkeep) fkeep[e] = v;
                        nsum += (double)v * (double)v;
                    }
                }
                const uint32_t dc = k - r * Pn;   // column (past D_dn: padding, not staged)
                if (dc < Dn) rows[(size_t)dc * R + r] = v;
            }
        }
        {   // elements beyond the register prefetch, loaded now
            const uint64_t nelem = (uint64_t)nr * pitch;
            const T* base = x + u0 * pitch;
            for (uint32_t k = threadIdx.x + (uint32_t)PER * kWideBlock; k < (uint32_t)R * Pn; k += kWideBlock) {
                const uint32_t r = row_of<R>(k, Pn);
                T v = (T)0;
                if (k < nelem) v = FUSE ? stage_elem(u0 * pitch, k) : base[k];
                const uint32_t dc = k - r * Pn;
                if (dc < Dn) rows[(size_t)dc * R + r] = v;
            }
        }
        __syncthreads();
        if (g + gridDim.x < ngroups) fetch(g + gridDim.x);
        uint32_t pu[R];
#pragma unroll
        for (int r = 0; r < R; ++r) pu[r] = a.up_states[u0 + (r < nr ? r : 0)];
        for (uint32_t d = threadIdx.x; d < Dn; d += kWideBlock) {
            const uint32_t pd = a.dn_states[d];
            T acc[R];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = a.U * (T)__builtin_popcount(pu[r] & pd) * rows[(size_t)d * R + r];
            const int cnt = a.dn_count[d];
            if (MAXH > 0) {
                // issue every table load of the column before the first use:
                // one L2 round trip per column instead of one per few hops
                // (16-bit tables only: two slots per 32-bit word)
                const uint32_t* w32 = reinterpret_cast<const uint32_t*>(a.dn_ell);
                uint32_t w[MAXH > 0 ? MAXH / 2 : 1];
#pragma unroll
                for (int k = 0; k < MAXH / 2; ++k) w[k] = (2 * k < cnt) ? w32[(uint32_t)k * Dn + d] : 0u;
#pragma unroll
                for (int h = 0; h < MAXH; ++h) {
                    if (h < cnt) {
                        const uint32_t e = (h & 1) ? (w[h >> 1] >> 16) : (w[h >> 1] & 0xFFFFu);
                        const T c = coef[e >> a.cshift];
                        const T* sv = rows + (e & a.tmask) * R;
#pragma unroll
                        for (int r = 0; r < R; ++r) acc[r] += c * sv[r];
                    }
                }
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (r < nr) {
                        __builtin_nontemporal_store(acc[r], y + (u0 + r) * pitch + d);
                        dsum += (double)rows[(size_t)d * R + r] * (double)acc[r];
                    }
                continue;
            }
            if constexpr (sizeof(E) == 2) {
                // Slot-pair words of four hops at a time, in two register
                // sets: the words of the group after next are loaded while a
                // group computes.  Slots past the count load pair 0 instead
                // (no branch around a load, so the wait before a group covers
                // only its own words).  Buffer loads (range-checked against
                // the table size) keep the compiler from merging the two
                // loads that feed a loop-carried word into one load at its
                // use, which would undo the prefetch.  The last one to three
                // hops form one group whose missing slots use entry 0 (an
                // address inside the staged rows) and add nothing.
                auto ld = [&](int slot) -> uint32_t {
                    const uint32_t pair = (uint32_t)(slot < cnt ? slot : 0) >> 1;
                    return __builtin_amdgcn_raw_buffer_load_b32(ell_rs, (pair * Dn + d) * 4u, 0, 0);
                };
                uint32_t a0 = ld(0), a1 = ld(2), b0 = ld(4), b1 = ld(6);
                int h = 0;
                for (; h + 8 <= cnt; h += 8) {
                    hops4<T, R>(acc, coef, rows, a0, a1, a.tmask, a.cshift);
                    a0 = ld(h + 8);
                    a1 = ld(h + 10);
                    __builtin_amdgcn_sched_barrier(0);   // issue them before the next group's work
                    hops4<T, R>(acc, coef, rows, b0, b1, a.tmask, a.cshift);
                    b0 = ld(h + 12);
                    b1 = ld(h + 14);
                    __builtin_amdgcn_sched_barrier(0);
                }
                const int left = cnt - h;   // 0 to 7: slots h.. in a0, a1, then b0, b1
                if (left >= 4) {
                    hops4<T, R>(acc, coef, rows, a0, a1, a.tmask, a.cshift);
                    if (left > 4) hops_tail<T, R>(acc, coef, rows, b0, b1, left - 4, a.tmask, a.cshift);
                } else if (left > 0) {
                    hops_tail<T, R>(acc, coef, rows, a0, a1, left, a.tmask, a.cshift);
                }
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (r < nr) {
                        __builtin_nontemporal_store(acc[r], y + (u0 + r) * pitch + d);
                        dsum += (double)rows[(size_t)d * R + r] * (double)acc[r];
                    }
                continue;
            }
            int h = 0;
            for (; h + 4 <= cnt; h += 4) {
                const uint32_t e0 = hop_entry(a.dn_ell, h + 0, d, D_dn), e1 = hop_entry(a.dn_ell, h + 1, d, D_dn);
                const uint32_t e2 = hop_entry(a.dn_ell, h + 2, d, D_dn), e3 = hop_entry(a.dn_ell, h + 3, d, D_dn);
                const T c0 = coef[e0 >> a.cshift], c1 = coef[e1 >> a.cshift];
                const T c2 = coef[e2 >> a.cshift], c3 = coef[e3 >> a.cshift];
                const T* s0 = rows + (size_t)(e0 & a.tmask) * R;
                const T* s1 = rows + (size_t)(e1 & a.tmask) * R;
                const T* s2 = rows + (size_t)(e2 & a.tmask) * R;
                const T* s3 = rows + (size_t)(e3 & a.tmask) * R;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    acc[r] += c0 * s0[r];
                    acc[r] += c1 * s1[r];
                    acc[r] += c2 * s2[r];
                    acc[r] += c3 * s3[r];
                }
            }
            for (; h < cnt; ++h) {
                const uint32_t e = hop_entry(a.dn_ell, h, d, D_dn);
                const T c = coef[e >> a.cshift];
                const T* sv = rows + (size_t)(e & a.tmask) * R;
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r] += c * sv[r];
            }
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (r < nr) {
                    __builtin_nontemporal_store(acc[r], y + (u0 + r) * pitch + d);
                    dsum += (double)rows[(size_t)d * R + r] * (double)acc[r];
                }
        }
    }
    if constexpr (FUSE)
        block_dot_store2<kWideBlock>(dsum, a.dotp + blockIdx.x, nsum, a.fnorm + blockIdx.x);
    else if (a.dotp)
        block_dot_store<kWideBlock>(dsum, a.dotp + blockIdx.x);
}

// Scheduled down pass (plans down 5, 6, 7: 1, 2 or 3 rows per group).  The
// group's rows are staged as planes of 32-bit words kSchedPlane words apart in
// a static LDS array, element d' of a row in bank d' mod 32 (FP64: a plane of
// low words and one of high words), and each wave's 64 columns gather in the
// steps of the sector's gather schedule (pdz_sched.cpp): at every step the 32
// lanes of a half-wave read 32 different banks, so no read waits on a bank
// conflict.  The hop magnitude of a step is the same in every lane; its sign
// comes with the lane's entry.  An element's sum: diagonal, then its hops in
// schedule order.  The next group's
// rows are partly loaded into registers while a group computes; the rest are
// loaded in unrolled batches once the group is done.  FUSE: the staged rows
// are q_{k+1}, formed from the previous step's parts as in k_hv_down_wide.
constexpr int kSchedMaxWords = kSchedMaxSteps / 2;   // schedule words a wave holds in registers

template <typename T>
struct SchedArgs {
    const uint32_t* words;
    const uint32_t* meta;  // per wave: word offset, steps | steps of the smaller magnitude << 16
    T mag0, mag1;          // hop magnitudes of the two step groups
};

// Sums of one double per thread over the work group (fixed order) into *out1
// and *out2 by thread 0, through `red` (LDS the work group no longer reads).
__device__ __forceinline__ void sched_block_sums(double v1, double* out1, double v2, double* out2, double* red) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        v1 += __shfl_xor(v1, m);
        v2 += __shfl_xor(v2, m);
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = v1;
        red[kWideBlock / 64 + (threadIdx.x >> 6)] = v2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t1 = 0.0, t2 = 0.0;
        for (int i = 0; i < kWideBlock / 64; ++i) {
            t1 += red[i];
            t2 += red[kWideBlock / 64 + i];
        }
        if (out1) *out1 = t1;
        if (out2) *out2 = t2;
    }
}

// Read-only data the kernels read at wave-uniform addresses, seen through the
// constant address space so that the reads are scalar loads.
template <typename U>
using CPtr = const U __attribute__((address_space(4)))*;
template <typename U>
__device__ __forceinline__ CPtr<U> const_ptr(const U* p) {
    return (CPtr<U>)p;
}


// GRP: the row groups come from a.goff / a.gnr (and fz is not read: the
// recurrence takes the whole H q_k from y); otherwise R consecutive rows.
template <typename T, typename E, int R, bool FUSE, bool GRP = false>
__global__ __launch_bounds__(kWideBlock) void k_hv_down_sched(const DownArgs<T, E> a, const SchedArgs<T> sc,
                                                              const T* __restrict__ x, T* __restrict__ y) {
    if (a.skip && *a.skip) return;
    constexpr int W = sizeof(T) / 4;      // 32-bit planes per row
    static_assert(R >= 1 && R <= 3 && (W == 1 || R == 1), "rows per group");
    constexpr uint32_t P = kSchedPlane;
    // staging by quads of four consecutive elements of the group: quads per thread loaded ahead
    // for the next group, and quads per batch of the remaining loads
    constexpr int PQ = FUSE ? 1 : 2;
    constexpr int NQ = FUSE ? (W == 1 ? 2 : 1) : 4;
    __shared__ __align__(16) uint32_t planes[R * W * P];   // plane (r, word) at (r * W + word) * P
    const unsigned char* lbase = reinterpret_cast<const unsigned char*>(planes);
    const uint64_t D_up = a.D_up, D_dn = a.D_dn;
    const uint32_t Dn = (uint32_t)D_dn;
    const uint64_t pitch = a.pitch;   // a group's rows are R * pitch consecutive elements (columns
    const uint32_t Pn = (uint32_t)pitch;   // past Dn: zeros, staged too, never gathered)
    const uint64_t ngroups = GRP ? a.ngroups : (D_up + R - 1) / R;
    const uint32_t nwaves = (Dn + 63) / 64;
    // rows and first element of group g
    auto grows = [&](uint64_t g) -> uint32_t {
        if constexpr (GRP && R == 1) {
            return 1u;
        } else if constexpr (GRP) {
            return const_ptr(a.gnr)[g];   // wave-uniform: scalar loads
        } else {
            const uint64_t u0 = g * R;
            return (uint32_t)((D_up - u0) < (uint64_t)R ? (D_up - u0) : (uint64_t)R);
        }
    };
    auto gstart = [&](uint64_t g) -> uint64_t {
        if constexpr (GRP) return const_ptr(a.goff)[g];
        else return g * R * pitch;
    };
    const int lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // zero pads: read by lanes without a hop at a step
    for (uint32_t k = threadIdx.x; k < (uint32_t)(R * W) * 32u; k += kWideBlock)
        planes[(k / 32u) * P + P - 32u + (k % 32u)] = 0u;
    double dsum = 0.0, nsum = 0.0;
    double fa = 0.0, fb = 0.0, fc = 0.0;
    T* fkeep = nullptr;
    if constexpr (FUSE) {
        const int k = *a.fkidx;
        fa = a.fsc[k];
        fb = a.falpha[k] * a.fsc[k];
        fc = k > 0 ? a.fbeta[k] * a.fsc[k - 1] : 0.0;
        if (a.fkeep && k + 1 < a.fkeep_cap) fkeep = a.fkeep + (uint64_t)(k + 1) * a.fkeep_ld;
    }
    // element k of a group lives in row k / pitch at column k mod pitch
    auto put = [&](uint32_t k, T v) {
        const uint32_t r = R == 1 ? 0u : (k >= 2 * Pn ? 2u : (k >= Pn ? 1u : 0u));
        const uint32_t d = k - r * Pn;
        if constexpr (W == 1) {
            planes[r * P + d] = __float_as_uint((float)v);
        } else {
            const unsigned long long b = (unsigned long long)__double_as_longlong((double)v);
            planes[d] = (uint32_t)b;
            planes[P + d] = (uint32_t)(b >> 32);
        }
    };
    // element of row r at byte address ba of plane r (ba = 4 d')
    auto get = [&](int r, uint32_t ba) -> T {
        const uint32_t* pr = reinterpret_cast<const uint32_t*>(lbase + ba);
        if constexpr (W == 1) {
            return (T)__uint_as_float(pr[(uint32_t)r * P]);
        } else {
            return (T)__longlong_as_double((long long)(((unsigned long long)pr[P] << 32) | pr[0]));
        }
    };
    // the four elements of quad k0 / 4 of the group (k0 + j < nelem of them exist)
    auto load4 = [&](const T* base, uint64_t e0, uint32_t k0, uint32_t nelem, T (&v)[4], bool stream) {
        if (k0 + 4 <= nelem) {
            if (stream) {
                typedef T vt __attribute__((ext_vector_type(4), aligned(sizeof(T))));
                const vt t = __builtin_nontemporal_load(reinterpret_cast<const vt*>(base + e0));
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] = t[j];
            } else {
                vec_load<T, 4>(base + e0, v);
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = (k0 + (uint32_t)j < nelem) ? base[e0 + j] : (T)0;
        }
    };
    T pre[PQ][4];
    T pz[FUSE ? PQ : 1][4], p1[FUSE ? PQ : 1][4], p2[FUSE ? PQ : 1][4];
    auto fetch = [&](uint64_t g) {
        const uint32_t nelem = grows(g) * Pn;
        const uint64_t off = gstart(g);
#pragma unroll
        for (int i = 0; i < PQ; ++i) {
            const uint32_t k0 = 4u * (threadIdx.x + (uint32_t)i * kWideBlock);
            if (k0 < nelem) {
                if constexpr (FUSE) {
                    load4(y, off + k0, k0, nelem, pre[i], false);
                    if constexpr (GRP) pz[i][0] = pz[i][1] = pz[i][2] = pz[i][3] = (T)0;
                    else load4(a.fz, off + k0, k0, nelem, pz[i], false);
                    load4(a.fq1, off + k0, k0, nelem, p1[i], false);
                    load4(a.fq2, off + k0, k0, nelem, p2[i], false);
                } else {
                    load4(x, off + k0, k0, nelem, pre[i], true);
                }
            }
        }
    };
    // q_{k+1} at the elements of quad k0 / 4 (FUSE), stored back and counted in |q_{k+1}|^2
    auto form4 = [&](uint64_t e0, uint32_t k0, uint32_t nelem, const T (&hd)[4], const T (&hu)[4], const T (&q1)[4],
                     const T (&q2)[4], T (&v)[4]) {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = lanczos_recurrence<T>(hd[j], hu[j], q1[j], q2[j], fa, fb, fc);
        if (k0 + 4 <= nelem) {
            vec_store<T, 4>(a.fq2 + e0, v);
            if (fkeep) vec_store<T, 4>(fkeep + e0, v);
#pragma unroll
            for (int j = 0; j < 4; ++j) nsum += (double)v[j] * (double)v[j];
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (k0 + (uint32_t)j < nelem) {
                    a.fq2[e0 + j] = v[j];
                    if (fkeep) fkeep[e0 + j] = v[j];
                    nsum += (double)v[j] * (double)v[j];
                }
        }
    };
    // the staged values of quad k0 / 4 into the planes (zeros past the group's last element)
    auto put4 = [&](uint32_t k0, uint32_t nelem, uint32_t nput, const T (&v)[4]) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t k = k0 + (uint32_t)j;
            if (k < nput) put(k, k < nelem ? v[j] : (T)0);
        }
    };
    // +-magnitude bits: FP32 the whole word, FP64 the high word (the low word is the same for both signs)
    auto hi_bits = [](T m) -> uint32_t {
        if constexpr (W == 1) return __float_as_uint((float)m);
        else return (uint32_t)((unsigned long long)__double_as_longlong((double)m) >> 32);
    };
    auto lo_bits = [](T m) -> uint32_t {
        if constexpr (W == 1) return 0u;
        else return (uint32_t)(unsigned long long)__double_as_longlong((double)m);
    };
    const uint32_t mp0 = hi_bits(sc.mag0), ml0 = lo_bits(sc.mag0);
    const uint32_t mp1 = hi_bits(sc.mag1), ml1 = lo_bits(sc.mag1);
    if (blockIdx.x < ngroups) fetch(blockIdx.x);
    for (uint64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const uint64_t u0 = g * R;
        const uint64_t g0 = gstart(g);   // first element of the group
        const int nr = (int)grows(g);
        const uint32_t nelem = (uint32_t)nr * Pn;
        const uint32_t nput = (uint32_t)R * Pn;   // rows past the last are staged as zeros
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PQ; ++i) {
            const uint32_t k0 = 4u * (threadIdx.x + (uint32_t)i * kWideBlock);
            if (k0 < nput) {
                T v[4];
                if constexpr (FUSE) {
                    if (k0 < nelem) form4(g0 + k0, k0, nelem, pre[i], pz[i], p1[i], p2[i], v);
                    put4(k0, nelem, nput, v);
                } else {
                    put4(k0, nelem, nput, pre[i]);
                }
            }
        }
#pragma nounroll
        for (uint32_t qb = threadIdx.x + (uint32_t)PQ * kWideBlock; 4u * qb < nput; qb += (uint32_t)NQ * kWideBlock) {
            // every load of the batch issued before the first store to LDS
            T v0[NQ][4], v1[FUSE ? NQ : 1][4], v2[FUSE ? NQ : 1][4], v3[FUSE ? NQ : 1][4];
#pragma unroll
            for (int j = 0; j < NQ; ++j) {
                const uint32_t k0 = 4u * (qb + (uint32_t)j * kWideBlock);
                if (k0 < nelem) {
                    const uint64_t e0 = g0 + k0;
                    if constexpr (FUSE) {
                        load4(y, e0, k0, nelem, v0[j], false);
                        if constexpr (GRP) v1[j][0] = v1[j][1] = v1[j][2] = v1[j][3] = (T)0;
                        else load4(a.fz, e0, k0, nelem, v1[j], false);
                        load4(a.fq1, e0, k0, nelem, v2[j], false);
                        load4(a.fq2, e0, k0, nelem, v3[j], false);
                    } else {
                        load4(x, e0, k0, nelem, v0[j], true);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < NQ; ++j) {
                const uint32_t k0 = 4u * (qb + (uint32_t)j * kWideBlock);
                if (k0 < nput) {
                    if constexpr (FUSE) {
                        T v[4];
                        if (k0 < nelem) form4(g0 + k0, k0, nelem, v0[j], v1[j], v2[j], v3[j], v);
                        put4(k0, nelem, nput, v);
                    } else {
                        put4(k0, nelem, nput, v0[j]);
                    }
                }
            }
        }
        __syncthreads();
        if (g + gridDim.x < ngroups) fetch(g + gridDim.x);
        uint32_t pu[R];
#pragma unroll
        for (int r = 0; r < R; ++r) pu[r] = a.up_states[u0 + (r < nr ? r : 0)];
        const CPtr<uint32_t> cmeta = const_ptr(sc.meta);
        uint32_t m_off = 0u, m_steps = 0u;   // the record of the wave's next column group
        if (wave < nwaves) {
            m_off = cmeta[2 * wave];
            m_steps = cmeta[2 * wave + 1];
        }
        for (uint32_t d0 = 0; d0 < Dn; d0 += kWideBlock) {
            const uint32_t wv = (d0 >> 6) + wave;
            if (wv >= nwaves) break;   // no barrier follows inside this loop
            // this wave's schedule words, all loaded before its steps start (its record was read
            // one column iteration ahead)
            const uint32_t so = m_off;
            const int n = (int)(m_steps & 0xFFFFu) / 2;   // words: a multiple of 2
            const int nb = (int)(m_steps >> 16) / 2;      // words of the smaller magnitude: a multiple of 2
            if (wv + kWideBlock / 64 < nwaves) {
                m_off = cmeta[2 * (wv + kWideBlock / 64)];
                m_steps = cmeta[2 * (wv + kWideBlock / 64) + 1];
            }
            // four words per lane in one 16-byte load (a last pair in one 8-byte load)
            const uint32_t* wp = sc.words + so;
            uint32_t wbuf[kSchedMaxWords];
#pragma unroll
            for (int q = 0; q < kSchedMaxWords / 4; ++q) {
                if (4 * q + 4 <= n) {
                    const uint4 w4 = *reinterpret_cast<const uint4*>(wp + (uint32_t)q * 256u + (uint32_t)lane * 4u);
                    wbuf[4 * q] = w4.x;
                    wbuf[4 * q + 1] = w4.y;
                    wbuf[4 * q + 2] = w4.z;
                    wbuf[4 * q + 3] = w4.w;
                } else if (4 * q < n) {
                    const uint2 w2 = *reinterpret_cast<const uint2*>(wp + (uint32_t)q * 256u + (uint32_t)lane * 2u);
                    wbuf[4 * q] = w2.x;
                    wbuf[4 * q + 1] = w2.y;
                    wbuf[4 * q + 2] = 0u;
                    wbuf[4 * q + 3] = 0u;
                } else {
                    wbuf[4 * q] = wbuf[4 * q + 1] = wbuf[4 * q + 2] = wbuf[4 * q + 3] = 0u;
                }
            }
            const uint32_t d = d0 + threadIdx.x;
            const bool live = d < Dn;
            const uint32_t pd = live ? a.dn_states[d] : 0u;
            T acc[R];
            if (a.add_y) {   // the up part of these elements, loaded with the schedule words
#pragma unroll
                for (int r = 0; r < R; ++r)
                    acc[r] = (live && r < nr) ? __builtin_nontemporal_load(y + g0 + r * pitch + d) : (T)0;
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const T dg = live ? a.U * (T)__builtin_popcount(pu[r] & pd) * get(r, d * 4u) : (T)0;
                acc[r] = a.add_y ? acc[r] + dg : dg;
            }
            // two words (four steps) per chunk, all of one magnitude: the chunk's reads are issued
            // before its multiply-adds; the words sit in registers, indexed statically, and only
            // the chunk tests branch (wave-uniform)
            auto chunk = [&](int cc, uint32_t mp, uint32_t ml) {
                uint32_t ba[4];
                T xv[4][R];
                uint32_t sh[4];   // signed magnitude bits of each step (mp has a clear sign bit,
                                  // so adding 2^31 sets it)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const uint32_t wj = wbuf[2 * cc + j];
                    ba[2 * j] = wj & 0xFFFCu;
                    ba[2 * j + 1] = (wj >> 16) & 0xFFFCu;
                    sh[2 * j] = (wj << 31) + mp;
                    sh[2 * j + 1] = mp ^ ((wj >> 16) << 31);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int r = 0; r < R; ++r) xv[q][r] = get(r, ba[q]);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t h = sh[q];
                    T c;
                    if constexpr (W == 1)
                        c = __uint_as_float(h);
                    else
                        c = __longlong_as_double((long long)(((unsigned long long)h << 32) | ml));
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[r] += c * xv[q][r];
                }
            };
            uint32_t vp = mp0, vl = ml0;   // magnitude of the current chunk
#pragma unroll
            for (int cc = 0; cc < kSchedMaxWords / 2; ++cc) {
                if (2 * cc < n) {
                    if (2 * cc == nb) {
                        vp = mp1;
                        vl = ml1;
                    }
                    chunk(cc, vp, vl);
                }
            }
            if (live) {
#pragma unroll
                for (int r = 0; r < R; ++r)
                    if (r < nr) {
                        __builtin_nontemporal_store(acc[r], y + g0 + r * pitch + d);
                        dsum += (double)get(r, d * 4u) * (double)acc[r];
                    }
            }
        }
    }
    // the planes are free now: the work group's sums go through them
    sched_block_sums(dsum, a.dotp ? a.dotp + blockIdx.x : nullptr, nsum, FUSE ? a.fnorm + blockIdx.x : nullptr,
                     reinterpret_cast<double*>(planes));
}

// Short rows: `rows` consecutive rows staged row-major; threads walk the
// flattened (row, column) index of the group.  STAGE = false gathers from
// global memory instead (rows too long for LDS).
template <typename T, typename E, bool STAGE>
__global__ __launch_bounds__(kNarrowBlock) void k_hv_down_narrow(const DownArgs<T, E> a, const T* __restrict__ x,
                                                                 T* __restrict__ y) {
    if (a.skip && *a.skip) return;
    extern __shared__ __align__(16) unsigned char smem[];
    T* coef = reinterpret_cast<T*>(smem);
    T* rows = coef + kMaxCoef;
    load_coef(coef, a.coef, a.ncoef);
    const uint64_t D_up = a.D_up, D_dn = a.D_dn;
    const int R = a.rows;
    const uint64_t ngroups = (D_up + R - 1) / R;
    double dsum = 0.0;
    for (uint64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const uint64_t u0 = g * (uint64_t)R;
        const int nr = (int)((D_up - u0) < (uint64_t)R ? (D_up - u0) : (uint64_t)R);
        const uint64_t nelem = (uint64_t)nr * D_dn;
        const T* xg = x + u0 * a.pitch;   // row r of the group at xg + r * pitch
        __syncthreads();
        if (STAGE)
            for (uint64_t k = threadIdx.x; k < nelem; k += blockDim.x) {
                const uint64_t r = k / D_dn;
                rows[k] = xg[r * a.pitch + (k - r * D_dn)];
            }
        __syncthreads();
        for (uint64_t k = threadIdx.x; k < nelem; k += blockDim.x) {
            const uint32_t r = (uint32_t)(k / D_dn);
            const uint32_t d = (uint32_t)(k - (uint64_t)r * D_dn);
            const T* xrow = STAGE ? rows + (uint64_t)r * D_dn : xg + (uint64_t)r * a.pitch;
            const uint32_t pu = a.up_states[u0 + r];
            const uint32_t pd = a.dn_states[d];
            T acc = a.U * (T)__builtin_popcount(pu & pd) * xrow[d];
            const int cnt = a.dn_count[d];
            // hops in order, eight table entries loaded before their multiply-adds
            constexpr int NB = 8;
            int h = 0;
            for (; h + NB <= cnt; h += NB) {
                uint32_t e[NB];
#pragma unroll
                for (int j = 0; j < NB; ++j) e[j] = hop_entry(a.dn_ell, (uint32_t)(h + j), d, D_dn);
#pragma unroll
                for (int j = 0; j < NB; ++j) acc += coef[e[j] >> a.cshift] * xrow[e[j] & a.tmask];
            }
            for (; h < cnt; ++h) {
                const uint32_t e = hop_entry(a.dn_ell, (uint32_t)h, d, D_dn);
                acc += coef[e >> a.cshift] * xrow[e & a.tmask];
            }
            y[(u0 + r) * a.pitch + d] = acc;
            dsum += (double)xrow[d] * (double)acc;
        }
    }
    if (a.dotp) block_dot_store<kNarrowBlock>(dsum, a.dotp + blockIdx.x);
}

// ------------------------------------------------------------------ up pass

// Block -> (column chunk, row tile).  map 1: blocks are dealt to the XCDs
// round robin (block b on XCD b % 8), so each XCD walks a pair of
// neighbouring chunks at a time through every row tile and keeps their slab
// in its L2; map 2: chunk-major order over all blocks; map 3: like map 1 with
// one chunk per XCD at a time (half the slab held in L2).
__device__ __forceinline__ void up_tile(uint32_t b, uint32_t rt, int map, uint32_t* chunk, uint32_t* tile) {
    if (map == 2) {
        *chunk = b / rt;
        *tile = b % rt;
        return;
    }
    constexpr int kXcd = 8;
    if (map == 3) {
        const uint32_t j = b / kXcd;
        *tile = j % rt;
        *chunk = (b % kXcd) + kXcd * (j / rt);
        return;
    }
    const uint32_t xcd = b % kXcd;
    const uint32_t j = b / kXcd;
    const uint32_t pair = j / (2 * rt);
    const uint32_t half = (j / rt) & 1u;
    *tile = j % rt;
    *chunk = 2 * (xcd + kXcd * pair) + half;
}

// One decoded up hop: element offset of the source row and its amplitude.
template <typename T>
struct UpHop;
template <>
struct __align__(8) UpHop<float> {
    uint32_t off;
    float c;
};
template <>
struct __align__(16) UpHop<double> {
    uint32_t off;
    uint32_t pad;
    double c;
};

// Tile = ROWS_PER_TILE rows x CW columns; a wave covers 64 / CW rows at once.
// Work groups are dealt to the XCDs round robin (block b runs on XCD b % 8);
// the tile order below gives each XCD a pair of neighbouring column chunks in
// turn, so the slab x[:, chunk] that all up hops of the chunk read stays in
// that XCD's L2, and both halves of every 128-byte line are used there.
// The tile's hop lists are decoded once into LDS.  IDX64 selects 64-bit
// element offsets (D >= 2^32).  BLK threads per work group (FP64 chunks of 128
// columns take 512, so that one pass covers the tile's eight rows).
template <typename T, typename E, int CW, int ROWS_PER_TILE, bool IDX64, int NB, int VECP = 0, int BLK = kUpBlock>
__global__ __launch_bounds__(BLK) void k_hv_up(const UpArgs<T, E> a, const T* __restrict__ x, T* __restrict__ y) {
    if (a.skip && *a.skip) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int maxh = a.max_hops;
    UpHop<T>* s_hop = reinterpret_cast<UpHop<T>*>(smem);                    // ROWS * maxh
    uint64_t* s_off64 = reinterpret_cast<uint64_t*>(s_hop + ROWS_PER_TILE * maxh);  // ROWS * maxh if IDX64
    int* s_cnt = reinterpret_cast<int*>(s_off64 + (IDX64 ? ROWS_PER_TILE * maxh : 0));
    uint32_t chunk, tile;
    up_tile(blockIdx.x, a.row_tiles, a.map, &chunk, &tile);
    if (chunk >= a.n_chunks) {   // padding block of the tile order
        if (a.dotp && threadIdx.x == 0) a.dotp[blockIdx.x] = 0.0;
        return;
    }
    const uint64_t D_up = a.D_up, D_dn = a.D_dn;
    const uint64_t u_begin = (uint64_t)tile * ROWS_PER_TILE;
    const int nrows = (int)((D_up - u_begin) < (uint64_t)ROWS_PER_TILE ? (D_up - u_begin) : (uint64_t)ROWS_PER_TILE);
    for (int r = threadIdx.x; r < nrows; r += BLK) s_cnt[r] = a.up_count[u_begin + r];
    __syncthreads();
    for (int k = threadIdx.x; k < nrows * maxh; k += BLK) {
        const int r = k / maxh, h = k - r * maxh;
        if (h >= s_cnt[r]) continue;   // slots past the count: neither loaded nor read
        const uint32_t e = hop_entry(a.up_ell, h, u_begin + r, D_up);
        const uint32_t ci = e >> a.cshift;
        s_hop[k].c = a.coef[ci < (uint32_t)a.ncoef ? ci : 0];
        if (IDX64)
            s_off64[k] = (uint64_t)(e & a.tmask) * a.pitch;
        else
            s_hop[k].off = (e & a.tmask) * (uint32_t)a.pitch;
    }
    __syncthreads();
    // each lane owns VEC consecutive columns: CW / VEC lanes per row segment
    // (VECP > 0: 16-byte lanes at any chunk width, several rows per wave)
    constexpr int VEC = VECP > 0 ? VECP : ((CW >= 256 && sizeof(T) == 4) ? 4 : (CW >= 128 ? 2 : 1));
    static_assert(CW % VEC == 0 && BLK % (CW / VEC) == 0, "lanes per row segment");
    constexpr int LANES = CW / VEC;
    const uint32_t lane = threadIdx.x % LANES;
    const uint64_t d = (uint64_t)chunk * CW + (uint64_t)lane * VEC;
    const bool active = d < D_dn;   // lanes past the last column idle (no early exit: a barrier follows)
    const int nv = !active ? 0 : ((d + VEC <= D_dn) ? VEC : (int)(D_dn - d));   // valid columns of this lane
    constexpr int kSlots = BLK / LANES;
    double dsum = 0.0;
    for (int r = threadIdx.x / LANES; active && r < nrows; r += kSlots) {
        const uint64_t u = u_begin + r;
        const int cnt = s_cnt[r];
        const UpHop<T>* hp = s_hop + r * maxh;
        const uint64_t* o64 = s_off64 + r * maxh;
        T* yr = y + u * a.pitch + d;
        // x at this row's own elements, for the x . out partial: loaded now, used after the hops
        T xo[VEC];
        if (a.dotp) {
            const T* xr = x + u * a.pitch + d;
            if (nv == VEC) {
                vec_load<T, VEC>(xr, xo);
            } else {
#pragma unroll
                for (int i = 0; i < VEC; ++i) xo[i] = (i < nv) ? xr[i] : (T)0;
            }
        }
        T acc[VEC];
        if (!a.add_y) {
#pragma unroll
            for (int i = 0; i < VEC; ++i) acc[i] = (T)0;
        } else if (VEC == 1) {
            acc[0] = __builtin_nontemporal_load(yr);   // streamed: keep the x slab in L2
        } else if (nv == VEC) {
            vec_load<T, VEC>(yr, acc);
        } else {
#pragma unroll
            for (int i = 0; i < VEC; ++i) acc[i] = (i < nv) ? yr[i] : (T)0;
        }
        int h = 0;
        if (nv == VEC) {
            for (; h + NB <= cnt; h += NB) {
                T v[NB][VEC];
                T c[NB];
#pragma unroll
                for (int q = 0; q < NB; ++q) {
                    const UpHop<T> hq = hp[h + q];
                    c[q] = hq.c;
                    const T* src = IDX64 ? x + o64[h + q] + d : x + (uint32_t)(hq.off + (uint32_t)d);
                    vec_load<T, VEC>(src, v[q]);
                }
#pragma unroll
                for (int q = 0; q < NB; ++q)
#pragma unroll
                    for (int i = 0; i < VEC; ++i) acc[i] += c[q] * v[q][i];
            }
            // the last cnt - h (< NB) hops in batches of NB/2, NB/4, ..., 1 taken
            // while they fit: exactly one load per hop, every load of a batch
            // issued before its first multiply-add, the hops in order
            auto tail = [&](auto bc) {
                constexpr int B = decltype(bc)::value;
                if constexpr (B >= 1 && B < NB) {
                    if (h + B <= cnt) {
                        T v[B][VEC];
                        T c[B];
#pragma unroll
                        for (int q = 0; q < B; ++q) {
                            const UpHop<T> hq = hp[h + q];
                            c[q] = hq.c;
                            const T* src = IDX64 ? x + o64[h + q] + d : x + (uint32_t)(hq.off + (uint32_t)d);
                            vec_load<T, VEC>(src, v[q]);
                        }
#pragma unroll
                        for (int q = 0; q < B; ++q)
#pragma unroll
                            for (int i = 0; i < VEC; ++i) acc[i] += c[q] * v[q][i];
                        h += B;
                    }
                }
            };
            tail(std::integral_constant<int, 8>{});
            tail(std::integral_constant<int, 4>{});
            tail(std::integral_constant<int, 2>{});
            tail(std::integral_constant<int, 1>{});
        }
        for (; h < cnt; ++h) {
            const UpHop<T> hq = hp[h];
            const T* src = IDX64 ? x + o64[h] + d : x + (uint32_t)(hq.off + (uint32_t)d);
#pragma unroll
            for (int i = 0; i < VEC; ++i)
                if (i < nv) acc[i] += hq.c * src[i];
        }
        if (VEC == 1) {
            __builtin_nontemporal_store(acc[0], yr);
        } else if (nv == VEC) {
            vec_store<T, VEC>(yr, acc);
        } else {
#pragma unroll
            for (int i = 0; i < VEC; ++i)
                if (i < nv) yr[i] = acc[i];
        }
        if (a.dotp) {
#pragma unroll
            for (int i = 0; i < VEC; ++i)
                if (i < nv) dsum += (double)xo[i] * (double)acc[i];
        }
    }
    if (a.dotp) block_dot_store<BLK>(dsum, a.dotp + blockIdx.x);
}

// Same tile order and decoded hop lists as k_hv_up, but every hop load of a
// row is issued before the first multiply-add (MAXH bounds the row's hop
// count): one memory round trip per row.  One column per lane, 32-bit offsets.
template <typename T, typename E, int CW, int ROWS_PER_TILE, int MAXH>
__global__ __launch_bounds__(kUpBlock) void k_hv_up_pre(const UpArgs<T, E> a, const T* __restrict__ x,
                                                        T* __restrict__ y) {
    if (a.skip && *a.skip) return;
    extern __shared__ __align__(16) unsigned char smem[];
    const int maxh = a.max_hops;
    UpHop<T>* s_hop = reinterpret_cast<UpHop<T>*>(smem);
    int* s_cnt = reinterpret_cast<int*>(s_hop + ROWS_PER_TILE * maxh);
    uint32_t chunk, tile;
    up_tile(blockIdx.x, a.row_tiles, a.map, &chunk, &tile);
    if (chunk >= a.n_chunks) {   // padding block of the tile order
        if (a.dotp && threadIdx.x == 0) a.dotp[blockIdx.x] = 0.0;
        return;
    }
    const uint64_t D_up = a.D_up, D_dn = a.D_dn;
    const uint64_t u_begin = (uint64_t)tile * ROWS_PER_TILE;
    const int nrows = (int)((D_up - u_begin) < (uint64_t)ROWS_PER_TILE ? (D_up - u_begin) : (uint64_t)ROWS_PER_TILE);
    for (int r = threadIdx.x; r < nrows; r += kUpBlock) s_cnt[r] = a.up_count[u_begin + r];
    for (int k = threadIdx.x; k < nrows * maxh; k += kUpBlock) {
        const int r = k / maxh, h = k - r * maxh;
        const uint32_t e = hop_entry(a.up_ell, h, u_begin + r, D_up);
        const uint32_t ci = e >> a.cshift;
        s_hop[k].c = a.coef[ci < (uint32_t)a.ncoef ? ci : 0];
        s_hop[k].off = (e & a.tmask) * (uint32_t)a.pitch;
    }
    __syncthreads();
    const uint32_t col = threadIdx.x % CW;
    const uint64_t d = (uint64_t)chunk * CW + col;
    const bool active = d < D_dn;   // no early exit: a barrier follows
    constexpr int kSlots = kUpBlock / CW;
    double dsum = 0.0;
    for (int r = threadIdx.x / CW; active && r < nrows; r += kSlots) {
        const uint64_t u = u_begin + r;
        const int cnt = s_cnt[r];
        const UpHop<T>* hp = s_hop + r * maxh;
        T v[MAXH];
#pragma unroll
        for (int h = 0; h < MAXH; ++h) v[h] = (h < cnt) ? x[(uint32_t)(hp[h].off + (uint32_t)d)] : (T)0;
        T acc = a.add_y ? __builtin_nontemporal_load(y + u * a.pitch + d) : (T)0;
#pragma unroll
        for (int h = 0; h < MAXH; ++h)
            if (h < cnt) acc += hp[h].c * v[h];
        __builtin_nontemporal_store(acc, y + u * a.pitch + d);
        if (a.dotp) dsum += (double)x[u * a.pitch + d] * (double)acc;
    }
    if (a.dotp) block_dot_store<kUpBlock>(dsum, a.dotp + blockIdx.x);
}

// ------------------------------------------------------------ fallback path

// Every sector rank and every hop target computed per element with the
// forward and backward maps (binomial table in LDS).
constexpr int kFlyNB = 8;   // bonds of an element whose targets are ranked and loaded together

struct FlyArgs {
    int N, n_up, n_dn, nb;
    uint64_t D_up, D_dn;
    const uint32_t* binom;
    const BondDev* bonds;
    const int* skip;
};

__device__ __forceinline__ uint32_t fly_rank(uint32_t phi, const uint32_t* sC) {
    uint32_t idx = 0;
    int m = 0;
    while (phi) {
        const int i = __builtin_ctz(phi);
        phi &= phi - 1u;
        ++m;
        idx += sC[i * kBinomStride + m];
    }
    return idx;
}

__device__ __forceinline__ uint32_t fly_unrank(uint32_t p, int n, int N, const uint32_t* sC) {
    uint32_t phi = 0;
    int m = n;
    for (int i = N - 1; i >= 0 && m > 0; --i) {
        const uint32_t c = sC[i * kBinomStride + m];
        if (p >= c) {
            phi |= 1u << i;
            p -= c;
            --m;
        }
    }
    return phi;
}

template <typename T>
__global__ __launch_bounds__(kFlyBlock) void k_hv_fly(const FlyArgs f, T U, const T* __restrict__ coef_g,
                                                     const T* __restrict__ x, T* __restrict__ y) {
    if (f.skip && *f.skip) return;
    __shared__ uint32_t sC[kBinomStride * kBinomStride];
    for (int k = threadIdx.x; k < kBinomStride * kBinomStride; k += blockDim.x) sC[k] = f.binom[k];
    __syncthreads();
    const uint64_t D = f.D_up * f.D_dn;
    for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < D;
         r += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t u = r / f.D_dn, d = r - u * f.D_dn;
        const uint32_t pu = fly_unrank((uint32_t)u, f.n_up, f.N, sC);
        const uint32_t pd = fly_unrank((uint32_t)d, f.n_dn, f.N, sC);
        T acc = U * (T)__builtin_popcount(pu & pd) * x[r];
        // bonds in order, kFlyNB at a time: the batch's targets are ranked and
        // their operands loaded before its first multiply-add (a bond that
        // moves no electron adds nothing)
        auto bonds = [&](uint32_t phi, bool down) {
            int b = 0;
            for (; b < f.nb; b += kFlyNB) {
                T cf[kFlyNB], xv[kFlyNB];
                bool hop[kFlyNB];
#pragma unroll
                for (int j = 0; j < kFlyNB; ++j) {
                    hop[j] = false;
                    cf[j] = (T)0;
                    xv[j] = (T)0;
                    if (b + j < f.nb) {
                        const BondDev bd = f.bonds[b + j];
                        const uint32_t o = phi & bd.mask;
                        hop[j] = o != 0u && o != bd.mask;
                        if (hop[j]) {
                            cf[j] = coef_g[(__builtin_popcount(phi & bd.between) & 1) ? bd.coef_neg : bd.coef_pos];
                            const uint64_t t = fly_rank(phi ^ bd.mask, sC);
                            xv[j] = down ? x[u * f.D_dn + t] : x[t * f.D_dn + d];
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < kFlyNB; ++j)
                    if (hop[j]) acc += cf[j] * xv[j];
            }
        };
        bonds(pd, true);
        bonds(pu, false);
        y[r] = acc;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_zero_fill(T* v, uint64_t n) {
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) v[i] = (T)0;
}

// ---------------------------------------------------------------- launches

template <typename T, typename E>
void fill_table_view(const SectorTables& t, bool compact, const E** ell, uint32_t* tmask, int* cshift) {
    if (compact) {
        *ell = reinterpret_cast<const E*>(t.ell16);
        *tmask = (1u << t.tbits16) - 1u;
        *cshift = t.tbits16;
    } else {
        *ell = reinterpret_cast<const E*>(t.ell);
        *tmask = kTargetMask;
        *cshift = (int)kTargetBits;
    }
}

// Down-pass variant: 1 = one row, table loaded up front (compile-time bound
// on the hop slots); 2 = one row, table in a loop; 3 = two rows, loop;
// 4 = three rows, loop.
template <typename T, typename E>
void launch_wide(int variant, int max_hops, uint64_t grid, size_t lds, hipStream_t s, const DownArgs<T, E>& da,
                 const T* x, T* y) {
    const dim3 g((unsigned)grid), b(kWideBlock);
    if (variant == 1 && sizeof(E) == 2 && max_hops <= 16)
        hipLaunchKernelGGL((k_hv_down_wide<T, E, 1, 16>), g, b, lds, s, da, x, y);
    else if (variant == 1 && sizeof(E) == 2 && max_hops <= 32)
        hipLaunchKernelGGL((k_hv_down_wide<T, E, 1, 32>), g, b, lds, s, da, x, y);
    else if (variant == 1 && sizeof(E) == 2 && max_hops <= 48)
        hipLaunchKernelGGL((k_hv_down_wide<T, E, 1, 48>), g, b, lds, s, da, x, y);
    else if (variant == 3)
        hipLaunchKernelGGL((k_hv_down_wide<T, E, 2, 0>), g, b, lds, s, da, x, y);
    else if (variant == 4)
        hipLaunchKernelGGL((k_hv_down_wide<T, E, 3, 0>), g, b, lds, s, da, x, y);
    else
        hipLaunchKernelGGL((k_hv_down_wide<T, E, 1, 0>), g, b, lds, s, da, x, y);
}

template <typename T, typename E, int R, int MAXH, bool FUSE = false>
pdz_status set_wide_lds() {
    PDZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hv_down_wide<T, E, R, MAXH, FUSE>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kDynLds));
    return ok();
}

// The looped down-pass variants (2, 3, 4) with the fused recurrence.
template <typename T, typename E>
void launch_wide_fused(int variant, uint64_t grid, size_t lds, hipStream_t s, const DownArgs<T, E>& da, T* y) {
    const dim3 g((unsigned)grid), b(kWideBlock);
    const T* x = da.fq2;
    if (variant == 3)
        hipLaunchKernelGGL((k_hv_down_wide<T, E, 2, 0, true>), g, b, lds, s, da, x, y);
    else if (variant == 4)
        hipLaunchKernelGGL((k_hv_down_wide<T, E, 3, 0, true>), g, b, lds, s, da, x, y);
    else
        hipLaunchKernelGGL((k_hv_down_wide<T, E, 1, 0, true>), g, b, lds, s, da, x, y);
}

// Scheduled down pass (plans down 5, 6, 7: 1, 2, 3 rows per group).
bool sched_plan(int variant) { return variant >= 5 && variant <= 7; }
int sched_rows(int variant) { return variant - 4; }
// LDS bytes of the row planes (a static array of the kernel)
size_t sched_lds(const pdz_problem_s* p, size_t es, int rows) {
    (void)p;
    return (size_t)rows * (es / 4) * kSchedPlane * 4;
}
bool sched_fits(const pdz_problem_s* p, size_t es, int rows) {
    return sched_lds(p, es, rows) <= kDynLds && p->up.D >= (uint64_t)rows;
}

template <typename T>
SchedArgs<T> sched_args(const pdz_problem_s* p) {
    SchedArgs<T> sa;
    sa.words = p->dn.sched.words;
    sa.meta = p->dn.sched.meta;
    sa.mag0 = (T)p->dn.sched.mag0;
    sa.mag1 = (T)p->dn.sched.mag1;
    return sa;
}

template <typename T, typename E, bool FUSE>
void launch_sched(const pdz_problem_s* p, int variant, uint64_t grid, size_t lds, hipStream_t s,
                  const DownArgs<T, E>& da, const T* x, T* y) {
    const dim3 g((unsigned)grid), b(kWideBlock);
    const SchedArgs<T> sa = sched_args<T>(p);
    (void)lds;   // the planes are a static LDS array
    lds = 0;
    if (variant == 7 && sizeof(T) == 4)
        hipLaunchKernelGGL((k_hv_down_sched<T, E, sizeof(T) == 4 ? 3 : 1, FUSE>), g, b, lds, s, da, sa, x, y);
    else if (variant == 6 && sizeof(T) == 4)
        hipLaunchKernelGGL((k_hv_down_sched<T, E, sizeof(T) == 4 ? 2 : 1, FUSE>), g, b, lds, s, da, sa, x, y);
    else
        hipLaunchKernelGGL((k_hv_down_sched<T, E, 1, FUSE>), g, b, lds, s, da, sa, x, y);
}

// Up-pass geometry: the x[:, chunk] slab one XCD streams over is
// D_up * CW * sizeof(T) bytes; narrower chunks stay in L2, wider ones issue
// fewer, longer requests.  The plan (autotuned or default) picks CW.
// Rows per tile: small tiles keep the rows in flight on one XCD to a small
// part of the chunk, so that the XCD's work groups stay on one column chunk
// at a time and its slab stays in that XCD's L2.
template <typename T>
constexpr int up_rows() { return 8; }

// Work-group size of the up pass with one column (two in FP64 at 128) per
// lane: 512 threads for FP64 chunks of 128 columns (measured faster there;
// FP32, and FP64 at narrower chunks, are faster at 256).
template <typename T, int CW>
constexpr int up_block() { return (sizeof(T) == 8 && CW >= 128) ? 512 : kUpBlock; }

// Wide lanes (plan up 4): 16 bytes per lane, so a wave covers 64 * 16 / (CW * sizeof(T)) rows of
// the chunk at once and a tile holds one row per lane group of the work group.
template <typename T, int CW>
constexpr int wide_rows() { return kUpBlock / (CW * (int)sizeof(T) / 16); }

template <typename T, typename E, int CW>
void launch_up_wide(uint64_t blocks, size_t lds, hipStream_t s, const UpArgs<T, E>& ua, const T* x, T* y) {
    hipLaunchKernelGGL((k_hv_up<T, E, CW, wide_rows<T, CW>(), false, 8, 16 / (int)sizeof(T)>), dim3((unsigned)blocks),
                       dim3(kUpBlock), lds, s, ua, x, y);
}

// nb: hop loads in flight per batch (8, or 16 with 32-bit offsets)
template <typename T, typename E, int CW>
void launch_up(bool idx64, int nb, uint64_t blocks, size_t lds, hipStream_t s, const UpArgs<T, E>& ua, const T* x,
               T* y) {
    const dim3 g((unsigned)blocks), b(kUpBlock), bb(up_block<T, CW>());
    if (idx64)
        hipLaunchKernelGGL((k_hv_up<T, E, CW, up_rows<T>(), true, 8>), g, b, lds, s, ua, x, y);
    else if (nb == 16)
        hipLaunchKernelGGL((k_hv_up<T, E, CW, up_rows<T>(), false, 16, 0, up_block<T, CW>()>), g, bb, lds, s, ua, x,
                           y);
    else
        hipLaunchKernelGGL((k_hv_up<T, E, CW, up_rows<T>(), false, 8, 0, up_block<T, CW>()>), g, bb, lds, s, ua, x,
                           y);
}

template <typename T, typename E, int CW>
void launch_up_pre(int max_hops, uint64_t blocks, size_t lds, hipStream_t s, const UpArgs<T, E>& ua, const T* x,
                   T* y) {
    const dim3 g((unsigned)blocks), b(kUpBlock);
    if (max_hops <= 16)
        hipLaunchKernelGGL((k_hv_up_pre<T, E, CW, up_rows<T>(), 16>), g, b, lds, s, ua, x, y);
    else if (max_hops <= 32)
        hipLaunchKernelGGL((k_hv_up_pre<T, E, CW, up_rows<T>(), 32>), g, b, lds, s, ua, x, y);
    else
        hipLaunchKernelGGL((k_hv_up_pre<T, E, CW, up_rows<T>(), 48>), g, b, lds, s, ua, x, y);
}

// Chunk widths offered per precision (columns).
constexpr int kUpCw32[] = {32, 64, 128, 256};
constexpr int kUpCw64[] = {16, 32, 64, 128};
constexpr int kNumCw = 4;

bool row_fits(const pdz_problem_s* p, size_t es, int rows) {
    const size_t lds_cap = kLdsBytes - kMaxCoef * es - 1024;
    return (size_t)rows * p->dn.D * es <= lds_cap;
}

bool wide_down(const pdz_problem_s* p, size_t es) { return p->dn.D >= (uint64_t)kWideBlock && row_fits(p, es, 1); }

HvPlan default_plan(const pdz_problem_s* p, pdz_dtype dt) {
    const size_t es = dt == PDZ_F64 ? 8 : 4;
    HvPlan d;
    const bool compact = p->up.tbits16 > 0 && p->dn.tbits16 > 0;
    if (wide_down(p, es) && p->dn.sched.words) {
        int r = es == 4 ? 3 : 1;
        while (r > 1 && !sched_fits(p, es, r)) --r;
        d.down = 4 + r;
    } else if (dt == PDZ_F32 && row_fits(p, es, 2) && p->up.D >= 2)
        d.down = 3;
    else if (compact && p->dn.max_hops <= 48)
        d.down = 1;
    else
        d.down = 2;
    d.up_cw = 128;
    d.up = 1;
    d.map = 3;
    return d;
}

HvPlan hv_resolve(const pdz_problem_s* p, pdz_dtype dt) {
    HvPlan pl = p->plan[dt == PDZ_F64 ? 0 : 1];
    const HvPlan d = default_plan(p, dt);
    if (pl.down == 0) pl.down = d.down;
    if (pl.up_cw == 0) pl.up_cw = d.up_cw;
    if (pl.up == 0) pl.up = d.up;
    if (pl.map == 0) pl.map = d.map;
    return pl;
}

int down_rows(int variant) { return sched_plan(variant) ? sched_rows(variant) : variant == 4 ? 3 : variant == 3 ? 2 : 1; }

// Down-pass launch geometry (also the number of x . y partial sums it writes).
struct DownGeom {
    bool wide = false;    // k_hv_down_wide (rows at least one work group wide, staged in LDS)
    bool stage = false;   // narrow kernel with rows staged in LDS
    int rows = 1;         // rows per group
    size_t lds = 0;       // dynamic LDS bytes
    uint64_t grid = 0;    // work groups
};

DownGeom down_geom(const pdz_problem_s* p, size_t es, const HvPlan& plan, unsigned cu) {
    DownGeom g;
    const uint64_t D_up = p->up.D, D_dn = p->dn.D;
    const size_t lds_cap = kLdsBytes - kMaxCoef * es - 1024;
    const size_t row_bytes = (size_t)D_dn * es;
    if (D_dn >= (uint64_t)kWideBlock && row_bytes <= lds_cap) {
        g.wide = g.stage = true;
        g.rows = down_rows(plan.down);
        g.lds = sched_plan(plan.down) ? sched_lds(p, es, g.rows) : kMaxCoef * es + (size_t)g.rows * row_bytes;
        const uint64_t ngroups = (D_up + g.rows - 1) / g.rows;
        const unsigned per_cu = (unsigned)(kLdsBytes / (g.lds + 256));
        g.grid = (uint64_t)cu * (per_cu < 1 ? 1 : per_cu);
        if (g.grid > ngroups) g.grid = ngroups;
        return g;
    }
    g.stage = row_bytes <= lds_cap;
    int R = 1;
    if (D_dn < 2 * (uint64_t)kNarrowBlock) R = (int)((2 * kNarrowBlock + D_dn - 1) / D_dn);
    if (g.stage) {
        const int rmax = (int)(lds_cap / row_bytes);
        if (R > rmax) R = rmax;
    }
    if ((uint64_t)R > D_up) R = (int)D_up;
    if (R < 1) R = 1;
    g.rows = R;
    g.lds = kMaxCoef * es + (g.stage ? (size_t)R * row_bytes : 0);
    const uint64_t ngroups = (D_up + R - 1) / R;
    const unsigned per_cu = g.stage ? (unsigned)(kLdsBytes / (g.lds + 256)) : 8u;
    g.grid = (uint64_t)cu * (per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu));
    if (g.grid > ngroups) g.grid = ngroups;
    return g;
}

uint64_t down_grid(const pdz_problem_s* p, size_t es, const HvPlan& plan, unsigned cu) {
    return down_geom(p, es, plan, cu).grid;
}

// Rows per up-pass tile: 8, or one per lane group with wide lanes (plan up 4).
int up_tile_rows(size_t es, const HvPlan& plan) {
    if (plan.up == 4) return kUpBlock / (int)((size_t)plan.up_cw * es / 16);
    return 8;
}

// Up-pass work groups (tile order padded to whole XCD rounds).
uint64_t up_blocks(const pdz_problem_s* p, size_t es, const HvPlan& plan) {
    constexpr uint64_t kXcd = 8;
    const uint64_t rows = (uint64_t)up_tile_rows(es, plan);
    const uint64_t rt = (p->up.D + rows - 1) / rows;
    const uint64_t nch = (p->dn.D + plan.up_cw - 1) / plan.up_cw;
    if (plan.map == 1) return kXcd * (((nch + 1) / 2 + kXcd - 1) / kXcd) * 2 * rt;
    if (plan.map == 3) return kXcd * ((nch + kXcd - 1) / kXcd) * rt;
    return nch * rt;
}

// Up pass of the table path: yout = (add_y ? yout : 0) + the up hops of x.
template <typename T, typename E>
pdz_status up_pass(const pdz_problem_s* p, const T* coef, const T* x, T* yout, hipStream_t s, const int* skip,
                   bool compact, const HvPlan& plan, int add_y, double* dotp, uint64_t pitch) {
    const uint64_t D_up = p->up.D, D_dn = p->dn.D;
    const int ncoef = (int)p->coef_host.size();
    UpArgs<T, E> ua;
    ua.D_up = D_up;
    ua.D_dn = D_dn;
    ua.pitch = pitch;
    ua.up_count = p->up.count;
    fill_table_view<T, E>(p->up, compact, &ua.up_ell, &ua.tmask, &ua.cshift);
    ua.coef = coef;
    ua.ncoef = ncoef;
    ua.skip = skip;
    ua.add_y = add_y;
    ua.dotp = dotp;
    const int CW = plan.up_cw;
    const int ROWS = up_tile_rows(sizeof(T), plan);
    const bool idx64 = D_up * pitch > 0xFFFFFFFFull;
    ua.row_tiles = (uint32_t)((D_up + ROWS - 1) / ROWS);
    ua.max_hops = p->up.max_hops;
    ua.n_chunks = (uint32_t)((D_dn + CW - 1) / CW);
    const size_t lds = (size_t)ROWS * ua.max_hops * (sizeof(UpHop<T>) + (idx64 ? 8 : 0)) + ROWS * sizeof(int);
    ua.map = plan.map;
    const uint64_t blocks = up_blocks(p, sizeof(T), plan);
    const int nb = plan.up == 3 ? 16 : 8;
    if (plan.up == 4 && !idx64) {
        if (sizeof(T) == 8) {
            if (CW == 16)
                launch_up_wide<T, E, 16>(blocks, lds, s, ua, x, yout);
            else if (CW == 32)
                launch_up_wide<T, E, 32>(blocks, lds, s, ua, x, yout);
            else
                launch_up_wide<T, E, 64>(blocks, lds, s, ua, x, yout);
        } else {
            if (CW == 32)
                launch_up_wide<T, E, 32>(blocks, lds, s, ua, x, yout);
            else if (CW == 64)
                launch_up_wide<T, E, 64>(blocks, lds, s, ua, x, yout);
            else
                launch_up_wide<T, E, 128>(blocks, lds, s, ua, x, yout);
        }
    } else if (plan.up == 2 && !idx64) {
        // preloaded rows: one column per lane (CW <= 64)
        if (sizeof(T) == 8 && CW == 16)
            launch_up_pre<T, E, 16>(ua.max_hops, blocks, lds, s, ua, x, yout);
        else if (CW == 32)
            launch_up_pre<T, E, 32>(ua.max_hops, blocks, lds, s, ua, x, yout);
        else
            launch_up_pre<T, E, 64>(ua.max_hops, blocks, lds, s, ua, x, yout);
    } else if (sizeof(T) == 8) {
        if (CW == 16)
            launch_up<T, E, 16>(idx64, nb, blocks, lds, s, ua, x, yout);
        else if (CW == 32)
            launch_up<T, E, 32>(idx64, nb, blocks, lds, s, ua, x, yout);
        else if (CW == 64)
            launch_up<T, E, 64>(idx64, nb, blocks, lds, s, ua, x, yout);
        else
            launch_up<T, E, 128>(idx64, nb, blocks, lds, s, ua, x, yout);
    } else {
        if (CW == 32)
            launch_up<T, E, 32>(idx64, nb, blocks, lds, s, ua, x, yout);
        else if (CW == 64)
            launch_up<T, E, 64>(idx64, nb, blocks, lds, s, ua, x, yout);
        else if (CW == 128)
            launch_up<T, E, 128>(idx64, nb, blocks, lds, s, ua, x, yout);
        else
            launch_up<T, E, 256>(idx64, nb, blocks, lds, s, ua, x, yout);
    }
    PDZ_HIP(hipGetLastError());
    return ok();
}


template <typename T, typename E>
pdz_status run_tables(const pdz_problem_s* p, const DeviceCtx* ctx, const T* coef, const T* x, T* y, hipStream_t s,
                      const int* skip, bool compact, unsigned passes, const HvSplit* split, uint64_t pitch) {
    const uint64_t D_up = p->up.D, D_dn = p->dn.D;
    const int ncoef = (int)p->coef_host.size();
    // ---- down pass
    DownArgs<T, E> da{};
    da.D_up = D_up;
    da.D_dn = D_dn;
    da.pitch = pitch;
    da.U = (T)p->U;
    da.up_states = p->up.states;
    da.dn_states = p->dn.states;
    da.dn_count = p->dn.count;
    fill_table_view<T, E>(p->dn, compact, &da.dn_ell, &da.tmask, &da.cshift);
    da.ell_bytes = compact ? (uint32_t)(((uint64_t)(p->dn.max_hops + 1) & ~1ull) * D_dn * sizeof(uint16_t)) : 0u;
    da.coef = coef;
    da.ncoef = ncoef;
    da.skip = skip;
    da.add_y = 0;
    da.dotp = split ? split->dotp_dn : nullptr;
    const bool fused = split && split->fq2;
    da.fz = fused ? static_cast<const T*>(split->fz) : nullptr;
    da.fq1 = fused ? static_cast<const T*>(split->fq1) : nullptr;
    da.fq2 = fused ? static_cast<T*>(split->fq2) : nullptr;
    da.fkeep = fused ? static_cast<T*>(split->fkeep) : nullptr;
    da.fkeep_ld = fused ? split->fkeep_ld : 0;
    da.fkeep_cap = fused ? split->fkeep_cap : 0;
    da.falpha = fused ? split->falpha : nullptr;
    da.fbeta = fused ? split->fbeta : nullptr;
    da.fsc = fused ? split->fsc : nullptr;
    da.fkidx = fused ? split->fkidx : nullptr;
    da.fnorm = fused ? split->fnorm : nullptr;
    const HvPlan plan = hv_resolve(p, sizeof(T) == 8 ? PDZ_F64 : PDZ_F32);
    const DownGeom gm = down_geom(p, sizeof(T), plan, (unsigned)ctx->cu_count);
    da.rows = gm.rows;
    if (gm.wide && sched_plan(plan.down) && pitch + 32 > (uint64_t)kSchedPlane)
        return fail(PDZ_EINVAL, "row pitch longer than the scheduled down pass's plane");
    if (fused) {
        if (!(passes & kPassDown) || (passes & kPassUp) || !gm.wide ||
            !(plan.down == 2 || plan.down == 3 || plan.down == 4 || sched_plan(plan.down)) || !split->dotp_dn ||
            !split->fnorm)
            return fail(PDZ_EINVAL, "fused recurrence needs the looped wide down pass, alone");
        if (sched_plan(plan.down))
            launch_sched<T, E, true>(p, plan.down, gm.grid, gm.lds, s, da, static_cast<const T*>(split->fq2), y);
        else
            launch_wide_fused<T, E>(plan.down, gm.grid, gm.lds, s, da, y);
        PDZ_HIP(hipGetLastError());
        return ok();
    }
    if (!split && gm.wide && sched_plan(plan.down) && p->up.max_hops > 0) {
        // the up pass writes y and the down pass adds its part as it stores
        // (so no pass re-reads y in its gathers); element sum: up hops, then
        // the diagonal, then the down hops
        if (passes & kPassUp) {
            const pdz_status st = up_pass<T, E>(p, coef, x, y, s, skip, compact, plan, 0, nullptr, pitch);
            if (st != PDZ_OK) return st;
        }
        if (passes & kPassDown) {
            da.add_y = 1;
            launch_sched<T, E, false>(p, plan.down, gm.grid, gm.lds, s, da, x, y);
            PDZ_HIP(hipGetLastError());
        }
        return ok();
    }
    if (!(passes & kPassDown)) {
        // up pass only
    } else if (gm.wide && sched_plan(plan.down)) {
        launch_sched<T, E, false>(p, plan.down, gm.grid, gm.lds, s, da, x, y);
    } else if (gm.wide) {
        launch_wide<T, E>(plan.down, p->dn.max_hops, gm.grid, gm.lds, s, da, x, y);
    } else if (gm.stage) {
        hipLaunchKernelGGL((k_hv_down_narrow<T, E, true>), dim3((unsigned)gm.grid), dim3(kNarrowBlock), gm.lds, s, da,
                           x, y);
    } else {
        hipLaunchKernelGGL((k_hv_down_narrow<T, E, false>), dim3((unsigned)gm.grid), dim3(kNarrowBlock), gm.lds, s,
                           da, x, y);
    }
    PDZ_HIP(hipGetLastError());
    if (p->up.max_hops == 0 || !(passes & kPassUp)) {
        if (split && split->z) {   // no up hops: the up term is zero
            hipLaunchKernelGGL(k_zero_fill<T>, dim3(1024), dim3(256), 0, s, static_cast<T*>(split->z), D_up * pitch);
            if (split->dotp_up) hipLaunchKernelGGL(k_zero_fill<double>, dim3(1), dim3(64), 0, s, split->dotp_up,
                                                   (uint64_t)1);
            PDZ_HIP(hipGetLastError());
        }
        return ok();
    }
    // split: the up term goes to its own buffer (no re-read of y); else it is added into y
    if (split && split->z)
        return up_pass<T, E>(p, coef, x, static_cast<T*>(split->z), s, skip, compact, plan, 0, split->dotp_up,
                             pitch);
    return up_pass<T, E>(p, coef, x, y, s, skip, compact, plan, 1, split ? split->dotp_up : nullptr, pitch);
}

template <typename T>
pdz_status run_hv(const pdz_problem_s* p, const T* coef, const T* x, T* y, hipStream_t s, const int* skip,
                  unsigned passes, const HvSplit* split, uint64_t pitch) {
    DeviceCtx* ctx = nullptr;
    pdz_status st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    if (pitch == 0) pitch = p->dn.D;
    if (pitch < p->dn.D) return fail(PDZ_EINVAL, "row pitch shorter than a row");
    if (p->hv_path == 0) {
        const bool compact = p->up.tbits16 > 0 && p->dn.tbits16 > 0;
        if (compact) return run_tables<T, uint16_t>(p, ctx, coef, x, y, s, skip, true, passes, split, pitch);
        return run_tables<T, uint32_t>(p, ctx, coef, x, y, s, skip, false, passes, split, pitch);
    }
    if (pitch != p->dn.D) return fail(PDZ_EINVAL, "the on-the-fly H.v takes unpadded rows");
    FlyArgs f;
    f.N = p->N;
    f.n_up = p->n_up;
    f.n_dn = p->n_dn;
    f.nb = p->n_bonds;
    f.D_up = p->up.D;
    f.D_dn = p->dn.D;
    f.binom = p->d_binom;
    f.bonds = p->d_bonds;
    f.skip = skip;
    uint64_t grid = (p->D + kFlyBlock - 1) / kFlyBlock;
    const uint64_t gmax = (uint64_t)ctx->cu_count * 16;
    if (grid > gmax) grid = gmax;
    hipLaunchKernelGGL(k_hv_fly<T>, dim3((unsigned)grid), dim3(kFlyBlock), 0, s, f, (T)p->U, coef, x, y);
    PDZ_HIP(hipGetLastError());
    return ok();
}

template <typename T, typename E, int CW>
pdz_status set_up_lds() {
    PDZ_HIP(hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k_hv_up<T, E, CW, up_rows<T>(), false, 8, 0, up_block<T, CW>()>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kDynLds));
    PDZ_HIP(hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k_hv_up<T, E, CW, up_rows<T>(), false, 16, 0, up_block<T, CW>()>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kDynLds));
    PDZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hv_up<T, E, CW, up_rows<T>(), true, 8>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kDynLds));
    return ok();
}

template <typename T, typename E, int CW>
pdz_status set_up_wide_lds() {
    PDZ_HIP(hipFuncSetAttribute(
        reinterpret_cast<const void*>(&k_hv_up<T, E, CW, wide_rows<T, CW>(), false, 8, 16 / (int)sizeof(T)>),
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)kDynLds));
    return ok();
}

template <typename T, typename E, int CW>
pdz_status set_up_pre_lds() {
    PDZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hv_up_pre<T, E, CW, up_rows<T>(), 16>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kDynLds));
    PDZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hv_up_pre<T, E, CW, up_rows<T>(), 32>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kDynLds));
    PDZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hv_up_pre<T, E, CW, up_rows<T>(), 48>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kDynLds));
    return ok();
}

template <typename T, typename E>
pdz_status prepare_one() {
    const int lds = (int)kDynLds;
    pdz_status st = set_wide_lds<T, E, 1, 0>();
    if (st == PDZ_OK) st = set_wide_lds<T, E, 2, 0>();
    if (sizeof(E) == 2) {
        if (st == PDZ_OK) st = set_wide_lds<T, E, 1, 16>();
        if (st == PDZ_OK) st = set_wide_lds<T, E, 1, 32>();
        if (st == PDZ_OK) st = set_wide_lds<T, E, 1, 48>();
    }
    if (st == PDZ_OK) st = set_wide_lds<T, E, 3, 0>();
    if (st == PDZ_OK) st = set_wide_lds<T, E, 1, 0, true>();
    if (st == PDZ_OK) st = set_wide_lds<T, E, 2, 0, true>();
    if (st == PDZ_OK) st = set_wide_lds<T, E, 3, 0, true>();
    if (st != PDZ_OK) return st;
    PDZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hv_down_narrow<T, E, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    if (st == PDZ_OK) st = set_up_lds<T, E, sizeof(T) == 8 ? 16 : 32>();
    if (st == PDZ_OK) st = set_up_lds<T, E, sizeof(T) == 8 ? 32 : 64>();
    if (st == PDZ_OK) st = set_up_lds<T, E, sizeof(T) == 8 ? 64 : 128>();
    if (st == PDZ_OK) st = set_up_lds<T, E, sizeof(T) == 8 ? 128 : 256>();
    if (st == PDZ_OK) st = set_up_wide_lds<T, E, sizeof(T) == 8 ? 16 : 32>();
    if (st == PDZ_OK) st = set_up_wide_lds<T, E, sizeof(T) == 8 ? 32 : 64>();
    if (st == PDZ_OK) st = set_up_wide_lds<T, E, sizeof(T) == 8 ? 64 : 128>();
    if (sizeof(T) == 8 && st == PDZ_OK) st = set_up_pre_lds<T, E, 16>();
    if (st == PDZ_OK) st = set_up_pre_lds<T, E, 32>();
    if (st == PDZ_OK) st = set_up_pre_lds<T, E, 64>();
    return st;
}

}  // namespace

pdz_status hv_prepare() {
    pdz_status st = prepare_one<double, uint16_t>();
    if (st == PDZ_OK) st = prepare_one<double, uint32_t>();
    if (st == PDZ_OK) st = prepare_one<float, uint16_t>();
    if (st == PDZ_OK) st = prepare_one<float, uint32_t>();
    return st;
}

std::vector<HvPlan> hv_candidates(const pdz_problem_s* p, pdz_dtype dt, bool every) {
    std::vector<HvPlan> out;
    const HvPlan d = default_plan(p, dt);
    out.push_back(d);
    if (p->hv_path != 0) return out;
    const size_t es = dt == PDZ_F64 ? 8 : 4;
    const bool compact = p->up.tbits16 > 0 && p->dn.tbits16 > 0;
    std::vector<int> downs;
    const bool sched = wide_down(p, es) && p->dn.sched.words;
    if (sched) {
        // the scheduled family: one summation order for every plan the tuner tries
        for (int r = 1; r <= (es == 4 ? 3 : 1); ++r)
            if (sched_fits(p, es, r)) downs.push_back(4 + r);
    }
    if (wide_down(p, es) && (!sched || every)) {
        if (compact && p->dn.max_hops <= 48) downs.push_back(1);
        downs.push_back(2);
        if (row_fits(p, es, 2) && p->up.D >= 2) downs.push_back(3);
        if (row_fits(p, es, 3) && p->up.D >= 3) downs.push_back(4);
    } else if (!sched) {
        downs.push_back(d.down);
    }
    const int* cws = dt == PDZ_F64 ? kUpCw64 : kUpCw32;
    const bool pre_ok = p->up.max_hops <= 48 && p->D <= 0xFFFFFFFFull;
    for (int dv : downs)
        for (int k = 0; k < kNumCw; ++k)
            for (int um = 1; um <= 4; ++um)
                for (int mp = 1; mp <= 3; ++mp) {
                    HvPlan c;
                    c.down = dv;
                    c.up_cw = cws[k];
                    c.up = um;
                    c.map = mp;
                    if (um == 2 && (!pre_ok || cws[k] > 64)) continue;
                    if (um == 3 && p->D > 0xFFFFFFFFull) continue;
                    // wide lanes: 16-byte lanes, at most 32 lanes per row segment
                    if (um == 4 && (p->D > 0xFFFFFFFFull || (size_t)cws[k] * es / 16 > 32)) continue;
                    if (c.down != d.down || c.up_cw != d.up_cw || c.up != d.up || c.map != d.map) out.push_back(c);
                }
    return out;
}

bool hv_plan_valid(const pdz_problem_s* p, pdz_dtype dt, const HvPlan& plan) {
    if (plan.down == 0 && plan.up_cw == 0 && plan.up == 0 && plan.map == 0) return true;
    for (const HvPlan& c : hv_candidates(p, dt, true))
        if ((plan.down == 0 || plan.down == c.down) && (plan.up_cw == 0 || plan.up_cw == c.up_cw) &&
            (plan.up == 0 || plan.up == c.up) && (plan.map == 0 || plan.map == c.map))
            return true;
    return false;
}

pdz_status launch_hv(const pdz_problem_s* p, pdz_dtype dt, const void* x, void* y, hipStream_t s,
                     const int* skip, unsigned passes, const HvSplit* split, uint64_t pitch) {
    if (split && p->hv_path != 0) return fail(PDZ_EINVAL, "split H.v needs the table path");
    if (dt == PDZ_F64)
        return run_hv<double>(p, p->d_coef64, static_cast<const double*>(x), static_cast<double*>(y), s, skip,
                              passes, split, pitch);
    return run_hv<float>(p, p->d_coef32, static_cast<const float*>(x), static_cast<float*>(y), s, skip, passes,
                         split, pitch);
}

bool hv_fused_available(const pdz_problem_s* p, pdz_dtype dt) {
    if (p->hv_path != 0) return false;
    DeviceCtx* ctx = nullptr;
    if (device_ctx(&ctx) != PDZ_OK) return false;
    const size_t es = dt == PDZ_F64 ? 8 : 4;
    const HvPlan plan = hv_resolve(p, dt);
    const DownGeom gm = down_geom(p, es, plan, (unsigned)ctx->cu_count);
    return gm.wide && (plan.down == 2 || plan.down == 3 || plan.down == 4 || sched_plan(plan.down));
}

size_t hv_dot_count_max(const pdz_problem_s* p, pdz_dtype dt) {
    if (p->hv_path != 0) return 0;
    DeviceCtx* ctx = nullptr;
    if (device_ctx(&ctx) != PDZ_OK) return 0;
    const size_t es = dt == PDZ_F64 ? 8 : 4;
    size_t best = 0;
    for (const HvPlan& c : hv_candidates(p, dt, true)) {
        const size_t n = (size_t)down_grid(p, es, c, (unsigned)ctx->cu_count) +
                         (p->up.max_hops == 0 ? 1 : (size_t)up_blocks(p, es, c));
        if (n > best) best = n;
    }
    return best;
}

namespace {

template <typename T, int R, bool FUSE>
void launch_groups_r(uint64_t grid, hipStream_t s, const DownArgs<T, uint16_t>& da, const SchedArgs<T>& sa,
                     const T* x, T* y) {
    hipLaunchKernelGGL((k_hv_down_sched<T, uint16_t, R, FUSE, true>), dim3((unsigned)grid), dim3(kWideBlock), 0, s, da,
                       sa, x, y);
}

template <typename T>
pdz_status run_sched_groups(const SchedGroups& gr, const T* x, T* y, hipStream_t s, const int* skip,
                            const HvSplit* f) {
    if (!gr.sched || !gr.sched->words) return fail(PDZ_EINVAL, "no gather schedule for these rows");
    if (gr.R < 1 || gr.R > 3 || (sizeof(T) == 8 && gr.R != 1)) return fail(PDZ_EINVAL, "rows per group");
    if (gr.D_dn + 32 > (uint64_t)kSchedPlane) return fail(PDZ_EINVAL, "rows longer than the schedule's plane");
    const bool fuse = f && f->fq2;
    if (fuse && (f->fz || !f->fnorm || !f->fq1)) return fail(PDZ_EINVAL, "fused recurrence arguments");
    DownArgs<T, uint16_t> da{};
    da.D_up = gr.ngroups * (uint64_t)gr.R;
    da.D_dn = gr.D_dn;
    da.pitch = gr.D_dn;
    da.U = (T)gr.U;
    da.up_states = gr.grp_up;
    da.dn_states = gr.col_dn;
    da.rows = gr.R;
    da.skip = skip;
    da.goff = gr.goff;
    da.gnr = gr.gnr;
    da.ngroups = gr.ngroups;
    if (fuse) {
        da.fq1 = static_cast<const T*>(f->fq1);
        da.fq2 = static_cast<T*>(f->fq2);
        da.fkeep = static_cast<T*>(f->fkeep);
        da.fkeep_ld = f->fkeep_ld;
        da.fkeep_cap = f->fkeep_cap;
        da.falpha = f->falpha;
        da.fbeta = f->fbeta;
        da.fsc = f->fsc;
        da.fkidx = f->fkidx;
        da.fnorm = f->fnorm;
    }
    SchedArgs<T> sa;
    sa.words = gr.sched->words;
    sa.meta = gr.sched->meta;
    sa.mag0 = (T)gr.sched->mag0;
    sa.mag1 = (T)gr.sched->mag1;
    const uint64_t grid = sched_groups_grid(gr);
    if (grid == 0) return ok();
    if constexpr (sizeof(T) == 4) {
        if (gr.R == 3) {
            if (fuse) launch_groups_r<T, 3, true>(grid, s, da, sa, x, y);
            else launch_groups_r<T, 3, false>(grid, s, da, sa, x, y);
            PDZ_HIP(hipGetLastError());
            return ok();
        }
        if (gr.R == 2) {
            if (fuse) launch_groups_r<T, 2, true>(grid, s, da, sa, x, y);
            else launch_groups_r<T, 2, false>(grid, s, da, sa, x, y);
            PDZ_HIP(hipGetLastError());
            return ok();
        }
    }
    {
        if (fuse) launch_groups_r<T, 1, true>(grid, s, da, sa, x, y);
        else launch_groups_r<T, 1, false>(grid, s, da, sa, x, y);
    }
    PDZ_HIP(hipGetLastError());
    return ok();
}

}  // namespace

uint64_t sched_groups_grid(const SchedGroups& g) {
    DeviceCtx* ctx = nullptr;
    if (device_ctx(&ctx) != PDZ_OK) return 0;
    const uint64_t cu = (uint64_t)ctx->cu_count;   // one work group per CU: the planes fill the LDS
    return g.ngroups < cu ? g.ngroups : cu;
}

pdz_status launch_sched_groups(const SchedGroups& g, pdz_dtype dt, const void* x, void* y, hipStream_t s,
                               const int* skip, const HvSplit* fuse) {
    if (dt == PDZ_F64)
        return run_sched_groups<double>(g, static_cast<const double*>(x), static_cast<double*>(y), s, skip, fuse);
    return run_sched_groups<float>(g, static_cast<const float*>(x), static_cast<float*>(y), s, skip, fuse);
}

bool hv_dot_counts(const pdz_problem_s* p, pdz_dtype dt, int* n_dn, int* n_up) {
    if (p->hv_path != 0) return false;
    DeviceCtx* ctx = nullptr;
    if (device_ctx(&ctx) != PDZ_OK) return false;
    const size_t es = dt == PDZ_F64 ? 8 : 4;
    const HvPlan plan = hv_resolve(p, dt);
    *n_dn = (int)down_grid(p, es, plan, (unsigned)ctx->cu_count);
    *n_up = p->up.max_hops == 0 ? 1 : (int)up_blocks(p, es, plan);
    return true;
}

}  // namespace pdz
