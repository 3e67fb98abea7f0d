// Perfect-hash kernels: the forward map (rank), the backward map (unrank) and
// the per-sector hop tables built from them (Sec. III).
//
// Forward map (Eq. 3): a string with set bits j_0 < j_1 < ... < j_{n-1} has
// index sum_m C(j_m, m+1); walking the bits upward, each set bit bumps the
// running count m and adds C(i, m).  Backward map: walk i from N-1 down; when
// the remaining rank p is at least C(i, m) the bit is set, p drops by C(i, m)
// and m by one.  C(i, m) = 0 for i < m.  Both are exact integer arithmetic;
// the binomial table is staged in LDS.
#include "pdz_internal.h"
#include "perfect_hash.h"

namespace pdz {

namespace {

constexpr int kHashBlock = 256;

__global__ __launch_bounds__(kHashBlock) void k_rank(const uint32_t* __restrict__ gC, int N, int n,
                                                     const uint32_t* __restrict__ bits, uint64_t count,
                                                     uint32_t* __restrict__ ranks, uint32_t* err) {
    __shared__ uint32_t sC[kBinomStride * kBinomStride];
    stage_binom(sC, gC);
    const uint32_t width_mask = (N >= 32) ? 0u : ~((1u << N) - 1u);
    bool bad = false;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < count;
         k += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t phi = bits[k];
        if (__builtin_popcount(phi) != n || (phi & width_mask)) {
            ranks[k] = kBadRank;
            bad = true;
        } else {
            ranks[k] = forward_map(phi, sC);
        }
    }
    if (bad) atomicOr(err, kErrRankInput);
}

__global__ __launch_bounds__(kHashBlock) void k_unrank(const uint32_t* __restrict__ gC, int N, int n,
                                                       const uint32_t* __restrict__ ranks, uint64_t count,
                                                       uint32_t* __restrict__ bits, uint32_t* err) {
    __shared__ uint32_t sC[kBinomStride * kBinomStride];
    stage_binom(sC, gC);
    const uint32_t D = sC[N * kBinomStride + n];
    bool bad = false;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < count;
         k += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t p = ranks[k];
        if (p >= D) {
            bits[k] = kBadRank;
            bad = true;
        } else {
            bits[k] = backward_map(p, n, N, sC);
        }
    }
    if (bad) atomicOr(err, kErrUnrankInput);
}

// Hops out of one sector state: a bond (i, j) acts when exactly one end is
// occupied.  The fermion sign of c+_a c_b on the normal-ordered string is
// (-1)^(occupied same-spin sites strictly between a and b); the operators of
// the other spin are passed twice and cancel.
__global__ __launch_bounds__(kHashBlock) void k_sector_count(const uint32_t* __restrict__ gC, int N, int n,
                                                             uint64_t D, const BondDev* __restrict__ bonds,
                                                             int nb, uint8_t* __restrict__ count,
                                                             unsigned int* max_hops,
                                                             unsigned long long* total) {
    __shared__ uint32_t sC[kBinomStride * kBinomStride];
    stage_binom(sC, gC);
    unsigned int local_max = 0;
    unsigned long long local_sum = 0;
    for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < D;
         s += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t phi = backward_map((uint32_t)s, n, N, sC);
        unsigned int c = 0;
        for (int b = 0; b < nb; ++b) {
            const uint32_t occ = phi & bonds[b].mask;
            c += (occ != 0u && occ != bonds[b].mask) ? 1u : 0u;
        }
        count[s] = (uint8_t)(c > 255u ? 255u : c);
        local_max = c > local_max ? c : local_max;
        local_sum += c;
    }
    atomicMax(max_hops, local_max);
    atomicAdd(total, local_sum);
}

__global__ __launch_bounds__(kHashBlock) void k_sector_fill(const uint32_t* __restrict__ gC, int N, int n,
                                                            uint64_t D, const BondDev* __restrict__ bonds,
                                                            int nb, uint32_t* __restrict__ states,
                                                            uint32_t* __restrict__ ell, uint32_t* err) {
    __shared__ uint32_t sC[kBinomStride * kBinomStride];
    stage_binom(sC, gC);
    bool bad = false;
    for (uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; s < D;
         s += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t phi = backward_map((uint32_t)s, n, N, sC);
        states[s] = phi;
        uint64_t h = 0;
        for (int b = 0; b < nb; ++b) {
            const BondDev bd = bonds[b];
            const uint32_t occ = phi & bd.mask;
            if (occ == 0u || occ == bd.mask) continue;
            const uint32_t target = forward_map(phi ^ bd.mask, sC);
            const bool odd = (__builtin_popcount(phi & bd.between) & 1) != 0;
            const uint32_t coef = (uint32_t)(odd ? bd.coef_neg : bd.coef_pos);
            if (target >= D || target > kTargetMask) bad = true;
            ell[h * D + s] = (target & kTargetMask) | (coef << kTargetBits);
            ++h;
        }
    }
    if (bad) atomicOr(err, kErrTable);
}

// 16-bit table in slot-pair layout: slots 2k and 2k+1 of state s share one
// 32-bit word, out[(k * D + s) * 2 + (h & 1)], so a column loads two slots
// per access.  Slots past the state's count are zero.
__global__ __launch_bounds__(kHashBlock) void k_compact(const uint32_t* __restrict__ ell, const uint8_t* __restrict__ cnt,
                                                        uint64_t D, int slots, int tbits, uint16_t* __restrict__ out) {
    const uint64_t n = (uint64_t)slots * D;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t h = (uint32_t)(k / D);
        const uint64_t st = k - (uint64_t)h * D;
        uint16_t v = 0;
        if (h < cnt[st]) {
            const uint32_t e = ell[k];
            v = (uint16_t)((e & kTargetMask) | ((e >> kTargetBits) << tbits));
        }
        out[(((uint64_t)(h >> 1) * D + st) << 1) + (h & 1u)] = v;
    }
}

int grid_for(uint64_t n, int block) {
    uint64_t g = (n + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

// 16-bit form of a sector's hop table: target in the low tbits bits, amplitude
// index above, when both fit.
pdz_status build_compact_table(SectorTables* st, int ncoef, hipStream_t s) {
    int cbits = 0;
    while ((1 << cbits) < ncoef) ++cbits;
    const int tbits = 16 - cbits;
    if (cbits > 15 || st->D > (1ull << tbits) || st->max_hops == 0) {
        st->tbits16 = 0;
        return ok();
    }
    const int slots = (st->max_hops + 1) & ~1;   // even: whole slot pairs
    const uint64_t n = (uint64_t)slots * st->D;
    PDZ_HIP(hipMalloc(&st->ell16, n * sizeof(uint16_t)));
    PDZ_HIP(hipMemsetAsync(st->ell16, 0, n * sizeof(uint16_t), s));
    hipLaunchKernelGGL(k_compact, dim3(grid_for((uint64_t)st->max_hops * st->D, kHashBlock)), dim3(kHashBlock), 0, s,
                       st->ell, st->count, st->D, st->max_hops, tbits, st->ell16);
    PDZ_HIP(hipGetLastError());
    st->tbits16 = tbits;
    return ok();
}

pdz_status launch_rank(const uint32_t* d_binom, int N, int n, const uint32_t* bits, uint64_t count,
                       uint32_t* ranks, uint32_t* err, hipStream_t s) {
    if (count == 0) return ok();
    hipLaunchKernelGGL(k_rank, dim3(grid_for(count, kHashBlock)), dim3(kHashBlock), 0, s, d_binom, N, n, bits,
                       count, ranks, err);
    PDZ_HIP(hipGetLastError());
    return ok();
}

pdz_status launch_unrank(const uint32_t* d_binom, int N, int n, const uint32_t* ranks, uint64_t count,
                         uint32_t* bits, uint32_t* err, hipStream_t s) {
    if (count == 0) return ok();
    hipLaunchKernelGGL(k_unrank, dim3(grid_for(count, kHashBlock)), dim3(kHashBlock), 0, s, d_binom, N, n,
                       ranks, count, bits, err);
    PDZ_HIP(hipGetLastError());
    return ok();
}

pdz_status build_sector_tables(const uint32_t* d_binom, int N, int n, const BondDev* d_bonds, int nb,
                               SectorTables* st, uint32_t* err, hipStream_t s) {
    const uint64_t D = st->D;
    unsigned int* d_max = nullptr;
    unsigned long long* d_total = nullptr;
    PDZ_HIP(hipMalloc(&d_max, sizeof(unsigned int) + sizeof(unsigned long long) + 8));
    d_total = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(d_max) + 8);
    PDZ_HIP(hipMemsetAsync(d_max, 0, 16, s));
    PDZ_HIP(hipMalloc(&st->count, D));
    PDZ_HIP(hipMalloc(&st->states, D * sizeof(uint32_t)));
    hipLaunchKernelGGL(k_sector_count, dim3(grid_for(D, kHashBlock)), dim3(kHashBlock), 0, s, d_binom, N, n, D,
                       d_bonds, nb, st->count, d_max, d_total);
    PDZ_HIP(hipGetLastError());
    unsigned int h_max = 0;
    unsigned long long h_total = 0;
    PDZ_HIP(hipMemcpyAsync(&h_max, d_max, sizeof(h_max), hipMemcpyDeviceToHost, s));
    PDZ_HIP(hipMemcpyAsync(&h_total, d_total, sizeof(h_total), hipMemcpyDeviceToHost, s));
    PDZ_HIP(hipStreamSynchronize(s));
    (void)hipFree(d_max);
    if (h_max > 255u) return fail(PDZ_ERANGE, "more than 255 hops out of one sector state");
    st->max_hops = (int)h_max;
    st->total_hops = h_total;
    const size_t ell_elems = (size_t)h_max * D;
    PDZ_HIP(hipMalloc(&st->ell, (ell_elems ? ell_elems : 1) * sizeof(uint32_t)));
    hipLaunchKernelGGL(k_sector_fill, dim3(grid_for(D, kHashBlock)), dim3(kHashBlock), 0, s, d_binom, N, n, D,
                       d_bonds, nb, st->states, st->ell, err);
    PDZ_HIP(hipGetLastError());
    return ok();
}

}  // namespace pdz
