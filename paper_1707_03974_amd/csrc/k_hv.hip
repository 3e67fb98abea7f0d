// y = H x for the Hubbard Hamiltonian (Eq. 1), matrix-free.
//
// Vector layout: X[i_up][i_dn], index i_up * D_dn + i_dn (composite index of
// Sec. III).  With this layout
//     y[u,d] = U popc(phi_up(u) & phi_dn(d)) x[u,d]
//            + sum_{up hops u->u'} a(u,u') x[u',d]      (rows of X, coalesced)
//            + sum_{dn hops d->d'} a(d,d') x[u,d']      (gathers inside row u)
// where a = -t_b * sign.  Each hop target index comes from the forward map
// (perfect hash) evaluated once per sector state when the problem is created
// (hop tables, k_hash.hip) or, on the fallback path, per element here.
//
// Each output element is summed by one thread in a fixed order (diagonal,
// down hops in bond order, up hops in bond order): no atomics, bitwise
// reproducible.
#include "pdz_internal.h"

namespace pdz {

namespace {

constexpr int kHvBlock = 256;

// Table path: a group of R consecutive rows of x is staged in LDS; every
// thread walks the elements of the group.
template <typename T, bool STAGE>
__global__ __launch_bounds__(kHvBlock) void k_hv_table(const HvArgs<T> a, const T* __restrict__ x,
                                                       T* __restrict__ y) {
    if (a.skip && *a.skip) return;
    extern __shared__ __align__(16) unsigned char smem[];
    T* coef = reinterpret_cast<T*>(smem);
    T* rows = coef + kMaxCoef;
    for (int k = threadIdx.x; k < a.ncoef; k += blockDim.x) coef[k] = a.coef[k];

    const uint64_t D_up = a.D_up, D_dn = a.D_dn;
    const int R = a.rows_per_group;
    const uint64_t ngroups = (D_up + R - 1) / R;
    for (uint64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        const uint64_t u0 = g * (uint64_t)R;
        const int nr = (int)((D_up - u0) < (uint64_t)R ? (D_up - u0) : (uint64_t)R);
        const uint64_t nelem = (uint64_t)nr * D_dn;
        const T* xg = x + u0 * D_dn;
        __syncthreads();
        if (STAGE) {
            for (uint64_t k = threadIdx.x; k < nelem; k += blockDim.x) rows[k] = xg[k];
        }
        __syncthreads();
        for (uint64_t k = threadIdx.x; k < nelem; k += blockDim.x) {
            const uint32_t r = (uint32_t)(k / D_dn);
            const uint32_t d = (uint32_t)(k - (uint64_t)r * D_dn);
            const uint64_t u = u0 + r;
            const T* xrow = STAGE ? rows + (uint64_t)r * D_dn : xg + (uint64_t)r * D_dn;
            const uint32_t pu = a.up_states[u];
            const uint32_t pd = a.dn_states[d];
            T acc = a.U * (T)__builtin_popcount(pu & pd) * xrow[d];
            const int cd = a.dn_count[d];
            for (int h = 0; h < cd; ++h) {
                const uint32_t e = a.dn_ell[(uint64_t)h * D_dn + d];
                acc += coef[e >> kTargetBits] * xrow[e & kTargetMask];
            }
            const int cu = a.up_count[u];
            for (int h = 0; h < cu; ++h) {
                const uint32_t e = a.up_ell[(uint64_t)h * D_up + u];
                acc += coef[e >> kTargetBits] * x[(uint64_t)(e & kTargetMask) * D_dn + d];
            }
            y[u * D_dn + d] = acc;
        }
    }
}

// Fallback path: every sector rank and every hop target is computed per
// element with the forward and backward maps (binomial table in LDS).
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
__global__ __launch_bounds__(kHvBlock) void k_hv_fly(const FlyArgs f, T U, const T* __restrict__ coef_g,
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
        for (int b = 0; b < f.nb; ++b) {
            const BondDev bd = f.bonds[b];
            const uint32_t od = pd & bd.mask;
            if (od != 0u && od != bd.mask) {
                const int c = (__builtin_popcount(pd & bd.between) & 1) ? bd.coef_neg : bd.coef_pos;
                acc += coef_g[c] * x[u * f.D_dn + fly_rank(pd ^ bd.mask, sC)];
            }
        }
        for (int b = 0; b < f.nb; ++b) {
            const BondDev bd = f.bonds[b];
            const uint32_t ou = pu & bd.mask;
            if (ou != 0u && ou != bd.mask) {
                const int c = (__builtin_popcount(pu & bd.between) & 1) ? bd.coef_neg : bd.coef_pos;
                acc += coef_g[c] * x[(uint64_t)fly_rank(pu ^ bd.mask, sC) * f.D_dn + d];
            }
        }
        y[r] = acc;
    }
}

template <typename T>
pdz_status run_hv(const pdz_problem_s* p, const T* coef, const T* x, T* y, hipStream_t s, const int* skip) {
    DeviceCtx* ctx = nullptr;
    pdz_status st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    if (p->hv_path == 0) {
        HvArgs<T> a;
        a.D_up = p->up.D;
        a.D_dn = p->dn.D;
        a.U = (T)p->U;
        a.up_states = p->up.states;
        a.up_count = p->up.count;
        a.up_ell = p->up.ell;
        a.dn_states = p->dn.states;
        a.dn_count = p->dn.count;
        a.dn_ell = p->dn.ell;
        a.coef = coef;
        a.ncoef = (int)p->coef_host.size();
        a.skip = skip;
        const size_t lds_cap = 160 * 1024 - kMaxCoef * sizeof(T) - 1024;
        const size_t row_bytes = (size_t)a.D_dn * sizeof(T);
        const bool stage = row_bytes <= lds_cap;
        int R = 1;
        if (a.D_dn < 2 * (uint64_t)kHvBlock) R = (int)((2 * kHvBlock + a.D_dn - 1) / a.D_dn);
        if (stage) {
            int rmax = (int)(lds_cap / row_bytes);
            if (R > rmax) R = rmax;
        }
        if ((uint64_t)R > a.D_up) R = (int)a.D_up;
        if (R < 1) R = 1;
        a.rows_per_group = R;
        const size_t lds = kMaxCoef * sizeof(T) + (stage ? (size_t)R * row_bytes : 0);
        const uint64_t ngroups = (a.D_up + R - 1) / R;
        const int per_cu = stage ? (int)((160 * 1024) / (lds + 512)) : 4;
        uint64_t grid = (uint64_t)ctx->cu_count * (per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu));
        if (grid > ngroups) grid = ngroups;
        if (grid < 1) grid = 1;
        if (stage) {
            hipLaunchKernelGGL((k_hv_table<T, true>), dim3((unsigned)grid), dim3(kHvBlock), lds, s, a, x, y);
        } else {
            hipLaunchKernelGGL((k_hv_table<T, false>), dim3((unsigned)grid), dim3(kHvBlock), lds, s, a, x, y);
        }
        PDZ_HIP(hipGetLastError());
        return ok();
    }
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
    uint64_t grid = (p->D + kHvBlock - 1) / kHvBlock;
    const uint64_t gmax = (uint64_t)ctx->cu_count * 16;
    if (grid > gmax) grid = gmax;
    hipLaunchKernelGGL(k_hv_fly<T>, dim3((unsigned)grid), dim3(kHvBlock), 0, s, f, (T)p->U, coef, x, y);
    PDZ_HIP(hipGetLastError());
    return ok();
}

}  // namespace

pdz_status hv_prepare() {
    const int lds = 160 * 1024;
    PDZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hv_table<double, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    PDZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_hv_table<float, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, lds));
    return ok();
}

pdz_status launch_hv(const pdz_problem_s* p, pdz_dtype dt, const void* x, void* y, hipStream_t s,
                     const int* skip) {
    if (dt == PDZ_F64)
        return run_hv<double>(p, p->d_coef64, static_cast<const double*>(x), static_cast<double*>(y), s, skip);
    return run_hv<float>(p, p->d_coef32, static_cast<const float*>(x), static_cast<float*>(y), s, skip);
}

}  // namespace pdz
