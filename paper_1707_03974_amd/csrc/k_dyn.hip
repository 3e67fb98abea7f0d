// Dynamical correlations by the Lanczos continued fraction (the method that
// Sec. I cites): fermion operators that carry a state between Hubbard
// sectors, and the continued fraction of the resolvent built from the Lanczos
// coefficients of the new sector.
//
// c_{j,s} (op 0) removes and c+_{j,s} (op 1) adds an electron of spin s at site
// j.  The operator acts on one spin's string only, so a target basis state
// (phi_up', phi_dn') has at most one source state, found by toggling bit j of
// that spin's string and ranking the result with the forward map (Eq. 3) of the
// source sector: no list, no search.  The sign follows the operator order of
// the Hamiltonian (Sec. II.A: up operators left of down operators, the site
// index growing from right to left): (-1)^(electrons of spin s above site j),
// times (-1)^(n_up) for a down operator, which passes every up operator.
#include <complex>

#include "pdz_internal.h"
#include "perfect_hash.h"

namespace pdz {

namespace {

constexpr int kDynBlock = 256;

struct FermArgs {
    const uint32_t* binom;
    const uint32_t* t_up;   // target sector strings, up and down
    const uint32_t* t_dn;
    uint64_t Dt_up, Dt_dn;  // target sector sizes
    uint64_t Ds_dn;         // source down-sector size (row length of x)
    int site, spin, op, n_up;
};

__device__ __forceinline__ bool odd_above(uint32_t phi, int site, int extra) {
    const uint32_t above = site + 1 < 32 ? (phi >> (site + 1)) : 0u;
    return ((__builtin_popcount(above) + extra) & 1) != 0;
}

// One work group per target row (grid-stride); threads over the row's columns.
template <typename T>
__global__ __launch_bounds__(kDynBlock) void k_fermion_apply(const FermArgs a, const T* __restrict__ x,
                                                             T* __restrict__ y) {
    __shared__ uint32_t sC[kBinomStride * kBinomStride];
    stage_binom(sC, a.binom);
    const uint32_t bit = 1u << a.site;
    for (uint64_t u = blockIdx.x; u < a.Dt_up; u += gridDim.x) {
        // up operator: the whole row has one source row and one sign
        bool row_zero = false, row_neg = false;
        uint64_t src_row = u;
        if (a.spin == 0) {
            const uint32_t phi_t = a.t_up[u];
            const bool has = (phi_t & bit) != 0;
            if (has == (a.op == 0)) {
                row_zero = true;
            } else {
                const uint32_t phi_s = a.op == 0 ? (phi_t | bit) : (phi_t & ~bit);
                src_row = forward_map(phi_s, sC);
                row_neg = odd_above(phi_s, a.site, 0);
            }
        }
        const T* xr = x + src_row * a.Ds_dn;
        T* yr = y + u * a.Dt_dn;
        for (uint64_t d = threadIdx.x; d < a.Dt_dn; d += kDynBlock) {
            T v = (T)0;
            if (a.spin == 0) {
                if (!row_zero) v = row_neg ? -xr[d] : xr[d];
            } else {
                const uint32_t phi_t = a.t_dn[d];
                const bool has = (phi_t & bit) != 0;
                if (has != (a.op == 0)) {
                    const uint32_t phi_s = a.op == 0 ? (phi_t | bit) : (phi_t & ~bit);
                    const T s = xr[forward_map(phi_s, sC)];
                    v = odd_above(phi_s, a.site, a.n_up) ? -s : s;
                }
            }
            yr[d] = v;
        }
    }
}

}  // namespace
}  // namespace pdz

using namespace pdz;

extern "C" {

pdz_status pdz_fermion_op(pdz_problem src, pdz_problem dst, int32_t site, int32_t spin, int32_t op, pdz_dtype dt,
                          const void* x, void* y, void* stream) {
    if (!src || !dst || !x || !y) return fail(PDZ_EINVAL, "NULL argument");
    if (src->ks || dst->ks || src->par || dst->par)
        return fail(PDZ_EINVAL, "fermion operators act on full real-space sectors");
    if (dt != PDZ_F64 && dt != PDZ_F32) return fail(PDZ_EINVAL, "dtype must be F64 or F32");
    if (src->N != dst->N) return fail(PDZ_EINVAL, "source and target differ in the number of sites");
    if (site < 0 || site >= src->N) return fail(PDZ_EINVAL, "site out of range");
    if (spin != 0 && spin != 1) return fail(PDZ_EINVAL, "spin must be 0 (up) or 1 (down)");
    if (op != 0 && op != 1) return fail(PDZ_EINVAL, "op must be 0 (annihilate) or 1 (create)");
    const int d = op == 0 ? -1 : 1;
    const int want_up = src->n_up + (spin == 0 ? d : 0), want_dn = src->n_dn + (spin == 1 ? d : 0);
    if (dst->n_up != want_up || dst->n_dn != want_dn)
        return fail(PDZ_EINVAL, "target sector must have one electron of that spin fewer (op 0) or more (op 1)");
    if (src->device != dst->device) return fail(PDZ_EINVAL, "problems live on different devices");
    int dev = 0;
    PDZ_HIP(hipGetDevice(&dev));
    if (dev != src->device) return fail(PDZ_EINVAL, "problem lives on another device");
    const size_t es = dt == PDZ_F64 ? 8 : 4;
    const uintptr_t xa = reinterpret_cast<uintptr_t>(x), ya = reinterpret_cast<uintptr_t>(y);
    if (xa < ya + dst->D * es && ya < xa + src->D * es) return fail(PDZ_EINVAL, "x and y overlap");
    DeviceCtx* ctx = nullptr;
    pdz_status st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    FermArgs a;
    a.binom = ctx->binom;
    a.t_up = dst->up.states;
    a.t_dn = dst->dn.states;
    a.Dt_up = dst->up.D;
    a.Dt_dn = dst->dn.D;
    a.Ds_dn = src->dn.D;
    a.site = site;
    a.spin = spin;
    a.op = op;
    a.n_up = src->n_up;
    uint64_t grid = a.Dt_up;
    const uint64_t gmax = (uint64_t)ctx->cu_count * 8;
    if (grid > gmax) grid = gmax;
    if (grid < 1) grid = 1;
    hipStream_t s = (hipStream_t)stream;
    if (dt == PDZ_F64)
        hipLaunchKernelGGL(k_fermion_apply<double>, dim3((unsigned)grid), dim3(kDynBlock), 0, s, a,
                           static_cast<const double*>(x), static_cast<double*>(y));
    else
        hipLaunchKernelGGL(k_fermion_apply<float>, dim3((unsigned)grid), dim3(kDynBlock), 0, s, a,
                           static_cast<const float*>(x), static_cast<float*>(y));
    PDZ_HIP(hipGetLastError());
    return ok();
}

pdz_status pdz_continued_fraction(const double* alpha, const double* beta, int32_t n, double norm2,
                                  const double* w_re, const double* w_im, int32_t nw, double* g_re, double* g_im) {
    if (!alpha || !beta || !w_re || !w_im || !g_re || !g_im) return fail(PDZ_EINVAL, "NULL argument");
    if (n < 1 || nw < 0) return fail(PDZ_EINVAL, "need n >= 1 coefficients and nw >= 0 points");
    for (int i = 0; i < nw; ++i) {
        const std::complex<double> w(w_re[i], w_im[i]);
        std::complex<double> g(0.0, 0.0);   // tail of the fraction, built from the last level up
        for (int j = n - 1; j >= 1; --j) g = (beta[j] * beta[j]) / (w - alpha[j] - g);
        const std::complex<double> r = norm2 / (w - alpha[0] - g);
        g_re[i] = r.real();
        g_im[i] = r.imag();
    }
    return ok();
}

}  // extern "C"
