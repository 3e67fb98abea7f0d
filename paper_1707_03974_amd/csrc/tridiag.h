// Lowest eigenpair of the Lanczos tridiagonal T_k (FP64), shared by the
// single-problem and the batched Lanczos kernels.
//
// T_k has diagonal a[0..k-1] and off-diagonal e[1..k-1] (e[0] = 0).  Its
// lowest eigenvalue comes from Sturm-count multisection over the Gershgorin
// interval: each round splits the bracket into blockDim + 1 pieces and keeps
// the one where the count of eigenvalues below the point first reaches one.
// The eigenvector comes from inverse iteration with a shift just below the
// bracket, so T_k - sigma I is positive definite and its LDL^T factorisation
// needs no pivoting.
#pragma once

#include <hip/hip_runtime.h>

namespace pdz {

// Number of eigenvalues of T below x (signs of the LDL^T pivots of T - x I).
__device__ inline int tridiag_sturm_count(const double* a, const double* e, int k, double x) {
    int cnt = 0;
    double q = a[0] - x;
    if (q < 0.0) ++cnt;
    for (int i = 1; i < k; ++i) {
        if (q == 0.0) q = 1e-300;
        q = (a[i] - x) - e[i] * e[i] / q;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// Whole work group: bracket [bounds[0], bounds[1]] of lambda_min(T_k) to a
// few ulps.  a, e in LDS; lo_s, hi_s: blockDim doubles of LDS; found, bounds
// in LDS.  Every thread must call it; bounds is valid for all on return.
__device__ inline void tridiag_bracket_min(const double* a, const double* e, int k, double* lo_s, double* hi_s,
                                           int* found, double* bounds) {
    double lo = 1e300, hi = -1e300;
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        const double r = fabs(e[i]) + (i + 1 < k ? fabs(e[i + 1]) : 0.0);
        lo = fmin(lo, a[i] - r);
        hi = fmax(hi, a[i] + r);
    }
    lo_s[threadIdx.x] = lo;
    hi_s[threadIdx.x] = hi;
    __syncthreads();
    for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            lo_s[threadIdx.x] = fmin(lo_s[threadIdx.x], lo_s[threadIdx.x + st]);
            hi_s[threadIdx.x] = fmax(hi_s[threadIdx.x], hi_s[threadIdx.x + st]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double pad = 1e-12 * fmax(1.0, fmax(fabs(lo_s[0]), fabs(hi_s[0])));
        bounds[0] = lo_s[0] - pad;
        bounds[1] = hi_s[0] + pad;
    }
    __syncthreads();
    for (int round = 0; round < 64; ++round) {
        lo = bounds[0];
        hi = bounds[1];
        if (!(hi - lo > 2.0 * 2.220446049250313e-16 * fmax(fabs(lo), fabs(hi)) + 1e-300)) break;
        const double x = lo + (hi - lo) * (double)(threadIdx.x + 1) / (double)(blockDim.x + 1);
        if (threadIdx.x == 0) *found = blockDim.x;
        __syncthreads();
        if (tridiag_sturm_count(a, e, k, x) >= 1) atomicMin(found, (int)threadIdx.x);
        __syncthreads();
        if (threadIdx.x == 0) {
            const int t = *found;
            const double nlo = (t == 0) ? lo : lo + (hi - lo) * (double)t / (double)(blockDim.x + 1);
            const double nhi = (t == (int)blockDim.x) ? hi : lo + (hi - lo) * (double)(t + 1) / (double)(blockDim.x + 1);
            bounds[0] = nlo;
            bounds[1] = nhi;
        }
        __syncthreads();
    }
}

// One thread: normalised eigenvector z[0..k-1] for the eigenvalue bracketed
// below by `lower`, by three steps of inverse iteration; dpiv holds k pivots.
__device__ inline void tridiag_min_vector(const double* a, const double* e, int k, double lower, double* z,
                                          double* dpiv) {
    const double sigma = lower - 4.0 * 2.220446049250313e-16 * fmax(1.0, fabs(lower));
    for (int i = 0; i < k; ++i) z[i] = 1.0;
    for (int it = 0; it < 3; ++it) {
        // (T - sigma I) = L D L^T: forward solve with L, then D, then L^T
        double d0 = a[0] - sigma;
        if (d0 == 0.0) d0 = 1e-300;
        dpiv[0] = d0;
        for (int i = 1; i < k; ++i) {
            const double l = e[i] / dpiv[i - 1];
            double di = (a[i] - sigma) - l * e[i];
            if (di == 0.0) di = 1e-300;
            dpiv[i] = di;
            z[i] -= l * z[i - 1];
        }
        z[k - 1] /= dpiv[k - 1];
        for (int i = k - 2; i >= 0; --i) z[i] = z[i] / dpiv[i] - (e[i + 1] / dpiv[i]) * z[i + 1];
        double nrm = 0.0;
        for (int i = 0; i < k; ++i) nrm += z[i] * z[i];
        nrm = sqrt(nrm);
        if (!(nrm > 0.0) || !isfinite(nrm)) break;
        for (int i = 0; i < k; ++i) z[i] /= nrm;
    }
}

}  // namespace pdz
