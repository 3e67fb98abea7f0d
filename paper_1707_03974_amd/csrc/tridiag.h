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

// 1/q in FP64 from the hardware reciprocal estimate and two steps of Newton's
// iteration r <- r + r (1 - q r), each of which doubles the number of correct
// bits; a few fused operations in place of a division on the serial chains
// below (q finite, |q| >= 1e-300: the callers lift smaller pivots to 1e-300).
__device__ inline double tridiag_recip(double q) {
    double r = __builtin_amdgcn_rcp(q);
    double t = fma(-q, r, 1.0);
    r = fma(r, t, r);
    t = fma(-q, r, 1.0);
    return fma(r, t, r);
}

// Operands read ahead of the serial steps below: the LDS reads of a batch are
// issued together, so one wait covers them, and the steps then run on
// registers (the arithmetic and its order are those of the plain loops).
constexpr int kTriBatch = 8;

// Number of eigenvalues of T below x (signs of the LDL^T pivots of T - x I).
__device__ inline int tridiag_sturm_count(const double* a, const double* e, int k, double x) {
    int cnt = 0;
    double q = a[0] - x;
    if (q < 0.0) ++cnt;
    auto step = [&](double am, double e2) {
        if (fabs(q) < 1e-300) q = q < 0.0 ? -1e-300 : 1e-300;   // the sign is counted already
        q = am - e2 * tridiag_recip(q);
        if (q < 0.0) ++cnt;
    };
    int i = 1;
    for (; i + kTriBatch <= k; i += kTriBatch) {
        double am[kTriBatch], e2[kTriBatch];
#pragma unroll
        for (int j = 0; j < kTriBatch; ++j) {
            am[j] = a[i + j] - x;
            e2[j] = e[i + j] * e[i + j];
        }
#pragma unroll
        for (int j = 0; j < kTriBatch; ++j) step(am[j], e2[j]);
    }
    for (; i < k; ++i) step(a[i] - x, e[i] * e[i]);
    return cnt;
}

// Whole work group: shrink [bounds[0], bounds[1]], which holds lambda_min,
// by splitting it into blockDim + 1 pieces per round.
__device__ inline void tridiag_multisect(const double* a, const double* e, int k, int* found, double* bounds) {
    double lo, hi;
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

// Whole work group: bracket [bounds[0], bounds[1]] of lambda_min(T_k) to a
// few ulps.  a, e in LDS; lo_s, hi_s: blockDim doubles of LDS; found, bounds
// in LDS.  Every thread must call it; bounds is valid for all on return.
// A hint [hint_lo, hint_hi] (hint_lo < hint_hi) replaces the Gershgorin
// interval when two Sturm counts confirm that it holds exactly the lowest
// eigenvalue's side: none below hint_lo, at least one below hint_hi.  In
// Lanczos the previous Ritz value bounds the new one from above (Cauchy
// interlacing), and the last change estimates how far it moves.
__device__ inline void tridiag_bracket_min(const double* a, const double* e, int k, double* lo_s, double* hi_s,
                                           int* found, double* bounds, double hint_lo = 0.0,
                                           double hint_hi = 0.0) {
    if (hint_lo < hint_hi) {
        if (threadIdx.x == 0) *found = 0;
        __syncthreads();
        if (threadIdx.x < 2) {
            const int c = tridiag_sturm_count(a, e, k, threadIdx.x == 0 ? hint_lo : hint_hi);
            const bool good = threadIdx.x == 0 ? (c == 0) : (c >= 1);
            if (good) atomicAdd(found, 1);
        }
        __syncthreads();
        const bool use = *found == 2;
        __syncthreads();
        if (use) {
            if (threadIdx.x == 0) {
                bounds[0] = hint_lo;
                bounds[1] = hint_hi;
            }
            __syncthreads();
            tridiag_multisect(a, e, k, found, bounds);
            return;
        }
    }
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
    tridiag_multisect(a, e, k, found, bounds);
}

// Bracket hint for lambda_min(T_k) from the Ritz values of the two previous
// steps: the new value lies below theta1 (interlacing; the pad covers the
// rounding of theta1) and, once the iteration settles, within a few times the
// last change of it.
__device__ inline void ritz_hint(double theta1, double theta2, double* lo, double* hi) {
    const double scale = fmax(1.0, fabs(theta1));
    const double w = fmax(8.0 * fabs(theta1 - theta2), 1e-12 * scale);
    *hi = theta1 + 8.0 * 2.220446049250313e-16 * scale;
    *lo = theta1 - w;
}

// One thread: normalised eigenvector z[0..k-1] for the eigenvalue bracketed
// below by `lower`.  T - sigma I = L D L^T is factored once (reciprocal
// pivots in rp), then three steps of inverse iteration reuse it.  a, e, z, rp
// should live in LDS: the sweeps are serial recurrences, so only the carried
// value stays on the critical path.
__device__ inline void tridiag_min_vector(const double* a, const double* e, int k, double lower, double* z,
                                          double* rp) {
    constexpr int B = kTriBatch;
    const double sigma = lower - 4.0 * 2.220446049250313e-16 * fmax(1.0, fabs(lower));
    double d = a[0] - sigma;
    if (fabs(d) < 1e-300) d = d < 0.0 ? -1e-300 : 1e-300;
    double r = tridiag_recip(d);
    rp[0] = r;
    z[0] = 1.0;
    auto pivot = [&](double am, double ei) {
        d = am - (ei * r) * ei;
        if (fabs(d) < 1e-300) d = d < 0.0 ? -1e-300 : 1e-300;
        r = tridiag_recip(d);
        return r;
    };
    int i = 1;
    for (; i + B <= k; i += B) {
        double am[B], ev[B], rv[B];
#pragma unroll
        for (int j = 0; j < B; ++j) {
            am[j] = a[i + j] - sigma;
            ev[j] = e[i + j];
        }
#pragma unroll
        for (int j = 0; j < B; ++j) rv[j] = pivot(am[j], ev[j]);
#pragma unroll
        for (int j = 0; j < B; ++j) {
            rp[i + j] = rv[j];
            z[i + j] = 1.0;
        }
    }
    for (; i < k; ++i) {
        rp[i] = pivot(a[i] - sigma, e[i]);
        z[i] = 1.0;
    }
    for (int it = 0; it < 3; ++it) {
        // L y = z (forward), then D L^T x = y (backward); x overwrites z
        double c = z[0];
        i = 1;
        for (; i + B <= k; i += B) {
            double zv[B], mv[B];
#pragma unroll
            for (int j = 0; j < B; ++j) {
                zv[j] = z[i + j];
                mv[j] = e[i + j] * rp[i + j - 1];
            }
#pragma unroll
            for (int j = 0; j < B; ++j) {
                c = zv[j] - mv[j] * c;
                zv[j] = c;
            }
#pragma unroll
            for (int j = 0; j < B; ++j) z[i + j] = zv[j];
        }
        for (; i < k; ++i) {
            c = z[i] - (e[i] * rp[i - 1]) * c;
            z[i] = c;
        }
        c = z[k - 1] * rp[k - 1];
        z[k - 1] = c;
        double nrm = c * c;
        i = k - 2;
        for (; i - B + 1 >= 0; i -= B) {   // i, i - 1, ..., i - B + 1
            double rv[B], zv[B], ev[B];
#pragma unroll
            for (int j = 0; j < B; ++j) {
                rv[j] = rp[i - j];
                zv[j] = z[i - j];
                ev[j] = e[i - j + 1];
            }
#pragma unroll
            for (int j = 0; j < B; ++j) {
                c = rv[j] * (zv[j] - ev[j] * c);
                zv[j] = c;
                nrm += c * c;
            }
#pragma unroll
            for (int j = 0; j < B; ++j) z[i - j] = zv[j];
        }
        for (; i >= 0; --i) {
            c = rp[i] * (z[i] - e[i + 1] * c);
            z[i] = c;
            nrm += c * c;
        }
        nrm = sqrt(nrm);
        if (!(nrm > 0.0) || !isfinite(nrm)) break;
        const double inv = 1.0 / nrm;
#pragma unroll 8
        for (int t = 0; t < k; ++t) z[t] *= inv;
    }
}

}  // namespace pdz
