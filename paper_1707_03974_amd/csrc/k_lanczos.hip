// Device-resident Lanczos for the lowest eigenvalue of H (the Krylov method
// cited in Sec. I).
//
// Recurrence (FP64 scalars):
//     w = H v_k;  alpha_k = <v_k, w>;  w -= alpha_k v_k + beta_k v_{k-1};
//     [full re-orthogonalisation against v_1..v_k, twice];
//     beta_{k+1} = |w|;  v_{k+1} = w / beta_{k+1}.
// T_k = tridiag(beta, alpha, beta).  Its lowest eigenvalue theta comes from
// Sturm-count multisection, its eigenvector s from inverse iteration, and the
// Ritz pair is accepted when beta_{k+1} |s_k| <= tol |theta|.
//
// Vectors may be stored in FP32 or FP64; every dot product multiplies in FP64
// and accumulates in FP64.  Reductions use a fixed grid and a fixed tree, so
// results are bitwise reproducible run to run.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "pdz_internal.h"
#include "tridiag.h"

namespace pdz {

namespace {

constexpr int kRedBlock = 256;
constexpr int kRedGrid = 1024;   // partial sums per reduction (fixed for determinism)
constexpr int kMaxIter = 2000;
constexpr int kMaxPartials = 4096;   // partial sums a fused H.v dot may write

struct Ctl {
    int k;          // completed Lanczos steps
    int done;       // non-zero: every later kernel of the run is a no-op
    int converged;  // tolerance met or invariant subspace
    int breakdown;  // beta_{k+1} vanished
    double theta;   // lowest Ritz value of T_k
    double resid;   // beta_{k+1} |s_k|
    double norm0;   // norm of the start vector
    double scratch[4];
};

__device__ __forceinline__ double block_sum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kRedBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Seeded start vector: element r of the basis (row r / dn, column r mod dn)
// draws SplitMix64 output r; the vector is stored with row pitch `pitch`
// (n = rows * pitch elements, zeros past column dn).
template <typename T>
__global__ __launch_bounds__(kRedBlock) void k_random_start(T* v, uint64_t n, uint64_t dn, uint64_t pitch,
                                                            uint64_t seed) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t u = i / pitch, d = i - u * pitch;
        v[i] = d < dn ? (T)splitmix_uniform(seed, u * dn + d) : (T)0;
    }
}

// dst (row pitch dp) <- src (row pitch sp), rows of dn elements; n = rows *
// dp destination elements, zeros past column dn.
template <typename TS, typename TD>
__global__ __launch_bounds__(kRedBlock) void k_repitch(const TS* __restrict__ s, uint64_t sp, TD* __restrict__ d,
                                                       uint64_t dp, uint64_t dn, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t u = i / dp, c = i - u * dp;
        d[i] = c < dn ? (TD)s[u * sp + c] : (TD)0;
    }
}

// Columns dn..pitch-1 of every row of `nslots` vectors `stride` elements apart set to zero.
template <typename T>
__global__ __launch_bounds__(kRedBlock) void k_zero_pad(T* v, uint64_t stride, int nslots, uint64_t rows,
                                                        uint64_t dn, uint64_t pitch) {
    const uint64_t w = pitch - dn, per = rows * w, n = per * (uint64_t)nslots;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t sl = i / per, j = i - sl * per, u = j / w;
        v[sl * stride + u * pitch + dn + (j - u * w)] = (T)0;
    }
}

template <typename TS, typename TD>
__global__ __launch_bounds__(kRedBlock) void k_copy(const TS* __restrict__ s, TD* __restrict__ d, uint64_t D) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < D; i += (uint64_t)gridDim.x * blockDim.x)
        d[i] = (TD)s[i];
}

template <typename T>
__global__ __launch_bounds__(kRedBlock) void k_fill_zero(T* v, uint64_t D) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < D; i += (uint64_t)gridDim.x * blockDim.x)
        v[i] = (T)0;
}

__global__ void k_set_step(Ctl* c, int k, int done) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->k = k;
        c->done = done;
    }
}

__global__ void k_clear_bits(uint32_t* err, uint32_t bits) {
    if (threadIdx.x == 0 && blockIdx.x == 0) atomicAnd(err, ~bits);
}

__global__ void k_init_ctl(Ctl* c, double* beta) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->k = 0;
        c->done = 0;
        c->converged = 0;
        c->breakdown = 0;
        c->theta = 0.0;
        c->resid = 0.0;
        c->norm0 = 0.0;
        beta[0] = 0.0;
    }
}

// partial[blockIdx] = sum over the block's strided elements of a[i] * b[i] (FP64)
template <typename TA, typename TB>
__global__ __launch_bounds__(kRedBlock) void k_dot_partial(const TA* __restrict__ a, const TB* __restrict__ b,
                                                           uint64_t D, double* partial, const int* skip) {
    if (skip && *skip) return;
    __shared__ double red[kRedBlock];
    double acc = 0.0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < D; i += (uint64_t)gridDim.x * blockDim.x)
        acc += (double)a[i] * (double)b[i];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

enum FinalMode { kStoreSum = 0, kStoreSqrt = 1 };

// out[index] = sum(partial) or sqrt(sum); index = *kidx + off when kidx != NULL.
__global__ __launch_bounds__(kRedBlock) void k_finalize(const double* partial, int n, double* out, const int* kidx,
                                                        int off, int mode, const int* skip, uint32_t* err) {
    if (skip && *skip) return;
    __shared__ double red[kRedBlock];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partial[i];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) {
        const double v = (mode == kStoreSqrt) ? sqrt(acc) : acc;
        out[(kidx ? *kidx : 0) + off] = v;
        if (!isfinite(v)) atomicOr(err, kErrNonFinite);
    }
}

// v *= 1 / s[*kidx + off]
template <typename T>
__global__ __launch_bounds__(kRedBlock) void k_scale(T* v, uint64_t D, const double* s, const int* kidx, int off,
                                                     const int* skip) {
    if (skip && *skip) return;
    const double inv = 1.0 / s[(kidx ? *kidx : 0) + off];
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < D; i += (uint64_t)gridDim.x * blockDim.x)
        v[i] = (T)((double)v[i] * inv);
}

// w -= alpha_k v + beta_k vprev, partial[] = |w|^2 of the stored result.
template <typename T>
__global__ __launch_bounds__(kRedBlock) void k_update(T* __restrict__ w, const T* __restrict__ v,
                                                      const T* __restrict__ vp, uint64_t D, const double* alpha,
                                                      const double* beta, const int* kidx, double* partial,
                                                      const int* skip) {
    if (skip && *skip) return;
    __shared__ double red[kRedBlock];
    const int k = *kidx;
    const double a = alpha[k], b = beta[k];
    double acc = 0.0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < D; i += (uint64_t)gridDim.x * blockDim.x) {
        const T r = (T)((double)w[i] - a * (double)v[i] - b * (double)vp[i]);
        w[i] = r;
        acc += (double)r * (double)r;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// Three-term recurrence on unnormalised vectors q_j with v_j = sc[j] q_j:
// on entry w + z = H q_k (z: the up-hop part kept apart by the split H.v, or
// NULL); on exit w = H v_k - alpha_k v_k - beta_k v_{k-1}
// = sc[k] w - alpha_k sc[k] q_k - beta_k sc[k-1] q_{k-1}, the next q, with
// partial[] = |w|^2.  No separate normalisation pass: sc[k+1] = 1 / beta_{k+1}.
template <typename T, bool HZ>
__device__ __forceinline__ T update_one(T wi, T zi, T qi, T qpi, double a, double b, double c, double& acc) {
    const T r = lanczos_recurrence<T>(wi, HZ ? zi : T(0), qi, qpi, a, b, c);   // H q_k from its two parts
    acc += (double)r * (double)r;
    return r;
}

// `vec`: every pointer is 16-byte aligned, so the body moves 16-byte vectors,
// two per thread and array in flight; the last D mod (16 / sizeof(T))
// elements go one per thread.  Each block's partial sums a fixed set of
// elements in a fixed order.
constexpr int kUpdBlock = 512;   // 32 waves per CU at kRedGrid work groups: more loads in flight

// Sum over a work group of BLOCK threads (fixed order), valid in thread 0.
template <int BLOCK>
__device__ __forceinline__ double block_sum_waves(double v) {
    __shared__ double ws[BLOCK / 64];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < BLOCK / 64; ++i) t += ws[i];
    return t;
}

// KEEP: the new vector is also stored as slot k + 1 of the kept basis (slots
// of keep_ld elements, keep_cap of them), the copy the refinement combines.
template <typename T, bool HZ, bool KEEP>
__global__ __launch_bounds__(kUpdBlock) void k_update_scaled(T* __restrict__ w, const T* __restrict__ z,
                                                             const T* __restrict__ q, const T* __restrict__ qp,
                                                             uint64_t D, const double* alpha, const double* beta,
                                                             const double* sc, const int* kidx, double* partial,
                                                             const int* skip, int vec, T* __restrict__ keep,
                                                             uint64_t keep_ld, int keep_cap) {
    if (skip && *skip) return;
    const int k = *kidx;
    const double a = sc[k];
    const double b = alpha[k] * sc[k];
    const double c = k > 0 ? beta[k] * sc[k - 1] : 0.0;
    const uint64_t tid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    T* kept = (KEEP && k + 1 < keep_cap) ? keep + (uint64_t)(k + 1) * keep_ld : nullptr;
    double acc = 0.0;
    uint64_t i = tid;
    if (vec) {
        constexpr int N = 16 / sizeof(T);
        typedef T V __attribute__((ext_vector_type(N)));
        V* wv = reinterpret_cast<V*>(w);
        const V* zv = reinterpret_cast<const V*>(z);
        const V* qv = reinterpret_cast<const V*>(q);
        const V* pv = reinterpret_cast<const V*>(qp);
        V* kv = reinterpret_cast<V*>(kept);
        const uint64_t nv = D / N;
        uint64_t j = tid;
        for (; j + stride < nv; j += 2 * stride) {
            const V w0 = wv[j], w1 = wv[j + stride];
            const V q0 = qv[j], q1 = qv[j + stride];
            const V p0 = pv[j], p1 = pv[j + stride];
            V z0 = w0, z1 = w1;
            if (HZ) {
                z0 = zv[j];
                z1 = zv[j + stride];
            }
            V r0, r1;
#pragma unroll
            for (int e = 0; e < N; ++e) r0[e] = update_one<T, HZ>(w0[e], z0[e], q0[e], p0[e], a, b, c, acc);
#pragma unroll
            for (int e = 0; e < N; ++e) r1[e] = update_one<T, HZ>(w1[e], z1[e], q1[e], p1[e], a, b, c, acc);
            wv[j] = r0;
            wv[j + stride] = r1;
            if (KEEP && kv) {
                kv[j] = r0;
                kv[j + stride] = r1;
            }
        }
        if (j < nv) {
            const V w0 = wv[j], q0 = qv[j], p0 = pv[j];
            const V z0 = HZ ? zv[j] : w0;
            V r0;
#pragma unroll
            for (int e = 0; e < N; ++e) r0[e] = update_one<T, HZ>(w0[e], z0[e], q0[e], p0[e], a, b, c, acc);
            wv[j] = r0;
            if (KEEP && kv) kv[j] = r0;
        }
        i = nv * N + tid;   // the ragged tail
    }
    for (; i < D; i += stride) {
        const T r = update_one<T, HZ>(w[i], HZ ? z[i] : T(0), q[i], qp[i], a, b, c, acc);
        w[i] = r;
        if (KEEP && kept) kept[i] = r;
    }
    acc = block_sum_waves<kUpdBlock>(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

template <typename T, bool KEEP>
void launch_update_scaled_k(T* w, const T* z, const T* q, const T* qp, uint64_t D, const double* alpha,
                            const double* beta, const double* sc, const int* kidx, double* partial, const int* skip,
                            hipStream_t s, int vec, T* keep, uint64_t keep_ld, int keep_cap) {
    if (z)
        hipLaunchKernelGGL((k_update_scaled<T, true, KEEP>), dim3(kRedGrid), dim3(kUpdBlock), 0, s, w, z, q, qp, D,
                           alpha, beta, sc, kidx, partial, skip, vec, keep, keep_ld, keep_cap);
    else
        hipLaunchKernelGGL((k_update_scaled<T, false, KEEP>), dim3(kRedGrid), dim3(kUpdBlock), 0, s, w, z, q, qp, D,
                           alpha, beta, sc, kidx, partial, skip, vec, keep, keep_ld, keep_cap);
}

// keep: NULL, or the kept basis (keep_cap slots of keep_ld elements)
template <typename T>
void launch_update_scaled(T* w, const T* z, const T* q, const T* qp, uint64_t D, const double* alpha,
                          const double* beta, const double* sc, const int* kidx, double* partial, const int* skip,
                          hipStream_t s, T* keep = nullptr, uint64_t keep_ld = 0, int keep_cap = 0) {
    auto al = [](const void* x) { return ((uintptr_t)x & 15) == 0; };
    const int vec = al(w) && al(q) && al(qp) && (!z || al(z)) && (!keep || (al(keep) && keep_ld % 4 == 0));
    if (keep)
        launch_update_scaled_k<T, true>(w, z, q, qp, D, alpha, beta, sc, kidx, partial, skip, s, vec, keep, keep_ld,
                                        keep_cap);
    else
        launch_update_scaled_k<T, false>(w, z, q, qp, D, alpha, beta, sc, kidx, partial, skip, s, vec, nullptr, 0, 0);
}

// y = sum_{j < m} (s_j sc_j) Q_j over kept unnormalised vectors, in j order
// (the sums the regenerating refinement forms one vector at a time).
template <typename T>
__global__ __launch_bounds__(kRedBlock) void k_combine_kept(double* __restrict__ y, const T* __restrict__ Q,
                                                            uint64_t ld, uint64_t D, int m, const double* __restrict__ s,
                                                            const double* __restrict__ sc) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < D; i += (uint64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
#pragma unroll 8
        for (int j = 0; j < m; ++j) acc += (s[j] * sc[j]) * (double)Q[(uint64_t)j * ld + i];
        y[i] = acc;
    }
}

// alpha[k] = sc[k]^2 * (sum(p1[0..n1)) + sum(p2[0..n2))): <v_k, H v_k> from
// partial sums of q_k . H q_k.
__global__ __launch_bounds__(kRedBlock) void k_finalize_alpha(const double* p1, int n1, const double* p2, int n2,
                                                              double* alpha, const double* sc, const int* kidx,
                                                              const int* skip, uint32_t* err) {
    if (skip && *skip) return;
    __shared__ double red[kRedBlock];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n1; i += blockDim.x) acc += p1[i];
    for (int i = threadIdx.x; i < n2; i += blockDim.x) acc += p2[i];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) {
        const int k = *kidx;
        const double v = sc[k] * sc[k] * acc;
        alpha[k] = v;
        if (!isfinite(v)) atomicOr(err, kErrNonFinite);
    }
}

// out[b] = sum of in[b], in[b + grid], in[b + 2 grid], ... (fixed order)
__global__ __launch_bounds__(kRedBlock) void k_sum_strided(const double* in, uint64_t n, double* out,
                                                           const int* skip) {
    if (skip && *skip) return;
    __shared__ double red[kRedBlock];
    double acc = 0.0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        acc += in[i];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

// sc[k] = 1 / beta[k] for the step counter k just advanced by k_tridiag.
__global__ void k_next_scale(const double* beta, double* sc, const Ctl* ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && !ctl->done) sc[ctl->k] = 1.0 / beta[ctl->k];
}

// sc[0] = 1 / norm0
__global__ void k_first_scale(double* sc, const Ctl* ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) sc[0] = 1.0 / ctl->norm0;
}

// Full re-orthogonalisation: c_j = <V_j, w> for j < nvec (grid.y = j).
template <typename T>
__global__ __launch_bounds__(kRedBlock) void k_dots_basis(const T* __restrict__ V, uint64_t ld, uint64_t D, int nvec,
                                                          const T* __restrict__ w, double* partial, const int* skip) {
    if (*skip) return;
    const int j = blockIdx.y;
    if (j >= nvec) return;
    __shared__ double red[kRedBlock];
    const T* q = V + (uint64_t)j * ld;
    double acc = 0.0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < D; i += (uint64_t)gridDim.x * blockDim.x)
        acc += (double)q[i] * (double)w[i];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partial[(uint64_t)j * gridDim.x + blockIdx.x] = acc;
}

__global__ __launch_bounds__(kRedBlock) void k_finalize_basis(const double* partial, int n, double* c,
                                                              const int* skip) {
    if (*skip) return;
    __shared__ double red[kRedBlock];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partial[(uint64_t)blockIdx.x * n + i];
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) c[blockIdx.x] = acc;
}

// w -= sum_j c_j V_j
template <typename T>
__global__ __launch_bounds__(kRedBlock) void k_sub_basis(const T* __restrict__ V, uint64_t ld, uint64_t D, int nvec,
                                                         const double* __restrict__ c, T* __restrict__ w,
                                                         const int* skip) {
    if (*skip) return;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < D; i += (uint64_t)gridDim.x * blockDim.x) {
        double acc = (double)w[i];
        for (int j = 0; j < nvec; ++j) acc -= c[j] * (double)V[(uint64_t)j * ld + i];
        w[i] = (T)acc;
    }
}

// y += s_j sc_j v (FP64 y; sc NULL = 1)
template <typename T>
__global__ __launch_bounds__(kRedBlock) void k_axpy_coef(double* __restrict__ y, const T* __restrict__ v, uint64_t D,
                                                         const double* s, const double* sc, int j) {
    const double c = sc ? s[j] * sc[j] : s[j];
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < D; i += (uint64_t)gridDim.x * blockDim.x)
        y[i] += c * (double)v[i];
}

// y = sum_j s_j V_j
template <typename T>
__global__ __launch_bounds__(kRedBlock) void k_combine_basis(double* __restrict__ y, const T* __restrict__ V,
                                                             uint64_t ld, uint64_t D, int m,
                                                             const double* __restrict__ s) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < D; i += (uint64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < m; ++j) acc += s[j] * (double)V[(uint64_t)j * ld + i];
        y[i] = acc;
    }
}

// partial[] = |Hy - theta y|^2, theta = *th
__global__ __launch_bounds__(kRedBlock) void k_resid_partial(const double* __restrict__ hy, const double* __restrict__ y,
                                                             uint64_t D, const double* th, double* partial) {
    __shared__ double red[kRedBlock];
    const double t = *th;
    double acc = 0.0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < D; i += (uint64_t)gridDim.x * blockDim.x) {
        const double r = hy[i] - t * y[i];
        acc += r * r;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// One block: theta = lambda_min(T_k), s = its normalised eigenvector, the
// convergence test, and the step counter.  alpha[0..k-1] is the diagonal,
// beta[1..k-1] the off-diagonal, beta[k] = beta_{k+1}.
__global__ __launch_bounds__(kRedBlock) void k_tridiag(const double* alpha, const double* beta, double* s_out,
                                                       double* theta_hist, Ctl* ctl, double tol, int max_iter,
                                                       uint32_t* err) {
    if (ctl->done) return;
    __shared__ double a[kMaxIter];
    __shared__ double e[kMaxIter];
    __shared__ double zs[kMaxIter];
    __shared__ double rp[kMaxIter];
    __shared__ double lo_s[kRedBlock], hi_s[kRedBlock];
    __shared__ int found;
    __shared__ double bounds[2];
    const int k = ctl->k + 1;
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        a[i] = alpha[i];
        e[i] = (i == 0) ? 0.0 : beta[i];
    }
    __syncthreads();
    double hint_lo = 0.0, hint_hi = 0.0;
    if (k >= 3) ritz_hint(theta_hist[k - 2], theta_hist[k - 3], &hint_lo, &hint_hi);
    tridiag_bracket_min(a, e, k, lo_s, hi_s, &found, bounds, hint_lo, hint_hi);
    if (threadIdx.x == 0) tridiag_min_vector(a, e, k, bounds[0], zs, rp);
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += blockDim.x) s_out[i] = zs[i];
    if (threadIdx.x == 0) {
        const double theta = 0.5 * (bounds[0] + bounds[1]);
        const double bk1 = beta[k];
        const double resid = fabs(bk1 * zs[k - 1]);
        theta_hist[k - 1] = theta;
        ctl->theta = theta;
        ctl->resid = resid;
        ctl->k = k;
        const double scale = fmax(fabs(theta), 1e-300);
        const bool breakdown = !(bk1 > 1e-14 * fmax(1.0, fabs(theta)));
        const bool conv = breakdown || resid <= tol * scale;
        if (!isfinite(theta) || !isfinite(bk1)) {
            atomicOr(err, kErrNonFinite);
            ctl->done = 1;
        }
        if (conv) {
            ctl->converged = 1;
            ctl->breakdown = breakdown ? 1 : 0;
            ctl->done = 1;
        }
        if (k >= max_iter) ctl->done = 1;
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Row pitch of the Lanczos vectors of a real-space table problem: rows of
// 1024 or more elements are padded to a multiple of 32 elements (128 bytes in
// FP32), so that every row starts on a cache line and the up pass's 16-byte
// loads are aligned; 0 (no padding) for shorter rows and the other H.v paths.
uint64_t lanczos_pitch(const pdz_problem_s* p) {
    if (p->hv_path != 0 || p->ks || p->par || p->dn.D < 1024) return 0;
    const uint64_t P = (p->dn.D + 31) / 32 * 32;
    return P == p->dn.D ? 0 : P;
}
// Elements of one Lanczos vector (D, or D_up * pitch).
uint64_t lanczos_len(const pdz_problem_s* p) {
    const uint64_t P = lanczos_pitch(p);
    return P ? p->up.D * P : p->D;
}

struct Layout {
    size_t vec = 0;
    size_t buf[3] = {0, 0, 0};
    size_t basis = 0;
    size_t y = 0, hy = 0;
    size_t alpha = 0, beta = 0, theta = 0, s = 0, sc = 0, partial = 0, partial2 = 0, partial3 = 0, coefs = 0, ctl = 0,
           z = 0;
    size_t total = 0;
    int nvec_basis = 0;
    size_t kept = 0;   // kept Lanczos vectors (keep_basis, three-term path): nkept slots
    int nkept = 0;
    size_t restart = 0;   // workspace of the FP64 restart (refine == 2)
};

// Eigenvalues of the k x k tridiagonal matrix (diagonal a[0..k), off-diagonal
// b[1..k)) below x, by the Sturm count (host, FP64).
int tridiag_count_below(const std::vector<double>& a, const std::vector<double>& b, int k, double x) {
    int c = 0;
    double q = a[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < k; ++i) {
        const double d = q != 0.0 ? q : 1e-300;
        q = a[i] - x - b[i] * b[i] / d;
        if (q < 0) ++c;
    }
    return c;
}

// The j-th smallest eigenvalue (j = 1, 2, ...) of the same matrix by bisection.
double tridiag_kth_host(const std::vector<double>& a, const std::vector<double>& b, int k, int j) {
    double lo = a[0], hi = a[0];
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(b[i]) : 0.0) + (i + 1 < k ? std::fabs(b[i + 1]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(lo) + std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (tridiag_count_below(a, b, k, mid) >= j) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// refine == 2 decision.  The Rayleigh quotient E of the Ritz vector with FP64
// residual r is within r^2 / gap of the eigenvalue, gap the distance to the
// next distinct eigenvalue.  Estimate: the first eigenvalue of T_k above the
// cluster of Ritz values within 1e-8 max(1, |theta_1|) of theta_1 (copies
// of theta_1 are ghosts of the same eigenvalue, or a degenerate level),
// divided by 10 since a Ritz value lies above the eigenvalue it approximates
// (Cauchy interlacing), so theta_next - theta_1 can exceed the true gap.
// No Ritz value above the cluster: the gap is unknown and the restart runs.
// Returns 1 when the FP64 restart must run; *gap_out receives the estimate
// (0 when unknown).
int refine_restart_needed(const std::vector<double>& a, const std::vector<double>& b, int k, double E, double r,
                          double* gap_out) {
    *gap_out = 0.0;
    if (k < 1) return 1;
    const double th1 = tridiag_kth_host(a, b, k, 1);
    const double delta = 1e-8 * std::max(1.0, std::fabs(th1));
    const int m = tridiag_count_below(a, b, k, th1 + delta);
    if (m >= k) return 1;
    const double gap = (tridiag_kth_host(a, b, k, m + 1) - th1) / 10.0;
    if (!(gap > 0.0) || !std::isfinite(gap)) return 1;
    *gap_out = gap;
    return r * r > 1e-8 * std::fabs(E) * gap ? 1 : 0;
}

// Options of the FP64 Lanczos restart from the Ritz vector (refine == 2).
pdz_lanczos_opts restart_opts(const pdz_lanczos_opts* o) {
    pdz_lanczos_opts r = *o;
    r.storage = PDZ_F64;
    r.reorth = 0;
    r.refine = 1;
    r.keep_basis = 0;
    r.tol = o->tol > 1e-12 ? o->tol : 1e-12;
    r.max_iter = o->max_iter > 300 ? o->max_iter : 300;
    return r;
}

Layout make_layout(const pdz_problem_s* p, const pdz_lanczos_opts* o) {
    const uint64_t D = lanczos_len(p);
    Layout L;
    const size_t es = o->storage == PDZ_F64 ? 8 : 4;
    L.vec = align256((size_t)D * es);
    size_t off = 0;
    if (o->reorth) {
        L.nvec_basis = o->max_iter + 1;
        L.basis = off;
        off += L.vec * (size_t)L.nvec_basis;
        L.buf[0] = off;   // zero vector for v_0
        off += L.vec;
    } else {
        for (int i = 0; i < 3; ++i) {
            L.buf[i] = off;
            off += L.vec;
        }
        L.z = off;   // up-hop part of H q_k
        off += L.vec;
        if (o->keep_basis) {
            L.nkept = o->max_iter + 1;
            L.kept = off;
            off += L.vec * (size_t)L.nkept;
        }
    }
    if (o->refine) {
        L.y = off;
        off += align256((size_t)D * 8);
        L.hy = off;
        off += align256((size_t)D * 8);
    }
    const size_t m = (size_t)o->max_iter + 8;
    L.alpha = off;
    off += align256(m * 8);
    L.beta = off;
    off += align256(m * 8);
    L.theta = off;
    off += align256(2 * m * 8);
    L.s = off;
    off += align256(m * 8);
    L.sc = off;
    off += align256(m * 8);
    L.partial = off;
    off += align256(std::max<size_t>(std::max<size_t>(std::max<size_t>((size_t)kRedGrid * (o->reorth ? m : 1),
                                                                          kMaxPartials),
                                                      hv_dot_count_max(p, (pdz_dtype)o->storage)),
                                     (size_t)parity_dot_count(p, (pdz_dtype)o->storage)) *
                    8);
    L.partial2 = off;
    off += align256((size_t)kRedGrid * 8);
    L.partial3 = off;   // |q_{k+1}|^2 per work group of the fused pass
    off += align256((size_t)kMaxPartials * 8);
    L.coefs = off;
    off += align256(m * 8);
    L.ctl = off;
    off += align256(sizeof(Ctl));
    if (o->refine == 2) {
        const pdz_lanczos_opts r = restart_opts(o);
        L.restart = off;
        off += align256(make_layout(p, &r).total);
    }
    L.total = off;
    return L;
}

unsigned grid_elems(uint64_t D) {
    uint64_t g = (D + kRedBlock - 1) / kRedBlock;
    if (g > (uint64_t)kRedGrid * 4) g = (uint64_t)kRedGrid * 4;
    return (unsigned)(g < 1 ? 1 : g);
}

template <typename T>
struct Run {
    const pdz_problem_s* p;
    const pdz_lanczos_opts* o;
    Layout L;
    char* ws;
    hipStream_t s;
    uint32_t* err;
    uint64_t D;              // elements of one vector (with the row padding)
    uint64_t pitch = 0;      // row pitch of the vectors, 0: unpadded (D elements, the basis order)
    bool v0_pitched = false; // v0 is already in the padded layout (the FP64 restart from y)
    T* buf(int i) const { return reinterpret_cast<T*>(ws + L.buf[i]); }
    T* basis(int j) const { return reinterpret_cast<T*>(ws + L.basis + (size_t)j * L.vec); }
    T* kept(int j) const { return L.nkept ? reinterpret_cast<T*>(ws + L.kept + (size_t)j * L.vec) : nullptr; }
    uint64_t ld() const { return L.vec / sizeof(T); }
    double* y() const { return reinterpret_cast<double*>(ws + L.y); }
    double* hy() const { return reinterpret_cast<double*>(ws + L.hy); }
    double* alpha() const { return reinterpret_cast<double*>(ws + L.alpha); }
    double* beta() const { return reinterpret_cast<double*>(ws + L.beta); }
    double* theta() const { return reinterpret_cast<double*>(ws + L.theta); }
    double* svec() const { return reinterpret_cast<double*>(ws + L.s); }
    double* sc() const { return reinterpret_cast<double*>(ws + L.sc); }
    double* partial2() const { return reinterpret_cast<double*>(ws + L.partial2); }
    double* partial3() const { return reinterpret_cast<double*>(ws + L.partial3); }
    T* zbuf() const { return reinterpret_cast<T*>(ws + L.z); }
    double* partial() const { return reinterpret_cast<double*>(ws + L.partial); }
    double* coefs() const { return reinterpret_cast<double*>(ws + L.coefs); }
    Ctl* ctl() const { return reinterpret_cast<Ctl*>(ws + L.ctl); }
    int* done() const { return &ctl()->done; }
    int* kptr() const { return &ctl()->k; }

    // Optional HIP events recorded between the launches of one step (timing).
    hipEvent_t* ev = nullptr;
    void mark(int i) {
        if (ev) (void)hipEventRecord(ev[i], s);
    }

    pdz_status launch_check() {
        PDZ_HIP(hipGetLastError());
        return ok();
    }

    // v_1 = v0 / |v0| into dst; zero vector into zero_dst.  scaled: keep
    // dst = v0 unnormalised and set sc[0] = 1 / |v0| instead.
    pdz_status start(const void* v0, T* dst, T* zero_dst, bool scaled) {
        const unsigned g = grid_elems(D);
        hipLaunchKernelGGL(k_clear_bits, dim3(1), dim3(1), 0, s, err, kErrNonFinite);
        hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(1), 0, s, ctl(), beta());
        const uint64_t dn = p->dn.D, rp = pitch ? pitch : dn;
        if (pitch) {
            // the H.v passes write columns below D_dn only: the padding of every vector they
            // write starts at zero and stays zero
            if (o->reorth)
                hipLaunchKernelGGL(k_zero_pad<T>, dim3(g), dim3(kRedBlock), 0, s, basis(0), ld(), L.nvec_basis,
                                   p->up.D, dn, pitch);
            hipLaunchKernelGGL(k_zero_pad<T>, dim3(g), dim3(kRedBlock), 0, s, buf(0), ld(), o->reorth ? 1 : 3,
                               p->up.D, dn, pitch);
            if (L.z)
                hipLaunchKernelGGL(k_zero_pad<T>, dim3(g), dim3(kRedBlock), 0, s, zbuf(), ld(), 1, p->up.D, dn,
                                   pitch);
            if (o->refine)
                hipLaunchKernelGGL(k_zero_pad<double>, dim3(g), dim3(kRedBlock), 0, s, hy(), (uint64_t)0, 1, p->up.D,
                                   dn, pitch);
        }
        if (v0 && (v0_pitched || !pitch))
            hipLaunchKernelGGL((k_copy<T, T>), dim3(g), dim3(kRedBlock), 0, s, static_cast<const T*>(v0), dst, D);
        else if (v0)
            hipLaunchKernelGGL((k_repitch<T, T>), dim3(g), dim3(kRedBlock), 0, s, static_cast<const T*>(v0), dn, dst,
                               pitch, dn, D);
        else
            hipLaunchKernelGGL(k_random_start<T>, dim3(g), dim3(kRedBlock), 0, s, dst, D, dn, rp, (uint64_t)o->seed);
        hipLaunchKernelGGL(k_fill_zero<T>, dim3(g), dim3(kRedBlock), 0, s, zero_dst, D);
        hipLaunchKernelGGL((k_dot_partial<T, T>), dim3(kRedGrid), dim3(kRedBlock), 0, s, dst, dst, D, partial(),
                           (const int*)nullptr);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedBlock), 0, s, partial(), kRedGrid, &ctl()->norm0,
                           (const int*)nullptr, 0, (int)kStoreSqrt, (const int*)nullptr, err);
        pdz_status st = launch_check();
        if (st != PDZ_OK) return st;
        Ctl h;
        PDZ_HIP(hipMemcpyAsync(&h, ctl(), sizeof(Ctl), hipMemcpyDeviceToHost, s));
        PDZ_HIP(hipStreamSynchronize(s));
        if (!(h.norm0 > 0.0) || !std::isfinite(h.norm0))
            return fail(PDZ_EINVAL, "start vector has zero or non-finite norm");
        if (scaled && kept(0))
            hipLaunchKernelGGL((k_copy<T, T>), dim3(g), dim3(kRedBlock), 0, s, dst, kept(0), D);
        if (scaled)
            hipLaunchKernelGGL(k_first_scale, dim3(1), dim3(1), 0, s, sc(), ctl());
        else
            hipLaunchKernelGGL(k_scale<T>, dim3(g), dim3(kRedBlock), 0, s, dst, D, &ctl()->norm0, (const int*)nullptr,
                               0, (const int*)nullptr);
        return launch_check();
    }

    // Split H.v layout of this run: partial-sum counts of its two passes
    // (ndn = 0: the on-the-fly path, which takes a separate dot kernel).
    // nwhole: partial sums of q . H q that the whole (unsplit) H.v writes (parity).
    struct SplitCounts {
        int ndn = 0, nup = 0, nwhole = 0;
    };
    SplitCounts split_counts() const {
        SplitCounts c;
        if (!hv_dot_counts(p, (pdz_dtype)o->storage, &c.ndn, &c.nup)) c.ndn = c.nup = 0;
        c.nwhole = parity_dot_count(p, (pdz_dtype)o->storage);
        return c;
    }

    // One step of the three-term recurrence on unnormalised vectors (v_k =
    // sc[k] q_k): q = q_k, qp = q_{k-1}, w receives q_{k+1}.  H q_k comes in
    // two parts (w: diagonal + down hops, z: up hops) that the update adds;
    // alpha comes from partial sums of q . (each part) written by the two
    // passes of H.v, so no pass re-reads a D-sized vector for them.
    pdz_status step_scaled(T* q, T* qp, T* w, const SplitCounts& c) {
        mark(0);
        if (c.ndn > 0) {
            HvSplit sd;   // down pass (no z: it would be cleared after a down-only launch)
            sd.dotp_dn = partial();
            pdz_status st = launch_hv_any(p, (pdz_dtype)o->storage, q, w, s, done(), kPassDown, &sd, pitch);
            if (st != PDZ_OK) return st;
            mark(1);
            HvSplit su;
            su.z = zbuf();
            su.dotp_up = partial() + c.ndn;
            st = launch_hv_any(p, (pdz_dtype)o->storage, q, w, s, done(), kPassUp, &su, pitch);
            if (st != PDZ_OK) return st;
            mark(2);
            hipLaunchKernelGGL(k_sum_strided, dim3(kRedGrid), dim3(kRedBlock), 0, s, partial() + c.ndn,
                               (uint64_t)c.nup, partial2(), done());
            hipLaunchKernelGGL(k_finalize_alpha, dim3(1), dim3(kRedBlock), 0, s, partial(), c.ndn, partial2(),
                               (int)kRedGrid, alpha(), sc(), kptr(), done(), err);
        } else if (c.nwhole > 0) {   // the H.v writes partial sums of q . H q
            HvSplit sw;
            sw.dotp_up = partial();
            pdz_status st = launch_hv_any(p, (pdz_dtype)o->storage, q, w, s, done(), kPassDown | kPassUp, &sw, pitch);
            if (st != PDZ_OK) return st;
            mark(1);
            mark(2);
            hipLaunchKernelGGL(k_sum_strided, dim3(kRedGrid), dim3(kRedBlock), 0, s, partial(), (uint64_t)c.nwhole,
                               partial2(), done());
            hipLaunchKernelGGL(k_finalize_alpha, dim3(1), dim3(kRedBlock), 0, s, partial(), 0, partial2(),
                               (int)kRedGrid, alpha(), sc(), kptr(), done(), err);
        } else {
            pdz_status st = launch_hv_any(p, (pdz_dtype)o->storage, q, w, s, done(), kPassDown | kPassUp, nullptr, pitch);
            if (st != PDZ_OK) return st;
            mark(1);
            mark(2);
            hipLaunchKernelGGL((k_dot_partial<T, T>), dim3(kRedGrid), dim3(kRedBlock), 0, s, q, w, D, partial(),
                               done());
            hipLaunchKernelGGL(k_finalize_alpha, dim3(1), dim3(kRedBlock), 0, s, partial(), (int)kRedGrid,
                               (const double*)nullptr, 0, alpha(), sc(), kptr(), done(), err);
        }
        mark(3);
        launch_update_scaled<T>(w, c.ndn > 0 ? (const T*)zbuf() : (const T*)nullptr, q, qp, D, alpha(), beta(), sc(),
                                kptr(), partial(), done(), s, kept(0), ld(), L.nkept);
        mark(4);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedBlock), 0, s, partial(), kRedGrid, beta(), kptr(), 1,
                           (int)kStoreSqrt, done(), err);
        hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(kRedBlock), 0, s, alpha(), beta(), svec(), theta(), ctl(), o->tol,
                           o->max_iter, err);
        hipLaunchKernelGGL(k_next_scale, dim3(1), dim3(1), 0, s, beta(), sc(), ctl());
        mark(5);
        return launch_check();
    }

    // The two passes of H q_k and alpha_k (the first half of step_scaled).
    pdz_status head_step(T* q, T* w, const SplitCounts& c) {
        if (p->par) {   // the whole H q_0 into w, alpha_0 from its x . y partials
            HvSplit sw;
            sw.dotp_up = partial();
            pdz_status st = launch_hv_any(p, (pdz_dtype)o->storage, q, w, s, done(), kPassDown | kPassUp, &sw, pitch);
            if (st != PDZ_OK) return st;
            hipLaunchKernelGGL(k_sum_strided, dim3(kRedGrid), dim3(kRedBlock), 0, s, partial(), (uint64_t)c.nwhole,
                               partial2(), done());
            hipLaunchKernelGGL(k_finalize_alpha, dim3(1), dim3(kRedBlock), 0, s, partial(), 0, partial2(),
                               (int)kRedGrid, alpha(), sc(), kptr(), done(), err);
            return launch_check();
        }
        HvSplit sp;
        sp.z = zbuf();
        sp.dotp_dn = partial();
        sp.dotp_up = partial() + c.ndn;
        pdz_status st = launch_hv_any(p, (pdz_dtype)o->storage, q, w, s, done(), kPassDown | kPassUp, &sp, pitch);
        if (st != PDZ_OK) return st;
        hipLaunchKernelGGL(k_sum_strided, dim3(kRedGrid), dim3(kRedBlock), 0, s, partial() + c.ndn, (uint64_t)c.nup,
                           partial2(), done());
        hipLaunchKernelGGL(k_finalize_alpha, dim3(1), dim3(kRedBlock), 0, s, partial(), c.ndn, partial2(),
                           (int)kRedGrid, alpha(), sc(), kptr(), done(), err);
        return launch_check();
    }

    // The same step as the update of step_scaled followed by the next step's
    // H.v and alpha, with the update carried out by the down pass while it
    // stages its rows: q1 = q_k, q2 = q_{k-1} (receives q_{k+1}), w = down
    // part of H q_k (receives that of H q_{k+1}), zbuf = up part of H q_k
    // (receives that of H q_{k+1}).  Between the two passes: beta_{k+1}, the
    // tridiagonal solve of T_{k+1} and sc[k+1], as in step_scaled.
    pdz_status fused_step(T* q1, T* q2, T* w, const SplitCounts& c) {
        if (p->par) return fused_step_parity(q1, q2, w, c);
        mark(0);
        HvSplit f;
        f.dotp_dn = partial();
        f.fq1 = q1;
        f.fq2 = q2;
        f.fz = zbuf();
        f.fkeep = kept(0);
        f.fkeep_ld = ld();
        f.fkeep_cap = L.nkept;
        f.falpha = alpha();
        f.fbeta = beta();
        f.fsc = sc();
        f.fkidx = kptr();
        f.fnorm = partial3();
        pdz_status st = launch_hv_any(p, (pdz_dtype)o->storage, q2, w, s, done(), kPassDown, &f, pitch);
        if (st != PDZ_OK) return st;
        mark(1);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedBlock), 0, s, partial3(), c.ndn, beta(), kptr(), 1,
                           (int)kStoreSqrt, done(), err);
        hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(kRedBlock), 0, s, alpha(), beta(), svec(), theta(), ctl(), o->tol,
                           o->max_iter, err);
        hipLaunchKernelGGL(k_next_scale, dim3(1), dim3(1), 0, s, beta(), sc(), ctl());
        mark(2);
        HvSplit u;
        u.z = zbuf();
        u.dotp_up = partial() + c.ndn;
        st = launch_hv_any(p, (pdz_dtype)o->storage, q2, w, s, done(), kPassUp, &u, pitch);
        if (st != PDZ_OK) return st;
        mark(3);
        hipLaunchKernelGGL(k_sum_strided, dim3(kRedGrid), dim3(kRedBlock), 0, s, partial() + c.ndn, (uint64_t)c.nup,
                           partial2(), done());
        hipLaunchKernelGGL(k_finalize_alpha, dim3(1), dim3(kRedBlock), 0, s, partial(), c.ndn, partial2(),
                           (int)kRedGrid, alpha(), sc(), kptr(), done(), err);
        mark(4);
        mark(5);
        return launch_check();
    }

    // fused_step on a parity subspace, whose H.v keeps its parts in y: w holds
    // the whole H q_k; the down pass forms q_{k+1} (over q2, the palindromic
    // rows included) and overwrites w with the down part of H q_{k+1}, to which
    // the up pass adds the rest (the palindromic rows whole), writing the x . y
    // partials of alpha_{k+1}.
    pdz_status fused_step_parity(T* q1, T* q2, T* w, const SplitCounts& c) {
        const pdz_dtype dt = (pdz_dtype)o->storage;
        mark(0);
        HvSplit f;
        f.fq1 = q1;
        f.fq2 = q2;
        f.fkeep = kept(0);
        f.fkeep_ld = ld();
        f.fkeep_cap = L.nkept;
        f.falpha = alpha();
        f.fbeta = beta();
        f.fsc = sc();
        f.fkidx = kptr();
        f.fnorm = partial3();
        pdz_status st = launch_hv_any(p, dt, q2, w, s, done(), kPassDown, &f);
        if (st != PDZ_OK) return st;
        mark(1);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedBlock), 0, s, partial3(), parity_fused_norms(p, dt), beta(),
                           kptr(), 1, (int)kStoreSqrt, done(), err);
        hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(kRedBlock), 0, s, alpha(), beta(), svec(), theta(), ctl(), o->tol,
                           o->max_iter, err);
        hipLaunchKernelGGL(k_next_scale, dim3(1), dim3(1), 0, s, beta(), sc(), ctl());
        mark(2);
        HvSplit u;
        u.dotp_up = partial();
        st = launch_hv_any(p, dt, q2, w, s, done(), kPassUp, &u);
        if (st != PDZ_OK) return st;
        mark(3);
        hipLaunchKernelGGL(k_sum_strided, dim3(kRedGrid), dim3(kRedBlock), 0, s, partial(), (uint64_t)c.nwhole,
                           partial2(), done());
        hipLaunchKernelGGL(k_finalize_alpha, dim3(1), dim3(kRedBlock), 0, s, partial(), 0, partial2(), (int)kRedGrid,
                           alpha(), sc(), kptr(), done(), err);
        mark(4);
        mark(5);
        return launch_check();
    }

    // Mean duration of each launch group over `steps` Lanczos steps from the
    // seeded start, stream launches with events between the groups.
    // ms[0] down pass (fused with the update on the fused path), ms[1] up
    // pass, ms[2] separate update (0 on the fused path), ms[3] scalar
    // kernels, ms[4] whole step.
    pdz_status timed_steps(int steps, double* ms, int* fused_out) {
        const bool fuse = fused_path();
        const SplitCounts counts = split_counts();
        pdz_status st = start(nullptr, buf(0), fuse ? buf(1) : buf(2), true);
        if (st != PDZ_OK) return st;
        if (fuse) {
            st = head_step(buf(0), buf(2), counts);
            if (st != PDZ_OK) return st;
        }
        hipEvent_t e[6];
        for (int i = 0; i < 6; ++i) PDZ_HIP(hipEventCreate(&e[i]));
        double acc[6] = {0, 0, 0, 0, 0, 0};
        ev = e;
        for (int t = 0; t < steps && st == PDZ_OK; ++t) {
            if (fuse) {
                const int a = t % 2;
                st = fused_step(buf(a), buf(1 - a), buf(2), counts);
            } else {
                const int a = t % 3;
                st = step_scaled(buf(a), buf((a + 2) % 3), buf((a + 1) % 3), counts);
            }
            if (st != PDZ_OK) break;
            hipError_t he = hipEventSynchronize(e[5]);
            float f[5];
            for (int i = 0; i < 5 && he == hipSuccess; ++i) he = hipEventElapsedTime(&f[i], e[i], e[i + 1]);
            if (he != hipSuccess) {
                st = hip_fail(he, "Lanczos step timing");
                break;
            }
            for (int i = 0; i < 5; ++i) acc[i] += f[i];
        }
        ev = nullptr;
        for (int i = 0; i < 6; ++i) (void)hipEventDestroy(e[i]);
        if (st != PDZ_OK) return st;
        const double n = steps > 0 ? steps : 1;
        if (fuse) {   // marks: 0 P 1 scalars 2 U 3 scalars 4 (5 = 4)
            ms[0] = acc[0] / n;
            ms[1] = acc[2] / n;
            ms[2] = 0.0;
            ms[3] = (acc[1] + acc[3]) / n;
        } else {      // marks: 0 D 1 U 2 scalars 3 update 4 scalars 5
            ms[0] = acc[0] / n;
            ms[1] = acc[1] / n;
            ms[2] = acc[3] / n;
            ms[3] = (acc[2] + acc[4]) / n;
        }
        ms[4] = (acc[0] + acc[1] + acc[2] + acc[3] + acc[4]) / n;
        *fused_out = fuse ? 1 : 0;
        return ok();
    }

    // One Lanczos step with v = v_k, vp = v_{k-1}, w the output slot.
    // rn > 0: re-orthogonalise w (classical Gram-Schmidt, twice) against the
    // rn consecutive basis slots from basis(rfirst): every earlier vector for
    // full re-orthogonalisation, v_{k-1} and v_k for local.
    pdz_status step(T* v, T* vp, T* w, int rfirst, int rn) {
        const unsigned g = grid_elems(D);
        pdz_status st = launch_hv_any(p, (pdz_dtype)o->storage, v, w, s, done(), kPassDown | kPassUp, nullptr, pitch);
        if (st != PDZ_OK) return st;
        hipLaunchKernelGGL((k_dot_partial<T, T>), dim3(kRedGrid), dim3(kRedBlock), 0, s, v, w, D, partial(), done());
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedBlock), 0, s, partial(), kRedGrid, alpha(), kptr(), 0,
                           (int)kStoreSum, done(), err);
        hipLaunchKernelGGL(k_update<T>, dim3(kRedGrid), dim3(kRedBlock), 0, s, w, v, vp, D, alpha(), beta(), kptr(),
                           partial(), done());
        if (rn > 0) {
            for (int pass = 0; pass < 2; ++pass) {
                hipLaunchKernelGGL(k_dots_basis<T>, dim3(kRedGrid, rn), dim3(kRedBlock), 0, s, basis(rfirst), ld(), D,
                                   rn, w, partial(), done());
                hipLaunchKernelGGL(k_finalize_basis, dim3(rn), dim3(kRedBlock), 0, s, partial(), kRedGrid, coefs(),
                                   done());
                hipLaunchKernelGGL(k_sub_basis<T>, dim3(g), dim3(kRedBlock), 0, s, basis(rfirst), ld(), D, rn, coefs(),
                                   w, done());
            }
            hipLaunchKernelGGL((k_dot_partial<T, T>), dim3(kRedGrid), dim3(kRedBlock), 0, s, w, w, D, partial(), done());
        }
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedBlock), 0, s, partial(), kRedGrid, beta(), kptr(), 1,
                           (int)kStoreSqrt, done(), err);
        hipLaunchKernelGGL(k_tridiag, dim3(1), dim3(kRedBlock), 0, s, alpha(), beta(), svec(), theta(), ctl(), o->tol,
                           o->max_iter, err);
        hipLaunchKernelGGL(k_scale<T>, dim3(g), dim3(kRedBlock), 0, s, w, D, beta(), kptr(), 0, done());
        return launch_check();
    }

    // The update rides on the down pass when the plan's down pass is the
    // looped wide kernel (the split H.v is available there too).
    bool fused_path() const {
        if (o->reorth) return false;
        const SplitCounts c = split_counts();
        if (p->par) {
            // parity: the recurrence rides on its down pass (two-pass form) in
            // FP64 storage, and in FP32 where that pass is the gather-scheduled
            // one; the looped FP32 pass (two rows share a CU) is faster with
            // the separate update
            const int nn = parity_fused_norms(p, (pdz_dtype)o->storage);
            const bool f32 = parity_sched_down(p, (pdz_dtype)o->storage);
            return (o->storage == PDZ_F64 || f32) && nn > 0 && nn <= kMaxPartials && c.nwhole > 0;
        }
        return c.ndn > 0 && c.ndn <= kMaxPartials && hv_fused_available(p, (pdz_dtype)o->storage);
    }

    pdz_status read_ctl(Ctl* h) {
        PDZ_HIP(hipMemcpyAsync(h, ctl(), sizeof(Ctl), hipMemcpyDeviceToHost, s));
        PDZ_HIP(hipStreamSynchronize(s));
        return ok();
    }

    pdz_status iterate(Ctl* h) {
        pdz_status st;
        if (o->reorth) {
            for (int k = 1; k <= o->max_iter; ++k) {
                // v_k = basis(k-1), v_{k-1} = basis(k-2) or the zero vector, w -> basis(k)
                T* vp = (k >= 2) ? basis(k - 2) : buf(0);
                // full (2): against v_0 .. v_{k-1}; local (1): against v_{k-2}, v_{k-1}
                const int rfirst = o->reorth == 2 ? 0 : (k >= 2 ? k - 2 : 0);
                const int rn = o->reorth == 2 ? k : (k >= 2 ? 2 : 1);
                st = step(basis(k - 1), vp, basis(k), rfirst, rn);
                if (st != PDZ_OK) return st;
                if (k % o->check_every == 0 || k == o->max_iter) {
                    st = read_ctl(h);
                    if (st != PDZ_OK) return st;
                    if (h->done) return ok();
                }
            }
            return read_ctl(h);
        }
        const SplitCounts counts = split_counts();
        // fused: q_k alternates between buf(0) and buf(1) (the update runs in
        // place over q_{k-1}), buf(2) holds the down part of H q_k; after the
        // first H.v, every step is one fused_step.  Otherwise three rotating
        // buffers.  A block of `period` steps keeps the rotation aligned.
        const bool fuse = fused_path();
        int period = o->check_every;
        const int rot = fuse ? 2 : 3;
        if (period % rot) period += rot - period % rot;
        if (fuse) {
            st = head_step(buf(0), buf(2), counts);
            if (st != PDZ_OK) return st;
        }
        auto enqueue_block = [&]() -> pdz_status {
            for (int t = 0; t < period; ++t) {
                pdz_status s2;
                if (fuse) {
                    const int a = t % 2;
                    s2 = fused_step(buf(a), buf(1 - a), buf(2), counts);
                } else {
                    const int a = t % 3;
                    s2 = step_scaled(buf(a), buf((a + 2) % 3), buf((a + 1) % 3), counts);
                }
                if (s2 != PDZ_OK) return s2;
            }
            return ok();
        };
        hipGraphExec_t exec = nullptr;
        hipGraph_t graph = nullptr;
        if (o->use_graph) {
            PDZ_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            st = enqueue_block();
            hipGraph_t g2 = nullptr;
            hipError_t e = hipStreamEndCapture(s, &g2);
            if (st != PDZ_OK) {
                if (g2) (void)hipGraphDestroy(g2);
                return st;
            }
            if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
            graph = g2;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(graph);
                return hip_fail(e, "hipGraphInstantiate");
            }
        }
        st = ok();
        for (int done_steps = 0; done_steps < o->max_iter; done_steps += period) {
            if (exec) {
                hipError_t e = hipGraphLaunch(exec, s);
                if (e != hipSuccess) {
                    st = hip_fail(e, "hipGraphLaunch");
                    break;
                }
            } else {
                st = enqueue_block();
                if (st != PDZ_OK) break;
            }
            st = read_ctl(h);
            if (st != PDZ_OK || h->done) break;
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (st != PDZ_OK) return st;
        return read_ctl(h);
    }

    // Ritz vector y = sum_j s_j v_j (FP64), normalised; FP64 Rayleigh quotient and residual.
    pdz_status refine(const void* v0, int m, double* E_ref, double* r_ref) {
        const unsigned g = grid_elems(D);
        if (o->reorth) {
            hipLaunchKernelGGL(k_combine_basis<T>, dim3(g), dim3(kRedBlock), 0, s, y(), basis(0), ld(), D, m, svec());
        } else if (kept(0) && m <= L.nkept) {
            hipLaunchKernelGGL(k_combine_kept<T>, dim3(g), dim3(kRedBlock), 0, s, y(), kept(0), ld(), D, m, svec(),
                               sc());
        } else {
            // regenerate v_1..v_m with the same kernels and the stored alpha, beta
            Ctl saved;
            pdz_status st = read_ctl(&saved);
            if (st != PDZ_OK) return st;
            std::vector<double> alpha_h(m + 1), beta_h(m + 2), sc_h(m + 1);
            PDZ_HIP(hipMemcpyAsync(alpha_h.data(), alpha(), (size_t)m * 8, hipMemcpyDeviceToHost, s));
            PDZ_HIP(hipMemcpyAsync(beta_h.data(), beta(), (size_t)(m + 1) * 8, hipMemcpyDeviceToHost, s));
            PDZ_HIP(hipMemcpyAsync(sc_h.data(), sc(), (size_t)m * 8, hipMemcpyDeviceToHost, s));
            PDZ_HIP(hipStreamSynchronize(s));
            st = start(v0, buf(0), buf(2), true);
            if (st != PDZ_OK) return st;
            // restore the recurrence coefficients overwritten by start()
            PDZ_HIP(hipMemcpyAsync(alpha(), alpha_h.data(), (size_t)m * 8, hipMemcpyHostToDevice, s));
            PDZ_HIP(hipMemcpyAsync(beta(), beta_h.data(), (size_t)(m + 1) * 8, hipMemcpyHostToDevice, s));
            PDZ_HIP(hipMemcpyAsync(sc(), sc_h.data(), (size_t)m * 8, hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_fill_zero<double>, dim3(g), dim3(kRedBlock), 0, s, y(), D);
            const SplitCounts counts = split_counts();
            for (int j = 0; j < m; ++j) {
                const int a = j % 3;
                T* q = buf(a);
                T* qp = buf((a + 2) % 3);
                T* w = buf((a + 1) % 3);
                hipLaunchKernelGGL(k_axpy_coef<T>, dim3(g), dim3(kRedBlock), 0, s, y(), q, D, svec(), sc(), j);
                if (j + 1 < m) {
                    // the step kernels read alpha/beta/sc at index *kptr: set k = j on the device
                    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, s, ctl(), j, 0);
                    HvSplit sp;
                    sp.z = zbuf();
                    st = launch_hv_any(p, (pdz_dtype)o->storage, q, w, s, nullptr, kPassDown | kPassUp,
                                       counts.ndn > 0 ? &sp : nullptr, pitch);
                    if (st != PDZ_OK) return st;
                    launch_update_scaled<T>(w, counts.ndn > 0 ? (const T*)zbuf() : (const T*)nullptr, q, qp, D,
                                            alpha(), beta(), sc(), kptr(), partial(), (const int*)nullptr, s);
                }
            }
            hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, s, ctl(), saved.k, saved.done);
        }
        double* scr = &ctl()->scratch[0];
        hipLaunchKernelGGL((k_dot_partial<double, double>), dim3(kRedGrid), dim3(kRedBlock), 0, s, y(), y(), D,
                           partial(), (const int*)nullptr);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedBlock), 0, s, partial(), kRedGrid, scr, (const int*)nullptr, 0,
                           (int)kStoreSqrt, (const int*)nullptr, err);
        hipLaunchKernelGGL(k_scale<double>, dim3(g), dim3(kRedBlock), 0, s, y(), D, scr, (const int*)nullptr, 0,
                           (const int*)nullptr);
        pdz_status st = launch_hv_any(p, PDZ_F64, y(), hy(), s, nullptr, kPassDown | kPassUp, nullptr, pitch);
        if (st != PDZ_OK) return st;
        hipLaunchKernelGGL((k_dot_partial<double, double>), dim3(kRedGrid), dim3(kRedBlock), 0, s, y(), hy(), D,
                           partial(), (const int*)nullptr);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedBlock), 0, s, partial(), kRedGrid, scr + 1,
                           (const int*)nullptr, 0, (int)kStoreSum, (const int*)nullptr, err);
        hipLaunchKernelGGL(k_resid_partial, dim3(kRedGrid), dim3(kRedBlock), 0, s, hy(), y(), D, scr + 1, partial());
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kRedBlock), 0, s, partial(), kRedGrid, scr + 2,
                           (const int*)nullptr, 0, (int)kStoreSqrt, (const int*)nullptr, err);
        st = launch_check();
        if (st != PDZ_OK) return st;
        double h[3];
        PDZ_HIP(hipMemcpyAsync(h, scr, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        PDZ_HIP(hipStreamSynchronize(s));
        *E_ref = h[1];
        *r_ref = h[2];
        return ok();
    }

    pdz_status run(const void* v0, double* ritz_out, pdz_lanczos_result* res) {
        T* v1 = o->reorth ? basis(0) : buf(0);
        T* zero = o->reorth ? buf(0) : (fused_path() ? buf(1) : buf(2));
        pdz_status st = start(v0, v1, zero, !o->reorth);
        if (st != PDZ_OK) return st;
        Ctl h;
        st = iterate(&h);
        if (st != PDZ_OK) return st;
        uint32_t word = 0;
        PDZ_HIP(hipMemcpyAsync(&word, err, sizeof(word), hipMemcpyDeviceToHost, s));
        PDZ_HIP(hipStreamSynchronize(s));
        if (word & kErrNonFinite) {
            hipLaunchKernelGGL(k_clear_bits, dim3(1), dim3(1), 0, s, err, kErrNonFinite);
            (void)hipStreamSynchronize(s);
            return fail(PDZ_EINVAL, "non-finite Lanczos scalar (start vector or H)");
        }
        res->E0 = h.theta;
        res->resid_est = h.resid;
        res->iters = h.k;
        res->converged = h.converged;
        res->E0_refined = h.theta;
        res->resid_refined = -1.0;
        if (o->refine && h.k > 0) {
            st = refine(v0, h.k, &res->E0_refined, &res->resid_refined);
            if (st != PDZ_OK) return st;
            if (o->refine == 2) {
                bool restarted = false;
                st = maybe_restart(h.k, ritz_out, res, &restarted);
                if (st != PDZ_OK && st != PDZ_ENOCONV) return st;
                if (restarted) return st;
            }
            if (ritz_out && pitch) {   // back to the basis order (unpadded rows)
                hipLaunchKernelGGL((k_repitch<double, double>), dim3(grid_elems(p->D)), dim3(kRedBlock), 0, s, y(),
                                   pitch, ritz_out, p->dn.D, p->dn.D, p->D);
                st = launch_check();
                if (st != PDZ_OK) return st;
            } else if (ritz_out) {
                PDZ_HIP(hipMemcpyAsync(ritz_out, y(), (size_t)D * 8, hipMemcpyDeviceToDevice, s));
            }
        }
        PDZ_HIP(hipStreamSynchronize(s));
        return h.converged ? ok() : fail(PDZ_ENOCONV, "max_iter reached before the tolerance");
    }

    // refine == 2: when the FP64 residual r of the Ritz vector y is too large
    // for its Rayleigh quotient to be within 1e-8 of the eigenvalue
    // (refine_restart_needed), run FP64 Lanczos from y (three-term
    // recurrence, tol at least 1e-12, at least 300 steps) and report its
    // refined energy.
    pdz_status maybe_restart(int k, double* ritz_out, pdz_lanczos_result* res, bool* restarted) {
        *restarted = false;
        std::vector<double> a(k), b(k + 1);
        PDZ_HIP(hipMemcpyAsync(a.data(), alpha(), (size_t)k * 8, hipMemcpyDeviceToHost, s));
        PDZ_HIP(hipMemcpyAsync(b.data(), beta(), (size_t)(k + 1) * 8, hipMemcpyDeviceToHost, s));
        PDZ_HIP(hipStreamSynchronize(s));
        double gap = 0.0;
        if (!refine_restart_needed(a, b, k, res->E0_refined, res->resid_refined, &gap)) return ok();
        const pdz_lanczos_opts ro = restart_opts(o);
        const Layout L2 = make_layout(p, &ro);
        Run<double> r2{p, &ro, L2, ws + L.restart, s, err, D};
        r2.pitch = pitch;
        r2.v0_pitched = true;   // y is in the padded layout
        pdz_lanczos_result rr;
        std::memset(&rr, 0, sizeof(rr));
        pdz_status st = r2.run(y(), ritz_out, &rr);
        if (st != PDZ_OK && st != PDZ_ENOCONV) return st;
        *restarted = true;
        res->E0_refined = rr.E0_refined;
        res->resid_refined = rr.resid_refined;
        res->restart_iters = rr.iters;
        return st;
    }
};

pdz_status check_opts(const pdz_lanczos_opts* o) {
    if (!o) return fail(PDZ_EINVAL, "opts is NULL");
    if (o->max_iter < 1 || o->max_iter > kMaxIter) return fail(PDZ_EINVAL, "max_iter must be in [1, 2000]");
    if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return fail(PDZ_EINVAL, "tol must be finite and >= 0");
    if (o->storage != PDZ_F64 && o->storage != PDZ_F32) return fail(PDZ_EINVAL, "storage must be F64 or F32");
    if (o->reorth < 0 || o->reorth > 2) return fail(PDZ_EINVAL, "reorth must be 0 (none), 1 (local) or 2 (full)");
    if (o->check_every < 1) return fail(PDZ_EINVAL, "check_every must be >= 1");
    if (o->refine < 0 || o->refine > 2) return fail(PDZ_EINVAL, "refine must be 0, 1 or 2");
    if (o->refine == 2 && o->reorth) return fail(PDZ_EINVAL, "refine = 2 restarts the three-term recurrence (reorth 0)");
    if (o->keep_basis != 0 && o->keep_basis != 1) return fail(PDZ_EINVAL, "keep_basis must be 0 or 1");
    return ok();
}

}  // namespace
}  // namespace pdz

using namespace pdz;

extern "C" {

pdz_status pdz_refine_decision(const double* alpha, const double* beta, int32_t k, double E, double resid,
                               int32_t* restart, double* gap) {
    if (!alpha || !beta || !restart || !gap || k < 1 || k > kMaxIter)
        return fail(PDZ_EINVAL, "pdz_refine_decision: null pointer or k outside [1, 2000]");
    std::vector<double> a(alpha, alpha + k), b(beta, beta + k + 1);
    *restart = refine_restart_needed(a, b, k, E, resid, gap);
    return ok();
}

pdz_status pdz_lanczos_default_opts(pdz_lanczos_opts* o) {
    if (!o) return fail(PDZ_EINVAL, "opts is NULL");
    std::memset(o, 0, sizeof(*o));
    o->max_iter = 300;
    o->tol = 1e-12;
    o->storage = PDZ_F64;
    o->reorth = 0;
    o->seed = 1;
    o->check_every = 10;
    o->use_graph = 1;
    o->refine = 0;
    o->keep_basis = 0;
    return ok();
}

pdz_status pdz_lanczos_workspace_size(pdz_problem p, const pdz_lanczos_opts* o, size_t* bytes) {
    if (!p || !bytes) return fail(PDZ_EINVAL, "NULL argument");
    pdz_status st = check_opts(o);
    if (st != PDZ_OK) return st;
    pdz_lanczos_opts oo = *o;
    *bytes = make_layout(p, &oo).total;
    return ok();
}

pdz_status pdz_lanczos_coefficients(pdz_problem p, const pdz_lanczos_opts* o, const void* ws, size_t ws_bytes,
                                    int32_t max_n, double* alpha, double* beta, double* norm0, int32_t* n_out) {
    if (!p || !ws || !alpha || !beta || !norm0 || !n_out) return fail(PDZ_EINVAL, "NULL argument");
    pdz_status st = check_opts(o);
    if (st != PDZ_OK) return st;
    pdz_lanczos_opts oo = *o;
    if (oo.reorth) oo.use_graph = 0;
    const Layout L = make_layout(p, &oo);
    if (ws_bytes < L.total) return fail(PDZ_EINVAL, "workspace smaller than pdz_lanczos_workspace_size");
    Ctl h;
    PDZ_HIP(hipMemcpy(&h, static_cast<const char*>(ws) + L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    int n = h.k < max_n ? h.k : max_n;
    if (n < 0) n = 0;
    if (n > 0) {
        PDZ_HIP(hipMemcpy(alpha, static_cast<const char*>(ws) + L.alpha, (size_t)n * sizeof(double),
                          hipMemcpyDeviceToHost));
        PDZ_HIP(hipMemcpy(beta, static_cast<const char*>(ws) + L.beta, (size_t)(n + 1) * sizeof(double),
                          hipMemcpyDeviceToHost));
    }
    *norm0 = h.norm0;
    *n_out = n;
    return ok();
}

pdz_status pdz_lanczos_history(pdz_problem p, const pdz_lanczos_opts* o, const void* ws, size_t ws_bytes,
                               int32_t max_n, double* theta_host, int32_t* n_out) {
    if (!p || !ws || !theta_host || !n_out) return fail(PDZ_EINVAL, "NULL argument");
    pdz_status st = check_opts(o);
    if (st != PDZ_OK) return st;
    pdz_lanczos_opts oo = *o;
    if (oo.reorth) oo.use_graph = 0;
    const Layout L = make_layout(p, &oo);
    if (ws_bytes < L.total) return fail(PDZ_EINVAL, "workspace smaller than pdz_lanczos_workspace_size");
    Ctl h;
    PDZ_HIP(hipMemcpy(&h, static_cast<const char*>(ws) + L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost));
    int n = h.k < max_n ? h.k : max_n;
    if (n < 0) n = 0;
    if (n > 0)
        PDZ_HIP(hipMemcpy(theta_host, static_cast<const char*>(ws) + L.theta, (size_t)n * sizeof(double),
                          hipMemcpyDeviceToHost));
    *n_out = n;
    return ok();
}

pdz_status pdz_lanczos_kernel_times(pdz_problem p, const pdz_lanczos_opts* o, void* ws, size_t ws_bytes,
                                    int32_t steps, double* ms, int32_t* fused, void* stream) {
    if (!p || !ms || !fused) return fail(PDZ_EINVAL, "NULL argument");
    pdz_status st = check_opts(o);
    if (st != PDZ_OK) return st;
    if (o->reorth) return fail(PDZ_EINVAL, "step timing covers the three-term recurrence (reorth must be 0)");
    if (steps < 1 || steps >= o->max_iter) return fail(PDZ_EINVAL, "steps must be in [1, max_iter)");
    const Layout L = make_layout(p, o);
    if (!ws || ws_bytes < L.total) return fail(PDZ_EINVAL, "workspace smaller than pdz_lanczos_workspace_size");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(PDZ_EINVAL, "workspace must be 256-byte aligned");
    int dev = 0;
    PDZ_HIP(hipGetDevice(&dev));
    if (dev != p->device) return fail(PDZ_EINVAL, "problem lives on another device");
    DeviceCtx* ctx = nullptr;
    st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    pdz_lanczos_opts oo = *o;
    oo.tol = 0.0;
    hipStream_t s = (hipStream_t)stream;
    int f = 0;
    if (oo.storage == PDZ_F64) {
        Run<double> r{p, &oo, L, static_cast<char*>(ws), s, ctx->err, lanczos_len(p)};
        r.pitch = lanczos_pitch(p);
        st = r.timed_steps(steps, ms, &f);
    } else {
        Run<float> r{p, &oo, L, static_cast<char*>(ws), s, ctx->err, lanczos_len(p)};
        r.pitch = lanczos_pitch(p);
        st = r.timed_steps(steps, ms, &f);
    }
    *fused = f;
    return st;
}

pdz_status pdz_lanczos(pdz_problem p, const pdz_lanczos_opts* o, const void* v0, void* ws, size_t ws_bytes,
                       double* ritz_out, pdz_lanczos_result* res, void* stream) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!p || !res) return fail(PDZ_EINVAL, "NULL problem or result");
    pdz_status st = check_opts(o);
    if (st != PDZ_OK) return st;
    std::memset(res, 0, sizeof(*res));
    pdz_lanczos_opts oo = *o;
    if (ritz_out && oo.refine == 0) oo.refine = 1;
    if (oo.reorth) oo.use_graph = 0;
    const Layout L = make_layout(p, &oo);
    if (!ws) return fail(PDZ_EINVAL, "workspace is NULL");
    if (ws_bytes < L.total) return fail(PDZ_EINVAL, "workspace smaller than pdz_lanczos_workspace_size");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(PDZ_EINVAL, "workspace must be 256-byte aligned");
    int dev = 0;
    PDZ_HIP(hipGetDevice(&dev));
    if (dev != p->device) return fail(PDZ_EINVAL, "problem lives on another device");
    DeviceCtx* ctx = nullptr;
    st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipStream_t own = nullptr;
    if (!s && oo.use_graph) {
        // capture needs a stream other than the legacy default stream
        PDZ_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
        PDZ_HIP(hipDeviceSynchronize());
        s = own;
    }
    if (oo.storage == PDZ_F64) {
        Run<double> r{p, &oo, L, static_cast<char*>(ws), s, ctx->err, lanczos_len(p)};
        r.pitch = lanczos_pitch(p);
        st = r.run(v0, ritz_out, res);
    } else {
        Run<float> r{p, &oo, L, static_cast<char*>(ws), s, ctx->err, lanczos_len(p)};
        r.pitch = lanczos_pitch(p);
        st = r.run(v0, ritz_out, res);
    }
    if (own) {
        (void)hipStreamSynchronize(own);
        (void)hipStreamDestroy(own);
    }
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return st;
}

}  // extern "C"
