// Batched H.v and Lanczos over many Hubbard clusters of uneven size.
//
// The clusters' vectors are packed back to back (each at a 64-element aligned
// offset).  One persistent launch applies every cluster's H: work groups pull
// tiles (cluster, group of rows) from an atomic work queue, largest clusters
// first, stage the tile's rows in LDS and compute each output element whole:
// diagonal, down hops gathered from LDS, up hops read from the (cache
// resident) packed vector.  Every element is summed by one thread in the same
// order as the single-cluster H.v, so the results are bitwise identical to
// pdz_hv on each cluster.  The queue is reset by a small kernel before each
// launch, which keeps the pair capturable in a HIP graph.
//
// Batched Lanczos runs the recurrence of k_lanczos.hip for all clusters in
// lockstep over the packed vectors: per-cluster alpha, beta, Ritz value and
// convergence flag on the device; a converged cluster's tiles and chunks are
// skipped by every later kernel.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "pdz_internal.h"
#include "tridiag.h"

namespace pdz {
namespace {

constexpr int kBatchMaxIter = 2000;
constexpr int kRed = 256;
constexpr uint64_t kAlign = 64;       // packed vector offsets, elements
constexpr uint64_t kChunk = 16384;    // reduction chunk, elements

struct BProb {
    uint64_t off;                 // element offset of the cluster's vector
    uint64_t D_up, D_dn;
    double U;
    const uint32_t* up_states;
    const uint32_t* dn_states;
    const uint8_t* up_count;
    const uint8_t* dn_count;
    const uint32_t* up_ell;       // 32-bit hop tables, slot major
    const uint32_t* dn_ell;
    const double* coef64;
    const float* coef32;
    int ncoef;
    int pad;
};

struct BTile {
    uint32_t prob;
    uint32_t u0;
    uint32_t nrows;
    uint32_t pad;
};

struct BChunk {                    // reduction chunk [begin, end) of one cluster
    uint32_t prob;
    uint32_t pad;
    uint64_t begin, end;
};

struct BCtl {                      // per-cluster Lanczos state
    int k;
    int done;
    int converged;
    int breakdown;
    double theta;
    double resid;
    double norm0;
    double theta_prev;   // Ritz value of the step before
};

__global__ void k_clear_bits1(uint32_t* w, uint32_t bits) {
    if (threadIdx.x == 0 && blockIdx.x == 0) atomicAnd(w, ~bits);
}

__global__ void k_queue_reset(unsigned* q) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *q = 0u;
}

template <typename T>
__device__ __forceinline__ const T* bcoef(const BProb& p);
template <>
__device__ __forceinline__ const double* bcoef<double>(const BProb& p) { return p.coef64; }
template <>
__device__ __forceinline__ const float* bcoef<float>(const BProb& p) { return p.coef32; }

constexpr int kBHopNB = 8;   // hops of one element whose loads are in flight together

// done: per-cluster flags with stride `dstride` ints (NULL: none skipped).
template <typename T, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_batch_hv(const BProb* __restrict__ probs, const BTile* __restrict__ tiles,
                                                    uint32_t ntiles, unsigned* queue, const int* done, int dstride,
                                                    const T* __restrict__ x, T* __restrict__ y) {
    extern __shared__ __align__(16) unsigned char smem[];
    T* coef = reinterpret_cast<T*>(smem);
    T* rows = coef + kMaxCoef;
    __shared__ uint32_t s_t;
    for (;;) {
        if (threadIdx.x == 0) s_t = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t t = s_t;
        __syncthreads();
        if (t >= ntiles) break;   // every wave of every group reaches this exit once the queue is drained
        const BTile tl = tiles[t];
        if (done && done[(size_t)tl.prob * dstride]) continue;
        const BProb pr = probs[tl.prob];
        const T* cg = bcoef<T>(pr);
        for (int k = threadIdx.x; k < pr.ncoef; k += BLOCK) coef[k] = cg[k];
        const uint64_t D_dn = pr.D_dn, D_up = pr.D_up;
        const uint32_t nelem = tl.nrows * (uint32_t)D_dn;
        const T* xp = x + pr.off;
        T* yp = y + pr.off;
        const T* xg = xp + (uint64_t)tl.u0 * D_dn;
        for (uint32_t k = threadIdx.x; k < nelem; k += BLOCK) rows[k] = xg[k];
        __syncthreads();
        const T U = (T)pr.U;
        for (uint32_t k = threadIdx.x; k < nelem; k += BLOCK) {
            const uint32_t r = k / (uint32_t)D_dn;
            const uint32_t d = k - r * (uint32_t)D_dn;
            const uint64_t u = tl.u0 + r;
            const T* xrow = rows + (size_t)r * D_dn;
            T acc = U * (T)__builtin_popcount(pr.up_states[u] & pr.dn_states[d]) * xrow[d];
            // the barriers keep the rounding of the two-pass H.v: the diagonal
            // product and the down-hop sum are rounded before the next term
            asm volatile("" : "+v"(acc));
            // hops in order, kBHopNB at a time: a batch's table entries (and, for
            // up hops, its operands) are loaded before its first multiply-add
            const int cd = pr.dn_count[d];
            int h = 0;
            for (; h + kBHopNB <= cd; h += kBHopNB) {
                uint32_t e[kBHopNB];
#pragma unroll
                for (int j = 0; j < kBHopNB; ++j) e[j] = pr.dn_ell[(uint64_t)(h + j) * D_dn + d];
#pragma unroll
                for (int j = 0; j < kBHopNB; ++j) acc += coef[e[j] >> kTargetBits] * xrow[e[j] & kTargetMask];
            }
            for (; h < cd; ++h) {
                const uint32_t e = pr.dn_ell[(uint64_t)h * D_dn + d];
                acc += coef[e >> kTargetBits] * xrow[e & kTargetMask];
            }
            asm volatile("" : "+v"(acc));
            const int cu = pr.up_count[u];
            h = 0;
            for (; h + kBHopNB <= cu; h += kBHopNB) {
                uint32_t e[kBHopNB];
                T v[kBHopNB];
#pragma unroll
                for (int j = 0; j < kBHopNB; ++j) e[j] = pr.up_ell[(uint64_t)(h + j) * D_up + u];
#pragma unroll
                for (int j = 0; j < kBHopNB; ++j) v[j] = xp[(uint64_t)(e[j] & kTargetMask) * D_dn + d];
#pragma unroll
                for (int j = 0; j < kBHopNB; ++j) acc += coef[e[j] >> kTargetBits] * v[j];
            }
            for (; h < cu; ++h) {
                const uint32_t e = pr.up_ell[(uint64_t)h * D_up + u];
                acc += coef[e >> kTargetBits] * xp[(uint64_t)(e & kTargetMask) * D_dn + d];
            }
            yp[u * D_dn + d] = acc;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ batched Lanczos

__device__ __forceinline__ double bsum(double v, double* red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kRed / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Clear two packed vectors (the padding between clusters stays zero).
template <typename T>
__global__ __launch_bounds__(kRed) void k_bzero(uint64_t total, T* a, T* b) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < total; i += (uint64_t)gridDim.x * blockDim.x) {
        a[i] = (T)0;
        b[i] = (T)0;
    }
}

// Start vector of cluster p: SplitMix64 stream seeded with seed + p, output r
// mapped to 2u - 1 (the single-problem start vector of that seed).
template <typename T>
__global__ __launch_bounds__(kRed) void k_bfill(const BChunk* ch, const BProb* probs, uint64_t seed, T* v) {
    const BChunk c = ch[blockIdx.x];
    const uint64_t off = probs[c.prob].off;
    for (uint64_t i = c.begin + threadIdx.x; i < c.end; i += blockDim.x)
        v[off + i] = (T)splitmix_uniform(seed + c.prob, i);
}

// partial[c] = sum over chunk c of a*b (FP64), skipped for done clusters.
template <typename T>
__global__ __launch_bounds__(kRed) void k_bdot(const BChunk* ch, const BProb* probs, const BCtl* ctl, const T* a,
                                               const T* b, double* partial) {
    __shared__ double red[kRed];
    const BChunk c = ch[blockIdx.x];
    if (ctl[c.prob].done) return;
    const uint64_t off = probs[c.prob].off;
    double acc = 0.0;
    for (uint64_t i = c.begin + threadIdx.x; i < c.end; i += blockDim.x) acc += (double)a[off + i] * (double)b[off + i];
    acc = bsum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// w -= alpha_k v + beta_k vp; partial[c] = |w|^2 over chunk c.
template <typename T>
__global__ __launch_bounds__(kRed) void k_bupdate(const BChunk* ch, const BProb* probs, const BCtl* ctl,
                                                  const double* alpha, const double* beta, int ld, T* w, const T* v,
                                                  const T* vp, double* partial) {
    __shared__ double red[kRed];
    const BChunk c = ch[blockIdx.x];
    const BCtl st = ctl[c.prob];
    if (st.done) return;
    const double a = alpha[(size_t)c.prob * ld + st.k], bt = beta[(size_t)c.prob * ld + st.k];
    const uint64_t off = probs[c.prob].off;
    double acc = 0.0;
    for (uint64_t i = c.begin + threadIdx.x; i < c.end; i += blockDim.x) {
        const T r = (T)((double)w[off + i] - a * (double)v[off + i] - bt * (double)vp[off + i]);
        w[off + i] = r;
        acc += (double)r * (double)r;
    }
    acc = bsum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// v *= 1 / s[p * ld + k + koff] (or 1 / norm0 when norm is set)
template <typename T>
__global__ __launch_bounds__(kRed) void k_bscale(const BChunk* ch, const BProb* probs, const BCtl* ctl, const double* s,
                                                 int ld, int koff, int use_norm, T* v) {
    const BChunk c = ch[blockIdx.x];
    const BCtl st = ctl[c.prob];
    if (st.done) return;
    const double inv = 1.0 / (use_norm ? st.norm0 : s[(size_t)c.prob * ld + st.k + koff]);
    const uint64_t off = probs[c.prob].off;
    for (uint64_t i = c.begin + threadIdx.x; i < c.end; i += blockDim.x) v[off + i] = (T)((double)v[off + i] * inv);
}

// One block per cluster: sum its chunk partials in order.
// mode 0: alpha[k] = sum; 1: beta[k+1] = sqrt(sum); 2: norm0 = sqrt(sum).
__global__ __launch_bounds__(kRed) void k_bfinal(const uint32_t* ch_begin, const double* partial, BCtl* ctl,
                                                 double* alpha, double* beta, int ld, int mode, uint32_t* err) {
    __shared__ double red[kRed];
    const uint32_t p = blockIdx.x;
    BCtl* st = ctl + p;
    if (st->done) return;
    double acc = 0.0;
    for (uint32_t c = ch_begin[p] + threadIdx.x; c < ch_begin[p + 1]; c += blockDim.x) acc += partial[c];
    acc = bsum(acc, red);
    if (threadIdx.x == 0) {
        const int k = st->k;
        double v = acc;
        if (mode == 0) {
            alpha[(size_t)p * ld + k] = v;
        } else {
            v = sqrt(acc);
            if (mode == 1)
                beta[(size_t)p * ld + k + 1] = v;
            else
                st->norm0 = v;
        }
        if (!isfinite(v)) atomicOr(err, kErrNonFinite);
    }
}

__global__ void k_binit(BCtl* ctl, double* beta, int ld, uint32_t n) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    BCtl c;
    c.k = 0;
    c.done = 0;
    c.converged = 0;
    c.breakdown = 0;
    c.theta = 0.0;
    c.resid = 0.0;
    c.norm0 = 0.0;
    c.theta_prev = 0.0;
    ctl[p] = c;
    beta[(size_t)p * ld] = 0.0;
}

// One block per cluster: lowest eigenpair of its T_k, convergence test, step
// counter.  Row p of svec receives the eigenvector.
__global__ __launch_bounds__(kRed) void k_btridiag(BCtl* ctl, const double* alpha, const double* beta, double* svec,
                                                   int ld, double tol, int max_iter, uint32_t* err) {
    const uint32_t p = blockIdx.x;
    BCtl* st = ctl + p;
    if (st->done) return;
    __shared__ double a[kBatchMaxIter];
    __shared__ double e[kBatchMaxIter];
    __shared__ double zs[kBatchMaxIter];
    __shared__ double rp[kBatchMaxIter];
    __shared__ double lo_s[kRed], hi_s[kRed];
    __shared__ int found;
    __shared__ double bounds[2];
    const int k = st->k + 1;
    const double* al = alpha + (size_t)p * ld;
    const double* be = beta + (size_t)p * ld;
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        a[i] = al[i];
        e[i] = (i == 0) ? 0.0 : be[i];
    }
    __syncthreads();
    double hint_lo = 0.0, hint_hi = 0.0;
    if (k >= 3) ritz_hint(st->theta, st->theta_prev, &hint_lo, &hint_hi);
    tridiag_bracket_min(a, e, k, lo_s, hi_s, &found, bounds, hint_lo, hint_hi);
    if (threadIdx.x == 0) tridiag_min_vector(a, e, k, bounds[0], zs, rp);
    __syncthreads();
    double* z = svec + (size_t)p * ld;
    for (int i = threadIdx.x; i < k; i += blockDim.x) z[i] = zs[i];
    if (threadIdx.x == 0) {
        const double theta = 0.5 * (bounds[0] + bounds[1]);
        const double bk1 = be[k];
        const double resid = fabs(bk1 * zs[k - 1]);
        st->theta_prev = st->theta;
        st->theta = theta;
        st->resid = resid;
        st->k = k;
        const bool breakdown = !(bk1 > 1e-14 * fmax(1.0, fabs(theta)));
        if (!isfinite(theta) || !isfinite(bk1)) {
            atomicOr(err, kErrNonFinite);
            st->done = 1;
        }
        if (breakdown || resid <= tol * fmax(fabs(theta), 1e-300)) {
            st->converged = 1;
            st->breakdown = breakdown ? 1 : 0;
            st->done = 1;
        }
        if (k >= max_iter) st->done = 1;
    }
}

// ---- FP64 refinement of the Ritz vectors (storage FP32 or FP64)

// kfin[p] = steps the run took; counters restart for the regeneration pass.
__global__ void k_bregen_init(BCtl* ctl, int* kfin, uint32_t n) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int k = ctl[p].k;
    kfin[p] = k;
    ctl[p].k = 0;
    ctl[p].done = k > 0 ? 0 : 1;
}

// y += s_k v_k (FP64) for every live cluster, s = row p of svec (eigenvector of T_kfin).
template <typename T>
__global__ __launch_bounds__(kRed) void k_baxpy_ritz(const BChunk* ch, const BProb* probs, const BCtl* ctl,
                                                     const double* svec, int ld, const T* v, double* y) {
    const BChunk c = ch[blockIdx.x];
    const BCtl st = ctl[c.prob];
    if (st.done) return;
    const double sk = svec[(size_t)c.prob * ld + st.k];
    const uint64_t off = probs[c.prob].off;
    for (uint64_t i = c.begin + threadIdx.x; i < c.end; i += blockDim.x) y[off + i] += sk * (double)v[off + i];
}

// A cluster whose last Lanczos vector has been added needs no further one.
__global__ void k_bregen_mark(BCtl* ctl, const int* kfin, uint32_t n) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n || ctl[p].done) return;
    if (ctl[p].k + 1 >= kfin[p]) ctl[p].done = 1;
}

// v_{k+1} from w = H v_k with the stored alpha_k, beta_k, beta_{k+1}: the same
// two roundings as the run (recurrence, then scaling), so the vectors are the
// run's bit for bit.
template <typename T>
__global__ __launch_bounds__(kRed) void k_bregen_update(const BChunk* ch, const BProb* probs, const BCtl* ctl,
                                                        const double* alpha, const double* beta, int ld, T* w,
                                                        const T* v, const T* vp) {
    const BChunk c = ch[blockIdx.x];
    const BCtl st = ctl[c.prob];
    if (st.done) return;
    const size_t row = (size_t)c.prob * ld;
    const double a = alpha[row + st.k], bt = beta[row + st.k];
    const double inv = 1.0 / beta[row + st.k + 1];
    const uint64_t off = probs[c.prob].off;
    for (uint64_t i = c.begin + threadIdx.x; i < c.end; i += blockDim.x) {
        const T r = (T)((double)w[off + i] - a * (double)v[off + i] - bt * (double)vp[off + i]);
        w[off + i] = (T)((double)r * inv);
    }
}

__global__ void k_bregen_next(BCtl* ctl, uint32_t n) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n || ctl[p].done) return;
    ctl[p].k += 1;
}

// Every cluster that ran at least one step is live again.
__global__ void k_bregen_reopen(BCtl* ctl, const int* kfin, uint32_t n) {
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    ctl[p].k = 0;
    ctl[p].done = kfin[p] > 0 ? 0 : 1;
}

// out[p] = sum of the chunk partials of cluster p (sqrt when root).
__global__ __launch_bounds__(kRed) void k_bsum_out(const uint32_t* ch_begin, const double* partial, const BCtl* ctl,
                                                   double* out, int root) {
    __shared__ double red[kRed];
    const uint32_t p = blockIdx.x;
    if (ctl[p].done) return;
    double acc = 0.0;
    for (uint32_t c = ch_begin[p] + threadIdx.x; c < ch_begin[p + 1]; c += blockDim.x) acc += partial[c];
    acc = bsum(acc, red);
    if (threadIdx.x == 0) out[p] = root ? sqrt(acc) : acc;
}

// partial[c] = |hy - E_p y|^2 over chunk c.
__global__ __launch_bounds__(kRed) void k_bresid(const BChunk* ch, const BProb* probs, const BCtl* ctl,
                                                 const double* hy, const double* y, const double* E, double* partial) {
    __shared__ double red[kRed];
    const BChunk c = ch[blockIdx.x];
    if (ctl[c.prob].done) return;
    const double e = E[c.prob];
    const uint64_t off = probs[c.prob].off;
    double acc = 0.0;
    for (uint64_t i = c.begin + threadIdx.x; i < c.end; i += blockDim.x) {
        const double r = hy[off + i] - e * y[off + i];
        acc += r * r;
    }
    acc = bsum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr size_t kBatchLds = 159 * 1024;   // dynamic LDS limit: 160 KiB less the static queue slot

template <typename T, int BLOCK>
pdz_status set_batch_lds() {
    PDZ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_hv<T, BLOCK>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBatchLds));
    return ok();
}

}  // namespace

pdz_status batch_prepare() {
    pdz_status st = set_batch_lds<double, 256>();
    if (st == PDZ_OK) st = set_batch_lds<double, 512>();
    if (st == PDZ_OK) st = set_batch_lds<double, 1024>();
    if (st == PDZ_OK) st = set_batch_lds<float, 256>();
    if (st == PDZ_OK) st = set_batch_lds<float, 512>();
    if (st == PDZ_OK) st = set_batch_lds<float, 1024>();
    return st;
}

}  // namespace pdz

using namespace pdz;

struct pdz_batch_s {
    int device = 0;
    int n = 0;
    std::vector<pdz_problem> problems;
    std::vector<uint64_t> offsets;   // n + 1, elements
    uint64_t total = 0;
    BProb* d_probs = nullptr;
    BTile* d_tiles = nullptr;        // tiles for the current plan
    uint32_t ntiles = 0;
    BChunk* d_chunks = nullptr;
    uint32_t* d_chunk_begin = nullptr;   // n + 1
    uint32_t nchunks = 0;
    unsigned* d_queue = nullptr;
    uint64_t max_D_dn = 0;
    pdz_batch_plan plan{0, 0, 0, 0};
    pdz_batch_plan tiles_for{-1, -1, -1, -1};
};

namespace {

pdz_batch_plan resolve(const pdz_batch_s* b) {
    pdz_batch_plan p = b->plan;
    if (p.tile_elems == 0) p.tile_elems = 4096;
    if (p.block == 0) p.block = 256;
    if (p.wgs_per_cu == 0) p.wgs_per_cu = 4;
    if (p.order == 0) p.order = 1;
    return p;
}

bool plan_ok(const pdz_batch_s* b, const pdz_batch_plan& p) {
    const bool te = p.tile_elems == 1024 || p.tile_elems == 2048 || p.tile_elems == 4096 || p.tile_elems == 8192;
    const bool bl = p.block == 256 || p.block == 512 || p.block == 1024;
    const bool wg = p.wgs_per_cu >= 1 && p.wgs_per_cu <= 8;
    const bool od = p.order == 1 || p.order == 2;
    // every tile must hold at least one full row in LDS for both precisions
    const bool fits = b->max_D_dn * 8 + kMaxCoef * 8 + 1024 <= 160 * 1024;
    return te && bl && wg && od && fits;
}

// Tiles: rows of each cluster in groups of about tile_elems elements;
// order 1 = largest clusters first, 2 = cluster order.
pdz_status build_tiles(pdz_batch_s* b, const pdz_batch_plan& p) {
    if (b->d_tiles && b->tiles_for.tile_elems == p.tile_elems && b->tiles_for.order == p.order) return ok();
    std::vector<int> idx(b->n);
    std::iota(idx.begin(), idx.end(), 0);
    if (p.order == 1)
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) { return b->problems[a]->D > b->problems[c]->D; });
    std::vector<BTile> tiles;
    const size_t lds_rows_cap = (160 * 1024 - kMaxCoef * 8 - 1024) / 8;   // elements, FP64 worst case
    for (int i : idx) {
        const pdz_problem q = b->problems[i];
        const uint64_t Dn = q->dn.D, Du = q->up.D;
        uint64_t rows = (uint64_t)p.tile_elems / Dn;
        if (rows < 1) rows = 1;
        if (rows * Dn > lds_rows_cap) rows = lds_rows_cap / Dn;
        if (rows < 1) return fail(PDZ_ERANGE, "a cluster row does not fit the batched kernel's LDS");
        for (uint64_t u0 = 0; u0 < Du; u0 += rows) {
            BTile t;
            t.prob = (uint32_t)i;
            t.u0 = (uint32_t)u0;
            t.nrows = (uint32_t)((Du - u0) < rows ? (Du - u0) : rows);
            t.pad = 0;
            tiles.push_back(t);
        }
    }
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    b->d_tiles = nullptr;
    PDZ_HIP(hipMalloc(&b->d_tiles, tiles.size() * sizeof(BTile)));
    PDZ_HIP(hipMemcpy(b->d_tiles, tiles.data(), tiles.size() * sizeof(BTile), hipMemcpyHostToDevice));
    b->ntiles = (uint32_t)tiles.size();
    b->tiles_for = p;
    return ok();
}

template <typename T>
pdz_status batch_hv_launch(pdz_batch_s* b, const pdz_batch_plan& p, const T* x, T* y, hipStream_t s, const int* done,
                           int dstride) {
    DeviceCtx* ctx = nullptr;
    pdz_status st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    size_t max_tile = 0;
    for (int i = 0; i < b->n; ++i) {
        const uint64_t Dn = b->problems[i]->dn.D;
        uint64_t rows = (uint64_t)p.tile_elems / Dn;
        if (rows < 1) rows = 1;
        const uint64_t Du = b->problems[i]->up.D;
        if (rows > Du) rows = Du;
        max_tile = std::max<size_t>(max_tile, rows * Dn);
    }
    const size_t lds = kMaxCoef * sizeof(T) + max_tile * sizeof(T);
    const unsigned grid = (unsigned)(ctx->cu_count * p.wgs_per_cu);
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(1), 0, s, b->d_queue);
    if (p.block == 1024)
        hipLaunchKernelGGL((k_batch_hv<T, 1024>), dim3(grid), dim3(1024), lds, s, b->d_probs, b->d_tiles, b->ntiles,
                           b->d_queue, done, dstride, x, y);
    else if (p.block == 512)
        hipLaunchKernelGGL((k_batch_hv<T, 512>), dim3(grid), dim3(512), lds, s, b->d_probs, b->d_tiles, b->ntiles,
                           b->d_queue, done, dstride, x, y);
    else
        hipLaunchKernelGGL((k_batch_hv<T, 256>), dim3(grid), dim3(256), lds, s, b->d_probs, b->d_tiles, b->ntiles,
                           b->d_queue, done, dstride, x, y);
    PDZ_HIP(hipGetLastError());
    return ok();
}

pdz_status batch_hv_any(pdz_batch_s* b, pdz_dtype dt, const void* x, void* y, hipStream_t s, const int* done,
                        int dstride) {
    const pdz_batch_plan p = resolve(b);
    pdz_status st = build_tiles(b, p);
    if (st != PDZ_OK) return st;
    if (dt == PDZ_F64)
        return batch_hv_launch<double>(b, p, static_cast<const double*>(x), static_cast<double*>(y), s, done,
                                       dstride);
    return batch_hv_launch<float>(b, p, static_cast<const float*>(x), static_cast<float*>(y), s, done, dstride);
}

struct BLayout {
    size_t vec = 0, buf[3] = {0, 0, 0}, alpha = 0, beta = 0, svec = 0, partial = 0, ctl = 0, total = 0;
    size_t y = 0, hy = 0, kfin = 0, eref = 0;   // refinement (refine == 1)
    int ld = 0;
};

BLayout blayout(const pdz_batch_s* b, const pdz_lanczos_opts* o) {
    BLayout L;
    const size_t es = o->storage == PDZ_F64 ? 8 : 4;
    L.vec = al256(b->total * es);
    size_t off = 0;
    for (int i = 0; i < 3; ++i) {
        L.buf[i] = off;
        off += L.vec;
    }
    L.ld = 2 * (o->max_iter + 8);
    const size_t per = (size_t)L.ld * b->n * 8;
    L.alpha = off;
    off += al256(per);
    L.beta = off;
    off += al256(per);
    L.svec = off;
    off += al256(per);
    L.partial = off;
    off += al256((size_t)b->nchunks * 8);
    L.ctl = off;
    off += al256((size_t)b->n * sizeof(BCtl));
    if (o->refine) {
        L.y = off;
        off += al256(b->total * 8);
        L.hy = off;
        off += al256(b->total * 8);
        L.kfin = off;
        off += al256((size_t)b->n * sizeof(int));
        L.eref = off;
        off += al256((size_t)b->n * 2 * 8);
    }
    L.total = off;
    return L;
}

template <typename T>
pdz_status batch_lanczos_run(pdz_batch_s* b, const pdz_lanczos_opts* o, char* ws, const BLayout& L,
                             pdz_lanczos_result* res, hipStream_t s, uint32_t* err) {
    T* buf[3];
    for (int i = 0; i < 3; ++i) buf[i] = reinterpret_cast<T*>(ws + L.buf[i]);
    double* alpha = reinterpret_cast<double*>(ws + L.alpha);
    double* beta = reinterpret_cast<double*>(ws + L.beta);
    double* svec = reinterpret_cast<double*>(ws + L.svec);
    double* partial = reinterpret_cast<double*>(ws + L.partial);
    BCtl* ctl = reinterpret_cast<BCtl*>(ws + L.ctl);
    const int ld = L.ld;
    const dim3 nch(b->nchunks), np(b->n), blk(kRed);
    const pdz_dtype dt = o->storage == PDZ_F64 ? PDZ_F64 : PDZ_F32;
    // start: v_1 = SplitMix64 vectors normalised per cluster, v_0 = 0
    hipLaunchKernelGGL(k_clear_bits1, dim3(1), dim3(1), 0, s, err, kErrNonFinite);
    hipLaunchKernelGGL(k_binit, dim3((b->n + 255) / 256), dim3(256), 0, s, ctl, beta, ld, (uint32_t)b->n);
    hipLaunchKernelGGL(k_bzero<T>, dim3(1024), blk, 0, s, b->total, buf[0], buf[2]);
    hipLaunchKernelGGL(k_bfill<T>, nch, blk, 0, s, b->d_chunks, b->d_probs, o->seed, buf[0]);
    hipLaunchKernelGGL(k_bdot<T>, nch, blk, 0, s, b->d_chunks, b->d_probs, ctl, buf[0], buf[0], partial);
    hipLaunchKernelGGL(k_bfinal, np, blk, 0, s, b->d_chunk_begin, partial, ctl, alpha, beta, ld, 2, err);
    hipLaunchKernelGGL(k_bscale<T>, nch, blk, 0, s, b->d_chunks, b->d_probs, ctl, beta, ld, 0, 1, buf[0]);
    PDZ_HIP(hipGetLastError());
    const int* done = &ctl[0].done;
    const int dstride = (int)(sizeof(BCtl) / sizeof(int));
    int period = o->check_every;
    if (period % 3) period += 3 - period % 3;
    auto step = [&](T* v, T* vp, T* w) -> pdz_status {
        pdz_status st = batch_hv_any(b, dt, v, w, s, done, dstride);
        if (st != PDZ_OK) return st;
        hipLaunchKernelGGL(k_bdot<T>, nch, blk, 0, s, b->d_chunks, b->d_probs, ctl, v, w, partial);
        hipLaunchKernelGGL(k_bfinal, np, blk, 0, s, b->d_chunk_begin, partial, ctl, alpha, beta, ld, 0, err);
        hipLaunchKernelGGL(k_bupdate<T>, nch, blk, 0, s, b->d_chunks, b->d_probs, ctl, alpha, beta, ld, w, v, vp,
                           partial);
        hipLaunchKernelGGL(k_bfinal, np, blk, 0, s, b->d_chunk_begin, partial, ctl, alpha, beta, ld, 1, err);
        hipLaunchKernelGGL(k_btridiag, np, blk, 0, s, ctl, alpha, beta, svec, ld, o->tol, o->max_iter, err);
        hipLaunchKernelGGL(k_bscale<T>, nch, blk, 0, s, b->d_chunks, b->d_probs, ctl, beta, ld, 0, 0, w);
        PDZ_HIP(hipGetLastError());
        return ok();
    };
    auto enqueue = [&]() -> pdz_status {
        for (int t = 0; t < period; ++t) {
            const int a = t % 3;
            pdz_status st = step(buf[a], buf[(a + 2) % 3], buf[(a + 1) % 3]);
            if (st != PDZ_OK) return st;
        }
        return ok();
    };
    // tiles for the current plan must exist before capture (no allocation inside a graph)
    pdz_status st = build_tiles(b, resolve(b));
    if (st != PDZ_OK) return st;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (o->use_graph) {
        PDZ_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        st = enqueue();
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
    std::vector<BCtl> h(b->n);
    st = ok();
    for (int steps = 0; steps < o->max_iter; steps += period) {
        if (exec) {
            hipError_t e = hipGraphLaunch(exec, s);
            if (e != hipSuccess) {
                st = hip_fail(e, "hipGraphLaunch");
                break;
            }
        } else {
            st = enqueue();
            if (st != PDZ_OK) break;
        }
        hipError_t e = hipMemcpyAsync(h.data(), ctl, b->n * sizeof(BCtl), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            st = hip_fail(e, "batched Lanczos flags");
            break;
        }
        bool all = true;
        for (const BCtl& c : h) all = all && c.done;
        if (all) break;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (st != PDZ_OK) return st;
    uint32_t word = 0;
    PDZ_HIP(hipMemcpyAsync(h.data(), ctl, b->n * sizeof(BCtl), hipMemcpyDeviceToHost, s));
    PDZ_HIP(hipMemcpyAsync(&word, err, sizeof(word), hipMemcpyDeviceToHost, s));
    PDZ_HIP(hipStreamSynchronize(s));
    if (word & kErrNonFinite) {
        hipLaunchKernelGGL(k_clear_bits1, dim3(1), dim3(1), 0, s, err, kErrNonFinite);
        (void)hipStreamSynchronize(s);
        return fail(PDZ_EINVAL, "non-finite Lanczos scalar (start vector or H)");
    }
    bool all_conv = true;
    int kmax = 0;
    for (int i = 0; i < b->n; ++i) {
        if (!(h[i].norm0 > 0.0) || !std::isfinite(h[i].norm0))
            return fail(PDZ_EINVAL, "a start vector has zero or non-finite norm");
        res[i].E0 = h[i].theta;
        res[i].resid_est = h[i].resid;
        res[i].E0_refined = h[i].theta;
        res[i].resid_refined = -1.0;
        res[i].iters = h[i].k;
        res[i].converged = h[i].converged;
        all_conv = all_conv && h[i].converged;
        kmax = std::max(kmax, h[i].k);
    }
    if (o->refine && kmax > 0) {
        // Ritz vector y_p = sum_j s_{p,j} v_{p,j} in FP64 from the regenerated
        // Lanczos vectors, normalised; its FP64 Rayleigh quotient and residual.
        double* y = reinterpret_cast<double*>(ws + L.y);
        double* hy = reinterpret_cast<double*>(ws + L.hy);
        int* kfin = reinterpret_cast<int*>(ws + L.kfin);
        double* eref = reinterpret_cast<double*>(ws + L.eref);
        const dim3 npg((b->n + 255) / 256), b256(256);
        hipLaunchKernelGGL(k_bregen_init, npg, b256, 0, s, ctl, kfin, (uint32_t)b->n);
        hipLaunchKernelGGL(k_bzero<T>, dim3(1024), blk, 0, s, b->total, buf[0], buf[2]);
        hipLaunchKernelGGL(k_bzero<double>, dim3(1024), blk, 0, s, b->total, y, hy);
        hipLaunchKernelGGL(k_bfill<T>, nch, blk, 0, s, b->d_chunks, b->d_probs, o->seed, buf[0]);
        hipLaunchKernelGGL(k_bdot<T>, nch, blk, 0, s, b->d_chunks, b->d_probs, ctl, buf[0], buf[0], partial);
        hipLaunchKernelGGL(k_bfinal, np, blk, 0, s, b->d_chunk_begin, partial, ctl, alpha, beta, ld, 2, err);
        hipLaunchKernelGGL(k_bscale<T>, nch, blk, 0, s, b->d_chunks, b->d_probs, ctl, beta, ld, 0, 1, buf[0]);
        for (int j = 0; j < kmax; ++j) {
            const int a = j % 3;
            T* v = buf[a];
            T* vp = buf[(a + 2) % 3];
            T* w = buf[(a + 1) % 3];
            hipLaunchKernelGGL(k_baxpy_ritz<T>, nch, blk, 0, s, b->d_chunks, b->d_probs, ctl, svec, ld, v, y);
            if (j + 1 >= kmax) break;
            hipLaunchKernelGGL(k_bregen_mark, npg, b256, 0, s, ctl, kfin, (uint32_t)b->n);
            st = batch_hv_any(b, dt, v, w, s, done, dstride);
            if (st != PDZ_OK) return st;
            hipLaunchKernelGGL(k_bregen_update<T>, nch, blk, 0, s, b->d_chunks, b->d_probs, ctl, alpha, beta, ld, w,
                               v, vp);
            hipLaunchKernelGGL(k_bregen_next, npg, b256, 0, s, ctl, (uint32_t)b->n);
        }
        hipLaunchKernelGGL(k_bregen_reopen, npg, b256, 0, s, ctl, kfin, (uint32_t)b->n);
        hipLaunchKernelGGL(k_bdot<double>, nch, blk, 0, s, b->d_chunks, b->d_probs, ctl, y, y, partial);
        hipLaunchKernelGGL(k_bfinal, np, blk, 0, s, b->d_chunk_begin, partial, ctl, alpha, beta, ld, 2, err);
        hipLaunchKernelGGL(k_bscale<double>, nch, blk, 0, s, b->d_chunks, b->d_probs, ctl, beta, ld, 0, 1, y);
        st = batch_hv_any(b, PDZ_F64, y, hy, s, done, dstride);
        if (st != PDZ_OK) return st;
        hipLaunchKernelGGL(k_bdot<double>, nch, blk, 0, s, b->d_chunks, b->d_probs, ctl, y, hy, partial);
        hipLaunchKernelGGL(k_bsum_out, np, blk, 0, s, b->d_chunk_begin, partial, ctl, eref, 0);
        hipLaunchKernelGGL(k_bresid, nch, blk, 0, s, b->d_chunks, b->d_probs, ctl, hy, y, eref, partial);
        hipLaunchKernelGGL(k_bsum_out, np, blk, 0, s, b->d_chunk_begin, partial, ctl, eref + b->n, 1);
        PDZ_HIP(hipGetLastError());
        std::vector<double> er(2 * (size_t)b->n);
        std::vector<int> kf(b->n);
        PDZ_HIP(hipMemcpyAsync(er.data(), eref, er.size() * 8, hipMemcpyDeviceToHost, s));
        PDZ_HIP(hipMemcpyAsync(kf.data(), kfin, kf.size() * sizeof(int), hipMemcpyDeviceToHost, s));
        PDZ_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < b->n; ++i)
            if (kf[i] > 0) {
                res[i].E0_refined = er[i];
                res[i].resid_refined = er[b->n + i];
            }
        // leave the control blocks as the run ended
        PDZ_HIP(hipMemcpyAsync(ctl, h.data(), b->n * sizeof(BCtl), hipMemcpyHostToDevice, s));
        PDZ_HIP(hipStreamSynchronize(s));
    }
    return all_conv ? ok() : fail(PDZ_ENOCONV, "max_iter reached before every cluster met the tolerance");
}

}  // namespace

extern "C" {

pdz_status pdz_batch_create(const pdz_problem* problems, int32_t n, pdz_batch* out) {
    if (!out) return fail(PDZ_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !problems) return fail(PDZ_EINVAL, "need at least one problem");
    int dev = 0;
    PDZ_HIP(hipGetDevice(&dev));
    for (int i = 0; i < n; ++i) {
        if (!problems[i]) return fail(PDZ_EINVAL, "NULL problem in batch");
        if (problems[i]->device != dev) return fail(PDZ_EINVAL, "batch problems must live on the current device");
        if (problems[i]->hv_path != 0) return fail(PDZ_ERANGE, "batched H.v needs sector hop tables");
    }
    pdz_batch_s* b = new pdz_batch_s();
    b->device = dev;
    b->n = n;
    b->problems.assign(problems, problems + n);
    b->offsets.resize(n + 1);
    uint64_t off = 0;
    std::vector<BProb> hp(n);
    std::vector<BChunk> chunks;
    std::vector<uint32_t> cb(n + 1);
    for (int i = 0; i < n; ++i) {
        const pdz_problem q = problems[i];
        b->offsets[i] = off;
        hp[i].off = off;
        hp[i].D_up = q->up.D;
        hp[i].D_dn = q->dn.D;
        hp[i].U = q->U;
        hp[i].up_states = q->up.states;
        hp[i].dn_states = q->dn.states;
        hp[i].up_count = q->up.count;
        hp[i].dn_count = q->dn.count;
        hp[i].up_ell = q->up.ell;
        hp[i].dn_ell = q->dn.ell;
        hp[i].coef64 = q->d_coef64;
        hp[i].coef32 = q->d_coef32;
        hp[i].ncoef = (int)q->coef_host.size();
        hp[i].pad = 0;
        b->max_D_dn = std::max<uint64_t>(b->max_D_dn, q->dn.D);
        cb[i] = (uint32_t)chunks.size();
        for (uint64_t s0 = 0; s0 < q->D; s0 += kChunk) {
            BChunk c;
            c.prob = (uint32_t)i;
            c.pad = 0;
            c.begin = s0;
            c.end = std::min<uint64_t>(q->D, s0 + kChunk);
            chunks.push_back(c);
        }
        off += (q->D + kAlign - 1) / kAlign * kAlign;
    }
    cb[n] = (uint32_t)chunks.size();
    b->offsets[n] = off;
    b->total = off;
    b->nchunks = (uint32_t)chunks.size();
    auto cleanup = [&](pdz_status code) {
        pdz_batch_destroy(b);
        return code;
    };
#define BCK(call)                                                   \
    do {                                                            \
        hipError_t e_ = (call);                                     \
        if (e_ != hipSuccess) return cleanup(hip_fail(e_, #call)); \
    } while (0)
    BCK(hipMalloc(&b->d_probs, n * sizeof(BProb)));
    BCK(hipMemcpy(b->d_probs, hp.data(), n * sizeof(BProb), hipMemcpyHostToDevice));
    BCK(hipMalloc(&b->d_chunks, chunks.size() * sizeof(BChunk)));
    BCK(hipMemcpy(b->d_chunks, chunks.data(), chunks.size() * sizeof(BChunk), hipMemcpyHostToDevice));
    BCK(hipMalloc(&b->d_chunk_begin, (n + 1) * sizeof(uint32_t)));
    BCK(hipMemcpy(b->d_chunk_begin, cb.data(), (n + 1) * sizeof(uint32_t), hipMemcpyHostToDevice));
    BCK(hipMalloc(&b->d_queue, 256));
#undef BCK
    if (!plan_ok(b, resolve(b))) return cleanup(fail(PDZ_ERANGE, "a cluster row does not fit the batched kernel's LDS"));
    pdz_status st = build_tiles(b, resolve(b));
    if (st != PDZ_OK) return cleanup(st);
    *out = b;
    return ok();
}

pdz_status pdz_batch_destroy(pdz_batch b) {
    if (!b) return ok();
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    if (b->d_probs) (void)hipFree(b->d_probs);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_chunks) (void)hipFree(b->d_chunks);
    if (b->d_chunk_begin) (void)hipFree(b->d_chunk_begin);
    if (b->d_queue) (void)hipFree(b->d_queue);
    (void)hipSetDevice(prev);
    delete b;
    return ok();
}

pdz_status pdz_batch_offsets(pdz_batch b, uint64_t* offsets) {
    if (!b || !offsets) return fail(PDZ_EINVAL, "NULL argument");
    for (int i = 0; i <= b->n; ++i) offsets[i] = b->offsets[i];
    return ok();
}

pdz_status pdz_batch_get_plan(pdz_batch b, pdz_batch_plan* out) {
    if (!b || !out) return fail(PDZ_EINVAL, "NULL argument");
    *out = resolve(b);
    return ok();
}

pdz_status pdz_batch_set_plan(pdz_batch b, const pdz_batch_plan* plan) {
    if (!b || !plan) return fail(PDZ_EINVAL, "NULL argument");
    pdz_batch_plan p = *plan;
    const pdz_batch_plan d = resolve(b);
    if (p.tile_elems == 0) p.tile_elems = d.tile_elems;
    if (p.block == 0) p.block = d.block;
    if (p.wgs_per_cu == 0) p.wgs_per_cu = d.wgs_per_cu;
    if (p.order == 0) p.order = d.order;
    if (!plan_ok(b, p)) return fail(PDZ_EINVAL, "batch plan out of range");
    pdz_status st = build_tiles(b, p);
    if (st != PDZ_OK) return st;
    b->plan = p;
    return ok();
}

pdz_status pdz_batch_hv(pdz_batch b, pdz_dtype dt, const void* x, void* y, void* stream) {
    if (!b) return fail(PDZ_EINVAL, "batch is NULL");
    if (dt != PDZ_F64 && dt != PDZ_F32) return fail(PDZ_EINVAL, "dtype must be PDZ_F64 or PDZ_F32");
    if (!x || !y) return fail(PDZ_EINVAL, "NULL vector");
    const size_t bytes = (size_t)b->total * (dt == PDZ_F64 ? 8 : 4);
    const char* xb = static_cast<const char*>(x);
    const char* yb = static_cast<const char*>(y);
    if (xb < yb + bytes && yb < xb + bytes) return fail(PDZ_EINVAL, "x and y overlap");
    return batch_hv_any(b, dt, x, y, (hipStream_t)stream, nullptr, 0);
}

pdz_status pdz_batch_tune(pdz_batch b, pdz_dtype dt, const void* x, void* y, int32_t reps, pdz_batch_trial* trials,
                          int32_t max_trials, int32_t* n_trials, pdz_batch_plan* best, void* stream) {
    if (!b || !x || !y) return fail(PDZ_EINVAL, "NULL argument");
    if (dt != PDZ_F64 && dt != PDZ_F32) return fail(PDZ_EINVAL, "dtype must be PDZ_F64 or PDZ_F32");
    if (reps < 1) return fail(PDZ_EINVAL, "reps must be >= 1");
    if (max_trials > 0 && !trials) return fail(PDZ_EINVAL, "trials is NULL");
    hipStream_t s = (hipStream_t)stream;
    const pdz_batch_plan saved = resolve(b);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PDZ_HIP(hipEventCreate(&e0));
    PDZ_HIP(hipEventCreate(&e1));
    double best_ms = 1e300;
    pdz_batch_plan bp = saved;
    int n = 0;
    pdz_status st = ok();
    const int tes[] = {1024, 2048, 4096, 8192};
    const int bls[] = {256, 512, 1024};
    const int wgs[] = {2, 4, 8};
    const int ods[] = {1, 2};
    for (int te : tes)
        for (int bl : bls)
            for (int wg : wgs)
                for (int od : ods) {
                    pdz_batch_plan c{te, bl, wg, od};
                    if (!plan_ok(b, c)) continue;
                    // prune: natural order only with the default tile size (largest-first wins by cost model)
                    if (od == 2 && te != 4096) continue;
                    st = pdz_batch_set_plan(b, &c);
                    if (st != PDZ_OK) break;
                    st = pdz_batch_hv(b, dt, x, y, stream);
                    if (st != PDZ_OK) break;
                    hipError_t e = hipEventRecord(e0, s);
                    for (int r = 0; r < reps && st == PDZ_OK; ++r) st = pdz_batch_hv(b, dt, x, y, stream);
                    if (st != PDZ_OK) break;
                    if (e == hipSuccess) e = hipEventRecord(e1, s);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    float ms = 0.f;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                    if (e != hipSuccess) {
                        st = hip_fail(e, "batch autotune timing");
                        break;
                    }
                    const double avg = (double)ms / reps;
                    if (n < max_trials) {
                        trials[n].plan = c;
                        trials[n].ms = avg;
                    }
                    ++n;
                    if (avg < best_ms) {
                        best_ms = avg;
                        bp = c;
                    }
                }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != PDZ_OK) {
        (void)pdz_batch_set_plan(b, &saved);
        return st;
    }
    st = pdz_batch_set_plan(b, &bp);
    if (st != PDZ_OK) return st;
    if (n_trials) *n_trials = n < max_trials ? n : max_trials;
    if (best) *best = bp;
    return ok();
}

pdz_status pdz_batch_lanczos_workspace_size(pdz_batch b, const pdz_lanczos_opts* o, size_t* bytes) {
    if (!b || !o || !bytes) return fail(PDZ_EINVAL, "NULL argument");
    if (o->max_iter < 1 || o->max_iter > kBatchMaxIter) return fail(PDZ_EINVAL, "max_iter must be in [1, 2000]");
    *bytes = blayout(b, o).total;
    return ok();
}

pdz_status pdz_batch_lanczos(pdz_batch b, const pdz_lanczos_opts* o, void* ws, size_t ws_bytes,
                             pdz_lanczos_result* results, void* stream) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!b || !o || !results) return fail(PDZ_EINVAL, "NULL argument");
    if (o->max_iter < 1 || o->max_iter > kBatchMaxIter) return fail(PDZ_EINVAL, "max_iter must be in [1, 2000]");
    if (!(o->tol >= 0.0) || !std::isfinite(o->tol)) return fail(PDZ_EINVAL, "tol must be finite and >= 0");
    if (o->storage != PDZ_F64 && o->storage != PDZ_F32) return fail(PDZ_EINVAL, "storage must be F64 or F32");
    if (o->check_every < 1) return fail(PDZ_EINVAL, "check_every must be >= 1");
    if (o->reorth != 0) return fail(PDZ_EINVAL, "batched Lanczos runs the three-term recurrence (reorth must be 0)");
    if (o->refine != 0 && o->refine != 1) return fail(PDZ_EINVAL, "refine must be 0 or 1");
    if (o->keep_basis != 0) return fail(PDZ_EINVAL, "keep_basis is not offered for batches (refine regenerates)");
    const BLayout L = blayout(b, o);
    if (!ws || ws_bytes < L.total) return fail(PDZ_EINVAL, "workspace smaller than pdz_batch_lanczos_workspace_size");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(PDZ_EINVAL, "workspace must be 256-byte aligned");
    DeviceCtx* ctx = nullptr;
    pdz_status st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipStream_t own = nullptr;
    if (!s && o->use_graph) {
        PDZ_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
        PDZ_HIP(hipDeviceSynchronize());
        s = own;
    }
    std::memset(results, 0, sizeof(pdz_lanczos_result) * b->n);
    if (o->storage == PDZ_F64)
        st = batch_lanczos_run<double>(b, o, static_cast<char*>(ws), L, results, s, ctx->err);
    else
        st = batch_lanczos_run<float>(b, o, static_cast<char*>(ws), L, results, s, ctx->err);
    if (own) {
        (void)hipStreamSynchronize(own);
        (void)hipStreamDestroy(own);
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < b->n; ++i) results[i].seconds = secs;
    return st;
}

}  // extern "C"
