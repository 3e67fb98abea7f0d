// Learned Lanczos start vector: a 32 -> 128 -> 128 -> 2 tanh network on
// occupation strings, its training kernels and its inference over a basis.
//
// Parameters live in one vector (W1 128x32, b1, W2 128x128, b2, W3 2x128, b3;
// 20,994 values): FP32 master copy for Adam, BF16 copy for the kernels.
// Dense products run on the BF16 matrix cores (16x16x32, FP32 accumulation):
// one wave multiplies a tile of 16 states by the weights; a tile's first
// hidden layer goes through LDS to change from the accumulator layout to the
// operand layout of the second product.  Stored activations are BF16.
//
// Training samples states with probability proportional to |psi|^2 using
// integer weights w_r = floor(2^32 psi_r^2 / max psi^2), an exact prefix sum
// and a SplitMix64 draw per sample, so the draws do not depend on summation
// order.
#include <cmath>
#include <mutex>
#include <vector>

#include "pdz_internal.h"

namespace pdz {
namespace {

constexpr int kIn = 32, kHid = 128, kOut = 2;
constexpr int kParams = kHid * kIn + kHid + kHid * kHid + kHid + kOut * kHid + kOut;   // 20,994
constexpr int oW1 = 0, oB1 = kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kOut * kHid;
static_assert(oB3 + kOut == kParams, "parameter layout");
constexpr int kLd1 = kIn + 8;    // padded LDS row of W1 (bf16 elements)
constexpr int kLd2 = kHid + 8;   // padded LDS row of W2 / W2^T / hidden tiles
constexpr int kSlice = 512;      // states per partial weight gradient
constexpr int kLossBlocks = 64;
constexpr int kScanChunk = 8192;   // elements per block of the sampler prefix sum (32 per thread)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(p));
}
__device__ __forceinline__ bf16x8 pack8(const uint16_t* v) {
    u32x4 u;
    u.x = v[0] | ((uint32_t)v[1] << 16);
    u.y = v[2] | ((uint32_t)v[3] << 16);
    u.z = v[4] | ((uint32_t)v[5] << 16);
    u.w = v[6] | ((uint32_t)v[7] << 16);
    return __builtin_bit_cast(bf16x8, u);
}
__device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
// tanh(x) = 1 - 2 / (exp(2x) + 1); saturates to +-1 for large |x|
__device__ __forceinline__ float tanh_fast(float x) {
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(__expf(2.0f * x) + 1.0f);
}
// 8 features (+-1 in BF16) of one operand slot: bits [off, off + 8) of `bits`
__device__ __forceinline__ bf16x8 feature8(uint32_t bits) {
    uint16_t v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = ((bits >> t) & 1u) ? (uint16_t)0x3F80 : (uint16_t)0xBF80;
    return pack8(v);
}
__device__ __forceinline__ float pick4(const float* p, int i) {
    return i == 0 ? p[0] : (i == 1 ? p[1] : (i == 2 ? p[2] : p[3]));
}

// Source of the states of a forward pass.
struct StateSrc {
    const uint32_t* occ;        // list mode: occ[2s] up bits, occ[2s+1] down bits
    const uint32_t* up_states;  // basis mode: state s = r is (up_states[r / D_dn], dn_states[r % D_dn])
    const uint32_t* dn_states;
    uint64_t D_dn;
};
template <bool BASIS>
__device__ __forceinline__ void state_of(const StateSrc& S, uint64_t s, uint32_t* up, uint32_t* dn) {
    if (BASIS) {
        const uint64_t iu = s / S.D_dn;
        *up = S.up_states[iu];
        *dn = S.dn_states[s - iu * S.D_dn];
    } else {
        *up = S.occ[2 * s];
        *dn = S.occ[2 * s + 1];
    }
}

struct Act {                 // saved activations of a training forward pass (BF16)
    uint16_t* h1;            // n x 128, state major
    uint16_t* h1t;           // 128 x n
    uint16_t* h2;            // n x 128
};

// Forward pass over n states.  BASIS = false: outputs (n x 2) and, when
// act.h1 != NULL, the activations; BASIS = true: the start vector
// v0[s] = sign * exp(min(o_0, 60)), sign = + for o_1 >= 0.
template <typename T, bool BASIS>
__global__ __launch_bounds__(256) void k_mlp_fwd(const uint16_t* __restrict__ prm, StateSrc src, uint64_t n,
                                                 float* __restrict__ out, Act act, T* __restrict__ v0) {
    __shared__ __align__(16) uint16_t sW1[kHid * kLd1];
    __shared__ __align__(16) uint16_t sW2[kHid * kLd2];
    __shared__ __align__(16) uint16_t sH[4][16 * kLd2];
    __shared__ float sb1[kHid], sb2[kHid], sW3[kOut * kHid], sb3[kOut];
    const int tid = threadIdx.x;
    for (int i = tid; i < kHid * kIn; i += 256) sW1[(i / kIn) * kLd1 + (i % kIn)] = prm[oW1 + i];
    for (int i = tid; i < kHid * kHid; i += 256) sW2[(i / kHid) * kLd2 + (i % kHid)] = prm[oW2 + i];
    for (int i = tid; i < kHid; i += 256) {
        sb1[i] = bf2f(prm[oB1 + i]);
        sb2[i] = bf2f(prm[oB2 + i]);
    }
    for (int i = tid; i < kOut * kHid; i += 256) sW3[i] = bf2f(prm[oW3 + i]);
    if (tid < kOut) sb3[tid] = bf2f(prm[oB3 + tid]);
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
    uint16_t* h = sH[wave];
    const uint64_t ngroups = (n + 63) / 64;
    for (uint64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {   // block-uniform trip count
        const uint64_t s0 = grp * 64 + (uint64_t)wave * 16;
        // ---- layer 1: operand A holds state s0 + c, features 8g .. 8g+7
        uint32_t up = 0, dn = 0;
        {
            const uint64_t sa = s0 + c;
            state_of<BASIS>(src, sa < n ? sa : n - 1, &up, &dn);
        }
        const bf16x8 A1 = feature8(((g < 2) ? up : dn) >> (8 * (g & 1)));
#pragma unroll
        for (int ct = 0; ct < 8; ++ct) {
            const int j = 16 * ct + c;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = mma(A1, ld8(sW1 + j * kLd1 + 8 * g), acc);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint16_t hb = f2bf(tanh_fast(acc[t] + sb1[j]));
                h[(4 * g + t) * kLd2 + j] = hb;
                const uint64_t s = s0 + 4 * g + t;
                if (!BASIS && act.h1 && s < n) {
                    act.h1[s * kHid + j] = hb;
                    act.h1t[(uint64_t)j * n + s] = hb;
                }
            }
        }
        __syncthreads();
        // ---- layer 2: operand A = row c of the tile, features 32kc + 8g ..
        bf16x8 A2[4];
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) A2[kc] = ld8(h + c * kLd2 + 32 * kc + 8 * g);
        float p0[4] = {0.f, 0.f, 0.f, 0.f}, p1[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ct = 0; ct < 8; ++ct) {
            const int j = 16 * ct + c;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) acc = mma(A2[kc], ld8(sW2 + j * kLd2 + 32 * kc + 8 * g), acc);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint16_t hb = f2bf(tanh_fast(acc[t] + sb2[j]));
                const float hq = bf2f(hb);
                const uint64_t s = s0 + 4 * g + t;
                if (!BASIS && act.h2 && s < n) act.h2[s * kHid + j] = hb;
                p0[t] += hq * sW3[j];
                p1[t] += hq * sW3[kHid + j];
            }
        }
        // ---- layer 3: sum the 16 lanes of each state group
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int m = 1; m < 16; m <<= 1) {
                p0[t] += __shfl_xor(p0[t], m);
                p1[t] += __shfl_xor(p1[t], m);
            }
        if (c < 4) {
            const uint64_t s = s0 + 4 * g + c;
            if (s < n) {
                const float o0 = pick4(p0, c) + sb3[0];
                const float o1 = pick4(p1, c) + sb3[1];
                if (BASIS) {
                    const double a = exp((double)fminf(o0, 60.0f));
                    v0[s] = (T)(o1 >= 0.0f ? a : -a);
                } else {
                    out[2 * s] = o0;
                    out[2 * s + 1] = o1;
                }
            }
        }
        __syncthreads();   // the tile buffer is rewritten by the next group
    }
}

// dout and the per-block loss partial sums.
__global__ __launch_bounds__(256) void k_mlp_loss(const float* __restrict__ out, const float* __restrict__ target,
                                                  uint64_t n, float* __restrict__ dout, double* partial) {
    __shared__ double red[256];
    double acc = 0.0;
    const float inv_n = 1.0f / (float)n;
    for (uint64_t s = blockIdx.x * 256ull + threadIdx.x; s < n; s += (uint64_t)gridDim.x * 256) {
        const float a = out[2 * s], z = out[2 * s + 1];
        const float la = target[2 * s];
        const float y = target[2 * s + 1] > 0.0f ? 1.0f : 0.0f;
        const float d = a - la;
        const float sp = fmaxf(z, 0.0f) + log1pf(expf(-fabsf(z)));   // softplus(z)
        acc += (double)(d * d) + (double)sp - (double)(y * z);
        dout[2 * s] = 2.0f * d * inv_n;
        dout[2 * s + 1] = (1.0f / (1.0f + expf(-z)) - y) * inv_n;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_sum_partials(const double* partial, int np, double scale, double* result) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < np; ++i) s += partial[i];
        *result = s * scale;
    }
}

// Backward, per state: dz2 = (dout W3) (1 - h2^2) and dz1 = (dz2 W2) (1 - h1^2),
// both stored transposed (BF16).  One wave per tile of 16 states; n % 16 == 0.
__global__ __launch_bounds__(256) void k_mlp_bwd_act(const uint16_t* __restrict__ prm, uint64_t n, Act act,
                                                     const float* __restrict__ dout, uint16_t* __restrict__ dz2t,
                                                     uint16_t* __restrict__ dz1t) {
    __shared__ __align__(16) uint16_t sW2t[kHid * kLd2];   // sW2t[j][o] = W2[o][j]
    __shared__ float sW3[kOut * kHid];
    const int tid = threadIdx.x;
    for (int i = tid; i < kHid * kHid; i += 256) sW2t[(i % kHid) * kLd2 + (i / kHid)] = prm[oW2 + i];
    for (int i = tid; i < kOut * kHid; i += 256) sW3[i] = bf2f(prm[oW3 + i]);
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63, g = lane >> 4, c = lane & 15;
    const uint64_t ntiles = n / 16;
    for (uint64_t tile = (uint64_t)blockIdx.x * 4 + wave; tile < ntiles; tile += (uint64_t)gridDim.x * 4) {
        const uint64_t s0 = tile * 16;
        // dz2 of state s0 + c, units 32kc + 8g + t, in operand layout
        const uint64_t sa = s0 + c;
        const float d0 = dout[2 * sa], d1 = dout[2 * sa + 1];
        bf16x8 A[4];
#pragma unroll
        for (int kc = 0; kc < 4; ++kc) {
            const int o0 = 32 * kc + 8 * g;
            const u32x4 hv = *reinterpret_cast<const u32x4*>(act.h2 + sa * kHid + o0);
            uint16_t v[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const uint32_t w = hv[t >> 1];
                const float h2 = bf2f((uint16_t)((t & 1) ? (w >> 16) : (w & 0xFFFFu)));
                const float dz = (d0 * sW3[o0 + t] + d1 * sW3[kHid + o0 + t]) * (1.0f - h2 * h2);
                v[t] = f2bf(dz);
                dz2t[(uint64_t)(o0 + t) * n + sa] = v[t];
            }
            A[kc] = pack8(v);
        }
        // dh1 = dz2 W2 on the matrix cores; accumulator rows 4g + t, column j
#pragma unroll
        for (int ct = 0; ct < 8; ++ct) {
            const int j = 16 * ct + c;
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kc = 0; kc < 4; ++kc) acc = mma(A[kc], ld8(sW2t + j * kLd2 + 32 * kc + 8 * g), acc);
            const uint64_t s = s0 + 4 * g;
            const uint2 h1w = *reinterpret_cast<const uint2*>(act.h1t + (uint64_t)j * n + s);
            uint16_t o[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t w = (t < 2) ? h1w.x : h1w.y;
                const float h1 = bf2f((uint16_t)((t & 1) ? (w >> 16) : (w & 0xFFFFu)));
                o[t] = f2bf(acc[t] * (1.0f - h1 * h1));
            }
            uint2 st;
            st.x = o[0] | ((uint32_t)o[1] << 16);
            st.y = o[2] | ((uint32_t)o[3] << 16);
            *reinterpret_cast<uint2*>(dz1t + (uint64_t)j * n + s) = st;
        }
    }
}

// Weight-gradient partials over one slice of states (one wave per job):
// jobs 0..63: 16x16 tiles of dW2 = dz2^T h1 (tiles of column block 0 also
// b2 = dz2^T 1, a second product with an all-ones operand); jobs 64..71:
// 16-unit rows of dW1 = dz1^T x (and b1 = dz1^T 1); jobs 72..79: 16 columns
// of W3 = dout^T h2 each, the 64 lanes as 16 columns x 4 interleaved sample
// streams (job 72 also b3 = dout^T 1).  part[slice * kParams + k].
constexpr int kGradJobs = 80;
__global__ __launch_bounds__(64) void k_mlp_bwd_grad(const uint32_t* __restrict__ occ, uint64_t n, Act act,
                                                     const float* __restrict__ dout,
                                                     const uint16_t* __restrict__ dz2t,
                                                     const uint16_t* __restrict__ dz1t, float* __restrict__ part) {
    const int job = blockIdx.x;
    const int slice = blockIdx.y;
    const uint64_t b0 = (uint64_t)slice * kSlice;
    const uint64_t b1 = (b0 + kSlice < n) ? b0 + kSlice : n;
    const int lane = threadIdx.x, g = lane >> 4, c = lane & 15;
    float* P = part + (size_t)slice * kParams;
    const uint16_t one8[8] = {0x3F80, 0x3F80, 0x3F80, 0x3F80, 0x3F80, 0x3F80, 0x3F80, 0x3F80};   // BF16 1.0
    const bf16x8 ones = pack8(one8);
    if (job < 64) {
        const int ot = job >> 3, jt = job & 7;
        const int o = 16 * ot + c, j = 16 * jt + c;
        const bool bias = jt == 0;   // wave-uniform
        f32x4 acc = {0.f, 0.f, 0.f, 0.f}, accb = {0.f, 0.f, 0.f, 0.f};
        for (uint64_t s = b0; s < b1; s += 32) {
            const bf16x8 a = ld8(dz2t + (uint64_t)o * n + s + 8 * g);
            acc = mma(a, ld8(act.h1t + (uint64_t)j * n + s + 8 * g), acc);
            if (bias) accb = mma(a, ones, accb);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) P[oW2 + (16 * ot + 4 * g + t) * kHid + j] = acc[t];
        if (bias && c == 0)   // every column of accb holds the row sums
#pragma unroll
            for (int t = 0; t < 4; ++t) P[oB2 + 16 * ot + 4 * g + t] = accb[t];
    } else if (job < 72) {
        const int ot = job - 64;
        const int o = 16 * ot + c;
        f32x4 accb = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            const int i = 16 * it + c;   // feature i: up site i (i < 16) or down site i - 16
            for (uint64_t s = b0; s < b1; s += 32) {
                uint16_t v[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const uint32_t bits = occ[2 * (s + 8 * g + t) + (i >> 4)];
                    v[t] = ((bits >> (i & 15)) & 1u) ? (uint16_t)0x3F80 : (uint16_t)0xBF80;
                }
                const bf16x8 a = ld8(dz1t + (uint64_t)o * n + s + 8 * g);
                acc = mma(a, pack8(v), acc);
                if (it == 0) accb = mma(a, ones, accb);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) P[oW1 + (16 * ot + 4 * g + t) * kIn + i] = acc[t];
        }
        if (c == 0)
#pragma unroll
            for (int t = 0; t < 4; ++t) P[oB1 + 16 * ot + 4 * g + t] = accb[t];
    } else {
        const int jt = job - 72;
        const int j = 16 * jt + c;
        float a0 = 0.f, a1 = 0.f;
        constexpr int U = 8;   // loads in flight per lane
        for (uint64_t s0 = b0 + (uint64_t)g; s0 < b1; s0 += 4 * U) {
            float h[U], d0[U], d1[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint64_t s = s0 + 4 * (uint64_t)u;
                const bool in = s < b1;
                h[u] = in ? bf2f(act.h2[s * kHid + j]) : 0.f;
                d0[u] = in ? dout[2 * s] : 0.f;
                d1[u] = in ? dout[2 * s + 1] : 0.f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                a0 += d0[u] * h[u];
                a1 += d1[u] * h[u];
            }
        }
        a0 += __shfl_xor(a0, 16);
        a0 += __shfl_xor(a0, 32);
        a1 += __shfl_xor(a1, 16);
        a1 += __shfl_xor(a1, 32);
        if (g == 0) {
            P[oW3 + j] = a0;
            P[oW3 + kHid + j] = a1;
        }
        if (jt == 0) {
            float e0 = 0.f, e1 = 0.f;
            for (uint64_t s = b0 + (uint64_t)lane; s < b1; s += 64) {
                e0 += dout[2 * s];
                e1 += dout[2 * s + 1];
            }
            for (int m = 32; m > 0; m >>= 1) {
                e0 += __shfl_xor(e0, m);
                e1 += __shfl_xor(e1, m);
            }
            if (lane == 0) {
                P[oB3] = e0;
                P[oB3 + 1] = e1;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_mlp_grad_reduce(const float* __restrict__ part, int slices,
                                                         float* __restrict__ grad) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= kParams) return;
    float s = 0.f;
    for (int i = 0; i < slices; ++i) s += part[(size_t)i * kParams + k];
    grad[k] = s;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ w, uint16_t* __restrict__ wb,
                                              const float* __restrict__ grad, float* __restrict__ m,
                                              float* __restrict__ v, uint64_t count, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
    const uint64_t k = blockIdx.x * 256ull + threadIdx.x;
    if (k >= count) return;
    const float gk = grad[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    const float wk = w[k] - lr * (mk / c1) / (sqrtf(vk / c2) + eps);
    w[k] = wk;
    wb[k] = f2bf(wk);
}

__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ w, uint16_t* __restrict__ wb,
                                                 uint64_t count) {
    const uint64_t k = blockIdx.x * 256ull + threadIdx.x;
    if (k < count) wb[k] = f2bf(w[k]);
}

// ------------------------------------------------------------------ sampler

__device__ __forceinline__ uint64_t qweight(double p, double m) {
    return (uint64_t)floor(p * p / m * 4294967296.0);
}

__global__ __launch_bounds__(256) void k_max_sq(const double* __restrict__ psi, uint64_t D, double* partial) {
    __shared__ double red[256];
    double mx = 0.0;
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < D; i += (uint64_t)gridDim.x * 256)
        mx = fmax(mx, psi[i] * psi[i]);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_max_final(const double* partial, int np, double* result) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double m = 0.0;
        for (int i = 0; i < np; ++i) m = fmax(m, partial[i]);
        *result = m;
    }
}

// sums[b] = sum of the weights of chunk b
__global__ __launch_bounds__(256) void k_chunk_sums(const double* __restrict__ psi, uint64_t D, const double* mx,
                                                    uint64_t* sums) {
    __shared__ uint64_t red[256];
    const double m = *mx;
    const uint64_t c0 = (uint64_t)blockIdx.x * kScanChunk;
    uint64_t acc = 0;
    for (uint64_t i = c0 + threadIdx.x; i < c0 + kScanChunk && i < D; i += 256) acc += qweight(psi[i], m);
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

// exclusive scan of the chunk sums in place (one block), total in *total
__global__ __launch_bounds__(256) void k_scan_sums(uint64_t* sums, uint64_t nchunks, uint64_t* total) {
    __shared__ uint64_t sh[256];
    uint64_t carry = 0;
    for (uint64_t base = 0; base < nchunks; base += 256) {
        const uint64_t i = base + threadIdx.x;
        const uint64_t v = i < nchunks ? sums[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {   // inclusive Hillis-Steele scan
            const uint64_t add = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nchunks) sums[i] = carry + sh[threadIdx.x] - v;
        carry += sh[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// prefix[r] = inclusive prefix sum of the weights; 32 consecutive elements per thread
__global__ __launch_bounds__(256) void k_chunk_scan(const double* __restrict__ psi, uint64_t D, const double* mx,
                                                    const uint64_t* offs, uint64_t* __restrict__ prefix) {
    __shared__ uint64_t sh[256];
    const double m = *mx;
    const uint64_t c0 = (uint64_t)blockIdx.x * kScanChunk + (uint64_t)threadIdx.x * 32;
    uint64_t w[32];
    uint64_t tot = 0;
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        const uint64_t i = c0 + q;
        w[q] = i < D ? qweight(psi[i], m) : 0;
        tot += w[q];
    }
    sh[threadIdx.x] = tot;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint64_t add = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    uint64_t run = offs[blockIdx.x] + sh[threadIdx.x] - tot;
#pragma unroll
    for (int q = 0; q < 32; ++q) {
        const uint64_t i = c0 + q;
        run += w[q];
        if (i < D) prefix[i] = run;
    }
}

__device__ __forceinline__ uint64_t splitmix_u64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_sample(const double* __restrict__ psi, const uint64_t* __restrict__ prefix,
                                                uint64_t D, const uint32_t* __restrict__ up_states,
                                                const uint32_t* __restrict__ dn_states, uint64_t D_dn, uint64_t seed,
                                                uint64_t first, uint64_t count, float gauge,
                                                uint32_t* __restrict__ occ, float* __restrict__ target,
                                                uint32_t* __restrict__ idx) {
    const uint64_t j = blockIdx.x * 256ull + threadIdx.x;
    if (j >= count) return;
    const uint64_t W = prefix[D - 1];
    const uint64_t t = __umul64hi(splitmix_u64(seed, first + j), W);
    uint64_t lo = 0, hi = D - 1;   // prefix[hi] = W > t
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (prefix[mid] > t)
            hi = mid;
        else
            lo = mid + 1;
    }
    const uint64_t r = lo;
    const uint64_t iu = r / D_dn;
    occ[2 * j] = up_states[iu];
    occ[2 * j + 1] = dn_states[r - iu * D_dn];
    const double p = psi[r];
    target[2 * j] = (float)log(fabs(p));
    target[2 * j + 1] = (p * gauge > 0.0) ? 1.0f : -1.0f;
    if (idx) idx[j] = (uint32_t)r;
}

// ----------------------------------------------------------------- vectors

template <typename T>
__global__ __launch_bounds__(256) void k_vdot(const T* __restrict__ a, const T* __restrict__ b, uint64_t n,
                                              double* partial) {
    __shared__ double red[256];
    double acc = 0.0;
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
        acc += (double)a[i] * (double)b[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct MlpWs {
    size_t dz2t = 0, dz1t = 0, part = 0, loss = 0, total = 0;
    int slices = 0;
};
MlpWs mlp_ws(uint64_t n) {
    MlpWs w;
    w.slices = (int)((n + kSlice - 1) / kSlice);
    size_t off = 0;
    w.dz2t = off;
    off += al256((size_t)n * kHid * 2);
    w.dz1t = off;
    off += al256((size_t)n * kHid * 2);
    w.part = off;
    off += al256((size_t)w.slices * kParams * 4);
    w.loss = off;
    off += al256(kLossBlocks * 8);
    w.total = off;
    return w;
}

struct SampWs {
    size_t prefix = 0, sums = 0, mx = 0, total = 0;
    uint64_t nchunks = 0;
};
SampWs samp_ws(uint64_t D) {
    SampWs w;
    w.nchunks = (D + kScanChunk - 1) / kScanChunk;
    size_t off = 0;
    w.prefix = off;
    off += al256((size_t)D * 8);
    w.sums = off;
    off += al256((size_t)(w.nchunks + 1) * 8);
    w.mx = off;
    off += al256(1024 * 8 + 8);
    w.total = off;
    return w;
}

int fwd_grid(uint64_t n) {
    DeviceCtx* ctx = nullptr;
    const int cu = (device_ctx(&ctx) == PDZ_OK && ctx) ? ctx->cu_count : 256;
    const uint64_t groups = (n + 63) / 64;
    const uint64_t g = (uint64_t)cu * 2;
    return (int)(groups < g ? groups : g);
}

Act act_views(void* act, uint64_t n) {
    Act a;
    uint16_t* base = static_cast<uint16_t*>(act);
    a.h1 = base;
    a.h1t = base ? base + (size_t)n * kHid : nullptr;
    a.h2 = base ? base + 2 * (size_t)n * kHid : nullptr;
    return a;
}

}  // namespace
}  // namespace pdz

using namespace pdz;

namespace {

// Partial sums of pdz_dot_noalloc: one array per device, held until the
// process ends.  Host code reaches it only through the address
// hipGetSymbolAddress returns on each device (dot_scratch_ptr).
constexpr int kDotPartials = 1024;
static __device__ __align__(256) double scratch[kDotPartials];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's array (the current device), looked up once per device.
pdz_status dot_scratch_ptr(double** out) {
    int dev = -1;
    PDZ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PDZ_EDEVICE, "device index outside the supported range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        PDZ_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(PDZ_EDEVICE, "no device address for the dot-product scratch array");
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return ok();
}

}  // namespace

extern "C" {

int32_t pdz_mlp_param_count(void) { return kParams; }

pdz_status pdz_mlp_init(float* params, uint16_t* params_bf16, uint64_t seed) {
    if (!params || !params_bf16) return fail(PDZ_EINVAL, "NULL argument");
    // weights uniform in +-1/sqrt(fan_in) from SplitMix64 output k of `seed`, biases zero
    std::vector<float> h(kParams, 0.0f);
    auto uni = [&](uint64_t k) {
        uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z = z ^ (z >> 31);
        return 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
    };
    for (int k = oW1; k < oB1; ++k) h[k] = (float)(uni(k) / std::sqrt((double)kIn));
    for (int k = oW2; k < oB2; ++k) h[k] = (float)(uni(k) / std::sqrt((double)kHid));
    for (int k = oW3; k < oB3; ++k) h[k] = (float)(uni(k) / std::sqrt((double)kHid));
    PDZ_HIP(hipMemcpy(params, h.data(), kParams * sizeof(float), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_to_bf16, dim3((kParams + 255) / 256), dim3(256), 0, 0, params, params_bf16,
                       (uint64_t)kParams);
    PDZ_HIP(hipGetLastError());
    PDZ_HIP(hipDeviceSynchronize());
    return ok();
}

pdz_status pdz_mlp_to_bf16(const float* params, uint16_t* params_bf16, void* stream) {
    if (!params || !params_bf16) return fail(PDZ_EINVAL, "NULL argument");
    hipLaunchKernelGGL(k_to_bf16, dim3((kParams + 255) / 256), dim3(256), 0, (hipStream_t)stream, params,
                       params_bf16, (uint64_t)kParams);
    PDZ_HIP(hipGetLastError());
    return ok();
}

pdz_status pdz_mlp_forward(const uint16_t* params_bf16, const uint32_t* occ, uint64_t n, float* out, void* act,
                           void* stream) {
    if (!params_bf16 || !out || (n > 0 && !occ)) return fail(PDZ_EINVAL, "NULL argument");
    if (n == 0) return ok();
    if (n > (1ull << 32)) return fail(PDZ_ERANGE, "at most 2^32 states per call");
    StateSrc src{occ, nullptr, nullptr, 1};
    const Act a = act_views(act, n);
    hipLaunchKernelGGL((k_mlp_fwd<float, false>), dim3(fwd_grid(n)), dim3(256), 0, (hipStream_t)stream, params_bf16,
                       src, n, out, a, (float*)nullptr);
    PDZ_HIP(hipGetLastError());
    return ok();
}

pdz_status pdz_mlp_workspace_size(uint64_t n, size_t* bytes) {
    if (!bytes) return fail(PDZ_EINVAL, "NULL argument");
    *bytes = mlp_ws(n).total;
    return ok();
}

pdz_status pdz_mlp_loss(const float* out, const float* target, uint64_t n, float* dout, double* loss, void* ws,
                        size_t ws_bytes, void* stream) {
    if (!out || !target || !dout || !loss || !ws) return fail(PDZ_EINVAL, "NULL argument");
    if (n == 0) return fail(PDZ_EINVAL, "empty batch");
    const MlpWs w = mlp_ws(n);
    if (ws_bytes < w.total) return fail(PDZ_EINVAL, "workspace smaller than pdz_mlp_workspace_size");
    double* part = reinterpret_cast<double*>(static_cast<char*>(ws) + w.loss);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_loss, dim3(kLossBlocks), dim3(256), 0, s, out, target, n, dout, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, part, kLossBlocks, 1.0 / (double)n, loss);
    PDZ_HIP(hipGetLastError());
    return ok();
}

pdz_status pdz_mlp_backward(const uint16_t* params_bf16, const uint32_t* occ, uint64_t n, const void* act,
                            const float* dout, float* grad, void* ws, size_t ws_bytes, void* stream) {
    if (!params_bf16 || !occ || !act || !dout || !grad || !ws) return fail(PDZ_EINVAL, "NULL argument");
    if (n == 0 || n % 32 != 0) return fail(PDZ_EINVAL, "the batch size must be a positive multiple of 32");
    if (n > (1ull << 24)) return fail(PDZ_ERANGE, "at most 2^24 states per training batch");
    const MlpWs w = mlp_ws(n);
    if (ws_bytes < w.total) return fail(PDZ_EINVAL, "workspace smaller than pdz_mlp_workspace_size");
    if (reinterpret_cast<uintptr_t>(ws) % 256 || reinterpret_cast<uintptr_t>(act) % 16)
        return fail(PDZ_EINVAL, "workspace must be 256-byte aligned and activations 16-byte aligned");
    char* base = static_cast<char*>(ws);
    uint16_t* dz2t = reinterpret_cast<uint16_t*>(base + w.dz2t);
    uint16_t* dz1t = reinterpret_cast<uint16_t*>(base + w.dz1t);
    float* part = reinterpret_cast<float*>(base + w.part);
    const Act a = act_views(const_cast<void*>(act), n);
    hipStream_t s = (hipStream_t)stream;
    const uint64_t tiles = n / 16;
    uint64_t grid = (tiles + 3) / 4;
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(k_mlp_bwd_act, dim3((unsigned)grid), dim3(256), 0, s, params_bf16, n, a, dout, dz2t, dz1t);
    hipLaunchKernelGGL(k_mlp_bwd_grad, dim3(kGradJobs, w.slices), dim3(64), 0, s, occ, n, a, dout, dz2t, dz1t, part);
    hipLaunchKernelGGL(k_mlp_grad_reduce, dim3((kParams + 255) / 256), dim3(256), 0, s, part, w.slices, grad);
    PDZ_HIP(hipGetLastError());
    return ok();
}

pdz_status pdz_adam_step(float* params, uint16_t* params_bf16, const float* grad, float* m, float* v, uint64_t count,
                         float lr, float beta1, float beta2, float eps, int32_t step, void* stream) {
    if (!params || !params_bf16 || !grad || !m || !v) return fail(PDZ_EINVAL, "NULL argument");
    if (step < 1) return fail(PDZ_EINVAL, "step counts from 1");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f && std::isfinite(lr)))
        return fail(PDZ_EINVAL, "Adam hyper-parameters out of range");
    if (count == 0) return ok();
    const float c1 = (float)(1.0 - std::pow((double)beta1, step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, step));
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, (hipStream_t)stream, params,
                       params_bf16, grad, m, v, count, lr, beta1, beta2, eps, c1, c2);
    PDZ_HIP(hipGetLastError());
    return ok();
}

pdz_status pdz_sampler_workspace_size(pdz_problem p, size_t* bytes) {
    if (!p || !bytes) return fail(PDZ_EINVAL, "NULL argument");
    *bytes = samp_ws(p->D).total;
    return ok();
}

pdz_status pdz_sampler_prepare(pdz_problem p, const double* psi, void* ws, size_t ws_bytes, void* stream) {
    if (!p || !psi || !ws) return fail(PDZ_EINVAL, "NULL argument");
    const SampWs w = samp_ws(p->D);
    if (ws_bytes < w.total) return fail(PDZ_EINVAL, "workspace smaller than pdz_sampler_workspace_size");
    if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(PDZ_EINVAL, "workspace must be 256-byte aligned");
    char* base = static_cast<char*>(ws);
    uint64_t* prefix = reinterpret_cast<uint64_t*>(base + w.prefix);
    uint64_t* sums = reinterpret_cast<uint64_t*>(base + w.sums);
    double* mx = reinterpret_cast<double*>(base + w.mx);   // [0] max, [1..1024] partials
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_max_sq, dim3(1024), dim3(256), 0, s, psi, p->D, mx + 1);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(64), 0, s, mx + 1, 1024, mx);
    hipLaunchKernelGGL(k_chunk_sums, dim3((unsigned)w.nchunks), dim3(256), 0, s, psi, p->D, mx, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, sums, w.nchunks, sums + w.nchunks);
    hipLaunchKernelGGL(k_chunk_scan, dim3((unsigned)w.nchunks), dim3(256), 0, s, psi, p->D, mx, sums, prefix);
    PDZ_HIP(hipGetLastError());
    return ok();
}

pdz_status pdz_sample(pdz_problem p, const double* psi, const void* ws, size_t ws_bytes, uint64_t seed,
                      uint64_t first, uint64_t count, double gauge, uint32_t* occ, float* target, uint32_t* idx,
                      void* stream) {
    if (!p || !psi || !ws || (count > 0 && (!occ || !target))) return fail(PDZ_EINVAL, "NULL argument");
    if (!(gauge == 1.0 || gauge == -1.0)) return fail(PDZ_EINVAL, "gauge must be +1 or -1");
    const SampWs w = samp_ws(p->D);
    if (ws_bytes < w.total) return fail(PDZ_EINVAL, "workspace smaller than pdz_sampler_workspace_size");
    if (count == 0) return ok();
    const uint64_t* prefix = reinterpret_cast<const uint64_t*>(static_cast<const char*>(ws) + w.prefix);
    hipLaunchKernelGGL(k_sample, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, (hipStream_t)stream, psi,
                       prefix, p->D, p->up.states, p->dn.states, p->dn.D, seed, first, count, (float)gauge, occ,
                       target, idx);
    PDZ_HIP(hipGetLastError());
    return ok();
}

pdz_status pdz_start_vector(pdz_problem p, const uint16_t* params_bf16, pdz_dtype dt, void* v0, void* stream) {
    if (!p || !params_bf16 || !v0) return fail(PDZ_EINVAL, "NULL argument");
    if (dt != PDZ_F64 && dt != PDZ_F32) return fail(PDZ_EINVAL, "dtype must be PDZ_F64 or PDZ_F32");
    if (p->N > 16) return fail(PDZ_ERANGE, "the network reads 16 sites per spin");
    StateSrc src{nullptr, p->up.states, p->dn.states, p->dn.D};
    const Act none = act_views(nullptr, 0);
    hipStream_t s = (hipStream_t)stream;
    if (dt == PDZ_F64)
        hipLaunchKernelGGL((k_mlp_fwd<double, true>), dim3(fwd_grid(p->D)), dim3(256), 0, s, params_bf16, src, p->D,
                           (float*)nullptr, none, static_cast<double*>(v0));
    else
        hipLaunchKernelGGL((k_mlp_fwd<float, true>), dim3(fwd_grid(p->D)), dim3(256), 0, s, params_bf16, src, p->D,
                           (float*)nullptr, none, static_cast<float*>(v0));
    PDZ_HIP(hipGetLastError());
    return ok();
}

pdz_status pdz_dot(pdz_dtype dt, const void* a, const void* b, uint64_t n, double* result, void* stream) {
    if (!a || !b || !result) return fail(PDZ_EINVAL, "NULL argument");
    if (dt != PDZ_F64 && dt != PDZ_F32) return fail(PDZ_EINVAL, "dtype must be PDZ_F64 or PDZ_F32");
    hipStream_t s = (hipStream_t)stream;
    double* d = nullptr;
    PDZ_HIP(hipMallocAsync((void**)&d, 1025 * sizeof(double), s));
    if (dt == PDZ_F64)
        hipLaunchKernelGGL(k_vdot<double>, dim3(1024), dim3(256), 0, s, static_cast<const double*>(a),
                           static_cast<const double*>(b), n, d + 1);
    else
        hipLaunchKernelGGL(k_vdot<float>, dim3(1024), dim3(256), 0, s, static_cast<const float*>(a),
                           static_cast<const float*>(b), n, d + 1);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, d + 1, 1024, 1.0, d);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(result, d, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFreeAsync(d, s);
    (void)hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "pdz_dot");
    return ok();
}

pdz_status pdz_dot_noalloc(pdz_dtype dt, const void* a, const void* b, uint64_t n, double* result, void* stream) {
    if (!a || !b || !result) return fail(PDZ_EINVAL, "NULL argument");
    if (dt != PDZ_F64 && dt != PDZ_F32) return fail(PDZ_EINVAL, "dtype must be PDZ_F64 or PDZ_F32");
    double* part = nullptr;
    pdz_status st = dot_scratch_ptr(&part);
    if (st != PDZ_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // every one of the kDotPartials work groups writes its partial sum, so
    // nothing of the previous call's contents is read
    if (dt == PDZ_F64)
        hipLaunchKernelGGL(k_vdot<double>, dim3(kDotPartials), dim3(256), 0, s, static_cast<const double*>(a),
                           static_cast<const double*>(b), n, part);
    else
        hipLaunchKernelGGL(k_vdot<float>, dim3(kDotPartials), dim3(256), 0, s, static_cast<const float*>(a),
                           static_cast<const float*>(b), n, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, part, kDotPartials, 1.0, result);
    PDZ_HIP(hipGetLastError());
    return ok();
}

}  // extern "C"
