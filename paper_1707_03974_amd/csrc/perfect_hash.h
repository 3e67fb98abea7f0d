// Device forms of the forward map (Eq. 3) and the backward map (Sec. III)
// over a binomial table staged in LDS (C[i * kBinomStride + m], exact integer
// arithmetic).  Shared by the hashing kernels and the fermion operators.
#pragma once
#include "pdz_internal.h"

namespace pdz {

__device__ __forceinline__ void stage_binom(uint32_t* sC, const uint32_t* __restrict__ gC) {
    for (int k = threadIdx.x; k < kBinomStride * kBinomStride; k += blockDim.x) sC[k] = gC[k];
    __syncthreads();
}

// rank of phi in the ascending list of strings with its popcount
__device__ __forceinline__ uint32_t forward_map(uint32_t phi, const uint32_t* sC) {
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

// string of rank p among the N-bit strings with n set bits
__device__ __forceinline__ uint32_t backward_map(uint32_t p, int n, int N, const uint32_t* sC) {
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

}  // namespace pdz
