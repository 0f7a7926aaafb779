// Device helpers shared by the kernel translation units of libcpgrad.
#pragma once

#include "cpg_internal.h"

namespace cpg {

// Khatri-Rao entry in float64: prod over modes m in [first, first+count) of
// A^(m)(i_m, r), (i_first, ...) = unravel(idx) with the first mode fastest
// (the row order of Notation 2.1's reverse-ordered products).
template <typename TC>
__device__ __forceinline__ double kr_entry_d(const FacSet<TC>& fs, int first, int count, int64_t idx, int r) {
    double v = 1.0;
    for (int m = 0; m < count; ++m) {
        const int64_t d = fs.dims[first + m];
        const int64_t q = idx / d;
        const int64_t i = idx - q * d;
        idx = q;
        v *= (double)fs.A[first + m][i * fs.R + r];
    }
    return v;
}

// Sum over the block (blockDim.x a power of two <= 1024); sbuf >= blockDim.x
// doubles.  Fixed tree order; every thread gets the total.
__device__ __forceinline__ double block_sum(double v, double* sbuf) {
    const int tid = threadIdx.x;
    sbuf[tid] = v;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if (tid < s) sbuf[tid] += sbuf[tid + s];
        __syncthreads();
    }
    const double t = sbuf[0];
    __syncthreads();
    return t;
}

// Uniform broadcast of lane `src`'s double (src must be wave-uniform).
__device__ __forceinline__ double readlane_d(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

}  // namespace cpg
