// Device helpers shared by the kernel translation units of libcpgrad.
#pragma once

#include "cpg_internal.h"

namespace cpg {

// Buffer resource over `bytes` bytes from `base` (raw addressing, stride 0).
// Loads at offsets >= bytes return zero and stores there are dropped, so
// ragged edges need no branches; kOOB is an offset that is always outside.
constexpr uint32_t kOOB = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

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

// Stores of split partials that another kernel reads: written through the
// L2 at system scope (cache policy sc0 sc1), so they stream out while the
// kernel runs instead of waiting in the L2 for the write-back at its end.
constexpr int kStoreThrough = 1 | 16;
__device__ __forceinline__ void store_through(float* p, float v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Uniform broadcast of lane `src`'s double (src must be wave-uniform).
__device__ __forceinline__ double readlane_d(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

}  // namespace cpg
