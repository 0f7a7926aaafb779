// Device side of the learned extrapolation step: factor copies, the step's
// features, the extrapolation A + sigma (A - A_start) and the accept test
// against the exactly evaluated cost.
#include <algorithm>

#include "cpg_device.h"

namespace cpg {

constexpr int kLearnThreads = 512;

template <typename TC>
__global__ __launch_bounds__(256) void k_copy_factors(FacSet<TC> dst, FacSet<TC> src) {
    const int n = blockIdx.y;
    const int64_t m = src.dims[n] * src.R;
    TC* d = (TC*)dst.A[n];
    const TC* s = src.A[n];
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < m; e += (int64_t)gridDim.x * 256) d[e] = s[e];
}

// out = A + sigma (A - As), sigma from *sigma_dev if non-null else sigma_val
template <typename TC>
__global__ __launch_bounds__(256) void k_extrapolate(FacSet<TC> out, FacSet<TC> A, FacSet<TC> As,
                                                     const float* __restrict__ sigma_dev, double sigma_val) {
    const int n = blockIdx.y;
    const int64_t m = A.dims[n] * A.R;
    const double sg = sigma_dev ? (double)*sigma_dev : sigma_val;
    TC* o = (TC*)out.A[n];
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < m; e += (int64_t)gridDim.x * 256) {
        const double a = (double)A.A[n][e];
        o[e] = (TC)(a + sg * (a - (double)As.A[n][e]));
    }
}

// keep the extrapolated factors if their cost is lower than the sweep's
template <typename TC>
__global__ __launch_bounds__(256) void k_accept(FacSet<TC> A, FacSet<TC> Aext, double* __restrict__ scal,
                                                int* __restrict__ accepted) {
    const double plain = scal[2], ext = scal[8];
    const bool take = ext < plain;   // NaN never accepted
    for (int n = 0; n < A.N; ++n) {
        const int64_t m = A.dims[n] * A.R;
        TC* a = (TC*)A.A[n];
        if (take)
            for (int64_t e = threadIdx.x; e < m; e += 256) a[e] = Aext.A[n][e];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        *accepted = take ? 1 : 0;
        if (take) {
            scal[2] = scal[8];
            scal[3] = scal[9];
        }
    }
}

struct FeatArgs {
    double costs[6];   // oldest first
    int ncost;
    const double* cur_cost;   // if set: appended as the newest cost (read on the device)
    int iteration;
    float last_sigma;
    int last_accept;
    int have_prev;     // the previous update Dp is valid
};

// Per-mode statistics of the update U = A - As and the previous update Dp,
// the feature vector, then Dp <- U.
template <typename TC>
__global__ __launch_bounds__(kLearnThreads) void k_features(FacSet<TC> A, FacSet<TC> As, FacSet<TC> Dp, FeatArgs fa,
                                                            float* __restrict__ feat) {
    constexpr int kWaves = kLearnThreads / 64;
    __shared__ double sw[CPG_MAX_MODES][4][kWaves];   // per-wave sums
    __shared__ double st[CPG_MAX_MODES][4];
    const int tid = threadIdx.x, w = tid >> 6;
    const int N = A.N, R = A.R;
    // per mode: each thread's terms in order, a butterfly in each wave, the
    // wave sums to LDS (no block barrier between modes); Dp <- A - As on the
    // way (each entry is read, then overwritten, by the same thread)
    for (int n = 0; n < N; ++n) {
        const int64_t m = A.dims[n] * R;
        TC* dp = (TC*)Dp.A[n];
        double uu = 0, aa = 0, ud = 0, dd = 0;
        for (int64_t e = tid; e < m; e += kLearnThreads) {
            const double a = (double)A.A[n][e];
            const double u = a - (double)As.A[n][e];
            const double d = fa.have_prev ? (double)dp[e] : 0.0;
            dp[e] = (TC)u;
            uu += u * u;
            aa += a * a;
            ud += u * d;
            dd += d * d;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            uu += __shfl_xor(uu, o);
            aa += __shfl_xor(aa, o);
            ud += __shfl_xor(ud, o);
            dd += __shfl_xor(dd, o);
        }
        if ((tid & 63) == 0) {
            sw[n][0][w] = uu;
            sw[n][1][w] = aa;
            sw[n][2][w] = ud;
            sw[n][3][w] = dd;
        }
    }
    __syncthreads();
    if (tid < 4 * N) {   // the waves in order
        const int n = tid >> 2, k = tid & 3;
        double v = 0.0;
        for (int ww = 0; ww < kWaves; ++ww) v += sw[n][k][ww];
        st[n][k] = v;
    }
    __syncthreads();
    if (tid == 0) {
        double costs[7];
        int nc = fa.ncost;
        for (int k = 0; k < nc; ++k) costs[k] = fa.costs[k];
        if (fa.cur_cost) costs[nc++] = *fa.cur_cost;
        float f[12];
        // relative cost decreases of the last four sweeps
        for (int k = 0; k < 4; ++k) {
            const int j = nc - 4 + k;   // decrease from costs[j-1] to costs[j]
            double rel = 1.0;
            if (j >= 1 && j < nc && costs[j - 1] > 0) rel = (costs[j - 1] - costs[j]) / costs[j - 1];
            rel = rel < 1e-12 ? 1e-12 : (rel > 1.0 ? 1.0 : rel);
            f[k] = (float)(log10(rel) / 12.0);
        }
        double lmean = 0, lmax = -1e30, cmean = 0, cmin = 1e30;
        for (int n = 0; n < N; ++n) {
            double ratio = sqrt(st[n][0]) / (sqrt(st[n][1]) + 1e-300);
            ratio = ratio < 1e-12 ? 1e-12 : ratio;
            const double lr = log10(ratio);
            lmean += lr / N;
            lmax = lr > lmax ? lr : lmax;
            double c = 0.0;
            if (fa.have_prev && st[n][0] > 0 && st[n][3] > 0) c = st[n][2] / sqrt(st[n][0] * st[n][3]);
            cmean += c / N;
            cmin = c < cmin ? c : cmin;
        }
        f[4] = (float)(lmean / 6.0);
        f[5] = (float)(lmax / 6.0);
        f[6] = (float)cmean;
        f[7] = (float)cmin;
        f[8] = (float)R / 20.f;
        f[9] = (float)(log10((double)fa.iteration + 1.0) / 4.0);
        f[10] = (float)(log1p((double)fa.last_sigma) / log1p(32.0));
        f[11] = (float)fa.last_accept;
        for (int k = 0; k < 12; ++k) feat[k] = f[k];
    }
}

static unsigned fac_blocks(int64_t maxm) { return (unsigned)std::min<int64_t>(64, (maxm + 255) / 256); }

template <typename TC>
static int64_t max_fac(const FacSet<TC>& f) {
    int64_t m = 0;
    for (int n = 0; n < f.N; ++n) m = std::max<int64_t>(m, f.dims[n] * f.R);
    return m;
}

hipError_t launch_copy_factors(int fdt, const void* dst, const void* src, hipStream_t s) {
    if (fdt == CPG_F64) {
        const auto& d = *(const FacSet<double>*)dst;
        hipLaunchKernelGGL(k_copy_factors<double>, dim3(fac_blocks(max_fac(d)), d.N), dim3(256), 0, s, d,
                           *(const FacSet<double>*)src);
    } else {
        const auto& d = *(const FacSet<float>*)dst;
        hipLaunchKernelGGL(k_copy_factors<float>, dim3(fac_blocks(max_fac(d)), d.N), dim3(256), 0, s, d,
                           *(const FacSet<float>*)src);
    }
    return hipGetLastError();
}

hipError_t launch_extrapolate(int fdt, const void* out, const void* A, const void* As, const float* sigma_dev,
                              double sigma_val, hipStream_t s) {
    if (fdt == CPG_F64) {
        const auto& o = *(const FacSet<double>*)out;
        hipLaunchKernelGGL(k_extrapolate<double>, dim3(fac_blocks(max_fac(o)), o.N), dim3(256), 0, s, o,
                           *(const FacSet<double>*)A, *(const FacSet<double>*)As, sigma_dev, sigma_val);
    } else {
        const auto& o = *(const FacSet<float>*)out;
        hipLaunchKernelGGL(k_extrapolate<float>, dim3(fac_blocks(max_fac(o)), o.N), dim3(256), 0, s, o,
                           *(const FacSet<float>*)A, *(const FacSet<float>*)As, sigma_dev, sigma_val);
    }
    return hipGetLastError();
}

hipError_t launch_accept(int fdt, const void* A, const void* Aext, double* scal, int* accepted, hipStream_t s) {
    if (fdt == CPG_F64)
        hipLaunchKernelGGL(k_accept<double>, dim3(1), dim3(256), 0, s, *(const FacSet<double>*)A,
                           *(const FacSet<double>*)Aext, scal, accepted);
    else
        hipLaunchKernelGGL(k_accept<float>, dim3(1), dim3(256), 0, s, *(const FacSet<float>*)A,
                           *(const FacSet<float>*)Aext, scal, accepted);
    return hipGetLastError();
}

hipError_t launch_features(int fdt, const void* A, const void* As, const void* Dp, const double* costs, int ncost,
                           const double* cur_cost_dev, int iteration, float last_sigma, int last_accept,
                           int have_prev, float* feat, hipStream_t s) {
    FeatArgs fa{};
    const int keep = ncost < 5 ? ncost : 5;
    for (int k = 0; k < keep; ++k) fa.costs[k] = costs[ncost - keep + k];
    fa.ncost = keep;
    fa.cur_cost = cur_cost_dev;
    fa.iteration = iteration;
    fa.last_sigma = last_sigma;
    fa.last_accept = last_accept;
    fa.have_prev = have_prev;
    if (fdt == CPG_F64)
        hipLaunchKernelGGL(k_features<double>, dim3(1), dim3(kLearnThreads), 0, s, *(const FacSet<double>*)A,
                           *(const FacSet<double>*)As, *(const FacSet<double>*)Dp, fa, feat);
    else
        hipLaunchKernelGGL(k_features<float>, dim3(1), dim3(kLearnThreads), 0, s, *(const FacSet<float>*)A,
                           *(const FacSet<float>*)As, *(const FacSet<float>*)Dp, fa, feat);
    return hipGetLastError();
}

}  // namespace cpg
