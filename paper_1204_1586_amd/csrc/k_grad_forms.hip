// Kernels that turn the CP gradients G^(n) = Y_(n) (⊙_{k≠n} A^(k)) into the
// other quantities the paper builds from them (Section 2.2):
//   * the full gradient of eq. 2.13 without its factor -2:
//       E^(n) = G^(n) - A^(n) Gamma^(n),  Gamma^(n) = ⊛_{k≠n} A^(k)T A^(k),
//     the quantity that all-at-once methods (eqs. 2.15 - 2.17) step along;
//   * the multiplicative nonnegative update of eq. 2.18:
//       A^(n) <- A^(n) ⊛ G^(n) ⊘ (A^(n) Gamma^(n)).
// Gamma^(n) is formed in float64 from the float64 Grams of the plan; the
// matrix products run in float64 and are rounded once to the factor type.
#include "cpg_device.h"

namespace cpg {

namespace {

// Gamma^(n) = Hadamard product of the Grams of every mode but n, into LDS.
__device__ __forceinline__ void form_gamma(const double* __restrict__ grams, int N, int n, int R, double* sGam) {
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
        double v = 1.0;
        for (int k = 0; k < N; ++k)
            if (k != n) v *= grams[(int64_t)k * R * R + e];
        sGam[e] = v;
    }
    __syncthreads();
}

}  // namespace

// Output pointers of every mode, passed to a kernel by value.
template <typename TC>
struct OutSet {
    TC* p[CPG_MAX_MODES];
};

// E[n](i, r) = G[n](i, r) - sum_s A[n](i, s) Gamma^(n)(s, r), in place on E
// (which holds G on entry).  Grid: x = row chunks of 256, y = mode.
template <typename TC>
__global__ __launch_bounds__(256) void k_egrad(FacSet<TC> fs, OutSet<TC> E, const double* __restrict__ grams) {
    __shared__ double sGam[CPG_MAX_RANK * CPG_MAX_RANK];
    const int n = blockIdx.y, R = fs.R;
    form_gamma(grams, fs.N, n, R, sGam);
    const int64_t I = fs.dims[n];
    const TC* __restrict__ A = fs.A[n];
    TC* __restrict__ En = E.p[n];
    const int64_t cells = I * R;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cells; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / R;
        const int r = (int)(e - i * R);
        double acc = 0.0;
        for (int s = 0; s < R; ++s) acc += (double)A[i * R + s] * sGam[s * R + r];
        En[e] = (TC)((double)En[e] - acc);
    }
}

// eq. 2.18 for one mode, one block: each thread takes whole rows, forms the
// row's denominators A(i,:) Gamma from the old row, then writes the new row;
// afterwards grams[n] <- A^T A of the stored (rounded) factor.  A denominator
// below the smallest normal number of the factor type is raised to it (the
// update is then 0 / tiny = 0 for a zero entry, the usual guard of the
// multiplicative rule).
template <typename TC>
__global__ __launch_bounds__(256) void k_ntf_update(const TC* __restrict__ G, TC* __restrict__ A,
                                                    double* __restrict__ grams, int N, int n, int64_t I, int R) {
    __shared__ double sGam[CPG_MAX_RANK * CPG_MAX_RANK];
    form_gamma(grams, N, n, R, sGam);
    const double tiny = sizeof(TC) == 8 ? 2.2250738585072014e-308 : 1.1754943508222875e-38;
    for (int64_t i = threadIdx.x; i < I; i += blockDim.x) {
        double row[CPG_MAX_RANK], den[CPG_MAX_RANK];
        for (int s = 0; s < R; ++s) row[s] = (double)A[i * R + s];
        for (int r = 0; r < R; ++r) {
            double acc = 0.0;
            for (int s = 0; s < R; ++s) acc += row[s] * sGam[s * R + r];
            den[r] = acc > tiny ? acc : tiny;
        }
        for (int r = 0; r < R; ++r) A[i * R + r] = (TC)(row[r] * (double)G[i * R + r] / den[r]);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
        const int r = e / R, c = e - (e / R) * R;
        double acc = 0.0;
        for (int64_t i = 0; i < I; ++i) acc += (double)A[i * R + r] * (double)A[i * R + c];
        grams[(int64_t)n * R * R + e] = acc;
    }
}

hipError_t launch_egrad(int fdt, const void* facset, void* const* E, const double* grams, int N, int64_t max_cells,
                        hipStream_t s) {
    const int64_t chunks = (max_cells + 255) / 256;
    const dim3 grid((unsigned)(chunks < 1024 ? chunks : 1024), (unsigned)N);
    if (fdt == CPG_F64) {
        OutSet<double> o{};
        for (int n = 0; n < N; ++n) o.p[n] = (double*)E[n];
        hipLaunchKernelGGL(k_egrad<double>, grid, dim3(256), 0, s, *(const FacSet<double>*)facset, o, grams);
    } else {
        OutSet<float> o{};
        for (int n = 0; n < N; ++n) o.p[n] = (float*)E[n];
        hipLaunchKernelGGL(k_egrad<float>, grid, dim3(256), 0, s, *(const FacSet<float>*)facset, o, grams);
    }
    return hipGetLastError();
}

hipError_t launch_ntf_update(int fdt, const void* G, void* A, double* grams, int N, int n, int64_t I, int R,
                             hipStream_t s) {
    if (fdt == CPG_F64)
        hipLaunchKernelGGL(k_ntf_update<double>, dim3(1), dim3(256), 0, s, (const double*)G, (double*)A, grams, N,
                           n, I, R);
    else
        hipLaunchKernelGGL(k_ntf_update<float>, dim3(1), dim3(256), 0, s, (const float*)G, (float*)A, grams, N, n,
                           I, R);
    return hipGetLastError();
}

}  // namespace cpg
