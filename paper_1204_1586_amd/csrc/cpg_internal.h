// Internal declarations shared by the host planner and the HIP kernels of
// libcpgrad.  Not part of the public C ABI (see include/cpgrad.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "cpgrad.h"

namespace cpg {

// Factor set handed to kernels by value: every mode's extent and factor
// pointer (I_n x R, row-major, r contiguous).
template <typename T>
struct FacSet {
    int N;
    int R;
    int64_t dims[CPG_MAX_MODES];
    const T* A[CPG_MAX_MODES];
};

// Tiling of one contraction pass over the J x K view Y_(1:n*).
struct Tiling {
    int kernel;        // 1 = generic vector ALU, 2 = MFMA
    int rt;            // rank tile (padded rank) used by the kernel
    int jtb;           // j-tiles (of 64 rows, or the MFMA kernel's row tile) per block
    int64_t ktb;       // k-tiles (of 64 columns) per block
    int64_t n_jr;      // blocks along J
    int64_t n_kc;      // blocks along K
};

// Launchers (defined in the kernel translation units).  All enqueue on
// `stream` and return a hipError_t.
//   roles: bit 0 = right contraction (P_R partials), bit 1 = left (P_L partials)
//   PRpart: [n_kc][J][R], PLpart: [n_jr][K][R]   (accumulation type)
hipError_t launch_contract_valu(int ydt, int fdt, const void* Y, int64_t J, int64_t K,
                                const void* facset, int nstar, const Tiling& t, int roles,
                                void* PRpart, void* PLpart, hipStream_t stream);
hipError_t launch_contract_mfma(int ydt, int mode, const void* Y, int64_t J, int64_t K,
                                const FacSet<float>& fs, int nstar, const Tiling& t, int roles,
                                float* PRpart, float* PLpart, hipStream_t stream);
bool mfma_supported(int ydt, int fdt, int mode, int R);

// out[row][r] = sum_p parts[p][row][r]  (summed in float64, fixed order)
hipError_t launch_reduce_parts(int fdt, const void* parts, int64_t nparts, int64_t rows, int R,
                               void* out, hipStream_t stream);

// mode product along the middle index of a (lo_n, I, hi_n) row space:
// out[lo + lo_n*hi][r] = sum_i in[lo + lo_n*(i + I*hi)][r] * a[i][r]
hipError_t launch_ttv(int fdt, const void* in, void* out, const void* a, int64_t lo_n, int64_t I,
                      int64_t hi_n, int R, hipStream_t stream);

// G(i, r) = sum_{lo, hi} Z[lo + lo_n*(i + I*hi)][r] * KR_lo(lo, r) * KR_hi(hi, r)
// KR_lo runs over modes [lo_first, lo_first+lo_count), KR_hi over
// [hi_first, hi_first+hi_count) (first listed mode fastest).
hipError_t launch_grad(int fdt, const void* Z, void* G, const void* facset, int64_t lo_n, int64_t I,
                       int64_t hi_n, int lo_first, int lo_count, int hi_first, int hi_count,
                       hipStream_t stream);

// float64 Gram matrices of every factor: grams[n][r][s]
hipError_t launch_grams(int fdt, const void* facset, double* grams, hipStream_t stream);

// eq. 2.14 for mode n: A[n] <- G Gamma^{-1}, Gamma = Hadamard of the other
// Grams; then grams[n] <- A[n]^T A[n].  Sets flags[0] |= 1 on failure.
hipError_t launch_als_update(int fdt, const void* G, void* A, double* grams, int N, int n, int64_t I,
                             int R, int* flags, hipStream_t stream);

// ||Y||^2 in float64 -> *out (two-stage, deterministic); scratch >= 1024 doubles
hipError_t launch_norm2(int ydt, const void* Y, int64_t n, double* scratch, double* out,
                        hipStream_t stream);

// inner = sum_{j<J, r} PR[j][r] * KR_left(j, r) (modes 0..nstar-1) -> *out
hipError_t launch_inner_kr(int fdt, const void* PR, int64_t J, const void* facset, int nstar,
                           double* scratch, double* out, hipStream_t stream);

// cost and fit in float64.  If G is non-null, inner = sum G .* A (I x R);
// otherwise inner is read from *inner_in.  scal: [0]=||Y||^2, writes [2]=cost,
// [3]=fit; flags[0] |= 2 if non-finite.
hipError_t launch_cost_fit(int fdt, const void* G, const void* A, int64_t I, int R,
                           const double* inner_in, const double* grams, int N, double* scal,
                           int* flags, hipStream_t stream);

}  // namespace cpg
