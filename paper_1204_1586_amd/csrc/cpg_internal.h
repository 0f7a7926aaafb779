// Internal declarations shared by the host planner and the HIP kernels of
// libcpgrad.  Not part of the public C ABI (see include/cpgrad.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "cpgrad.h"
#include "cpg_fastdiv.h"

struct cpmlp_s;

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

// One side of the peel-off of Algorithm 2 run by a single block (the chain
// epilogue): for the modes n_first, n_first -/+ 1, ... (right chain going
// down, left chain going up) it forms each mode's gradient from its chain
// tensor (cp_gradient 'right' / 'left'), then either writes it to Gout or
// applies eq. 2.14 to that factor, and steps the chain (eqs. 3.20, 3.22).
template <typename TC>
struct EpiArgs {
    FacSet<TC> fs;                 // factors; updated in place when `update`
    int side;                      // 0 = right chain (modes n_first, n_first-1, ...), 1 = left chain
    int n_first;                   // paper's 1-based first mode
    int n_count;                   // number of modes processed
    const TC* Z;                   // chain tensor of mode n_first (R^(n) rows J_n, or L^(n) rows K_{n-1})
    TC* buf[2];                    // chain ping-pong buffers
    const TC* Gpre;                // if set: gradient of mode n_first given (Z unused for it)
    TC* Gout[CPG_MAX_MODES];       // gradients out (when !update), by 0-based mode
    int ld;                        // row stride of Z and the chain buffers
    int update;                    // apply eq. 2.14 after each gradient
    int init;                      // first: clear flags and (unless grams_ready) all float64 Grams
    int grams_ready;               // the Grams were computed before this launch
    int cost;                      // last: cost of eq. 2.12 and fit from G^(N)
    double* grams;                 // [N][R][R] float64
    double* scal;                  // [0] = ||Y||^2 in; [2] cost, [3] fit, [4] <Y,Yhat>, [5] ||Yhat||^2 out
    int* flags;                    // bit 0: not SPD, bit 1: non-finite cost
    int64_t Jn[CPG_MAX_MODES + 1];
    int64_t Kn[CPG_MAX_MODES + 1];
};

constexpr int kEpiGCap = 4096;     // largest I_n * (padded R) the epilogue keeps in LDS
constexpr int kEpiKRCap = 4096;    // largest (terms x ld) of Khatri-Rao rows / factor entries it stages

// Launch `nsides` (1 or 2) epilogue blocks; args[b] drives block b.
hipError_t launch_epilogue(int fdt, int R, const void* args, int nsides, hipStream_t stream);

// ALS update of a side with exactly two modes on many blocks (float32
// factors, R <= 16): the side's first mode n1 from its precomputed gradient,
// then the last mode n2, whose gradient is the chain step of the first
// (eq. 3.20: right, n2 = 1; eq. 3.22: left, n2 = N) and whose rows are
// independent: block b forms and solves rows [b rows, (b + 1) rows).  The
// Gram of the new A^(n2) is not formed (the next pass's reduction forms every
// Gram); with `cost` a second launch adds up the cost of eq. 2.12.
struct EpiRows {
    FacSet<float> fs;
    int side;              // 0 = right (n2 = n1 - 1 = 1), 1 = left (n2 = n1 + 1 = N)
    int n1, n2;            // paper's 1-based modes
    const float* Z;        // P_R (rows i_1 + I_1 i_2) or P_L (rows i_{N-1} + I_{N-1} i_N), stride ld
    int ld;
    const float* Gpre;     // G^(n1), I_n1 x R
    int rows;              // rows of A^(n2) per block
    int cost;              // last pass of a sweep: cost of eq. 2.12 and fit
    double* grams;         // [N][R][R], read; grams[n1], grams[n2] written
    double* scal;          // as in EpiArgs
    int* flags;            // bit 0: not SPD, bit 1: non-finite cost
    double* part;          // two float64 per block (cost partials)
};
constexpr int kEpiRowsMaxBlocks = 16;
constexpr int kEpiRowsCells = 512;   // rows x rank tile of one block's slice
hipError_t launch_epi_rows(const EpiRows& a, hipStream_t stream);

// Tiling of one contraction pass over the J x K view Y_(1:n*).
struct Tiling {
    int kernel;        // 1 = generic vector ALU, 2 = float32 MFMA, 3 = bf16 MFMA, 4 = scaled fp16 MFMA
    int rt;            // rank tile (padded rank) used by the kernel
    int jtb;           // j-tiles (of 64 rows, or the MFMA kernel's row tile) per block
    int64_t ktb;       // k-tiles (of 64 columns) per block
    int64_t n_jr;      // blocks along J
    int64_t n_kc;      // blocks along K
};

// Launchers (defined in the kernel translation units).  All enqueue on
// `stream` and return a hipError_t.
//   roles: bit 0 = right contraction (P_R partials), bit 1 = left (P_L partials)
//   PRpart: [n_kc][J][ld], PLpart: [n_jr][K][ld]   (accumulation type)
// Every internal chain buffer (P_R, P_L, chain tensors, partials) stores its
// rows with the padded stride ld = 4 * ceil(R / 4); entries r >= R of a row are
// never read into a result.
hipError_t launch_contract_valu(int ydt, int fdt, const void* Y, int64_t J, int64_t K,
                                const void* facset, int nstar, const Tiling& t, int roles, int ld,
                                void* PRpart, void* PLpart, hipStream_t stream);
// What a kernel needs to generate Khatri-Rao rows (eq. 3.3) itself: the
// float32 factors, the mode sizes as multiply-shift divisors, R and n*.
struct KrGen {
    const float* A[CPG_MAX_MODES];
    FastDiv fd[CPG_MAX_MODES];
    int N;
    int R;
    int nstar;
};
// Buffers of the MFMA contractions: the split partials they write.
struct MfmaBufs {
    float* PRpart;
    float* PLpart;
    int ld;             // row stride (padded rank) of the partials
    KrGen kg;           // factors for the Khatri-Rao rows
    hipEvent_t ev0;     // if set: recorded at the kernel's start and end (launch-attached timing)
    hipEvent_t ev1;
    int fac_stage;      // float32 MFMA kernel: LDS floats for staging every factor (fac_stage_floats), 0 = none
};
// LDS floats the float32 MFMA contraction uses to stage all factors (each
// rounded up to 64 floats), or 0 when they exceed kFacStageMax.
constexpr int64_t kFacStageMax = 8192;
inline int64_t fac_stage_floats(int N, const int64_t* dims, int R) {
    int64_t f = 0;
    for (int m = 0; m < N; ++m) f += (dims[m] * R + 63) / 64 * 64;
    return f <= kFacStageMax ? f : 0;
}
hipError_t launch_contract_mfma(int ydt, int mode, const void* Y, int64_t J, int64_t K, const Tiling& t,
                                int roles, const MfmaBufs& bufs, hipStream_t stream);
// 16-bit matrix-core contraction: bf16 modes (kind 3) and the scaled fp16 modes (kind 4)
hipError_t launch_contract_bf16(int ydt, int mode, const void* Y, int64_t J, int64_t K, const Tiling& t,
                                int roles, const MfmaBufs& bufs, hipStream_t stream);
bool mfma_supported(int ydt, int fdt, int mode, int R);
// widest column chunk (a multiple of 32) the float32 / bf16 MFMA kernels hold in LDS
int64_t mfma_f32_max_cols(int rt, int roles, int64_t fac_stage = 0);
int64_t mfma_bf16_max_cols(int rt, int roles, bool ylo, bool klo, bool f16);

// One side of the fused partial reduction (float32): output row i of a side is
//   G(i, r) = sum_t Z(row(i, t), r) KR(t, r),  Z = sum_p parts[p]  (float64, p in order)
// with KR the Khatri-Rao rows of modes kr_first.. (one mode: a single chain
// step, eqs. 3.20 / 3.22; the side's other modes: its first gradient, eqs.
// 3.12 / 3.16).
struct ReduceFirst {
    const float* parts;   // nparts x rows x ld split partials of the side's chain tensor
    int64_t nparts;
    int64_t rows;         // J (right) or K (left)
    int ld;
    int side;             // term t of output row i sits in row T*i + t (0) or i + I*t (1)
    int64_t I;            // output rows (one block each)
    int64_t T;            // terms per output row
    int kr_first;         // modes (0-based) whose Khatri-Rao rows weight the terms
    int kr_count;
    float* Z;             // rows x ld reduced chain tensor (out), or null when nothing reads it
    float* G;             // I x out_ld result (out)
    int out_ld;           // R (a gradient) or ld (a chain buffer: columns R..ld-1 written as zero)
};
constexpr int kMaxReduceSides = 4;
// Output rows per block of a side: where the terms of one output row lie
// I rows apart (side 1), neighbouring output rows share each 128-byte line, so
// a block takes as many as fill one line.
inline __host__ __device__ int rf_rows_per_block(int side, int ld) {
    int r = 1;   // a power of two
    if (side == 1)
        while (2 * r * ld * 4 <= 128) r *= 2;
    return r;
}
// `clear_flags`, if set: flags[0..7] are zeroed by the kernel (the start of an ALS sweep).
hipError_t launch_reduce_first(const ReduceFirst* sides, int nsides, const KrGen& kg, double* grams,
                               hipStream_t stream, int* clear_flags = nullptr);

// out[row][r] = sum_p parts[p][row][r] over rows x ld entries (float64, fixed order)
hipError_t launch_reduce_parts(int fdt, const void* parts, int64_t nparts, int64_t rows, int ld,
                               void* out, hipStream_t stream);

// mode product along the middle index of a (lo_n, I, hi_n) row space:
// out[lo + lo_n*hi][r] = sum_i in[lo + lo_n*(i + I*hi)][r] * a[i][r]
hipError_t launch_ttv(int fdt, const void* in, void* out, const void* a, int64_t lo_n, int64_t I,
                      int64_t hi_n, int R, int ld, hipStream_t stream);

// G(i, r) = sum_{lo, hi} Z[lo + lo_n*(i + I*hi)][r] * KR_lo(lo, r) * KR_hi(hi, r)
// KR_lo runs over modes [lo_first, lo_first+lo_count), KR_hi over
// [hi_first, hi_first+hi_count) (first listed mode fastest).
hipError_t launch_grad(int fdt, const void* Z, int ld, void* G, const void* facset, int64_t lo_n, int64_t I,
                       int64_t hi_n, int lo_first, int lo_count, int hi_first, int hi_count,
                       hipStream_t stream);

// float64 Gram matrices of every factor: grams[n][r][s]
hipError_t launch_grams(int fdt, const void* facset, double* grams, hipStream_t stream);

// eq. 2.14 for mode n: A[n] <- G Gamma^{-1}, Gamma = Hadamard of the other
// Grams; then grams[n] <- A[n]^T A[n].  Sets flags[0] |= 1 on failure.
hipError_t launch_als_update(int fdt, const void* G, void* A, double* grams, int N, int n, int64_t I,
                             int R, int* flags, hipStream_t stream);

// E[n] <- E[n] - A[n] Gamma^(n) for every mode (E[n] holds G^(n) on entry;
// E is a host array of N device pointers), Gamma^(n) from the float64 Grams.
hipError_t launch_egrad(int fdt, const void* facset, void* const* E, const double* grams, int N, int64_t max_cells,
                        hipStream_t stream);
// eq. 2.18 for mode n: A[n] <- A[n] .* G ./ (A[n] Gamma^(n)); then grams[n] <- A[n]^T A[n].
hipError_t launch_ntf_update(int fdt, const void* G, void* A, double* grams, int N, int n, int64_t I, int R,
                             hipStream_t stream);

// ||Y||^2 in float64 -> *out (two-stage, deterministic); scratch >= 1024 doubles
hipError_t launch_norm2(int ydt, const void* Y, int64_t n, double* scratch, double* out,
                        hipStream_t stream);

// inner = sum_{j<J, r} PR[j][r] * KR_left(j, r) (modes 0..nstar-1) -> *out
hipError_t launch_inner_kr(int fdt, const void* PR, int ld, int64_t J, const void* facset, int nstar,
                           double* scratch, double* out, hipStream_t stream);

// cost and fit in float64.  If G is non-null, inner = sum G .* A (I x R);
// otherwise inner is read from *inner_in.  scal: [0]=||Y||^2, writes [2]=cost,
// [3]=fit (or [out_slot], [out_slot+1]); flags[0] |= 2 if non-finite.
hipError_t launch_cost_fit(int fdt, const void* G, const void* A, int64_t I, int R,
                           const double* inner_in, const double* grams, int N, double* scal,
                           int* flags, hipStream_t stream, int out_slot = 2);

// learned extrapolation step (k_learn.hip); factor sets are FacSet<T> of the plan's type
hipError_t launch_copy_factors(int fdt, const void* dst, const void* src, hipStream_t stream);
hipError_t launch_extrapolate(int fdt, const void* out, const void* A, const void* As, const float* sigma_dev,
                              double sigma_val, hipStream_t stream);
hipError_t launch_accept(int fdt, const void* A, const void* Aext, double* scal, int* accepted,
                         hipStream_t stream);
hipError_t launch_features(int fdt, const void* A, const void* As, const void* Dp, const double* costs, int ncost,
                           const double* cur_cost_dev, int iteration, float last_sigma, int last_accept,
                           int have_prev, float* feat, hipStream_t stream);
// the step-size network (k_mlp.hip)
hipError_t launch_mlp_forward(struct ::cpmlp_s* m, const float* X, int batch, float* sigma, hipStream_t stream);
int mlp_num_inputs(struct ::cpmlp_s* m);

}  // namespace cpg
