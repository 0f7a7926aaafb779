/*
 * cpgrad.h — C ABI of libcpgrad: the fast all-mode CP gradient and the CP_ALS
 * sweep built on it, for one MI355X (gfx950) GPU.
 *
 * Reference: A.-H. Phan, P. Tichavsky, A. Cichocki, "On fast computation of
 * gradients for CANDECOMP/PARAFAC algorithms" (arXiv 1204.1586).
 *
 * What is computed
 *   For a dense N-way tensor Y (I_1 x ... x I_N) and factors A^(n) (I_n x R),
 *   the CP gradient of mode n is G^(n) = Y_(n) (A^(N) (.) ... (.) A^(n+1) (.)
 *   A^(n-1) (.) ... (.) A^(1))  (eq. 2.13 / eq. 3.1; Khatri-Rao order of
 *   Notation 2.1).  All N of them are computed by Algorithm 2 (Section 3.3):
 *   two partial contractions of the free matrix view Y_(1:n*) (eq. 2.3, n* of
 *   Algorithm 2 step 1) followed by the per-mode peel-off chains
 *   (eqs. 3.19-3.22).  The ALS sweep applies the update of eq. 2.14 inside
 *   that loop in the order of Section 4 (n*, n*-1, ..., 1, n*+1, ..., N).
 *
 * Memory layout (all tensors are DEVICE memory owned by the caller)
 *   Y    : vec(Y) with mode 1 fastest (ivec of eq. 2.1) — a C-contiguous
 *          torch tensor of shape (I_N, ..., I_1).  Element type y_dtype.
 *   A[n] : I_n x R, row-major (r contiguous) — torch shape (I_n, R).
 *          Element type factor_dtype.
 *   G[n] : I_n x R, row-major, element type factor_dtype.
 *   The pointer arrays A and G themselves are HOST arrays of N device
 *   pointers.  The library never frees or reallocates caller memory.
 *   Y must be 16-byte aligned (any fresh torch or hipMalloc allocation is);
 *   a misaligned Y is rejected with CPG_ERR_INVALID.
 *
 * Supported type combinations
 *   y_dtype  factor_dtype  mode
 *   F64      F64           NATIVE          float64 throughout
 *   F32      F32           NATIVE          float32 contraction (MFMA), fp32 chains
 *   F32      F32           BF16            bf16 MFMA on rounded Y and Khatri-Rao tiles
 *   F32      F32           BF16_REFINED    + residual terms (hi*lo + lo*hi) in the same pass
 *   BF16     F32           BF16            Y stored bf16, Khatri-Rao tiles bf16
 *   BF16     F32           BF16_REFINED    + Y*KR_lo term (Y is exact in bf16)
 *   F32      F32           F16_SCALED      fp16 MFMA: each wave's 64 x 32 tile of Y in a step
 *                                          is scaled by a power of two from its largest
 *                                          magnitude, each Khatri-Rao column r by a power of
 *                                          two from prod_m max_i |A^(m)(i,r)| (its exact
 *                                          largest magnitude); results unscaled exactly
 *   F32      F32           F16_SCALED_REFINED  + residual terms (hi*lo + lo*hi), same pass
 *   BF16/F16 F32           F16_SCALED(_REFINED)  Y stored bf16 or fp16 (converts to scaled
 *                                          fp16 exactly); refinement adds Y*KR_lo
 *   Gram matrices, the normal-equation solve of eq. 2.14, ||Y||^2 and the
 *   cost of eq. 2.12 are float64 in every mode.
 *   The reduced-precision modes run only on the matrix cores: a plan whose
 *   shape they cannot take (J = I_1...I_n* not a multiple of 8, or beyond the
 *   kernels' 32-bit index and grid limits) is refused with
 *   CPG_ERR_UNSUPPORTED instead of silently running in full precision.  The
 *   native float32 form falls back to the vector-ALU kernel (same precision)
 *   for such shapes.
 *
 * Status codes: every call returns a cpg_status (0 = success, < 0 = error).
 * On error no caller buffer is freed; outputs are unspecified unless stated.
 * A plan is bound to one HIP stream and is not thread-safe.
 */
#ifndef CPGRAD_H
#define CPGRAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPG_MAX_MODES 16
#define CPG_MAX_RANK 64

typedef struct cpgrad_plan_s* cpgrad_plan_t;

typedef enum { CPG_F64 = 0, CPG_F32 = 1, CPG_BF16 = 2, CPG_F16 = 3 } cpg_dtype;

typedef enum {
    CPG_MODE_NATIVE = 0,             /* contraction in the tensor's own precision          */
    CPG_MODE_BF16 = 1,               /* bf16 MFMA, fp32 accumulation, no refinement         */
    CPG_MODE_BF16_REFINED = 2,       /* bf16 MFMA + one residual refinement term, same pass */
    CPG_MODE_F16_SCALED = 3,         /* fp16 MFMA on power-of-two scaled tiles, fp32 accum. */
    CPG_MODE_F16_SCALED_REFINED = 4  /* + the residual refinement terms, same pass          */
} cpg_mode;

typedef enum {
    CPG_OK = 0,
    CPG_ERR_INVALID = -1,      /* bad argument: N<2 or N>16, R<1 or R>64, dims<1, int64
                                  overflow of prod(dims), NULL pointer, bad dtype/mode */
    CPG_ERR_NOMEM = -2,        /* device workspace allocation failed                  */
    CPG_ERR_HIP = -3,          /* a HIP runtime call failed                           */
    CPG_ERR_NOT_SPD = -4,      /* eq. 2.14 matrix not positive definite after one
                                  jittered retry; that mode's factor is left as it was */
    CPG_ERR_UNSUPPORTED = -5,  /* valid but unsupported combination                   */
    CPG_ERR_NONFINITE = -6,    /* the cost came out NaN or infinite                   */
    CPG_ERR_SCRATCH = -7       /* cpgrad_all_modes_noalloc: the shape needs more
                                  workspace than the static scratch array holds       */
} cpg_status;

/* Plan options (cpgrad_set_option). */
typedef enum {
    CPG_OPT_FORCE_NSTAR = 1,   /* value in [1, N-1]: use this split instead of Algorithm
                                  2's n* (any split gives the same gradients, eqs. 3.7 =
                                  3.8); 0 restores the default                         */
    CPG_OPT_KERNEL = 2,        /* 0 = automatic, 1 = force the generic vector-ALU
                                  contraction (native mode only), 2 = force the MFMA
                                  contraction; CPG_ERR_UNSUPPORTED (settings kept)
                                  when the plan cannot honour it                      */
    CPG_OPT_PROFILE = 3,       /* 1: bracket every big-contraction launch with a pair of
                                  HIP events on the plan's stream (read them with
                                  cpgrad_profile_read); 0: off (default)               */
    CPG_OPT_MFMA_COLS = 4      /* columns of Y per block of the matrix-core contractions
                                  (a multiple of 32); 0 = automatic (default)           */
} cpg_option;

/* Create a plan for tensors of shape dims[0..N-1] (dims[0] = I_1 is the fastest
 * mode) and rank R.  Chooses n* (Algorithm 2, step 1: the largest n in [1, N-1]
 * with I_1...I_n <= I_{n+1}...I_N, or 1 if none), the tiling of the Y_(1:n*)
 * view and allocates the plan's device workspace (partials, chain buffers,
 * float64 Gram matrices).  stream: a hipStream_t, NULL for the null stream.
 * Errors: CPG_ERR_INVALID, CPG_ERR_UNSUPPORTED, CPG_ERR_NOMEM, CPG_ERR_HIP. */
int cpgrad_plan(cpgrad_plan_t* out, int N, const int64_t* dims, int R,
                int y_dtype, int factor_dtype, int mode, void* stream);

/* Plan facts: n* (1-based, as in the paper), bytes of device workspace the
 * plan owns, and the algorithmic work of one all-mode gradient: multiply-adds
 * x2 (flops) of Algorithm 2 and the bytes one fused pass must move (Y once +
 * factors + gradients).  Any output pointer may be NULL. */
int cpgrad_plan_info(cpgrad_plan_t p, int* n_star, size_t* workspace_bytes,
                     double* alg_flops_all_modes, double* alg_bytes_all_modes);

/* Which kernels the plan runs (host query, no device work): the contraction
 * kernel of its passes (1 = generic vector-ALU kernel, 2 = float32 matrix
 * cores, 3 = bf16 matrix cores, 4 = scaled fp16 matrix cores) and whether the split partials are reduced by
 * the fused multi-block reduction (1) or the generic one (0).  Either output
 * pointer may be NULL.  Errors: CPG_ERR_INVALID. */
int cpgrad_plan_path(cpgrad_plan_t p, int* contraction_kernel, int* fused_reduction);

/* Host-only planning query (touches no device): the n* that a plan for this
 * shape would use (Algorithm 2, step 1; force_nstar in [1, N-1] overrides it,
 * 0 = automatic) and the algorithmic flops / bytes of one all-mode gradient,
 * as cpgrad_plan_info reports them.  Errors: CPG_ERR_INVALID. */
int cpgrad_query(int N, const int64_t* dims, int R, int y_dtype, int factor_dtype, int force_nstar,
                 int* n_star, double* alg_flops_all_modes, double* alg_bytes_all_modes);

/* Set a plan option (cpg_option).  Re-tiles the plan if needed. */
int cpgrad_set_option(cpgrad_plan_t p, int option, int64_t value);

/* With CPG_OPT_PROFILE on: wait for the plan's stream and return the summed
 * duration (milliseconds, HIP events) and the number of big-contraction
 * launches recorded since the option was last set, restricted to `roles`
 * (1 = right pass, 2 = left pass, 3 = fused all-mode pass, 0 = all).  Setting
 * CPG_OPT_PROFILE (to 0 or 1) clears the records.  Errors: CPG_ERR_INVALID,
 * CPG_ERR_HIP. */
int cpgrad_profile_read(cpgrad_plan_t p, int roles, double* total_ms, int64_t* launches);

/* Bind a tensor: computes ||Y||_F^2 in float64 (needed by the cost of eq.
 * 2.12) and remembers the pointer; cpals_step and cp_fit must be called with
 * the bound pointer.  Y must stay alive and unchanged while bound.
 * Enqueued on the plan's stream; returns without waiting. */
int cpgrad_bind(cpgrad_plan_t p, const void* Y);

/* All N CP gradients (Algorithm 2): G[n] <- Y_(n) (⊙_{k≠n} A^(k)) for every
 * n, in one fused pass over Y plus the peel-off chains.  Asynchronous on the
 * plan's stream.  G[n] must not alias A[k] or Y. */
int cpgrad_all_modes(cpgrad_plan_t p, const void* Y, const void* const* A, void* const* G);

/* One CP_ALS sweep (eq. 2.14 in the Section 4 order) on the bound tensor Y:
 * pass 1 over Y gives Y_(1:n*) (A^(N) (.) ... (.) A^(n*+1)), the right chain
 * updates A^(n*), ..., A^(1); pass 2 gives (A^(n*) (.) ... (.) A^(1))^T Y_(1:n*)
 * with the updated factors and the left chain updates A^(n*+1), ..., A^(N).
 * A is updated in place.  Then the cost D = ||Y - Yhat||_F^2 (eq. 2.12) and
 * fit = 1 - sqrt(D)/||Y||_F are formed in float64 on the device.
 * If cost_out and fit_out are both NULL the call is asynchronous and the
 * values stay on the device (read them with cpgrad_last_fit); otherwise it
 * waits for the stream and returns them, together with CPG_ERR_NOT_SPD or
 * CPG_ERR_NONFINITE if the sweep hit either condition. */
int cpals_step(cpgrad_plan_t p, const void* Y, void* const* A,
               double* cost_out, double* fit_out);

/* Cost (eq. 2.12) and fit of the model [[A]] against the bound Y, without
 * changing A: one pass over Y for <Y, Yhat> plus float64 Gram matrices for
 * ||Yhat||^2.  Waits for the stream. */
int cp_fit(cpgrad_plan_t p, const void* Y, const void* const* A,
           double* cost_out, double* fit_out);

/* Wait for the plan's stream and return the cost and fit of the last
 * cpals_step / cp_fit, with its status (CPG_ERR_NOT_SPD / CPG_ERR_NONFINITE). */
int cpgrad_last_fit(cpgrad_plan_t p, double* cost_out, double* fit_out);

/* The full gradient of eq. 2.13 for all modes at once, without its factor -2
 * (the gradient all-at-once methods step along, eqs. 2.15 - 2.17):
 *   E[n] <- Y_(n) (⊙_{k≠n} A^(k)) - A^(n) Gamma^(n),
 *   Gamma^(n) = ⊛_{k≠n} A^(k)T A^(k)  (float64 Grams),
 * i.e. the CP gradients of cpgrad_all_modes (one fused pass over Y, Algorithm
 * 2) minus A^(n) Gamma^(n), formed in float64 and rounded once to the factor
 * type.  E (host array of N device pointers, I_n x R row-major) must not alias
 * A or Y.  Vanishes at an exact model Y = [[A]].  Asynchronous.
 * Errors: CPG_ERR_INVALID, CPG_ERR_HIP. */
int cpgrad_e_gradient(cpgrad_plan_t p, const void* Y, const void* const* A, void* const* E);

/* The CP gradient of one mode n (1-based) by Section 3.2: one pass over Y.
 * If J_n <= K_{n-1} (and n < N, or n = 1) the right-to-left way: P_R =
 * Y_(1:n) (A^(N) (.) ... (.) A^(n+1)) (eq. 3.10), then the leading J_{n-1}
 * rows contracted with A^(n-1) (.) ... (.) A^(1) (eq. 3.12); otherwise the
 * left-to-right way: P_L = (A^(n-1) (.) ... (.) A^(1))^T Y_(1:n-1) (eq. 3.9),
 * then the trailing K_n columns contracted with A^(N) (.) ... (.) A^(n+1)
 * (eq. 3.16).  G: I_n x R device buffer (row-major, factor type).
 * direction (may be NULL) receives 0 for right-to-left, 1 for left-to-right.
 * The plan allocates the buffers of that pass on first use (grown as needed).
 * A reduced-precision plan takes the other way if its matrix cores cannot
 * take the first split.  Asynchronous.
 * Errors: CPG_ERR_INVALID (n outside [1, N], NULL), CPG_ERR_UNSUPPORTED,
 * CPG_ERR_NOMEM, CPG_ERR_HIP. */
int cpgrad_mode_gradient(cpgrad_plan_t p, const void* Y, const void* const* A, int n, void* G, int* direction);

/* One sweep of the multiplicative nonnegative update of eq. 2.18 on the bound
 * tensor, with the gradients from the fast chains of Algorithm 2 in the
 * Section 4 order (n*, ..., 1, n*+1, ..., N; each mode's gradient uses the
 * factors updated before it):
 *   A^(n) <- A^(n) ⊛ G^(n) ⊘ (A^(n) Gamma^(n))
 * (float64 arithmetic, one rounding to the factor type; a denominator below
 * the factor type's smallest normal number is raised to it).  Meant for
 * nonnegative Y and factors, which it keeps nonnegative.  Then the cost of
 * eq. 2.12 and the fit, as cpals_step (NULL outputs: asynchronous).
 * Errors: CPG_ERR_INVALID (Y not the bound tensor), CPG_ERR_NONFINITE,
 * CPG_ERR_HIP. */
int cpntf_step(cpgrad_plan_t p, const void* Y, void* const* A, double* cost_out, double* fit_out);

/* Allocation-free variant of cpgrad_all_modes, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  No plan is created: the shape, types and
 * stream are passed directly (same meaning and checks as cpgrad_plan), and
 * every intermediate (split partials, chain buffers) lives in one static
 * device array of CPG_NOALLOC_SCRATCH_BYTES bytes that the library holds on
 * each GPU it runs on until the process ends.  The call performs no
 * hipMalloc / hipFree / hipMemset and no host allocation; it enqueues the
 * same kernels as cpgrad_all_modes on `stream` and returns without waiting.
 * Y, A (host array of N device pointers) and G are as for cpgrad_all_modes;
 * the HIP device current on the calling thread must be the stream's device.
 * The scratch array is shared by every call on that GPU and keeps the last
 * call's contents: calls that overlap on one GPU (other streams, other host
 * threads) race and must be serialised by the caller.
 * Errors: CPG_ERR_INVALID / CPG_ERR_UNSUPPORTED as cpgrad_plan and
 * cpgrad_all_modes; CPG_ERR_SCRATCH if the shape needs more workspace than
 * the array holds (cpgrad_plan_info's workspace_bytes of an equal plan tells
 * what a shape needs); CPG_ERR_HIP. */
#define CPG_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int cpgrad_all_modes_noalloc(int N, const int64_t* dims, int R, int y_dtype, int factor_dtype, int mode,
                             const void* Y, const void* const* A, void* const* G, void* stream);

/* Release the plan's workspace.  NULL is accepted. */
int cpgrad_destroy(cpgrad_plan_t p);

/* Human-readable name of a status code (static storage). */
const char* cpgrad_status_string(int status);

/* Library version string (static storage). */
const char* cpgrad_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CPGRAD_H */
