// Host side of libcpgrad: argument checking, the plan (n*, tiling,
// workspace) and the enqueue order of Algorithm 2 and of the fast ALS sweep
// (Section 4).  Every arithmetic step runs in the HIP kernels of this
// library; the host only validates, plans and launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "cpg_internal.h"
#include "cpmlp.h"

using namespace cpg;

struct cpgrad_plan_s {
    int N = 0, R = 0;
    int ld = 4;                            // row stride of internal chain buffers: 4 * ceil(R / 4)
    int64_t dims[CPG_MAX_MODES] = {0};
    int ydt = 0, fdt = 0, mode = 0;
    hipStream_t stream = nullptr;
    int nstar_auto = 1, nstar = 1;
    int force_nstar = 0, kernel_opt = 0;
    int64_t opt_cols = 0;                  // MFMA column chunk override (0 = automatic)
    int64_t Jn[CPG_MAX_MODES + 1] = {0};   // Jn[n] = I_1 ... I_n   (Jn[0] = 1)
    int64_t Kn[CPG_MAX_MODES + 1] = {0};   // Kn[n] = I_{n+1} ... I_N (Kn[N] = 1)
    int64_t J = 0, K = 0, numel = 0;
    Tiling t_fused{}, t_right{}, t_left{};
    size_t acc = 8;                        // bytes of the accumulation / factor type
    // device workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    bool ws_external = false;              // ws is the library's static scratch array (never freed or grown)
    void* PR = nullptr;
    void* PL = nullptr;
    void* chain[4] = {nullptr, nullptr, nullptr, nullptr};
    size_t prpart_bytes = 0, plpart_bytes = 0;   // sizes of the split-partial buffers
    void* PRpart = nullptr;
    void* PLpart = nullptr;
    FastDiv fd[CPG_MAX_MODES];  // mode sizes as multiply-shift divisors (kernels unravel row indices)
    bool fused_first = false; // partial reduction fused with each side's first gradient
    void* Gtmp = nullptr;
    double* grams = nullptr;
    double* scal = nullptr;   // [0]=||Y||^2 [2]=cost [3]=fit [4]=inner [5]=||Yhat||^2 [6]=inner(cp_fit)
    double* red = nullptr;    // reduction scratch (1024 doubles)
    int* flags = nullptr;     // [0] status bits
    double* rpart = nullptr;  // per-block cost partials of the many-block ALS epilogue
    double* host = nullptr;   // pinned readback: scal[0..7], flags
    const void* bound = nullptr;
    // learned extrapolation step: start / previous-update / extrapolated factors, features, sigma
    char* lws = nullptr;
    size_t lws_bytes = 0;
    int64_t fac_off[CPG_MAX_MODES] = {0};   // element offset of each mode in a factor set
    void* l_start = nullptr;
    void* l_dprev = nullptr;
    void* l_ext = nullptr;
    float* l_feat = nullptr;
    float* l_sigma = nullptr;
    int* l_accept = nullptr;
    int have_prev = 0;
    // single-mode gradient (Section 3.2): partial buffers of a one-sided pass at another split
    char* sws = nullptr;
    size_t sws_bytes = 0;
    // optional HIP-event timing of the big contraction launches
    int profile = 0;
    std::vector<hipEvent_t> ev_start, ev_stop;
    std::vector<int> ev_roles;
    size_t ev_used = 0;
};

namespace {

constexpr int kRedScratch = 1024;

int rank_tile(int R) {
    if (R <= 4) return 4;
    if (R <= 16) return 16;
    if (R <= 32) return 32;
    return 64;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

namespace cpg {
int valu_max_jtb(int fdt, int rt);
int64_t mfma_bf16_max_cols_shared(int rt, int roles, bool ylo, bool klo, bool f16, int blocks_per_cu);
hipError_t launch_grad_split(int fdt, const void* Z, int ld, void* G, const void* facset, int64_t lo_n, int64_t I,
                             int64_t hi_n, int lo_first, int lo_count, int hi_first, int hi_count, void* scratch,
                             size_t scratch_bytes, hipStream_t s);
}

// Tiling of one pass for the generic kernel: 64 x 64 tiles, up to `jtb`
// j-tiles per block, enough blocks to give every compute unit a few.
static Tiling tile_valu(int64_t J, int64_t K, int R, int fdt, int roles) {
    Tiling t{};
    t.kernel = 1;
    t.rt = rank_tile(R);
    const int64_t tJ = cdiv(J, 64), tK = cdiv(K, 64);
    const int maxj = valu_max_jtb(fdt, t.rt);
    t.jtb = (int)std::min<int64_t>(maxj, tJ);
    t.n_jr = cdiv(tJ, t.jtb);
    const int64_t target = 1024;
    t.ktb = std::max<int64_t>(1, (tK * t.n_jr) / target);
    (void)roles;
    t.n_kc = cdiv(tK, t.ktb);
    return t;
}

// Tiling of one pass for the MFMA kernel: 256-row blocks, column chunks of
// whole 32-column steps, about two blocks per compute unit.
static Tiling tile_mfma(int64_t J, int64_t K, int R, int roles, int kernel, int64_t cols, bool ylo, bool klo,
                        int64_t fac_stage) {
    Tiling t{};
    t.kernel = kernel;
    t.rt = 16 * (int)cdiv(R, 16);
    t.jtb = 1;
    t.n_jr = cdiv(J, 256);
    const int64_t steps = cdiv(K, 32);
    // about one block per CU: long-running blocks whose interleaved column
    // steps sweep Y as one moving window (measured best for 64^4, rank 16).
    // On a large tensor (32 or more steps per block at that grid) the
    // one-sided 16-bit passes run two blocks per CU (their registers allow it)
    // and measured fastest with four or more blocks per CU over the grid
    // (48^5, rank 32: left pass 189 -> 127 us, right pass 235 -> 185 us; on
    // 64^4 and 10^7 the same grids were slower).
    const bool b16 = kernel == 3 || kernel == 4;
    const bool b16_one = b16 && roles != 3 && cdiv(steps * t.n_jr, 256) >= 32;
    const int64_t target = b16_one ? 1024 : 256;
    t.ktb = cols > 0 ? cdiv(cols, 32) : std::max<int64_t>(1, cdiv(steps * t.n_jr, target));
    // LDS holds the KR_R rows of a block's steps
    if (kernel == 2) t.ktb = std::min<int64_t>(t.ktb, mfma_f32_max_cols(t.rt, roles, fac_stage) / 32);
    if (b16)
        t.ktb = std::min<int64_t>(t.ktb, mfma_bf16_max_cols_shared(t.rt, roles, ylo, klo, kernel == 4,
                                                                  b16_one && cols <= 0 ? 2 : 1) / 32);
    t.ktb = std::max<int64_t>(1, t.ktb);
    t.n_kc = cdiv(steps, t.ktb);
    return t;
}

// Can the matrix-core kernels take a J x K view at all?  32-bit buffer
// offsets (a 32-column step of Y below 2 GiB), row and column indices that
// the kernels unravel by 32-bit multiply-shift division (below 2^31), and a
// grid whose column dimension stays within 65535 blocks.
static bool refined_mode(int mode) { return mode == CPG_MODE_BF16_REFINED || mode == CPG_MODE_F16_SCALED_REFINED; }
static bool f16_mode(int mode) { return mode == CPG_MODE_F16_SCALED || mode == CPG_MODE_F16_SCALED_REFINED; }

static bool mfma_shape_ok(const cpgrad_plan_s* p, int kind) {
    const int64_t lim = int64_t(1) << 31;
    if (p->J * 4 * 32 >= lim || p->J >= lim || p->K >= lim) return false;
    const bool klo = refined_mode(p->mode);
    for (int roles = 1; roles <= 3; ++roles) {
        const Tiling t = tile_mfma(p->J, p->K, p->R, roles, kind, p->opt_cols, klo && p->ydt == CPG_F32, klo,
                                   fac_stage_floats(p->N, p->dims, p->R));
        if (t.n_kc > 65535 || t.n_jr > 0x7fffffff) return false;
    }
    return true;
}

// The matrix-core kind a plan's types and mode ask for: 2 = float32 MFMA
// (native float32), 3 = bf16 MFMA (the bf16 modes), 4 = scaled fp16 MFMA (the
// fp16 modes), 0 = none (float64).
static int wanted_kind(const cpgrad_plan_s* p) {
    if (f16_mode(p->mode)) return 4;
    if (p->mode != CPG_MODE_NATIVE) return 3;
    return (p->ydt == CPG_F32 && p->fdt == CPG_F32) ? 2 : 0;
}

// 0 = generic kernel, 2 = float32 MFMA, 3 / 4 = 16-bit MFMA (reduced-precision modes).
// The native float32 form falls back to the generic kernel (same precision)
// when the matrix cores cannot take the shape; a reduced-precision mode never
// does (plan_kind_ok refuses the plan instead).
static int mfma_kind(const cpgrad_plan_s* p) {
    const int kind = wanted_kind(p);
    if (kind == 0 || p->kernel_opt == 1) return 0;
    const int64_t align = kind == 2 ? 4 : 8;   // rows per MFMA operand chunk
    if (p->J % align != 0 || !mfma_shape_ok(p, kind)) return 0;
    return kind;
}

// A plan whose mode or forced kernel cannot be honoured is refused: the
// reduced-precision modes need their 16-bit matrix cores (J a multiple of 8
// and a shape they can take), CPG_OPT_KERNEL = 2 needs a matrix-core kind,
// and the reduced-precision modes cannot be forced onto the generic
// (full-precision) kernel.
static int plan_kind_ok(const cpgrad_plan_s* p) {
    const int kind = mfma_kind(p);
    if (p->mode != CPG_MODE_NATIVE && kind != wanted_kind(p)) return CPG_ERR_UNSUPPORTED;
    if (p->kernel_opt == 2 && kind == 0) return CPG_ERR_UNSUPPORTED;
    return CPG_OK;
}

static Tiling tile_pass(const cpgrad_plan_s* p, int roles) {
    const int kind = mfma_kind(p);
    if (kind) {
        const bool klo = refined_mode(p->mode);
        return tile_mfma(p->J, p->K, p->R, roles, kind, p->opt_cols, klo && p->ydt == CPG_F32, klo,
                         fac_stage_floats(p->N, p->dims, p->R));
    }
    return tile_valu(p->J, p->K, p->R, p->fdt, roles);
}

static int hip_status(hipError_t e) { return e == hipSuccess ? CPG_OK : CPG_ERR_HIP; }

static void release(cpgrad_plan_s* p) {
    if (p->ws && !p->ws_external) (void)hipFree(p->ws);
    p->ws = nullptr;
    p->ws_bytes = 0;
}

static bool fused_first_ok(const cpgrad_plan_s* p);

// Choose n*, tile every pass and (re)allocate the workspace.
static int configure(cpgrad_plan_s* p) {
    const int N = p->N;
    p->nstar = p->force_nstar ? p->force_nstar : p->nstar_auto;
    p->J = p->Jn[p->nstar];
    p->K = p->Kn[p->nstar];
    {
        const int st = plan_kind_ok(p);
        if (st) return st;
    }
    p->t_fused = tile_pass(p, 3);
    p->t_right = tile_pass(p, 1);
    p->t_left = tile_pass(p, 2);
    const size_t a = p->acc, R = (size_t)p->ld;
    int64_t chain_rows = 0;
    if (p->nstar >= 2) chain_rows = std::max<int64_t>(chain_rows, p->Jn[p->nstar - 1]);
    if (p->nstar + 1 < N) chain_rows = std::max<int64_t>(chain_rows, p->Kn[p->nstar + 1]);
    int64_t maxI = 0;
    for (int n = 0; n < N; ++n) maxI = std::max<int64_t>(maxI, p->dims[n]);
    const int64_t nkc = std::max(p->t_fused.n_kc, p->t_right.n_kc);
    const int64_t njr = std::max(p->t_fused.n_jr, p->t_left.n_jr);
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    size_t off = 0;
    const size_t oPR = off;     off += al(p->J * R * a);
    const size_t oPL = off;     off += al(p->K * R * a);
    const size_t oC0 = off;     off += al(chain_rows * R * a);
    const size_t oC1 = off;     off += al(chain_rows * R * a);
    const size_t oC2 = off;     off += al(chain_rows * R * a);
    const size_t oC3 = off;     off += al(chain_rows * R * a);
    const size_t oPRp = off;    off += al(nkc * p->J * R * a);
    const size_t oPLp = off;    off += al(njr * p->K * R * a);
    p->fused_first = fused_first_ok(p);
    for (int n = 0; n < N; ++n) p->fd[n] = make_fastdiv((uint32_t)p->dims[n]);
    const size_t oG = off;      off += al(maxI * R * a);
    const size_t oGr = off;     off += al((size_t)N * p->R * p->R * 8);
    // scal (16 doubles) and flags (16 ints) back to back: one copy reads both back
    const size_t oS = off;      off += al(16 * 8 + 16 * sizeof(int));
    const size_t oRed = off;    off += al(kRedScratch * 8);
    const size_t oRp = off;     off += al(2 * kEpiRowsMaxBlocks * 8);
    if (off > p->ws_bytes) {
        if (p->ws_external) return CPG_ERR_SCRATCH;
        release(p);
        void* mem = nullptr;
        if (hipMalloc(&mem, off) != hipSuccess) {
            (void)hipGetLastError();
            return CPG_ERR_NOMEM;
        }
        p->ws = (char*)mem;
        p->ws_bytes = off;
    }
    char* b = p->ws;
    p->PR = b + oPR;
    p->PL = b + oPL;
    p->chain[0] = b + oC0;
    p->chain[1] = b + oC1;
    p->chain[2] = b + oC2;
    p->chain[3] = b + oC3;
    p->PRpart = b + oPRp;
    p->PLpart = b + oPLp;
    p->prpart_bytes = oPLp - oPRp;
    p->plpart_bytes = oG - oPLp;
    p->Gtmp = b + oG;
    p->grams = (double*)(b + oGr);
    p->scal = (double*)(b + oS);
    p->red = (double*)(b + oRed);
    p->flags = (int*)(b + oS + 16 * 8);
    p->rpart = (double*)(b + oRp);

    p->bound = nullptr;
    if (p->ws_external) return CPG_OK;   // the all-mode gradient reads neither scal nor flags
    if (hipMemsetAsync(p->scal, 0, 16 * 8, p->stream) != hipSuccess) return CPG_ERR_HIP;
    if (hipMemsetAsync(p->flags, 0, 16 * sizeof(int), p->stream) != hipSuccess) return CPG_ERR_HIP;
    return CPG_OK;
}

template <typename T>
static FacSet<T> make_facset(const cpgrad_plan_s* p, const void* const* A) {
    FacSet<T> fs{};
    fs.N = p->N;
    fs.R = p->R;
    for (int n = 0; n < p->N; ++n) {
        fs.dims[n] = p->dims[n];
        fs.A[n] = (const T*)A[n];
    }
    return fs;
}

// A type-erased factor set: FacSet<double> or FacSet<float> by the plan's type.
struct AnyFacSet {
    FacSet<double> d;
    FacSet<float> f;
    const void* ptr(int fdt) const { return fdt == CPG_F64 ? (const void*)&d : (const void*)&f; }
};

static AnyFacSet facsets(const cpgrad_plan_s* p, const void* const* A) {
    AnyFacSet s{};
    if (p->fdt == CPG_F64)
        s.d = make_facset<double>(p, A);
    else
        s.f = make_facset<float>(p, A);
    return s;
}

static KrGen kr_gen(const cpgrad_plan_s* p, const FacSet<float>& fs) {
    KrGen g{};
    for (int n = 0; n < p->N; ++n) {
        g.A[n] = fs.A[n];
        g.fd[n] = p->fd[n];
    }
    g.N = p->N;
    g.R = p->R;
    g.nstar = p->nstar;
    return g;
}

static hipError_t launch_contract(cpgrad_plan_s* p, const void* Y, const AnyFacSet& fs, const Tiling& t,
                                  int roles, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr) {
    if (t.n_kc > 65535) return hipErrorInvalidConfiguration;
    if (t.kernel >= 2) {
        MfmaBufs o{(float*)p->PRpart, (float*)p->PLpart, p->ld, kr_gen(p, fs.f), ev0, ev1,
                   (int)fac_stage_floats(p->N, p->dims, p->R)};
        if (t.kernel >= 3)
            return launch_contract_bf16(p->ydt, p->mode, Y, p->J, p->K, t, roles, o, p->stream);
        return launch_contract_mfma(p->ydt, p->mode, Y, p->J, p->K, t, roles, o, p->stream);
    }
    return launch_contract_valu(p->ydt, p->fdt, Y, p->J, p->K, fs.ptr(p->fdt), p->nstar, t, roles, p->ld,
                                p->PRpart, p->PLpart, p->stream);
}

// Launch one big contraction; with profiling on, time it with HIP events on
// the plan's stream (attached to the launch for the matrix-core kernels, so
// they bracket exactly the kernel's execution; recorded around it otherwise).
static hipError_t run_contract(cpgrad_plan_s* p, const void* Y, const AnyFacSet& fs, const Tiling& t, int roles) {
    if (!p->profile) return launch_contract(p, Y, fs, t, roles);
    if (p->ev_used == p->ev_start.size()) {
        if (p->ev_used >= 65536) return launch_contract(p, Y, fs, t, roles);  // pool full: stop recording
        hipEvent_t a, b;
        hipError_t e = hipEventCreate(&a);
        if (e != hipSuccess) return e;
        e = hipEventCreate(&b);
        if (e != hipSuccess) return e;
        p->ev_start.push_back(a);
        p->ev_stop.push_back(b);
        p->ev_roles.push_back(0);
    }
    const size_t i = p->ev_used++;
    p->ev_roles[i] = roles;
    if (t.kernel >= 2)   // events attached to the kernel launch itself
        return launch_contract(p, Y, fs, t, roles, p->ev_start[i], p->ev_stop[i]);
    hipError_t e = hipEventRecord(p->ev_start[i], p->stream);
    if (e != hipSuccess) return e;
    e = launch_contract(p, Y, fs, t, roles);
    if (e != hipSuccess) return e;
    return hipEventRecord(p->ev_stop[i], p->stream);
}

#define CPG_TRY(x)                                   \
    do {                                             \
        hipError_t _e = (x);                         \
        if (_e != hipSuccess) return CPG_ERR_HIP;    \
    } while (0)

// Reduce the partials of a pass into P_R and/or P_L.  On the fused path a
// side whose first gradient is wanted (Gr: G^(n*), Gl: G^(n*+1)) gets it from
// the same kernel, which also computes every Gram when `grams` is set.  With
// `Gall` (the all-mode gradient, both sides fused) the kernel also takes the
// first chain step of each side straight from the partials: its result is
// the next mode's gradient (Gall) or the chain buffer the epilogue continues
// from, and P_R / P_L are not stored, since nothing reads them afterwards.
// Returns CPG_OK; *fused tells whether the gradients were formed.
static int finish_partials(cpgrad_plan_s* p, const FacSet<float>* fs, const Tiling& t, int roles, void* Gr = nullptr,
                           void* Gl = nullptr, bool grams = false, bool* fused = nullptr, void* const* Gall = nullptr,
                           int* clear_flags = nullptr) {
    const bool fr = p->fused_first && fs && (roles & 1) && Gr;
    const bool fl = p->fused_first && fs && (roles & 2) && Gl;
    if (fused) *fused = fr || fl;
    if (fr || fl) {
        const bool tail = Gall && fr && fl;
        const int N = p->N, ns = p->nstar, R = p->R, ld = p->ld;
        ReduceFirst sd[kMaxReduceSides];
        int n = 0;
        if (fr)
            sd[n++] = ReduceFirst{(const float*)p->PRpart, t.n_kc, p->J, ld, 0, p->dims[ns - 1], p->Jn[ns - 1],
                                  0, ns - 1, tail ? nullptr : (float*)p->PR, (float*)Gr, R};
        if (fl)
            sd[n++] = ReduceFirst{(const float*)p->PLpart, t.n_jr, p->K, ld, 1, p->dims[ns], p->Kn[ns + 1],
                                  ns + 1, N - ns - 1, tail ? nullptr : (float*)p->PL, (float*)Gl, R};
        if (tail && ns >= 2) {
            // right (eq. 3.20): out(t, r) = sum_i Z(t + T i, r) A^(n*)(i, r), T = J_{n*-1};
            // G^(1) itself when n* = 2
            const bool last = ns == 2;
            sd[n++] = ReduceFirst{(const float*)p->PRpart, t.n_kc, p->J, ld, 1, p->Jn[ns - 1], p->dims[ns - 1],
                                  ns - 1, 1, nullptr, last ? (float*)Gall[0] : (float*)p->chain[0], last ? R : ld};
        }
        if (tail && N - ns >= 2) {
            // left (eq. 3.22): out(t, r) = sum_i Z(i + I t, r) A^(n*+1)(i, r), I = I_{n*+1};
            // G^(N) itself when n* = N - 2
            const bool last = ns + 2 == N;
            sd[n++] = ReduceFirst{(const float*)p->PLpart, t.n_jr, p->K, ld, 0, p->Kn[ns + 1], p->dims[ns],
                                  ns, 1, nullptr, last ? (float*)Gall[N - 1] : (float*)p->chain[2], last ? R : ld};
        }
        CPG_TRY(launch_reduce_first(sd, n, kr_gen(p, *fs), grams ? p->grams : nullptr, p->stream, clear_flags));
    }
    if ((roles & 1) && !fr) CPG_TRY(launch_reduce_parts(p->fdt, p->PRpart, t.n_kc, p->J, p->ld, p->PR, p->stream));
    if ((roles & 2) && !fl) CPG_TRY(launch_reduce_parts(p->fdt, p->PLpart, t.n_jr, p->K, p->ld, p->PL, p->stream));
    return CPG_OK;
}

// Chain tensors bigger than this go through the multi-block grad / ttv
// kernels for their first step; smaller ones are walked by one epilogue block.
constexpr size_t kEpiLargeBytes = size_t(2) << 20;

static int epi_rank_tile(int R) { return rank_tile(R); }

// Terms of the gradient of paper mode n from its chain tensor: J_{n-1} on the
// right side (n <= n*), K_n on the left side.
static int64_t grad_terms(const cpgrad_plan_s* p, int n) { return n <= p->nstar ? p->Jn[n - 1] : p->Kn[n]; }

// Is a side's first chain tensor (P_R or P_L) small enough for one epilogue block?
static bool side_rows_small(const cpgrad_plan_s* p, int side, size_t elem) {
    const int64_t rows = side == 0 ? p->J : p->K;
    return (size_t)rows * p->ld * elem <= kEpiLargeBytes;
}

// Does the first mode of a side go through the single-block epilogue, or does
// its chain tensor (or its Khatri-Rao block) call for the multi-block kernels?
// (With the first gradient precomputed by the fused reduction, only the chain
// tensor's size matters: the epilogue then forms no Khatri-Rao block for it.)
static bool side_first_small(const cpgrad_plan_s* p, int side, size_t elem) {
    const int n = side == 0 ? p->nstar : p->nstar + 1;
    return side_rows_small(p, side, elem) && grad_terms(p, n) * p->ld <= kEpiKRCap;
}

// Can the single-block epilogue hold every mode's gradient, factor and the
// Khatri-Rao blocks of every mode after the first of each side?
static bool epilogue_fits(const cpgrad_plan_s* p) {
    const int rt = epi_rank_tile(p->R);
    for (int n = 0; n < p->N; ++n)
        if (p->dims[n] * rt > kEpiGCap || p->dims[n] * p->ld > kEpiKRCap) return false;
    for (int n = 1; n <= p->N; ++n) {
        if (n == p->nstar || n == p->nstar + 1) continue;
        if (grad_terms(p, n) * p->ld > kEpiKRCap) return false;
    }
    return true;
}

// The fused reduction + first gradients: float32 factors on an MFMA kind, and
// both sides walked by the single-block epilogue after their first gradient
// (the reduction forms the first gradients with Khatri-Rao weights of any
// length, generated from the factors).
static bool fused_first_ok(const cpgrad_plan_s* p) {
    const int kind = mfma_kind(p);
    return kind >= 2 && p->fdt == CPG_F32 && epilogue_fits(p) && side_rows_small(p, 0, 4) &&
           side_rows_small(p, 1, 4);
}

template <typename TC>
static EpiArgs<TC> epi_base(const cpgrad_plan_s* p, const FacSet<TC>& fs) {
    EpiArgs<TC> a{};
    a.fs = fs;
    a.grams = p->grams;
    a.ld = p->ld;
    a.scal = p->scal;
    a.flags = p->flags;
    for (int n = 0; n <= p->N; ++n) {
        a.Jn[n] = p->Jn[n];
        a.Kn[n] = p->Kn[n];
    }
    return a;
}

// One side of the peel-off (Algorithm 2 steps 4-5, 9-12 on the right, steps
// 7-8, 13-16 on the left; with `update`, eq. 2.14 after each gradient in the
// Section 4 order).  Small chain tensors: one epilogue block for the whole
// side.  A large first chain tensor: its gradient and its chain step run on
// the multi-block kernels, the rest in the epilogue.
template <typename TC>
static int run_side(cpgrad_plan_s* p, const FacSet<TC>& fs, int side, void* const* A, void* const* G, bool update,
                    bool init, bool cost, const TC* Gpre0 = nullptr, bool grams_ready = false) {
    const int N = p->N, R = p->R;
    const int n_first = side == 0 ? p->nstar : p->nstar + 1;
    const int n_count = side == 0 ? p->nstar : N - p->nstar;
    const void* Z = side == 0 ? p->PR : p->PL;
    const int64_t rows = side == 0 ? p->J : p->K;
    EpiArgs<TC> a = epi_base<TC>(p, fs);
    a.side = side;
    a.update = update ? 1 : 0;
    for (int n = 0; n < N; ++n) a.Gout[n] = G ? (TC*)G[n] : nullptr;
    (void)rows;
    if (Gpre0 ? side_rows_small(p, side, sizeof(TC)) : side_first_small(p, side, sizeof(TC))) {
        a.n_first = n_first;
        a.n_count = n_count;
        a.Z = (const TC*)Z;
        a.buf[0] = (TC*)p->chain[0];
        a.buf[1] = (TC*)p->chain[1];
        a.init = init ? 1 : 0;
        a.grams_ready = grams_ready ? 1 : 0;
        a.cost = cost ? 1 : 0;
        a.Gpre = Gpre0;
        CPG_TRY(launch_epilogue(p->fdt, R, &a, 1, p->stream));
        return CPG_OK;
    }
    // first mode of the side on the multi-block kernels
    const int n = n_first;
    void* g = update ? p->Gtmp : G[n - 1];
    // the side's split partials are summed by now: their buffer holds the gradient's parts
    if (side == 0)
        CPG_TRY(launch_grad_split(p->fdt, Z, p->ld, g, &fs, p->Jn[n - 1], p->dims[n - 1], 1, 0, n - 1, 0, 0,
                                  p->PRpart, p->prpart_bytes, p->stream));
    else
        CPG_TRY(launch_grad_split(p->fdt, Z, p->ld, g, &fs, 1, p->dims[n - 1], p->Kn[n], 0, 0, n, N - n, p->PLpart,
                                  p->plpart_bytes, p->stream));
    if (update || init) {
        EpiArgs<TC> b = a;
        b.n_first = n;
        b.n_count = update ? 1 : 0;
        b.Gpre = (const TC*)g;
        b.init = init ? 1 : 0;
        b.cost = (cost && n_count == 1) ? 1 : 0;
        CPG_TRY(launch_epilogue(p->fdt, R, &b, 1, p->stream));
    }
    if (n_count == 1) return CPG_OK;
    // next chain tensor with the (updated) factor, then the rest of the side
    const int nn = side == 0 ? n - 1 : n + 1;
    if (side == 0)
        CPG_TRY(launch_ttv(p->fdt, Z, p->chain[0], A[nn], p->Jn[nn], p->dims[nn], 1, R, p->ld, p->stream));
    else
        CPG_TRY(launch_ttv(p->fdt, Z, p->chain[0], A[nn - 2], 1, p->dims[nn - 2], p->Kn[nn - 1], R, p->ld,
                           p->stream));
    EpiArgs<TC> c = a;
    c.n_first = nn;
    c.n_count = n_count - 1;
    c.Z = (const TC*)p->chain[0];
    c.buf[0] = (TC*)p->chain[1];
    c.buf[1] = (TC*)p->chain[0];
    c.cost = cost ? 1 : 0;
    CPG_TRY(launch_epilogue(p->fdt, R, &c, 1, p->stream));
    return CPG_OK;
}

// All-mode gradient after the fused reduction, which wrote G^(n*), G^(n*+1)
// and the first chain step of each side (the next mode's gradient, or the
// chain buffer when modes are left): the single-block epilogue for the modes
// left after that.
static int all_modes_tail(cpgrad_plan_s* p, const FacSet<float>& fs, void* const* G) {
    const int N = p->N, ns = p->nstar;
    const bool right_more = ns > 2, left_more = N - ns > 2;
    EpiArgs<float> a[2];
    int na = 0;
    if (right_more) {
        EpiArgs<float> e = epi_base<float>(p, fs);
        e.side = 0;
        e.n_first = ns - 1;
        e.n_count = ns - 1;
        e.Z = (const float*)p->chain[0];
        e.buf[0] = (float*)p->chain[1];
        e.buf[1] = (float*)p->chain[0];
        for (int n = 0; n < N; ++n) e.Gout[n] = (float*)G[n];
        a[na++] = e;
    }
    if (left_more) {
        EpiArgs<float> e = epi_base<float>(p, fs);
        e.side = 1;
        e.n_first = ns + 2;
        e.n_count = N - ns - 1;
        e.Z = (const float*)p->chain[2];
        e.buf[0] = (float*)p->chain[3];
        e.buf[1] = (float*)p->chain[2];
        for (int n = 0; n < N; ++n) e.Gout[n] = (float*)G[n];
        a[na++] = e;
    }
    if (na) CPG_TRY(launch_epilogue(p->fdt, p->R, a, na, p->stream));
    return CPG_OK;
}

// All-mode gradient without the fused reduction: the two chains are
// independent, so a side whose first chain tensor is large first takes its
// first gradient and chain step on the multi-block kernels (into the side's
// own chain buffers), then one epilogue launch walks what is left of both
// sides, one block each.
template <typename TC>
static int run_both_sides(cpgrad_plan_s* p, const FacSet<TC>& fs, void* const* A, void* const* G) {
    const int N = p->N, R = p->R;
    EpiArgs<TC> a[2];
    int na = 0;
    for (int s = 0; s < 2; ++s) {
        const int n = s == 0 ? p->nstar : p->nstar + 1;       // the side's first mode
        const int n_count = s == 0 ? p->nstar : N - p->nstar;
        const void* Z = s == 0 ? p->PR : p->PL;
        EpiArgs<TC> e = epi_base<TC>(p, fs);
        e.side = s;
        for (int m = 0; m < N; ++m) e.Gout[m] = (TC*)G[m];
        if (side_first_small(p, s, sizeof(TC))) {
            e.n_first = n;
            e.n_count = n_count;
            e.Z = (const TC*)Z;
            e.buf[0] = (TC*)p->chain[2 * s];
            e.buf[1] = (TC*)p->chain[2 * s + 1];
            a[na++] = e;
            continue;
        }
        // the side's split partials are summed by now: their buffer holds the gradient's parts
        if (s == 0)
            CPG_TRY(launch_grad_split(p->fdt, Z, p->ld, G[n - 1], &fs, p->Jn[n - 1], p->dims[n - 1], 1, 0, n - 1, 0,
                                      0, p->PRpart, p->prpart_bytes, p->stream));
        else
            CPG_TRY(launch_grad_split(p->fdt, Z, p->ld, G[n - 1], &fs, 1, p->dims[n - 1], p->Kn[n], 0, 0, n, N - n,
                                      p->PLpart, p->plpart_bytes, p->stream));
        if (n_count == 1) continue;
        const int nn = s == 0 ? n - 1 : n + 1;
        if (s == 0)
            CPG_TRY(launch_ttv(p->fdt, Z, p->chain[0], A[nn], p->Jn[nn], p->dims[nn], 1, R, p->ld, p->stream));
        else
            CPG_TRY(launch_ttv(p->fdt, Z, p->chain[2], A[nn - 2], 1, p->dims[nn - 2], p->Kn[nn - 1], R, p->ld,
                               p->stream));
        e.n_first = nn;
        e.n_count = n_count - 1;
        e.Z = (const TC*)p->chain[2 * s];
        e.buf[0] = (TC*)p->chain[2 * s + 1];
        e.buf[1] = (TC*)p->chain[2 * s];
        a[na++] = e;
    }
    if (na) CPG_TRY(launch_epilogue(p->fdt, R, a, na, p->stream));
    return CPG_OK;
}

// What a chain does with each gradient it forms: store it, or update that
// mode's factor from it (eq. 2.14 ALS, or eq. 2.18 multiplicative).
enum ChainUpdate { kStore = 0, kAls = 1, kNtf = 2 };

static hipError_t chain_update(cpgrad_plan_s* p, int kind, const void* g, void* A, int m) {
    if (kind == kAls)
        return launch_als_update(p->fdt, g, A, p->grams, p->N, m, p->dims[m], p->R, p->flags, p->stream);
    return launch_ntf_update(p->fdt, g, A, p->grams, p->N, m, p->dims[m], p->R, p->stream);
}

// Per-kernel chains (one launch per step), used when a gradient does not fit
// the epilogue's LDS and by the multiplicative update.
static int right_chain(cpgrad_plan_s* p, const AnyFacSet& fs, void* const* A, void* const* G, int update) {
    const void* cur = p->PR;
    int buf = 0;
    for (int n = p->nstar; n >= 1; --n) {          // paper's 1-based mode n
        if (n < p->nstar) {
            // next chain tensor: contract R^(n+1) with the rank columns of A^(n+1)   (eq. 3.20)
            CPG_TRY(launch_ttv(p->fdt, cur, p->chain[buf], A[n], p->Jn[n], p->dims[n], 1, p->R, p->ld, p->stream));
            cur = p->chain[buf];
            buf ^= 1;
        }
        void* g = update ? p->Gtmp : G[n - 1];
        // gradient of mode n from R^(n) and the Khatri-Rao rows of modes 1..n-1   (eq. 3.12)
        CPG_TRY(launch_grad(p->fdt, cur, p->ld, g, fs.ptr(p->fdt), p->Jn[n - 1], p->dims[n - 1], 1, 0, n - 1, 0,
                            0, p->stream));
        if (update) CPG_TRY(chain_update(p, update, g, A[n - 1], n - 1));
    }
    return CPG_OK;
}

static int left_chain(cpgrad_plan_s* p, const AnyFacSet& fs, void* const* A, void* const* G, int update) {
    const void* cur = p->PL;
    int buf = 0;
    for (int n = p->nstar + 1; n <= p->N; ++n) {
        if (n > p->nstar + 1) {
            // next chain tensor: contract L^(n-1) with the rank columns of A^(n-1)   (eq. 3.22)
            CPG_TRY(launch_ttv(p->fdt, cur, p->chain[buf], A[n - 2], 1, p->dims[n - 2], p->Kn[n - 1], p->R,
                               p->ld, p->stream));
            cur = p->chain[buf];
            buf ^= 1;
        }
        void* g = update ? p->Gtmp : G[n - 1];
        // gradient of mode n from L^(n) and the Khatri-Rao rows of modes n+1..N   (eq. 3.16)
        CPG_TRY(launch_grad(p->fdt, cur, p->ld, g, fs.ptr(p->fdt), 1, p->dims[n - 1], p->Kn[n], 0, 0, n,
                            p->N - n, p->stream));
        if (update) CPG_TRY(chain_update(p, update, g, A[n - 1], n - 1));
    }
    return CPG_OK;
}

static int readback(cpgrad_plan_s* p, double* cost_out, double* fit_out) {
    // scal[0..15] and flags[0] in one copy (they are contiguous on the device)
    if (hipMemcpyAsync(p->host, p->scal, 16 * sizeof(double) + sizeof(int), hipMemcpyDeviceToHost, p->stream) !=
        hipSuccess)
        return CPG_ERR_HIP;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return CPG_ERR_HIP;
    int fl = 0;
    std::memcpy(&fl, p->host + 16, sizeof(int));
    if (cost_out) *cost_out = p->host[2];
    if (fit_out) *fit_out = p->host[3];
    if (fl & 1) return CPG_ERR_NOT_SPD;
    if (fl & 2) return CPG_ERR_NONFINITE;
    return CPG_OK;
}

// Algorithmic work of one all-mode gradient at split n* (1-based):
// multiply-adds of the two big contractions (2 R J_N), of the chain steps of
// eqs. 3.20 / 3.22 and of the per-mode gradients of eqs. 3.12 / 3.16, times 2;
// bytes: vec(Y) read once plus every factor read and every gradient written.
static void alg_tally(int N, const int64_t* dims, int R, int ydt, int fdt, int nstar, double* flops,
                      double* bytes) {
    int64_t Jn[CPG_MAX_MODES + 1], Kn[CPG_MAX_MODES + 1];
    Jn[0] = 1;
    for (int n = 1; n <= N; ++n) Jn[n] = Jn[n - 1] * dims[n - 1];
    Kn[N] = 1;
    for (int n = N - 1; n >= 0; --n) Kn[n] = Kn[n + 1] * dims[n];
    const double r = R;
    double mac = 2.0 * (double)Jn[N] * r;
    for (int n = nstar; n >= 1; --n) {
        if (n < nstar) mac += (double)Jn[n + 1] * r;
        mac += (double)Jn[n] * r;
    }
    for (int n = nstar + 1; n <= N; ++n) {
        if (n > nstar + 1) mac += (double)Kn[n - 2] * r;
        mac += (double)Kn[n - 1] * r;
    }
    if (flops) *flops = 2.0 * mac;
    if (bytes) {
        const double by = ydt == CPG_F64 ? 8 : (ydt == CPG_F32 ? 4 : 2);
        const double bf = fdt == CPG_F64 ? 8 : 4;
        double sumI = 0;
        for (int n = 0; n < N; ++n) sumI += (double)dims[n];
        *bytes = (double)Jn[N] * by + 2.0 * sumI * r * bf;
    }
}

static int default_nstar(int N, const int64_t* dims) {
    int64_t J = 1;
    int best = 1;
    for (int n = 1; n <= N - 1; ++n) {
        J *= dims[n - 1];
        int64_t K = 1;
        for (int m = n; m < N; ++m) K *= dims[m];
        if (J <= K) best = n;
    }
    return best;
}

static int check_shape(int N, const int64_t* dims, int R) {
    if (!dims || N < 2 || N > CPG_MAX_MODES || R < 1 || R > CPG_MAX_RANK) return CPG_ERR_INVALID;
    int64_t total = 1;
    for (int n = 0; n < N; ++n) {
        if (dims[n] < 1) return CPG_ERR_INVALID;
        if (total > INT64_MAX / dims[n]) return CPG_ERR_INVALID;
        total *= dims[n];
    }
    return CPG_OK;
}

__global__ void k_zero_flags(int* f) {
    if (threadIdx.x < 16) f[threadIdx.x] = 0;
}

// One ALS sweep enqueued on the plan's stream (no host wait): cost and fit end
// in scal[2], scal[3], failures in flags.
// A side of the ALS sweep with exactly two modes goes through the many-block
// epilogue (float32 factors, R <= 16, first gradient precomputed): rows of
// the side's last mode per block, at most kEpiRowsMaxBlocks blocks.
static int rows_per_block(int64_t I) { return (int)((I + kEpiRowsMaxBlocks - 1) / kEpiRowsMaxBlocks); }

static bool rows_side_ok(const cpgrad_plan_s* p, int side) {
    if (p->fdt != CPG_F32 || p->R > 16 || !p->fused_first) return false;
    if ((side == 0 ? p->nstar : p->N - p->nstar) != 2) return false;
    const int64_t rt = p->R <= 4 ? 4 : 16;
    const int64_t I1 = p->dims[side == 0 ? p->nstar - 1 : p->nstar], I2 = p->dims[side == 0 ? 0 : p->N - 1];
    return I1 * rt <= kEpiGCap && I2 * rt <= kEpiGCap && rows_per_block(I2) * rt <= kEpiRowsCells;
}

static int run_rows(cpgrad_plan_s* p, const FacSet<float>& fs, int side, bool cost) {
    EpiRows e{};
    e.fs = fs;
    e.side = side;
    e.n1 = side == 0 ? p->nstar : p->nstar + 1;
    e.n2 = side == 0 ? 1 : p->N;
    e.Z = (const float*)(side == 0 ? p->PR : p->PL);
    e.ld = p->ld;
    e.Gpre = (const float*)p->Gtmp;
    e.rows = rows_per_block(p->dims[e.n2 - 1]);
    e.cost = cost ? 1 : 0;
    e.grams = p->grams;
    e.scal = p->scal;
    e.flags = p->flags;
    e.part = p->rpart;
    CPG_TRY(launch_epi_rows(e, p->stream));
    return CPG_OK;
}

static int als_sweep_core(cpgrad_plan_s* p, const void* Y, void* const* A) {
    const AnyFacSet fs = facsets(p, (const void* const*)A);
    const bool epi = epilogue_fits(p);
    if (!epi) {
        hipLaunchKernelGGL(k_zero_flags, dim3(1), dim3(64), 0, p->stream, p->flags);
        CPG_TRY(hipGetLastError());
        CPG_TRY(launch_grams(p->fdt, fs.ptr(p->fdt), p->grams, p->stream));
    }
    // pass 1 over Y: P_R with the current A^(n*+1..N), then modes n*, ..., 1
    CPG_TRY(run_contract(p, Y, fs, p->t_right, 1));
    const FacSet<float>* fsf = p->fdt == CPG_F32 ? &fs.f : nullptr;
    bool pre = false;
    int st = finish_partials(p, fsf, p->t_right, 1, p->Gtmp, nullptr, true, &pre, nullptr, p->flags);
    if (st) return st;
    const bool rows_r = epi && pre && rows_side_ok(p, 0);
    if (rows_r)
        st = run_rows(p, fs.f, 0, false);   // leaves the Gram of A^(1) to the left pass's reduction
    else if (epi)
        st = p->fdt == CPG_F64 ? run_side<double>(p, fs.d, 0, A, nullptr, true, true, false)
                               : run_side<float>(p, fs.f, 0, A, nullptr, true, true, false,
                                                 pre ? (const float*)p->Gtmp : nullptr, pre);
    else
        st = right_chain(p, fs, A, nullptr, kAls);
    if (st) return st;
    // pass 2 over Y: P_L with the updated A^(1..n*), then modes n*+1, ..., N and the cost
    CPG_TRY(run_contract(p, Y, fs, p->t_left, 2));
    st = finish_partials(p, fsf, p->t_left, 2, nullptr, p->Gtmp, rows_r, &pre);
    if (st) return st;
    if (epi && pre && rows_side_ok(p, 1)) {
        st = run_rows(p, fs.f, 1, true);
        if (st) return st;
    } else if (epi) {
        st = p->fdt == CPG_F64 ? run_side<double>(p, fs.d, 1, A, nullptr, true, false, true)
                               : run_side<float>(p, fs.f, 1, A, nullptr, true, false, true,
                                                 pre ? (const float*)p->Gtmp : nullptr);
        if (st) return st;
    } else {
        st = left_chain(p, fs, A, nullptr, kAls);
        if (st) return st;
        // cost of eq. 2.12: Gtmp holds G^(N) (taken before the A^(N) update)
        CPG_TRY(launch_cost_fit(p->fdt, p->Gtmp, A[p->N - 1], p->dims[p->N - 1], p->R, nullptr, p->grams, p->N,
                                p->scal, p->flags, p->stream));
    }
    return CPG_OK;
}

// Cost of eq. 2.12 of the model given by the factor set `fs` against Y, into
// scal[slot], scal[slot+1] (no host wait).  Recomputes every Gram.
static int fit_core(cpgrad_plan_s* p, const void* Y, const AnyFacSet& fs, int slot) {
    CPG_TRY(launch_grams(p->fdt, fs.ptr(p->fdt), p->grams, p->stream));
    CPG_TRY(run_contract(p, Y, fs, p->t_right, 1));
    int st = finish_partials(p, nullptr, p->t_right, 1);
    if (st) return st;
    CPG_TRY(launch_inner_kr(p->fdt, p->PR, p->ld, p->J, fs.ptr(p->fdt), p->nstar, p->red, p->scal + 6,
                            p->stream));
    CPG_TRY(launch_cost_fit(p->fdt, nullptr, nullptr, 0, p->R, p->scal + 6, p->grams, p->N, p->scal, p->flags,
                            p->stream, slot));
    return CPG_OK;
}

// Scratch of the learned step: three factor sets of the plan's type, the
// features, sigma and the accept flag.
static int ensure_learn(cpgrad_plan_s* p) {
    if (p->lws) return CPG_OK;
    int64_t tot = 0;
    for (int n = 0; n < p->N; ++n) {
        p->fac_off[n] = tot;
        tot += ((p->dims[n] * p->R + 63) / 64) * 64;
    }
    const size_t fb = (size_t)tot * p->acc;
    const size_t bytes = 3 * fb + 256;
    if (hipMalloc((void**)&p->lws, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p->lws = nullptr;
        return CPG_ERR_NOMEM;
    }
    p->lws_bytes = bytes;
    p->l_start = p->lws;
    p->l_dprev = p->lws + fb;
    p->l_ext = p->lws + 2 * fb;
    p->l_feat = (float*)(p->lws + 3 * fb);
    // sigma and the accept flag sit in scal[12], scal[13], so the readback copy carries them
    p->l_sigma = (float*)(p->scal + 12);
    p->l_accept = (int*)(p->scal + 13);
    p->have_prev = 0;
    return hipMemsetAsync(p->lws, 0, bytes, p->stream) == hipSuccess ? CPG_OK : CPG_ERR_HIP;
}

static AnyFacSet plan_facset(const cpgrad_plan_s* p, void* base) {
    const void* ptrs[CPG_MAX_MODES];
    for (int n = 0; n < p->N; ++n) ptrs[n] = (const char*)base + p->fac_off[n] * p->acc;
    return facsets(p, ptrs);
}

// Shape, types and split of a plan (no device work, no allocation).
static int plan_init(cpgrad_plan_s* p, int N, const int64_t* dims, int R, int y_dtype, int factor_dtype, int mode,
                     void* stream) {
    if (!dims) return CPG_ERR_INVALID;
    {
        const int st = check_shape(N, dims, R);
        if (st) return st;
    }
    int64_t total = 1;
    for (int n = 0; n < N; ++n) total *= dims[n];
    if (y_dtype < CPG_F64 || y_dtype > CPG_F16 || factor_dtype < CPG_F64 || factor_dtype > CPG_F16 ||
        mode < CPG_MODE_NATIVE || mode > CPG_MODE_F16_SCALED_REFINED)
        return CPG_ERR_INVALID;
    // supported combinations (see the header)
    const bool f64 = (y_dtype == CPG_F64 && factor_dtype == CPG_F64 && mode == CPG_MODE_NATIVE);
    const bool f32 = (y_dtype == CPG_F32 && factor_dtype == CPG_F32);
    const bool b16 = (y_dtype == CPG_BF16 && factor_dtype == CPG_F32 && mode != CPG_MODE_NATIVE);
    const bool h16 = (y_dtype == CPG_F16 && factor_dtype == CPG_F32 && f16_mode(mode));
    if (!(f64 || f32 || b16 || h16)) return CPG_ERR_UNSUPPORTED;
    if (factor_dtype == CPG_BF16 || factor_dtype == CPG_F16) return CPG_ERR_UNSUPPORTED;
    p->N = N;
    p->R = R;
    p->ld = 4 * ((R + 3) / 4);
    for (int n = 0; n < N; ++n) p->dims[n] = dims[n];
    p->ydt = y_dtype;
    p->fdt = factor_dtype;
    p->mode = mode;
    p->stream = (hipStream_t)stream;
    p->acc = (factor_dtype == CPG_F64) ? 8 : 4;
    p->numel = total;
    p->Jn[0] = 1;
    for (int n = 1; n <= N; ++n) p->Jn[n] = p->Jn[n - 1] * dims[n - 1];
    p->Kn[N] = 1;
    for (int n = N - 1; n >= 0; --n) p->Kn[n] = p->Kn[n + 1] * dims[n];
    // Algorithm 2, step 1: n* = max{n : J_n <= K_n}, n in [1, N-1]; 1 if none
    p->nstar_auto = default_nstar(N, dims);
    p->nstar = p->nstar_auto;
    p->J = p->Jn[p->nstar];
    p->K = p->Kn[p->nstar];
    return plan_kind_ok(p);
}

// Enqueue the all-mode gradient on a configured plan.
static int all_modes_core(cpgrad_plan_s* p, const void* Y, const void* const* A, void* const* G) {
    const AnyFacSet fs = facsets(p, A);
    CPG_TRY(run_contract(p, Y, fs, p->t_fused, 3));
    bool pre = false;
    const bool tail = p->fdt == CPG_F32 && epilogue_fits(p);
    int st = finish_partials(p, p->fdt == CPG_F32 ? &fs.f : nullptr, p->t_fused, 3, G[p->nstar - 1], G[p->nstar],
                             false, &pre, tail ? G : nullptr);
    if (st) return st;
    if (epilogue_fits(p)) {
        if (p->fdt == CPG_F64) return run_both_sides<double>(p, fs.d, (void* const*)A, G);
        if (pre) return all_modes_tail(p, fs.f, G);
        return run_both_sides<float>(p, fs.f, (void* const*)A, G);
    }
    st = right_chain(p, fs, (void* const*)A, G, kStore);
    if (st) return st;
    return left_chain(p, fs, (void* const*)A, G, kStore);
}

// The same tensor viewed at split s (1-based) for one one-sided pass
// (roles 1: P_R = Y_(1:s) KR(s+1..N), eq. 3.10; roles 2: P_L =
// KR(1..s)^T Y_(1:s), eq. 3.9), with partial and result buffers from the
// plan's single-mode workspace (grown on first need).
static int split_view(cpgrad_plan_s* p, int s, int roles, cpgrad_plan_s* v) {
    v->N = p->N;
    v->R = p->R;
    v->ld = p->ld;
    for (int n = 0; n < p->N; ++n) {
        v->dims[n] = p->dims[n];
        v->fd[n] = p->fd[n];
    }
    for (int n = 0; n <= p->N; ++n) {
        v->Jn[n] = p->Jn[n];
        v->Kn[n] = p->Kn[n];
    }
    v->ydt = p->ydt;
    v->fdt = p->fdt;
    v->mode = p->mode;
    v->stream = p->stream;
    v->acc = p->acc;
    v->numel = p->numel;
    v->kernel_opt = p->kernel_opt;
    v->opt_cols = p->opt_cols;
    v->nstar = s;
    v->J = p->Jn[s];
    v->K = p->Kn[s];
    if (plan_kind_ok(v)) return CPG_ERR_UNSUPPORTED;
    const Tiling t = tile_pass(v, roles);
    if (roles == 1) v->t_right = t;
    else v->t_left = t;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const int64_t rows = roles == 1 ? v->J : v->K, parts = roles == 1 ? t.n_kc : t.n_jr;
    const size_t res = al((size_t)rows * v->ld * v->acc);
    const size_t need = res + al((size_t)parts * rows * v->ld * v->acc);
    if (need > p->sws_bytes) {
        if (p->sws) (void)hipFree(p->sws);
        p->sws = nullptr;
        p->sws_bytes = 0;
        if (hipMalloc((void**)&p->sws, need) != hipSuccess) {
            (void)hipGetLastError();
            p->sws = nullptr;
            return CPG_ERR_NOMEM;
        }
        p->sws_bytes = need;
    }
    if (roles == 1) {
        v->PR = p->sws;
        v->PRpart = p->sws + res;
    } else {
        v->PL = p->sws;
        v->PLpart = p->sws + res;
    }
    v->fused_first = false;
    return CPG_OK;
}

// Section 3.2: the gradient of one mode n (1-based) from one pass over Y.
// Right to left (eqs. 3.10, 3.12: split n, then contract the J_{n-1} leading
// rows with the Khatri-Rao rows of modes 1..n-1) when J_n <= K_{n-1};
// left to right (eqs. 3.9, 3.16: split n-1, then contract the K_n trailing
// columns with the Khatri-Rao rows of modes n+1..N) otherwise.  Mode 1 can
// only go right to left and mode N only left to right.
static int mode_gradient_core(cpgrad_plan_s* p, const void* Y, const void* const* A, int n, void* G, int* dir) {
    const int N = p->N;
    const bool can_r = n <= N - 1, can_l = n >= 2;
    bool right = can_r && (!can_l || p->Jn[n] <= p->Kn[n - 1]);
    cpgrad_plan_s v;
    int st = split_view(p, right ? n : n - 1, right ? 1 : 2, &v);
    if (st == CPG_ERR_UNSUPPORTED && (right ? can_l : can_r)) {
        right = !right;   // the matrix-core kind of a reduced-precision mode cannot take that split
        st = split_view(p, right ? n : n - 1, right ? 1 : 2, &v);
    }
    if (st) return st;
    const AnyFacSet fs = facsets(&v, A);
    if (right) {
        CPG_TRY(run_contract(&v, Y, fs, v.t_right, 1));
        st = finish_partials(&v, nullptr, v.t_right, 1);
        if (st) return st;
        CPG_TRY(launch_grad(v.fdt, v.PR, v.ld, G, fs.ptr(v.fdt), v.Jn[n - 1], v.dims[n - 1], 1, 0, n - 1, 0, 0,
                            v.stream));
    } else {
        CPG_TRY(run_contract(&v, Y, fs, v.t_left, 2));
        st = finish_partials(&v, nullptr, v.t_left, 2);
        if (st) return st;
        CPG_TRY(launch_grad(v.fdt, v.PL, v.ld, G, fs.ptr(v.fdt), 1, v.dims[n - 1], v.Kn[n], 0, 0, n, N - n,
                            v.stream));
    }
    if (dir) *dir = right ? 0 : 1;
    return CPG_OK;
}

// Static scratch of the allocation-free entry point: one copy per GPU, held
// until the process ends.  Host code never uses the array's name as an
// address: its device address is looked up once per device (with that device
// current) and kept in scratch_dev[].
static __device__ __align__(256) char scratch[CPG_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static void* scratch_dev[kMaxDevices];
static std::mutex scratch_mu;

static int scratch_ptr(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return CPG_ERR_HIP;
    if (dev < 0 || dev >= kMaxDevices) return CPG_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return CPG_ERR_HIP;
        }
        scratch_dev[dev] = ptr;
    }
    *out = scratch_dev[dev];
    return CPG_OK;
}

extern "C" {

const char* cpgrad_version(void) { return "cpgrad 0.1 (gfx950)"; }

const char* cpgrad_status_string(int s) {
    switch (s) {
        case CPG_OK: return "CPG_OK";
        case CPG_ERR_INVALID: return "CPG_ERR_INVALID: invalid argument";
        case CPG_ERR_NOMEM: return "CPG_ERR_NOMEM: device allocation failed";
        case CPG_ERR_HIP: return "CPG_ERR_HIP: HIP runtime error";
        case CPG_ERR_NOT_SPD: return "CPG_ERR_NOT_SPD: normal equations not positive definite";
        case CPG_ERR_UNSUPPORTED: return "CPG_ERR_UNSUPPORTED: unsupported type/mode combination";
        case CPG_ERR_NONFINITE: return "CPG_ERR_NONFINITE: non-finite cost";
        case CPG_ERR_SCRATCH:
            return "CPG_ERR_SCRATCH: the shape needs more workspace than the static scratch array holds";
        default: return "unknown cpgrad status";
    }
}

int cpgrad_plan(cpgrad_plan_t* out, int N, const int64_t* dims, int R, int y_dtype, int factor_dtype, int mode,
                void* stream) {
    if (!out) return CPG_ERR_INVALID;
    *out = nullptr;
    cpgrad_plan_s* p = new (std::nothrow) cpgrad_plan_s();
    if (!p) return CPG_ERR_NOMEM;
    int st = plan_init(p, N, dims, R, y_dtype, factor_dtype, mode, stream);
    if (st) {
        delete p;
        return st;
    }
    void* h = nullptr;
    if (hipHostMalloc(&h, 32 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        delete p;
        return CPG_ERR_NOMEM;
    }
    p->host = (double*)h;
    st = configure(p);
    if (st != CPG_OK) {
        release(p);
        (void)hipHostFree(p->host);
        delete p;
        return st;
    }
    *out = p;
    return CPG_OK;
}

int cpgrad_query(int N, const int64_t* dims, int R, int y_dtype, int factor_dtype, int force_nstar, int* n_star,
                 double* alg_flops_all_modes, double* alg_bytes_all_modes) {
    const int st = check_shape(N, dims, R);
    if (st) return st;
    if (y_dtype < CPG_F64 || y_dtype > CPG_F16 || factor_dtype < CPG_F64 || factor_dtype > CPG_F32)
        return CPG_ERR_INVALID;
    if (force_nstar != 0 && (force_nstar < 1 || force_nstar > N - 1)) return CPG_ERR_INVALID;
    const int ns = force_nstar ? force_nstar : default_nstar(N, dims);
    if (n_star) *n_star = ns;
    alg_tally(N, dims, R, y_dtype, factor_dtype, ns, alg_flops_all_modes, alg_bytes_all_modes);
    return CPG_OK;
}

int cpgrad_plan_info(cpgrad_plan_t p, int* n_star, size_t* workspace_bytes, double* alg_flops, double* alg_bytes) {
    if (!p) return CPG_ERR_INVALID;
    if (n_star) *n_star = p->nstar;
    if (workspace_bytes) *workspace_bytes = p->ws_bytes;
    alg_tally(p->N, p->dims, p->R, p->ydt, p->fdt, p->nstar, alg_flops, alg_bytes);
    return CPG_OK;
}

int cpgrad_plan_path(cpgrad_plan_t p, int* contraction_kernel, int* fused_reduction) {
    if (!p) return CPG_ERR_INVALID;
    if (contraction_kernel) *contraction_kernel = p->t_fused.kernel;
    if (fused_reduction) *fused_reduction = p->fused_first ? 1 : 0;
    return CPG_OK;
}

int cpgrad_profile_read(cpgrad_plan_t p, int roles, double* total_ms, int64_t* launches) {
    if (!p || roles < 0 || roles > 3) return CPG_ERR_INVALID;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return CPG_ERR_HIP;
    double tot = 0.0;
    int64_t cnt = 0;
    for (size_t i = 0; i < p->ev_used; ++i) {
        if (roles != 0 && p->ev_roles[i] != roles) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->ev_start[i], p->ev_stop[i]) != hipSuccess) return CPG_ERR_HIP;
        tot += ms;
        ++cnt;
    }
    if (total_ms) *total_ms = tot;
    if (launches) *launches = cnt;
    return CPG_OK;
}

int cpgrad_set_option(cpgrad_plan_t p, int option, int64_t value) {
    if (!p) return CPG_ERR_INVALID;
    if (option == CPG_OPT_PROFILE) {
        if (value < 0 || value > 1) return CPG_ERR_INVALID;
        p->profile = (int)value;
        p->ev_used = 0;
        return CPG_OK;
    }
    const int old_nstar = p->force_nstar, old_kernel = p->kernel_opt;
    const int64_t old_cols = p->opt_cols;
    if (option == CPG_OPT_FORCE_NSTAR) {
        if (value != 0 && (value < 1 || value > p->N - 1)) return CPG_ERR_INVALID;
        p->force_nstar = (int)value;
    } else if (option == CPG_OPT_KERNEL) {
        if (value < 0 || value > 2) return CPG_ERR_INVALID;
        p->kernel_opt = (int)value;
    } else if (option == CPG_OPT_MFMA_COLS) {
        if (value < 0 || value % 32 != 0 || value > (int64_t(1) << 30)) return CPG_ERR_INVALID;
        p->opt_cols = value;
    } else {
        return CPG_ERR_INVALID;
    }
    const void* b = p->bound;
    int st = configure(p);
    if (st == CPG_ERR_UNSUPPORTED) {
        // the option cannot be honoured for this plan: keep the previous settings
        p->force_nstar = old_nstar;
        p->kernel_opt = old_kernel;
        p->opt_cols = old_cols;
        const int st2 = configure(p);
        if (st2) return st2;
    }
    if (b) {
        const int sb = cpgrad_bind(p, b);
        if (sb) return sb;
    }
    return st;
}

int cpgrad_bind(cpgrad_plan_t p, const void* Y) {
    if (!p || !Y) return CPG_ERR_INVALID;
    if (((uintptr_t)Y & 15) != 0) return CPG_ERR_INVALID;
    if (launch_norm2(p->ydt, Y, p->numel, p->red, p->scal, p->stream) != hipSuccess) return CPG_ERR_HIP;
    p->bound = Y;
    p->have_prev = 0;
    return CPG_OK;
}

int cpgrad_all_modes(cpgrad_plan_t p, const void* Y, const void* const* A, void* const* G) {
    if (!p || !Y || !A || !G) return CPG_ERR_INVALID;
    if (((uintptr_t)Y & 15) != 0) return CPG_ERR_INVALID;
    for (int n = 0; n < p->N; ++n)
        if (!A[n] || !G[n]) return CPG_ERR_INVALID;
    return all_modes_core(p, Y, A, G);
}

int cpgrad_all_modes_noalloc(int N, const int64_t* dims, int R, int y_dtype, int factor_dtype, int mode,
                             const void* Y, const void* const* A, void* const* G, void* stream) {
    if (!Y || !A || !G) return CPG_ERR_INVALID;
    if (((uintptr_t)Y & 15) != 0) return CPG_ERR_INVALID;
    cpgrad_plan_s p;   // on the stack: its vectors stay empty (no profiling), nothing is allocated
    int st = plan_init(&p, N, dims, R, y_dtype, factor_dtype, mode, stream);
    if (st) return st;
    for (int n = 0; n < N; ++n)
        if (!A[n] || !G[n]) return CPG_ERR_INVALID;
    void* ws = nullptr;
    st = scratch_ptr(&ws);
    if (st) return st;
    p.ws = (char*)ws;
    p.ws_bytes = CPG_NOALLOC_SCRATCH_BYTES;
    p.ws_external = true;
    st = configure(&p);
    if (st) return st;
    return all_modes_core(&p, Y, A, G);
}

int cpgrad_e_gradient(cpgrad_plan_t p, const void* Y, const void* const* A, void* const* E) {
    if (!p || !Y || !A || !E) return CPG_ERR_INVALID;
    if (((uintptr_t)Y & 15) != 0) return CPG_ERR_INVALID;
    for (int n = 0; n < p->N; ++n)
        if (!A[n] || !E[n]) return CPG_ERR_INVALID;
    int st = all_modes_core(p, Y, A, E);
    if (st) return st;
    const AnyFacSet fs = facsets(p, A);
    CPG_TRY(launch_grams(p->fdt, fs.ptr(p->fdt), p->grams, p->stream));
    int64_t maxI = 0;
    for (int n = 0; n < p->N; ++n) maxI = std::max<int64_t>(maxI, p->dims[n]);
    CPG_TRY(launch_egrad(p->fdt, fs.ptr(p->fdt), E, p->grams, p->N, maxI * p->R, p->stream));
    return CPG_OK;
}

int cpgrad_mode_gradient(cpgrad_plan_t p, const void* Y, const void* const* A, int n, void* G, int* direction) {
    if (!p || !Y || !A || !G || n < 1 || n > p->N) return CPG_ERR_INVALID;
    if (((uintptr_t)Y & 15) != 0) return CPG_ERR_INVALID;
    for (int m = 0; m < p->N; ++m)
        if (!A[m]) return CPG_ERR_INVALID;
    return mode_gradient_core(p, Y, A, n, G, direction);
}

int cpntf_step(cpgrad_plan_t p, const void* Y, void* const* A, double* cost_out, double* fit_out) {
    if (!p || !Y || !A) return CPG_ERR_INVALID;
    if (Y != p->bound) return CPG_ERR_INVALID;
    for (int n = 0; n < p->N; ++n)
        if (!A[n]) return CPG_ERR_INVALID;
    const AnyFacSet fs = facsets(p, (const void* const*)A);
    hipLaunchKernelGGL(k_zero_flags, dim3(1), dim3(64), 0, p->stream, p->flags);
    CPG_TRY(hipGetLastError());
    CPG_TRY(launch_grams(p->fdt, fs.ptr(p->fdt), p->grams, p->stream));
    // pass 1: P_R with the current A^(n*+1..N), then modes n*, ..., 1 (eq. 2.18 after each gradient)
    CPG_TRY(run_contract(p, Y, fs, p->t_right, 1));
    int st = finish_partials(p, nullptr, p->t_right, 1);
    if (st) return st;
    st = right_chain(p, fs, A, nullptr, kNtf);
    if (st) return st;
    // pass 2: P_L with the updated A^(1..n*), then modes n*+1, ..., N
    CPG_TRY(run_contract(p, Y, fs, p->t_left, 2));
    st = finish_partials(p, nullptr, p->t_left, 2);
    if (st) return st;
    st = left_chain(p, fs, A, nullptr, kNtf);
    if (st) return st;
    // cost of eq. 2.12: Gtmp holds G^(N) (taken before the A^(N) update)
    CPG_TRY(launch_cost_fit(p->fdt, p->Gtmp, A[p->N - 1], p->dims[p->N - 1], p->R, nullptr, p->grams, p->N, p->scal,
                            p->flags, p->stream));
    if (!cost_out && !fit_out) return CPG_OK;
    return readback(p, cost_out, fit_out);
}

int cpals_step(cpgrad_plan_t p, const void* Y, void* const* A, double* cost_out, double* fit_out) {
    if (!p || !Y || !A) return CPG_ERR_INVALID;
    if (Y != p->bound) return CPG_ERR_INVALID;
    for (int n = 0; n < p->N; ++n)
        if (!A[n]) return CPG_ERR_INVALID;
    const int st = als_sweep_core(p, Y, A);
    if (st) return st;
    if (!cost_out && !fit_out) return CPG_OK;
    return readback(p, cost_out, fit_out);
}

int cp_fit(cpgrad_plan_t p, const void* Y, const void* const* A, double* cost_out, double* fit_out) {
    if (!p || !Y || !A) return CPG_ERR_INVALID;
    if (Y != p->bound) return CPG_ERR_INVALID;
    for (int n = 0; n < p->N; ++n)
        if (!A[n]) return CPG_ERR_INVALID;
    const AnyFacSet fs = facsets(p, A);
    hipLaunchKernelGGL(k_zero_flags, dim3(1), dim3(64), 0, p->stream, p->flags);
    CPG_TRY(hipGetLastError());
    const int st = fit_core(p, Y, fs, 2);
    if (st) return st;
    return readback(p, cost_out, fit_out);
}

int cpals_features(cpgrad_plan_t p, const void* const* A, const void* const* A_start, const double* costs,
                   int ncost, int iteration, float last_sigma, int last_accept, float* feat) {
    if (!p || !A || !A_start || !feat || ncost < 0 || (ncost > 0 && !costs)) return CPG_ERR_INVALID;
    for (int n = 0; n < p->N; ++n)
        if (!A[n] || !A_start[n]) return CPG_ERR_INVALID;
    int st = ensure_learn(p);
    if (st) return st;
    const AnyFacSet a = facsets(p, A), s0 = facsets(p, A_start), d = plan_facset(p, p->l_dprev);
    CPG_TRY(launch_features(p->fdt, a.ptr(p->fdt), s0.ptr(p->fdt), d.ptr(p->fdt), costs, ncost, nullptr, iteration,
                            last_sigma, last_accept, p->have_prev, feat, p->stream));
    p->have_prev = 1;
    return CPG_OK;
}

int cp_fit_extrapolated(cpgrad_plan_t p, const void* Y, const void* const* A, const void* const* A_start,
                        double sigma, double* cost_out, double* fit_out) {
    if (!p || !Y || !A || !A_start) return CPG_ERR_INVALID;
    if (Y != p->bound) return CPG_ERR_INVALID;
    for (int n = 0; n < p->N; ++n)
        if (!A[n] || !A_start[n]) return CPG_ERR_INVALID;
    int st = ensure_learn(p);
    if (st) return st;
    const AnyFacSet a = facsets(p, A), s0 = facsets(p, A_start), e = plan_facset(p, p->l_ext);
    CPG_TRY(launch_extrapolate(p->fdt, e.ptr(p->fdt), a.ptr(p->fdt), s0.ptr(p->fdt), nullptr, sigma, p->stream));
    hipLaunchKernelGGL(k_zero_flags, dim3(1), dim3(64), 0, p->stream, p->flags);
    CPG_TRY(hipGetLastError());
    st = fit_core(p, Y, e, 2);
    if (st) return st;
    return readback(p, cost_out, fit_out);
}

int cpals_extrapolate(cpgrad_plan_t p, const void* Y, void* const* A_new, const void* const* A_prev, double sigma,
                      int* accepted, double* cost_out, double* fit_out) {
    if (!p || !Y || !A_new || !A_prev || !(sigma >= 0.0) || !std::isfinite(sigma)) return CPG_ERR_INVALID;
    if (Y != p->bound) return CPG_ERR_INVALID;
    for (int n = 0; n < p->N; ++n)
        if (!A_new[n] || !A_prev[n]) return CPG_ERR_INVALID;
    int st = ensure_learn(p);
    if (st) return st;
    const AnyFacSet a = facsets(p, (const void* const*)A_new), s0 = facsets(p, A_prev),
                    e = plan_facset(p, p->l_ext);
    CPG_TRY(launch_extrapolate(p->fdt, e.ptr(p->fdt), a.ptr(p->fdt), s0.ptr(p->fdt), nullptr, sigma, p->stream));
    st = fit_core(p, Y, e, 8);      // exact cost of the extrapolated factors in scal[8]
    if (st) return st;
    CPG_TRY(launch_accept(p->fdt, a.ptr(p->fdt), e.ptr(p->fdt), p->scal, p->l_accept, p->stream));
    st = readback(p, cost_out, fit_out);   // waits for the stream; carries the accept flag
    int acc = 0;
    std::memcpy(&acc, p->host + 13, sizeof(int));
    if (accepted) *accepted = acc;
    return st;
}

int cpals_learned_step(cpgrad_plan_t p, cpmlp_t m, const void* Y, void* const* A, const double* costs, int ncost,
                       int iteration, float last_sigma, int last_accept, double* cost_out, double* fit_out,
                       int* accepted, float* sigma_out) {
    if (!p || !m || !Y || !A || ncost < 0 || (ncost > 0 && !costs)) return CPG_ERR_INVALID;
    if (Y != p->bound || mlp_num_inputs(m) != CPG_NFEAT) return CPG_ERR_INVALID;
    for (int n = 0; n < p->N; ++n)
        if (!A[n]) return CPG_ERR_INVALID;
    int st = ensure_learn(p);
    if (st) return st;
    const AnyFacSet a = facsets(p, (const void* const*)A), s0 = plan_facset(p, p->l_start),
                    d = plan_facset(p, p->l_dprev), e = plan_facset(p, p->l_ext);
    CPG_TRY(launch_copy_factors(p->fdt, s0.ptr(p->fdt), a.ptr(p->fdt), p->stream));
    st = als_sweep_core(p, Y, A);   // A <- plain ALS sweep, cost in scal[2]
    if (st) return st;
    CPG_TRY(launch_features(p->fdt, a.ptr(p->fdt), s0.ptr(p->fdt), d.ptr(p->fdt), costs, ncost, p->scal + 2,
                            iteration, last_sigma, last_accept, p->have_prev, p->l_feat, p->stream));
    p->have_prev = 1;
    CPG_TRY(launch_mlp_forward(m, p->l_feat, 1, p->l_sigma, p->stream));
    CPG_TRY(launch_extrapolate(p->fdt, e.ptr(p->fdt), a.ptr(p->fdt), s0.ptr(p->fdt), p->l_sigma, 0.0, p->stream));
    st = fit_core(p, Y, e, 8);      // exact cost of the extrapolated factors in scal[8]
    if (st) return st;
    CPG_TRY(launch_accept(p->fdt, a.ptr(p->fdt), e.ptr(p->fdt), p->scal, p->l_accept, p->stream));
    st = readback(p, cost_out, fit_out);   // waits for the stream
    float sg = 0.f;
    int acc = 0;
    std::memcpy(&sg, p->host + 12, sizeof(float));
    std::memcpy(&acc, p->host + 13, sizeof(int));
    if (accepted) *accepted = acc;
    if (sigma_out) *sigma_out = sg;
    return st;
}

int cpgrad_last_fit(cpgrad_plan_t p, double* cost_out, double* fit_out) {
    if (!p) return CPG_ERR_INVALID;
    return readback(p, cost_out, fit_out);
}

int cpgrad_destroy(cpgrad_plan_t p) {
    if (!p) return CPG_OK;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    else (void)hipDeviceSynchronize();
    release(p);
    if (p->lws) (void)hipFree(p->lws);
    if (p->sws) (void)hipFree(p->sws);
    if (p->host) (void)hipHostFree(p->host);
    for (size_t i = 0; i < p->ev_start.size(); ++i) {
        (void)hipEventDestroy(p->ev_start[i]);
        (void)hipEventDestroy(p->ev_stop[i]);
    }
    delete p;
    return CPG_OK;
}

}  // extern "C"
