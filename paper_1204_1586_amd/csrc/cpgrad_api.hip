// Host side of libcpgrad: argument checking, the plan (n*, tiling,
// workspace) and the enqueue order of Algorithm 2 and of the fast ALS sweep
// (Section 4).  Every arithmetic step runs in the HIP kernels of this
// library; the host only validates, plans and launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "cpg_internal.h"

using namespace cpg;

struct cpgrad_plan_s {
    int N = 0, R = 0;
    int64_t dims[CPG_MAX_MODES] = {0};
    int ydt = 0, fdt = 0, mode = 0;
    hipStream_t stream = nullptr;
    int nstar_auto = 1, nstar = 1;
    int force_nstar = 0, kernel_opt = 0;
    int64_t Jn[CPG_MAX_MODES + 1] = {0};   // Jn[n] = I_1 ... I_n   (Jn[0] = 1)
    int64_t Kn[CPG_MAX_MODES + 1] = {0};   // Kn[n] = I_{n+1} ... I_N (Kn[N] = 1)
    int64_t J = 0, K = 0, numel = 0;
    Tiling t_fused{}, t_right{}, t_left{};
    size_t acc = 8;                        // bytes of the accumulation / factor type
    // device workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    void* PR = nullptr;
    void* PL = nullptr;
    void* chain[2] = {nullptr, nullptr};
    void* PRpart = nullptr;
    void* PLpart = nullptr;
    void* Gtmp = nullptr;
    double* grams = nullptr;
    double* scal = nullptr;   // [0]=||Y||^2 [2]=cost [3]=fit [4]=inner [5]=||Yhat||^2 [6]=inner(cp_fit)
    double* red = nullptr;    // reduction scratch (1024 doubles)
    int* flags = nullptr;
    double* host = nullptr;   // pinned readback: scal[0..7], flags
    const void* bound = nullptr;
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

static Tiling tile_pass(const cpgrad_plan_s* p, int roles) {
    (void)roles;
    return tile_valu(p->J, p->K, p->R, p->fdt, roles);
}

static int hip_status(hipError_t e) { return e == hipSuccess ? CPG_OK : CPG_ERR_HIP; }

static void release(cpgrad_plan_s* p) {
    if (p->ws) (void)hipFree(p->ws);
    p->ws = nullptr;
    p->ws_bytes = 0;
}

// Choose n*, tile every pass and (re)allocate the workspace.
static int configure(cpgrad_plan_s* p) {
    const int N = p->N;
    p->nstar = p->force_nstar ? p->force_nstar : p->nstar_auto;
    p->J = p->Jn[p->nstar];
    p->K = p->Kn[p->nstar];
    p->t_fused = tile_pass(p, 3);
    p->t_right = tile_pass(p, 1);
    p->t_left = tile_pass(p, 2);
    const size_t a = p->acc, R = (size_t)p->R;
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
    const size_t oPRp = off;    off += al(nkc * p->J * R * a);
    const size_t oPLp = off;    off += al(njr * p->K * R * a);
    const size_t oG = off;      off += al(maxI * R * a);
    const size_t oGr = off;     off += al((size_t)N * R * R * 8);
    const size_t oS = off;      off += al(16 * 8);
    const size_t oRed = off;    off += al(kRedScratch * 8);
    const size_t oF = off;      off += al(16 * sizeof(int));
    if (off > p->ws_bytes) {
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
    p->PRpart = b + oPRp;
    p->PLpart = b + oPLp;
    p->Gtmp = b + oG;
    p->grams = (double*)(b + oGr);
    p->scal = (double*)(b + oS);
    p->red = (double*)(b + oRed);
    p->flags = (int*)(b + oF);
    if (hipMemsetAsync(p->scal, 0, 16 * 8, p->stream) != hipSuccess) return CPG_ERR_HIP;
    if (hipMemsetAsync(p->flags, 0, 16 * sizeof(int), p->stream) != hipSuccess) return CPG_ERR_HIP;
    p->bound = nullptr;
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

static hipError_t run_contract(cpgrad_plan_s* p, const void* Y, const AnyFacSet& fs, const Tiling& t, int roles) {
    if (t.kernel == 2)
        return launch_contract_mfma(p->ydt, p->mode, Y, p->J, p->K, fs.f, p->nstar, t, roles, (float*)p->PRpart,
                                    (float*)p->PLpart, p->stream);
    return launch_contract_valu(p->ydt, p->fdt, Y, p->J, p->K, fs.ptr(p->fdt), p->nstar, t, roles, p->PRpart,
                                p->PLpart, p->stream);
}

#define CPG_TRY(x)                                   \
    do {                                             \
        hipError_t _e = (x);                         \
        if (_e != hipSuccess) return CPG_ERR_HIP;    \
    } while (0)

// Reduce the partials of a pass into P_R and/or P_L.
static int finish_partials(cpgrad_plan_s* p, const Tiling& t, int roles) {
    if (roles & 1) CPG_TRY(launch_reduce_parts(p->fdt, p->PRpart, t.n_kc, p->J, p->R, p->PR, p->stream));
    if (roles & 2) CPG_TRY(launch_reduce_parts(p->fdt, p->PLpart, t.n_jr, p->K, p->R, p->PL, p->stream));
    return CPG_OK;
}

// Right chain of Algorithm 2 (steps 4-5 and 9-12): modes n*, ..., 1.
// If `update`, eq. 2.14 is applied to each mode right after its gradient and
// the next chain step uses the updated factor; otherwise G[n] receives the
// gradient.
static int right_chain(cpgrad_plan_s* p, const AnyFacSet& fs, void* const* A, void* const* G, bool update) {
    const void* cur = p->PR;
    int buf = 0;
    for (int n = p->nstar; n >= 1; --n) {          // paper's 1-based mode n
        if (n < p->nstar) {
            // vec R^(r,n) = reshape(R^(r,n+1), [J_n, I_{n+1}]) a_r^(n+1)   (eq. 3.20)
            CPG_TRY(launch_ttv(p->fdt, cur, p->chain[buf], A[n], p->Jn[n], p->dims[n], 1, p->R, p->stream));
            cur = p->chain[buf];
            buf ^= 1;
        }
        void* g = update ? p->Gtmp : G[n - 1];
        // g_r^(n) = reshape(R^(r,n), [J_{n-1}, I_n])^T (a_r^(n-1) (x) ... (x) a_r^(1))   (eq. 3.12)
        CPG_TRY(launch_grad(p->fdt, cur, g, fs.ptr(p->fdt), p->Jn[n - 1], p->dims[n - 1], 1, 0, n - 1, 0, 0,
                            p->stream));
        if (update)
            CPG_TRY(launch_als_update(p->fdt, g, A[n - 1], p->grams, p->N, n - 1, p->dims[n - 1], p->R, p->flags,
                                      p->stream));
    }
    return CPG_OK;
}

// Left chain of Algorithm 2 (steps 7-8 and 13-16): modes n*+1, ..., N.
static int left_chain(cpgrad_plan_s* p, const AnyFacSet& fs, void* const* A, void* const* G, bool update) {
    const void* cur = p->PL;
    int buf = 0;
    for (int n = p->nstar + 1; n <= p->N; ++n) {
        if (n > p->nstar + 1) {
            // vec L^(r,n) = reshape(L^(r,n-1), [I_{n-1}, K_{n-1}])^T a_r^(n-1)   (eq. 3.22)
            CPG_TRY(launch_ttv(p->fdt, cur, p->chain[buf], A[n - 2], 1, p->dims[n - 2], p->Kn[n - 1], p->R,
                               p->stream));
            cur = p->chain[buf];
            buf ^= 1;
        }
        void* g = update ? p->Gtmp : G[n - 1];
        // g_r^(n) = reshape(L^(r,n), [I_n, K_n]) (a_r^(N) (x) ... (x) a_r^(n+1))   (eq. 3.16)
        CPG_TRY(launch_grad(p->fdt, cur, g, fs.ptr(p->fdt), 1, p->dims[n - 1], p->Kn[n], 0, 0, n, p->N - n,
                            p->stream));
        if (update)
            CPG_TRY(launch_als_update(p->fdt, g, A[n - 1], p->grams, p->N, n - 1, p->dims[n - 1], p->R, p->flags,
                                      p->stream));
    }
    return CPG_OK;
}

static int readback(cpgrad_plan_s* p, double* cost_out, double* fit_out) {
    if (hipMemcpyAsync(p->host, p->scal, 8 * sizeof(double), hipMemcpyDeviceToHost, p->stream) != hipSuccess)
        return CPG_ERR_HIP;
    if (hipMemcpyAsync(p->host + 8, p->flags, sizeof(int), hipMemcpyDeviceToHost, p->stream) != hipSuccess)
        return CPG_ERR_HIP;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return CPG_ERR_HIP;
    int fl = 0;
    std::memcpy(&fl, p->host + 8, sizeof(int));
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
        default: return "unknown cpgrad status";
    }
}

int cpgrad_plan(cpgrad_plan_t* out, int N, const int64_t* dims, int R, int y_dtype, int factor_dtype, int mode,
                void* stream) {
    if (!out || !dims) return CPG_ERR_INVALID;
    *out = nullptr;
    {
        const int st = check_shape(N, dims, R);
        if (st) return st;
    }
    int64_t total = 1;
    for (int n = 0; n < N; ++n) total *= dims[n];
    if (y_dtype < CPG_F64 || y_dtype > CPG_BF16 || factor_dtype < CPG_F64 || factor_dtype > CPG_BF16 ||
        mode < CPG_MODE_NATIVE || mode > CPG_MODE_BF16_REFINED)
        return CPG_ERR_INVALID;
    // supported combinations (see the header)
    const bool f64 = (y_dtype == CPG_F64 && factor_dtype == CPG_F64 && mode == CPG_MODE_NATIVE);
    const bool f32 = (y_dtype == CPG_F32 && factor_dtype == CPG_F32);
    const bool b16 = (y_dtype == CPG_BF16 && factor_dtype == CPG_F32 && mode != CPG_MODE_NATIVE);
    if (!(f64 || f32 || b16)) return CPG_ERR_UNSUPPORTED;
    if (factor_dtype == CPG_BF16) return CPG_ERR_UNSUPPORTED;

    cpgrad_plan_s* p = new (std::nothrow) cpgrad_plan_s();
    if (!p) return CPG_ERR_NOMEM;
    p->N = N;
    p->R = R;
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
    void* h = nullptr;
    if (hipHostMalloc(&h, 16 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        delete p;
        return CPG_ERR_NOMEM;
    }
    p->host = (double*)h;
    const int st = configure(p);
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
    if (y_dtype < CPG_F64 || y_dtype > CPG_BF16 || factor_dtype < CPG_F64 || factor_dtype > CPG_F32)
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

int cpgrad_set_option(cpgrad_plan_t p, int option, int64_t value) {
    if (!p) return CPG_ERR_INVALID;
    if (option == CPG_OPT_FORCE_NSTAR) {
        if (value != 0 && (value < 1 || value > p->N - 1)) return CPG_ERR_INVALID;
        p->force_nstar = (int)value;
    } else if (option == CPG_OPT_KERNEL) {
        if (value < 0 || value > 2) return CPG_ERR_INVALID;
        p->kernel_opt = (int)value;
    } else {
        return CPG_ERR_INVALID;
    }
    const void* b = p->bound;
    const int st = configure(p);
    if (st == CPG_OK && b) return cpgrad_bind(p, b);
    return st;
}

int cpgrad_bind(cpgrad_plan_t p, const void* Y) {
    if (!p || !Y) return CPG_ERR_INVALID;
    if (launch_norm2(p->ydt, Y, p->numel, p->red, p->scal, p->stream) != hipSuccess) return CPG_ERR_HIP;
    p->bound = Y;
    return CPG_OK;
}

int cpgrad_all_modes(cpgrad_plan_t p, const void* Y, const void* const* A, void* const* G) {
    if (!p || !Y || !A || !G) return CPG_ERR_INVALID;
    for (int n = 0; n < p->N; ++n)
        if (!A[n] || !G[n]) return CPG_ERR_INVALID;
    const AnyFacSet fs = facsets(p, A);
    CPG_TRY(run_contract(p, Y, fs, p->t_fused, 3));
    int st = finish_partials(p, p->t_fused, 3);
    if (st) return st;
    st = right_chain(p, fs, (void* const*)A, G, false);
    if (st) return st;
    return left_chain(p, fs, (void* const*)A, G, false);
}

int cpals_step(cpgrad_plan_t p, const void* Y, void* const* A, double* cost_out, double* fit_out) {
    if (!p || !Y || !A) return CPG_ERR_INVALID;
    if (Y != p->bound) return CPG_ERR_INVALID;
    for (int n = 0; n < p->N; ++n)
        if (!A[n]) return CPG_ERR_INVALID;
    const AnyFacSet fs = facsets(p, (const void* const*)A);
    hipLaunchKernelGGL(k_zero_flags, dim3(1), dim3(64), 0, p->stream, p->flags);
    CPG_TRY(hipGetLastError());
    CPG_TRY(launch_grams(p->fdt, fs.ptr(p->fdt), p->grams, p->stream));
    // pass 1 over Y: P_R with the current A^(n*+1..N), then modes n*, ..., 1
    CPG_TRY(run_contract(p, Y, fs, p->t_right, 1));
    int st = finish_partials(p, p->t_right, 1);
    if (st) return st;
    st = right_chain(p, fs, A, nullptr, true);
    if (st) return st;
    // pass 2 over Y: P_L with the updated A^(1..n*), then modes n*+1, ..., N
    CPG_TRY(run_contract(p, Y, fs, p->t_left, 2));
    st = finish_partials(p, p->t_left, 2);
    if (st) return st;
    st = left_chain(p, fs, A, nullptr, true);
    if (st) return st;
    // cost of eq. 2.12: Gtmp holds G^(N) (taken before the A^(N) update)
    CPG_TRY(launch_cost_fit(p->fdt, p->Gtmp, A[p->N - 1], p->dims[p->N - 1], p->R, nullptr, p->grams, p->N,
                            p->scal, p->flags, p->stream));
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
    CPG_TRY(launch_grams(p->fdt, fs.ptr(p->fdt), p->grams, p->stream));
    CPG_TRY(run_contract(p, Y, fs, p->t_right, 1));
    int st = finish_partials(p, p->t_right, 1);
    if (st) return st;
    CPG_TRY(launch_inner_kr(p->fdt, p->PR, p->J, fs.ptr(p->fdt), p->nstar, p->red, p->scal + 6, p->stream));
    CPG_TRY(launch_cost_fit(p->fdt, nullptr, nullptr, 0, p->R, p->scal + 6, p->grams, p->N, p->scal, p->flags,
                            p->stream));
    return readback(p, cost_out, fit_out);
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
    if (p->host) (void)hipHostFree(p->host);
    delete p;
    return CPG_OK;
}

}  // extern "C"
