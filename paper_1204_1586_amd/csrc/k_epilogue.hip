// The chain epilogue of Algorithm 2 in one block: after a big contraction has
// produced P_R (= R^(n*), eq. 3.10) or P_L (= L^(n*+1), eq. 3.9), one block of
// 512 threads walks that side's modes.  For each mode it
//   * forms G^(n) from the chain tensor (cp_gradient 'right', eq. 3.12, or
//     'left', eq. 3.16) in float64 in LDS,
//   * either writes it out (all-mode gradient) or applies the ALS update of
//     eq. 2.14 with the Section 4 order: Gamma = Hadamard product of the other
//     modes' float64 Grams, Cholesky (one wave, rows in registers, one
//     jittered retry), W = L^{-1}, Gamma^{-1} = W^T W, A^(n) = G Gamma^{-1},
//     then the Gram of the new factor,
//   * steps the chain with the (updated) factor: eq. 3.20 on the right,
//     eq. 3.22 on the left.
// The left epilogue of an ALS sweep ends with the cost of eq. 2.12 and the
// fit.  Small chain tensors (hundreds of KB) are latency-bound work, so one
// block replaces a dozen dependent kernel launches.
#include "cpg_device.h"

// Optional phase timestamps for profiling builds; compiled out by default.
#ifndef CPG_EPI_MARK
#define CPG_EPI_MARK(k)
#endif
#ifndef CPG_EPI_WMARK
#define CPG_EPI_WMARK(k)
#endif

namespace cpg {

constexpr int kEpiThreads = 512;

__device__ __forceinline__ void wave_lds_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

struct d4 {
    double x, y, z, w;
};
__device__ __forceinline__ d4 operator+(d4 a, d4 b) { return d4{a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w}; }


// Four consecutive chain-tensor entries as loaded (16-byte aligned: rows
// have stride ld = 4k), converted to float64 when weighted.
template <typename TC>
struct Raw4;
template <>
struct Raw4<float> {
    float4 v;
    __device__ __forceinline__ static Raw4 load(const float* p) { return Raw4{*(const float4*)p}; }
    __device__ __forceinline__ d4 mul(const double* w) const {
        return d4{(double)v.x * w[0], (double)v.y * w[1], (double)v.z * w[2], (double)v.w * w[3]};
    }
};
template <>
struct Raw4<double> {
    double2 a, b;
    __device__ __forceinline__ static Raw4 load(const double* p) {
        return Raw4{*(const double2*)p, *(const double2*)(p + 2)};
    }
    __device__ __forceinline__ d4 mul(const double* w) const {
        return d4{a.x * w[0], a.y * w[1], b.x * w[2], b.y * w[3]};
    }
};

// LDS staging of n float64 entries, kStageBatch per thread in flight:
// load(e) is called with a valid e (tails are clamped, so no load sits behind
// a branch) and store(e, v) only for e < n.
constexpr int kStageBatch = 4;
template <typename Load, typename Store>
__device__ __forceinline__ void stage_batched(int64_t n, Load load, Store store) {
    for (int64_t e0 = threadIdx.x; e0 < n; e0 += kStageBatch * kEpiThreads) {
        double v[kStageBatch];
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int64_t e = e0 + u * kEpiThreads;
            v[u] = load(e < n ? e : n - 1);
        }
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int64_t e = e0 + u * kEpiThreads;
            if (e < n) store(e, v[u]);
        }
    }
}

// Khatri-Rao rows t (Notation 2.1 order, modes first..first+count-1) into
// sKR[t*ld + r], zero for r >= R; one mode at a time over a batch of entries,
// so each mode costs one round of loads.
template <typename TC>
__device__ __forceinline__ void stage_kr(const FacSet<TC>& fs, int first, int count, int64_t T, int ld, double* sKR) {
    const int R = fs.R;
    const int64_t n = T * ld;
    for (int64_t e0 = threadIdx.x; e0 < n; e0 += kStageBatch * kEpiThreads) {
        double v[kStageBatch];
        int64_t idx[kStageBatch];
        int r[kStageBatch];
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int64_t e = min(e0 + u * kEpiThreads, n - 1);
            idx[u] = e / ld;
            r[u] = (int)(e - idx[u] * ld);
            v[u] = r[u] < R ? 1.0 : 0.0;
            r[u] = r[u] < R ? r[u] : R - 1;
        }
        for (int m = 0; m < count; ++m) {
            const int64_t d = fs.dims[first + m];
            const TC* A = fs.A[first + m];
            TC x[kStageBatch];
#pragma unroll
            for (int u = 0; u < kStageBatch; ++u) {
                const int64_t q = idx[u] / d;
                x[u] = A[(idx[u] - q * d) * R + r[u]];
                idx[u] = q;
            }
#pragma unroll
            for (int u = 0; u < kStageBatch; ++u) v[u] *= (double)x[u];
        }
#pragma unroll
        for (int u = 0; u < kStageBatch; ++u) {
            const int64_t e = e0 + u * kEpiThreads;
            if (e < n) sKR[e] = v[u];
        }
    }
}

constexpr int kEpiBatch = 16;   // chain-tensor loads in flight per thread

// For O outputs (each four consecutive ranks) sum T weighted terms: term t of
// output o is the four entries at addr(o, t) times the four float64 weights at
// wt(o, t); store(o, d4) receives the sum.  Loads go out kEpiBatch at a time
// before any is used (the chain tensors are streamed from memory by this one
// block, so the loads in flight set its speed).  Few outputs: the terms of
// one output are split over several threads and the parts summed in fixed
// order.
template <typename TC, typename Addr, typename Wt, typename Store>
__device__ __forceinline__ void block_sum_terms(int64_t O, int64_t T, Addr addr, Wt wt, Store store, d4* spart) {
    const int tid = threadIdx.x;
    auto run = [&](int64_t o, int64_t t0, int64_t tstep) {
        d4 a0{0, 0, 0, 0}, a1{0, 0, 0, 0};
        int64_t t = t0;
        // full batches without branches (so the loads stay in flight together), then the tail
        for (; t + (kEpiBatch - 1) * tstep < T; t += kEpiBatch * tstep) {
            Raw4<TC> v[kEpiBatch];
#pragma unroll
            for (int u = 0; u < kEpiBatch; ++u) v[u] = Raw4<TC>::load(addr(o, t + u * tstep));
#pragma unroll
            for (int u = 0; u < kEpiBatch; u += 2) {
                a0 = a0 + v[u].mul(wt(o, t + u * tstep));
                a1 = a1 + v[u + 1].mul(wt(o, t + (u + 1) * tstep));
            }
        }
        for (; t < T; t += tstep) a0 = a0 + Raw4<TC>::load(addr(o, t)).mul(wt(o, t));
        return a0 + a1;
    };
    if (O >= kEpiThreads) {
        for (int64_t o = tid; o < O; o += kEpiThreads) store(o, run(o, 0, 1));
        __syncthreads();
    } else {
        const int g = kEpiThreads / (int)O;
        d4 acc{0, 0, 0, 0};
        if (tid < g * O) acc = run(tid % O, tid / (int)O, g);
        spart[tid] = acc;
        __syncthreads();
        if (tid < O) {
            d4 tot{0, 0, 0, 0};
            for (int p = 0; p < g; ++p) tot = tot + spart[p * O + tid];
            store(tid, tot);
        }
        __syncthreads();
    }
}

// sG[i*RT + r] = sum_t Z[(i*si + t*st)*ld + r] * KR(t, r)  (cp_gradient 'right' / 'left'):
// right: si = J_{n-1}, st = 1, KR over modes 1..n-1; left: si = 1, st = I_n, KR over modes n+1..N.
template <typename TC, int RT>
__device__ __forceinline__ void block_grad(const TC* __restrict__ Z, int ld, const FacSet<TC>& fs, int64_t I,
                                           int64_t T, int64_t si, int64_t st, int kr_first, int kr_count,
                                           double* sG, double* sKR, d4* spart) {
    // the host guarantees T * ld <= kEpiKRCap
    const int R = fs.R;
    const int nq = ld >> 2;
    {
        stage_kr(fs, kr_first, kr_count, T, ld, sKR);
        __syncthreads();
        block_sum_terms<TC>(
            I * nq, T,
            [&](int64_t o, int64_t t) {
                const int64_t i = o / nq;
                const int q4 = 4 * (int)(o - i * nq);
                return Z + (i * si + t * st) * ld + q4;
            },
            [&](int64_t o, int64_t t) {
                const int64_t i = o / nq;
                const int q4 = 4 * (int)(o - i * nq);
                return (const double*)(sKR + t * ld + q4);
            },
            [&](int64_t o, d4 v) {
                const int64_t i = o / nq;
                const int q4 = 4 * (int)(o - i * nq);
                double* g = sG + i * RT + q4;
                g[0] = v.x;
                if (q4 + 1 < RT) g[1] = v.y;
                if (q4 + 2 < RT) g[2] = v.z;
                if (q4 + 3 < RT) g[3] = v.w;
            },
            spart);
    }
}

// out[(lo + lo_n*hi)*ld + r] = sum_i in[(lo + lo_n*(i + I*hi))*ld + r] * a[i*R + r]
template <typename TC>
__device__ __forceinline__ void block_ttv(const TC* __restrict__ in, TC* __restrict__ out, const TC* __restrict__ a,
                                          int64_t lo_n, int64_t I, int64_t hi_n, int R, int ld, double* sA,
                                          d4* spart) {
    const int nq = ld >> 2;
    stage_batched(
        I * ld,
        [&](int64_t e) {
            const int64_t i = e / ld;
            const int r = (int)(e - i * ld);
            const double x = (double)a[i * R + (r < R ? r : R - 1)];
            return r < R ? x : 0.0;
        },
        [&](int64_t e, double v) { sA[e] = v; });
    __syncthreads();
    block_sum_terms<TC>(
        lo_n * hi_n * nq, I,
        [&](int64_t o, int64_t i) {
            const int64_t row = o / nq;
            const int q4 = 4 * (int)(o - row * nq);
            const int64_t hi = row / lo_n, lo = row - (row / lo_n) * lo_n;
            return in + (lo + lo_n * (i + I * hi)) * ld + q4;
        },
        [&](int64_t o, int64_t i) {
            const int64_t row = o / nq;
            const int q4 = 4 * (int)(o - row * nq);
            return (const double*)(sA + i * ld + q4);
        },
        [&](int64_t o, d4 v) {
            const int64_t row = o / nq;
            const int q4 = 4 * (int)(o - row * nq);
            TC* d = out + row * ld + q4;
            d[0] = (TC)v.x;
            d[1] = (TC)v.y;
            d[2] = (TC)v.z;
            d[3] = (TC)v.w;
        },
        spart);
}

// Gram entries of one or more staged factors: sA holds the factors back to
// back (mode m at sA + off[m], I_m x R, float64); entry e of the flat list
// (mode m, r, c) = sum_i A(i,r) A(i,c).  All entries of all staged modes are
// spread over the block; each entry's terms may be split over two threads.
__device__ __forceinline__ void block_gram_staged(const double* sA, const int64_t* off, const int64_t* I, int m0,
                                                  int m1, int R, double* grams, double* spart) {
    const int tid = threadIdx.x;
    const int RR = R * R;
    const int E = (m1 - m0) * RR;
    const int g = E * 2 <= kEpiThreads ? 2 : 1;      // threads per entry
    double acc = 0.0;
    int e = tid % (E > 0 ? E : 1);
    const int part = tid / (E > 0 ? E : 1);
    for (int ee = tid; ee < E * g; ee += kEpiThreads) {
        e = ee % E;
        const int h = ee / E;
        const int m = m0 + e / RR;
        const int rc = e - (e / RR) * RR;
        const int r = rc / R, c = rc - (rc / R) * R;
        const double* A = sA + off[m];
        double a0 = 0.0, a1 = 0.0;
        int64_t i = h;
        for (; i + g < I[m]; i += 2 * g) {
            a0 += A[i * R + r] * A[i * R + c];
            a1 += A[(i + g) * R + r] * A[(i + g) * R + c];
        }
        if (i < I[m]) a0 += A[i * R + r] * A[i * R + c];
        acc = a0 + a1;
        if (g == 1) grams[(int64_t)m * RR + rc] = acc;
    }
    (void)part;
    if (g == 2) {
        spart[tid] = tid < 2 * E ? acc : 0.0;
        __syncthreads();
        if (tid < E) {
            const int m = m0 + tid / RR;
            grams[(int64_t)m * RR + (tid - (tid / RR) * RR)] = spart[tid] + spart[tid + E];
        }
    }
    __syncthreads();
}

// All N Grams in float64, staging as many factors at a time as fit in sA.
template <typename TC>
__device__ __forceinline__ void block_grams_all(const FacSet<TC>& fs, double* grams, double* sA, double* spart) {
    const int R = fs.R, N = fs.N;
    int64_t off[CPG_MAX_MODES], I[CPG_MAX_MODES];
    for (int m = 0; m < N; ++m) I[m] = fs.dims[m];
    int m0 = 0;
    while (m0 < N) {
        int m1 = m0;
        int64_t used = 0;
        while (m1 < N && used + I[m1] * R <= kEpiKRCap) {
            off[m1] = used;
            used += I[m1] * R;
            ++m1;
        }
        __syncthreads();
        for (int m = m0; m < m1; ++m) {
            const TC* A = fs.A[m];
            stage_batched(
                I[m] * R, [&](int64_t e) { return (double)A[e]; }, [&](int64_t e, double v) { sA[off[m] + e] = v; });
        }
        __syncthreads();
        block_gram_staged(sA, off, I, m0, m1, R, grams, spart);
        m0 = m1;
    }
}

// eq. 2.14 for mode n (0-based) with G^(n) in sG, wide rank tiles: A^(n) <- G Gamma^{-1} by a
// float64 Cholesky factorisation Gamma = L L^T (right-looking, one block
// barrier per column; one retry with Gamma + 1e-12 tr(Gamma)/R I) and, for
// every row g of G, the two triangular solves L z = g^T, L^T x = z.  Returns
// false (leaving A^(n) and grams[n] untouched) if Gamma is not SPD.
template <typename TC, int RT>
__device__ __forceinline__ bool block_solve_lds(const EpiArgs<TC>& a, int n, const double* sG, double* sGam, double* sL,
                                            double* sA, double* spart, int* sOk) {
    constexpr int LD = RT + 1;
    const int tid = threadIdx.x;
    const int R = a.fs.R;
    const int N = a.fs.N;
    const int64_t I = a.fs.dims[n];
    for (int e = tid; e < R * R; e += kEpiThreads) {
        double g[CPG_MAX_MODES];
#pragma unroll
        for (int k = 0; k < CPG_MAX_MODES; ++k) g[k] = (k < N && k != n) ? a.grams[(int64_t)k * R * R + e] : 1.0;
        double v = 1.0;
#pragma unroll
        for (int k = 0; k < CPG_MAX_MODES; ++k) v *= g[k];
        sGam[e] = v;
    }
    __syncthreads();
    CPG_EPI_MARK(20);
    double tr = 0.0;
    for (int c = 0; c < R; ++c) tr += sGam[c * R + c];
    bool good = false;
    for (int attempt = 0; attempt < 2 && !good; ++attempt) {
        const double jit = attempt == 0 ? 0.0 : 1e-12 * tr / R;
        for (int e = tid; e < R * R; e += kEpiThreads) {
            const int i = e / R, j = e - (e / R) * R;
            sL[i * LD + j] = sGam[e] + (i == j ? jit : 0.0);
        }
        __syncthreads();
        bool bad = false;
        // column c: trailing update a_ij -= a_ic a_jc / a_cc (c < j <= i), one barrier
        for (int c = 0; c < R; ++c) {
            const double d = sL[c * LD + c];
            bad = bad || !(d > 0.0) || !isfinite(d);
            const double inv = bad ? 0.0 : 1.0 / d;
            const int m = R - 1 - c;
            for (int e = tid; e < m * m; e += kEpiThreads) {
                const int i = c + 1 + e / m, j = c + 1 + (e - (e / m) * m);
                if (j <= i) sL[i * LD + j] -= sL[i * LD + c] * sL[j * LD + c] * inv;
            }
            __syncthreads();
        }
        good = !bad;
        if (good) {
            // scale the columns: L_ic = a_ic / sqrt(a_cc); keep 1/L_cc on the diagonal
            for (int e = tid; e < R * R; e += kEpiThreads) {
                const int i = e / R, c = e - (e / R) * R;
                if (i > c) sL[i * LD + c] = sL[i * LD + c] / sqrt(sL[c * LD + c]);
            }
            __syncthreads();
            for (int c = tid; c < R; c += kEpiThreads) sL[c * LD + c] = 1.0 / sqrt(sL[c * LD + c]);
            __syncthreads();
        }
    }
    CPG_EPI_MARK(21);
    if (!good) return false;
    // W = L^{-1}, one row per step: w_ij = (delta_ij - sum_{j<=k<i} L_ik w_kj) / L_ii  (W in sGam)
    for (int i = 0; i < R; ++i) {
        for (int j = tid; j <= i; j += kEpiThreads) {
            double v = (i == j) ? 1.0 : 0.0;
            for (int k = j; k < i; ++k) v -= sL[i * LD + k] * sGam[k * RT + j];
            sGam[i * RT + j] = v * sL[i * LD + i];
        }
        __syncthreads();
    }
    // Gamma^{-1} = W^T W (W lower triangular) -> sL (stride LD); L is no longer needed
    for (int e = tid; e < R * R; e += kEpiThreads) {
        const int r = e / R, c = e - (e / R) * R;
        double acc = 0.0;
        for (int i = (r > c ? r : c); i < R; ++i) acc += sGam[i * RT + r] * sGam[i * RT + c];
        sL[r * LD + c] = acc;
    }
    __syncthreads();
    // A^(n) = G Gamma^{-1}
    TC* A = (TC*)a.fs.A[n];
    for (int64_t o = tid; o < I * R; o += kEpiThreads) {
        const int64_t i = o / R;
        const int c = (int)(o - i * R);
        double a0 = 0.0, a1 = 0.0;
        int s = 0;
        for (; s + 2 <= R; s += 2) {
            a0 += sG[i * RT + s] * sL[s * LD + c];
            a1 += sG[i * RT + s + 1] * sL[(s + 1) * LD + c];
        }
        if (s < R) a0 += sG[i * RT + s] * sL[s * LD + c];
        const TC v = (TC)(a0 + a1);
        A[o] = v;
        sA[o] = (double)v;   // the stored (rounded) factor, for its Gram
    }
    __syncthreads();
    CPG_EPI_MARK(22);
    CPG_EPI_MARK(23);
    int64_t off0 = 0, In[CPG_MAX_MODES];
    In[n] = I;
    int64_t offs[CPG_MAX_MODES];
    offs[n] = off0;
    block_gram_staged(sA, offs, In, n, n + 1, R, a.grams, spart);
    return true;
}

// 1/sqrt(d) in float64: hardware estimate refined by two Newton steps
__device__ __forceinline__ double rsqrt_d(double d) {
    double y = __builtin_amdgcn_rsq(d);
    y = y * (1.5 - 0.5 * d * y * y);
    y = y * (1.5 - 0.5 * d * y * y);
    return y;
}

// Gamma (R x R, stride RT) = Hadamard product of the float64 Grams of every
// mode but n (eq. 2.14).
template <typename TC, int RT>
__device__ __forceinline__ void block_gamma(const EpiArgs<TC>& a, int n, double* sGam) {
    const int R = a.fs.R;
    const int N = a.fs.N;
    for (int e = threadIdx.x; e < R * R; e += kEpiThreads) {
        double g[CPG_MAX_MODES];
#pragma unroll
        for (int k = 0; k < CPG_MAX_MODES; ++k) g[k] = (k < N && k != n) ? a.grams[(int64_t)k * R * R + e] : 1.0;
        double v = 1.0;
#pragma unroll
        for (int k = 0; k < CPG_MAX_MODES; ++k) v *= g[k];
        const int i = e / R;
        sGam[i * RT + (e - i * R)] = v;
    }
}

// One wave: W = L^{-1} for Gamma = L L^T (Gamma in sGam, stride RT), written
// to sW (stride RT, zero above the diagonal); rows and columns R..RT-1 are
// padded with the identity.  Cholesky in the row (dot-product) form
//   L_jj = sqrt(Gamma_jj - sum_{k<j} L_jk^2),
//   L_ij = (Gamma_ij - sum_{k<j} L_ik L_jk) / L_jj          (i > j):
// lane i keeps row i in registers and publishes each new entry L_ij to LDS
// (sLs, stride RT; 1/L_jj after the RT x RT entries); at column j every lane
// reads row j back as a broadcast and forms the pivot itself, so no lane
// waits on another beyond the wave's in-order LDS traffic.  Then W column by
// column, lane c independently:
//   W_cc = 1/L_cc,  W_ic = -(sum_{c<=k<i} L_ik W_kc) / L_ii   (i > c),
// with the rows of L read from LDS.  Returns false on a pivot that is not
// positive and finite (uniform over the wave).
template <int RT>
__device__ __forceinline__ bool wave_chol_inverse(const double* sGam, int R, double jit, double* sLs, double* sW) {
    // lane id read here (not hoistable): the lane masks of the unrolled
    // columns then live only inside this function instead of the whole kernel
    int l;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
    double* sDinv = sLs + RT * RT;
    auto gam = [&](int i, int k) -> double {
        return (i < R && k < R) ? sGam[i * RT + k] + (i == k ? jit : 0.0) : (i == k ? 1.0 : 0.0);
    };
    double x[RT], diag[RT];
#pragma unroll
    for (int k = 0; k < RT; ++k) {
        x[k] = l < RT ? gam(l, k) : 0.0;
        diag[k] = gam(k, k);
    }
    bool bad = false;
    CPG_EPI_WMARK(0);
#pragma unroll
    for (int j = 0; j < RT; ++j) {
        double Lj[j > 0 ? j : 1];
#pragma unroll
        for (int k = 0; k < j; ++k) Lj[k] = sLs[j * RT + k];
        const double gjj = diag[j];
        double sv[4] = {0.0, 0.0, 0.0, 0.0}, st[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < j; ++k) {
            sv[k & 3] += Lj[k] * Lj[k];
            st[k & 3] += x[k] * Lj[k];
        }
        const double v = gjj - ((sv[0] + sv[1]) + (sv[2] + sv[3]));
        const double t = x[j] - ((st[0] + st[1]) + (st[2] + st[3]));
        bad = bad || !(v > 0.0) || !isfinite(v);
        const double y = rsqrt_d(v);
        x[j] = l > j ? t * y : (l == j ? v * y : x[j]);
        if (l >= j && l < RT) sLs[l * RT + j] = x[j];
        if (l == j) sDinv[j] = y;
        wave_lds_sync();
        __builtin_amdgcn_sched_barrier(0);
    }
    CPG_EPI_WMARK(1);
    if (bad) return false;
    double wv[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < i; ++k) acc[k & 3] += sLs[i * RT + k] * wv[k];
        const double di = sDinv[i];
        wv[i] = l == i ? di : (l < i ? -((acc[0] + acc[1]) + (acc[2] + acc[3])) * di : 0.0);
        __builtin_amdgcn_sched_barrier(0);   // one row of L in registers at a time
    }
    CPG_EPI_WMARK(2);
    if (l < RT) {
#pragma unroll
        for (int i = 0; i < RT; ++i) sW[i * RT + l] = wv[i];
    }
    CPG_EPI_WMARK(3);
    return true;
}

// eq. 2.14 for mode n (0-based) with G^(n) in sG: A^(n) <- G Gamma^{-1}.
// Gamma by the block; W = L^{-1} by one wave (one jittered retry with
// Gamma + 1e-12 tr(Gamma)/R I); Gamma^{-1} = W^T W and A^(n) = G Gamma^{-1}
// by the block, then the Gram of the new factor: five block barriers per
// mode.  Returns false (leaving A^(n) and grams[n] untouched) if Gamma is not
// positive definite.
template <typename TC, int RT>
__device__ __forceinline__ bool block_solve(const EpiArgs<TC>& a, int n, const double* sG, double* sGam, double* sL,
                                            double* sA, double* spart, int* sOk) {
    if constexpr (RT > 16) {
        return block_solve_lds<TC, RT>(a, n, sG, sGam, sL, sA, spart, sOk);
    } else {
        static_assert(2 * RT * RT <= kEpiThreads, "two threads per Gram entry");
        static_assert(RT * RT + RT <= kEpiThreads, "Cholesky scratch fits the partial-sum buffer");
        const int tid = threadIdx.x;
        const int R = a.fs.R;
        const int64_t I = a.fs.dims[n];
        block_gamma<TC, RT>(a, n, sGam);
        __syncthreads();
        CPG_EPI_MARK(20);
        if (tid < 64) {
            bool good = wave_chol_inverse<RT>(sGam, R, 0.0, spart, sL);
            if (!good) {
                double tr = 0.0;
                for (int c = 0; c < R; ++c) tr += sGam[c * RT + c];
                good = wave_chol_inverse<RT>(sGam, R, 1e-12 * tr / R, spart, sL);
            }
            if (tid == 0) *sOk = good ? 1 : 0;
        }
        __syncthreads();
        CPG_EPI_MARK(21);
        if (!*sOk) return false;
        // Gamma^{-1} = W^T W into sGam (W: lower triangular, zero above the
        // diagonal and in the padding, so the sums run over the whole tile)
        for (int e = tid; e < R * R; e += kEpiThreads) {
            const int r = e / R, c = e - (e / R) * R;
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < RT; ++i) acc[i & 3] += sL[i * RT + r] * sL[i * RT + c];
            sGam[r * RT + c] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        }
        __syncthreads();
        // A^(n) = G Gamma^{-1}
        TC* A = (TC*)a.fs.A[n];
        for (int64_t o = tid; o < I * R; o += kEpiThreads) {
            const int64_t i = o / R;
            const int c = (int)(o - i * R);
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < RT; ++s)
                if (s < R) acc[s & 3] += sG[i * RT + s] * sGam[s * RT + c];
            const TC v = (TC)((acc[0] + acc[1]) + (acc[2] + acc[3]));
            A[o] = v;
            sA[o] = (double)v;   // the stored (rounded) factor, for its Gram
        }
        __syncthreads();
        CPG_EPI_MARK(22);
        CPG_EPI_MARK(23);
        // Gram of the new factor: entry (r, c) over two threads, rows split by parity
        {
            const int E = R * R;
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            if (tid < 2 * E) {
                const int e = tid % E, h = tid / E;
                const int r = e / R, c = e - (e / R) * R;
                int64_t i = h;
                for (; i + 6 < I; i += 8) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) acc[u] += sA[(i + 2 * u) * R + r] * sA[(i + 2 * u) * R + c];
                }
                for (; i < I; i += 2) acc[0] += sA[i * R + r] * sA[i * R + c];
            }
            spart[tid] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
            __syncthreads();
            if (tid < E) a.grams[(int64_t)n * E + tid] = spart[tid] + spart[tid + E];
            __syncthreads();
        }
        return true;
    }
}

template <typename TC, int RT>
__device__ __forceinline__ void epilogue_body(const EpiArgs<TC>& a, double* sG, double* sGam, double* sW,
                                              double* spart, double* sKR, d4* spart4, int* sOkp) {
    int& sOk = *sOkp;
    const int tid = threadIdx.x;
    CPG_EPI_MARK(0);
    const int R = a.fs.R;
    const int N = a.fs.N;

    if (a.init) {
        if (tid < 16) a.flags[tid] = 0;
        if (!a.grams_ready) block_grams_all(a.fs, a.grams, sKR, spart);
        CPG_EPI_MARK(1);
    }

    const TC* cur = a.Z;
    int buf = 0;
    for (int step = 0; step < a.n_count; ++step) {
        const int n = (a.side == 0) ? a.n_first - step : a.n_first + step;   // paper's mode
        const int64_t I = a.fs.dims[n - 1];
        if (step > 0) {
            if (a.side == 0) {
                // vec R^(r,n) = reshape(R^(r,n+1), [J_n, I_{n+1}]) a_r^(n+1)   (eq. 3.20)
                block_ttv(cur, a.buf[buf], a.fs.A[n], a.Jn[n], a.fs.dims[n], (int64_t)1, R, a.ld, sKR, spart4);
            } else {
                // vec L^(r,n) = reshape(L^(r,n-1), [I_{n-1}, K_{n-1}])^T a_r^(n-1)   (eq. 3.22)
                block_ttv(cur, a.buf[buf], a.fs.A[n - 2], (int64_t)1, a.fs.dims[n - 2], a.Kn[n - 1], R, a.ld, sKR,
                          spart4);
            }
            cur = a.buf[buf];
            buf ^= 1;
        }
        CPG_EPI_MARK(2 + 3 * step);
        if (step == 0 && a.Gpre) {
            for (int64_t o = tid; o < I * R; o += kEpiThreads) {
                const int64_t i = o / R;
                sG[i * RT + (o - i * R)] = (double)a.Gpre[o];
            }
            __syncthreads();
        } else if (a.side == 0) {
            // g_r^(n) = reshape(R^(r,n), [J_{n-1}, I_n])^T (a_r^(n-1) (x) ... (x) a_r^(1))   (eq. 3.12)
            block_grad<TC, RT>(cur, a.ld, a.fs, I, a.Jn[n - 1], a.Jn[n - 1], 1, 0, n - 1, sG, sKR, spart4);
        } else {
            // g_r^(n) = reshape(L^(r,n), [I_n, K_n]) (a_r^(N) (x) ... (x) a_r^(n+1))   (eq. 3.16)
            block_grad<TC, RT>(cur, a.ld, a.fs, I, a.Kn[n], 1, I, n, N - n, sG, sKR, spart4);
        }
        CPG_EPI_MARK(3 + 3 * step);
        if (a.update) {
            if (!block_solve<TC, RT>(a, n - 1, sG, sGam, sW, sKR, spart, &sOk)) {
                if (tid == 0) atomicOr(a.flags, 1);
            }
        } else if (!(step == 0 && a.Gpre == a.Gout[n - 1])) {
            TC* G = a.Gout[n - 1];
            for (int64_t o = tid; o < I * R; o += kEpiThreads) {
                const int64_t i = o / R;
                G[o] = (TC)sG[i * RT + (o - i * R)];
            }
        }
        __syncthreads();
        CPG_EPI_MARK(4 + 3 * step);
    }

    if (a.cost) {
        // eq. 2.12: D = ||Y||^2 - 2 <Y, Yhat> + ||Yhat||^2 with <Y,Yhat> = sum G^(N) .* A^(N)
        const int64_t I = a.fs.dims[N - 1];
        const TC* A = a.fs.A[N - 1];
        double acc = 0.0;
        for (int64_t o = tid; o < I * R; o += kEpiThreads) {
            const int64_t i = o / R;
            acc += sG[i * RT + (o - i * R)] * (double)A[o];
        }
        const double inner = block_sum(acc, spart);
        double h = 0.0;
        for (int e = tid; e < R * R; e += kEpiThreads) {
            double g[CPG_MAX_MODES];
#pragma unroll
            for (int k = 0; k < CPG_MAX_MODES; ++k) g[k] = (k < N) ? a.grams[(int64_t)k * R * R + e] : 1.0;
            double v = 1.0;
#pragma unroll
            for (int k = 0; k < CPG_MAX_MODES; ++k) v *= g[k];
            h += v;
        }
        const double nrm = block_sum(h, spart);
        if (tid == 0) {
            const double y2 = a.scal[0];
            const double D = y2 - 2.0 * inner + nrm;
            a.scal[2] = D;
            a.scal[3] = 1.0 - sqrt(D > 0.0 ? D : 0.0) / sqrt(y2);
            a.scal[4] = inner;
            a.scal[5] = nrm;
            if (!isfinite(D)) atomicOr(a.flags, 2);
        }
    }
}

template <typename TC, int RT>
__global__ __launch_bounds__(kEpiThreads) void k_epilogue(EpiArgs<TC> a0, EpiArgs<TC> a1) {
    __shared__ double sG[kEpiGCap];
    __shared__ double sGam[RT * RT];
    __shared__ double sW[RT * (RT + 1)];
    __shared__ double spart[kEpiThreads];
    __shared__ double sKR[kEpiKRCap];
    __shared__ d4 spart4[kEpiThreads];
    __shared__ int sOk;
    // two inlined copies so that each reads its own kernel argument directly
    if (blockIdx.x == 0)
        epilogue_body<TC, RT>(a0, sG, sGam, sW, spart, sKR, spart4, &sOk);
    else
        epilogue_body<TC, RT>(a1, sG, sGam, sW, spart, sKR, spart4, &sOk);
}

template <typename TC>
static hipError_t epi_dispatch(int R, const EpiArgs<TC>* args, int nsides, hipStream_t s) {
    const EpiArgs<TC>& a0 = args[0];
    const EpiArgs<TC>& a1 = args[nsides > 1 ? 1 : 0];
    if (R <= 4)
        hipLaunchKernelGGL((k_epilogue<TC, 4>), dim3(nsides), dim3(kEpiThreads), 0, s, a0, a1);
    else if (R <= 16)
        hipLaunchKernelGGL((k_epilogue<TC, 16>), dim3(nsides), dim3(kEpiThreads), 0, s, a0, a1);
    else if (R <= 32)
        hipLaunchKernelGGL((k_epilogue<TC, 32>), dim3(nsides), dim3(kEpiThreads), 0, s, a0, a1);
    else
        hipLaunchKernelGGL((k_epilogue<TC, 64>), dim3(nsides), dim3(kEpiThreads), 0, s, a0, a1);
    return hipGetLastError();
}

hipError_t launch_epilogue(int fdt, int R, const void* args, int nsides, hipStream_t stream) {
    if (fdt == CPG_F64) return epi_dispatch<double>(R, (const EpiArgs<double>*)args, nsides, stream);
    return epi_dispatch<float>(R, (const EpiArgs<float>*)args, nsides, stream);
}

}  // namespace cpg
