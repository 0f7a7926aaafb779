// The chain epilogue of Algorithm 2 in one block: after a big contraction has
// produced P_R (= R^(n*), eq. 3.10) or P_L (= L^(n*+1), eq. 3.9), one block of
// 512 threads walks that side's modes.  For each mode it
//   * forms G^(n) from the chain tensor (cp_gradient 'right', eq. 3.12, or
//     'left', eq. 3.16) in float64 in LDS,
//   * either writes it out (all-mode gradient) or applies the ALS update of
//     eq. 2.14 with the Section 4 order: Gamma = Hadamard product of the other
//     modes' float64 Grams, A^(n) = G Gamma^{-1} by Gauss-Jordan elimination
//     of [Gamma | G^T] in registers (one jittered retry), then the Gram of the
//     new factor,
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
#ifndef CPG_ROWS_MARK
#define CPG_ROWS_MARK(k)
#endif

namespace cpg {

constexpr int kEpiThreads = 512;

__device__ __forceinline__ void wave_lds_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

// A block barrier for LDS data only: this wave's LDS operations complete, then
// the barrier; its global stores stay in flight (a full __syncthreads waits
// for them too).  Used where no thread reads global data another thread of
// the block wrote since the last full barrier.
__device__ __forceinline__ void block_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

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

// q = x / d for the small non-negative values of the index arithmetic below
// (32-bit division when both fit)
__device__ __forceinline__ int64_t div_small(int64_t x, int64_t d) {
    if (((uint64_t)x | (uint64_t)d) <= 0xffffffffull) return (int64_t)((uint32_t)x / (uint32_t)d);
    return x / d;
}

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
            idx[u] = div_small(e, ld);
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
                const int64_t q = div_small(idx[u], d);
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
constexpr int kEpiTail = 4;     // ... in a batch's tail

// The terms of one output: term t is the four entries at z + t zs times the
// four float64 weights at w + t ws.
template <typename TC>
struct TermRun {
    const TC* z;
    int64_t zs;
    const double* w;
    int64_t ws;
};

// For O outputs (each four consecutive ranks) sum T weighted terms; prep(o)
// gives output o's TermRun and store(o, d4) receives the sum (into LDS when
// LDS_OUT: the closing barrier then leaves global stores in flight).  Loads go out
// kEpiBatch at a time before any is used (the chain tensors are streamed by
// this one block, so the loads in flight set its speed).  Few outputs: the
// terms of one output are split over several threads and the parts summed
// in fixed order.
template <typename TC, bool LDS_OUT, typename Prep, typename Store>
__device__ __forceinline__ void block_sum_terms(int64_t O, int64_t T, Prep prep, Store store, d4* spart) {
    auto close = [] {
        if constexpr (LDS_OUT)
            block_lds_sync();
        else
            __syncthreads();
    };
    const int tid = threadIdx.x;
    auto run = [&](int64_t o, int64_t t0, int64_t tstep) {
        const TermRun<TC> tr = prep(o);
        const TC* z = tr.z + t0 * tr.zs;
        const double* w = tr.w + t0 * tr.ws;
        const int64_t zs = tstep * tr.zs, ws = tstep * tr.ws;
        d4 a0{0, 0, 0, 0}, a1{0, 0, 0, 0};
        int64_t t = t0;
        // full batches without branches (so the loads stay in flight together), then the tail
        constexpr int kB = sizeof(TC) == 8 ? kEpiBatch / 2 : kEpiBatch;   // float64: half, within registers
        for (; t + (kB - 1) * tstep < T; t += kB * tstep) {
            Raw4<TC> v[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) v[u] = Raw4<TC>::load(z + u * zs);
#pragma unroll
            for (int u = 0; u < kB; u += 2) {
                a0 = a0 + v[u].mul(w + u * ws);
                a1 = a1 + v[u + 1].mul(w + (u + 1) * ws);
            }
            z += kB * zs;
            w += kB * ws;
        }
        // the tail (under kEpiBatch terms) four terms per round trip: their
        // loads, clamped to the last term, go out before any is used; the
        // terms past T are not added
        for (; t < T; t += kEpiTail * tstep) {
            const int left = (int)div_small(T - 1 - t, tstep);   // the last term: t + left * tstep
            Raw4<TC> v[kEpiTail];
            double wv[kEpiTail][4];
#pragma unroll
            for (int u = 0; u < kEpiTail; ++u) {
                v[u] = Raw4<TC>::load(z + min(u, left) * zs);
                const double* wu = w + min(u, left) * ws;
#pragma unroll
                for (int c = 0; c < 4; ++c) wv[u][c] = wu[c];
            }
#pragma unroll
            for (int u = 0; u < kEpiTail; ++u)
                if (u <= left) a0 = a0 + v[u].mul(wv[u]);
            z += kEpiTail * zs;
            w += kEpiTail * ws;
        }
        return a0 + a1;
    };
    if (O >= kEpiThreads) {
        for (int64_t o = tid; o < O; o += kEpiThreads) store(o, run(o, 0, 1));
        close();
    } else {
        const int g = kEpiThreads / (int)O;
        d4 acc{0, 0, 0, 0};
        if (tid < g * O) acc = run(tid % O, tid / (int)O, g);
        spart[tid] = acc;
        block_lds_sync();
        if (tid < O) {
            // the parts in order, eight LDS reads in flight
            d4 tot{0, 0, 0, 0};
            int p = 0;
            for (; p + 8 <= g; p += 8) {
                d4 u[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) u[k] = spart[(p + k) * O + tid];
#pragma unroll
                for (int k = 0; k < 8; ++k) tot = tot + u[k];
            }
            for (; p < g; ++p) tot = tot + spart[p * O + tid];
            store(tid, tot);
        }
        close();
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
        CPG_EPI_WMARK(53);
        stage_kr(fs, kr_first, kr_count, T, ld, sKR);
        block_lds_sync();
        CPG_EPI_WMARK(54);
        block_sum_terms<TC, true>(
            I * nq, T,
            [&](int64_t o) {
                const int64_t i = div_small(o, nq);
                const int q4 = 4 * (int)(o - i * nq);
                return TermRun<TC>{Z + i * si * ld + q4, st * ld, (const double*)(sKR + q4), (int64_t)ld};
            },
            [&](int64_t o, d4 v) {
                const int64_t i = div_small(o, nq);
                const int q4 = 4 * (int)(o - i * nq);
                double* g = sG + i * RT + q4;
                g[0] = v.x;
                if (q4 + 1 < RT) g[1] = v.y;
                if (q4 + 2 < RT) g[2] = v.z;
                if (q4 + 3 < RT) g[3] = v.w;
            },
            spart);
        CPG_EPI_WMARK(55);
    }
}

// out[(lo + lo_n*hi)*ld + r] = sum_i in[(lo + lo_n*(i + I*hi))*ld + r] * a[i*R + r]
template <typename TC>
__device__ __forceinline__ void block_ttv(const TC* __restrict__ in, TC* __restrict__ out, const TC* __restrict__ a,
                                          int64_t lo_n, int64_t I, int64_t hi_n, int R, int ld, double* sA,
                                          d4* spart) {
    const int nq = ld >> 2;
    CPG_EPI_WMARK(50);
    stage_batched(
        I * ld,
        [&](int64_t e) {
            const int64_t i = div_small(e, ld);
            const int r = (int)(e - i * ld);
            const double x = (double)a[i * R + (r < R ? r : R - 1)];
            return r < R ? x : 0.0;
        },
        [&](int64_t e, double v) { sA[e] = v; });
    block_lds_sync();
    CPG_EPI_WMARK(51);
    block_sum_terms<TC, false>(
        lo_n * hi_n * nq, I,
        [&](int64_t o) {
            const int64_t row = div_small(o, nq);
            const int q4 = 4 * (int)(o - row * nq);
            const int64_t hi = div_small(row, lo_n), lo = row - hi * lo_n;
            return TermRun<TC>{in + (lo + lo_n * I * hi) * ld + q4, lo_n * ld, (const double*)(sA + q4),
                               (int64_t)ld};
        },
        [&](int64_t o, d4 v) {
            const int64_t row = div_small(o, nq);
            const int q4 = 4 * (int)(o - row * nq);
            TC* d = out + row * ld + q4;
            d[0] = (TC)v.x;
            d[1] = (TC)v.y;
            d[2] = (TC)v.z;
            d[3] = (TC)v.w;
        },
        spart);
    CPG_EPI_WMARK(52);
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

// Gamma (R x R, stride RT) = Hadamard product of the float64 Grams of every
// mode but n (eq. 2.14); mode `ovr_mode`'s Gram, if any, is read from `ovr`
// (R x R) instead of `grams`.
template <int RT>
__device__ __forceinline__ void gamma_into(const double* grams, int N, int R, int n, double* sGam, int ovr_mode = -1,
                                           const double* ovr = nullptr) {
    for (int e = threadIdx.x; e < R * R; e += kEpiThreads) {
        double g[CPG_MAX_MODES];
#pragma unroll
        for (int k = 0; k < CPG_MAX_MODES; ++k)
            g[k] = (k < N && k != n) ? (k == ovr_mode ? ovr[e] : grams[(int64_t)k * R * R + e]) : 1.0;
        double v = 1.0;
#pragma unroll
        for (int k = 0; k < CPG_MAX_MODES; ++k) v *= g[k];
        const int i = e / R;
        sGam[i * RT + (e - i * R)] = v;
    }
}
template <typename TC, int RT>
__device__ __forceinline__ void block_gamma(const EpiArgs<TC>& a, int n, double* sGam) {
    gamma_into<RT>(a.grams, a.fs.N, a.fs.R, n, sGam);
}

// Gram of a solved factor held as rows of stride RT (float64): entry (r, c)
// summed over rows i = h, h + g, ... by g threads, the g partial sums then
// added in order h = 0, 1, ...
template <int RT>
__device__ __forceinline__ void block_gram_rows(const double* X, int64_t I, int R, double* gout, double* spart) {
    const int tid = threadIdx.x;
    const int E = R * R;
    if (E > kEpiThreads) {
        for (int e = tid; e < E; e += kEpiThreads) {
            const int r = e / R, c = e - (e / R) * R;
            double s[4] = {0.0, 0.0, 0.0, 0.0};
            int64_t i = 0;
            for (; i + 3 < I; i += 4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) s[u] += X[(i + u) * RT + r] * X[(i + u) * RT + c];
            }
            for (; i < I; ++i) s[0] += X[i * RT + r] * X[i * RT + c];
            gout[e] = (s[0] + s[1]) + (s[2] + s[3]);
        }
        __syncthreads();
        return;
    }
    int g = 1;
    while (g < 8 && 2 * g * E <= kEpiThreads) g *= 2;
    double acc = 0.0;
    if (tid < g * E) {
        const int e = tid % E, h = tid / E;
        const int r = e / R, c = e - (e / R) * R;
        double s[4] = {0.0, 0.0, 0.0, 0.0};
        int64_t i = h;
        for (; i + 3 * g < I; i += 4 * g) {
#pragma unroll
            for (int u = 0; u < 4; ++u) s[u] += X[(i + u * g) * RT + r] * X[(i + u * g) * RT + c];
        }
        for (; i < I; i += g) s[0] += X[i * RT + r] * X[i * RT + c];
        acc = (s[0] + s[1]) + (s[2] + s[3]);
    }
    spart[tid] = acc;
    __syncthreads();
    if (tid < E) {
        double v = spart[tid];
        for (int h = 1; h < g; ++h) v += spart[h * E + tid];
        gout[tid] = v;
    }
    __syncthreads();
}

// 1/d in float64: hardware estimate refined by two Newton steps
__device__ __forceinline__ double rcp_d(double d) {
    double y = __builtin_amdgcn_rcp(d);
    y = __builtin_fma(y, __builtin_fma(-d, y, 1.0), y);
    y = __builtin_fma(y, __builtin_fma(-d, y, 1.0), y);
    return y;
}

typedef double v4d __attribute__((ext_vector_type(4)));

// Rank tiles up to 32: the elimination below in the registers of single
// waves.  Lane l of a wave holds column l of Gamma' (lanes < R) and columns
// i = 64 (8 q + w) + l of G^T; at step k the multipliers Gamma'_sk and the pivot
// come from lane k by readlane, so a step needs no LDS and no barrier.  Every
// wave with columns of G^T repeats the (small) elimination of Gamma', with
// identical results.  *sFlag carries the outcome to the other waves.
// I rows of G (stride RT) in sG; the solved rows are stored to A (I x R, when
// not null) and, rounded to TC, to sF (stride RT).  The registers hold the
// first RE <= RT columns (R <= RE): the entries past R are zero and stay zero,
// so a smaller RE only drops work on them.
template <typename TC, int RT, int RE = RT>
__device__ __forceinline__ bool wave_eliminate(int R, int64_t I, const double* sG, const double* sGam, TC* A,
                                               double* sF, int* sFlag) {
    static_assert(RE <= RT, "register columns within the stride");
    constexpr int kSets = (kEpiGCap / RT + kEpiThreads - 1) / kEpiThreads;   // columns of G^T per lane
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    if ((int64_t)w * 64 < I) {
        double gc[RE], xc[kSets][RE];
#pragma unroll
        for (int s = 0; s < RE; ++s) gc[s] = (l < R && s < R) ? sGam[s * RT + l] : 0.0;
#pragma unroll
        for (int q = 0; q < kSets; ++q) {
            const int64_t i = (int64_t)(q * (kEpiThreads / 64) + w) * 64 + l;
#pragma unroll
            for (int s = 0; s < RE; ++s) xc[q][s] = (i < I && s < R) ? sG[i * RT + s] : 0.0;
        }
        bool ok = true;
#pragma unroll
        for (int k = 0; k < RE; ++k) {
            if (k < R) {
                // the pivot and its reciprocal estimate first, then all the
                // step's multipliers Gamma'_sk (uniform, in scalar registers),
                // so their latencies overlap instead of stalling each update.
                // No branch on the pivot: after a bad one the remaining steps
                // run on values that are discarded (ok false)
                const double piv = readlane_d(gc[k], k);
                ok = ok && piv > 0.0 && isfinite(piv);
                double rp = __builtin_amdgcn_rcp(piv);
                // pinned here for 17-20 register columns: the compiler otherwise
                // emits the estimate after the multipliers, on the step's critical
                // path (measured faster there; no gain with fewer columns, and
                // spills with 32)
                if constexpr (RE > 16 && RE <= 20) asm volatile("" : "+v"(rp));
                __builtin_amdgcn_sched_barrier(0);
                double mk[RE];
#pragma unroll
                for (int s = 0; s < RE; ++s) mk[s] = s == k ? 0.0 : readlane_d(gc[s], k);
                __builtin_amdgcn_sched_barrier(0);
                rp = __builtin_fma(rp, __builtin_fma(-piv, rp, 1.0), rp);   // two Newton steps
                rp = __builtin_fma(rp, __builtin_fma(-piv, rp, 1.0), rp);
                const double tg = gc[k] * rp;
                double tx[kSets];
#pragma unroll
                for (int q = 0; q < kSets; ++q) tx[q] = xc[q][k] * rp;
                // row k + 1 first: the next step's pivot is ready early
#pragma unroll
                for (int d = 1; d < RE; ++d) {
                    const int s = (k + d) % RE;
                    gc[s] -= mk[s] * tg;
#pragma unroll
                    for (int q = 0; q < kSets; ++q) xc[q][s] -= mk[s] * tx[q];
                }
                gc[k] = tg;
#pragma unroll
                for (int q = 0; q < kSets; ++q) xc[q][k] = tx[q];
            }
        }
        if (ok) {
#pragma unroll
            for (int q = 0; q < kSets; ++q) {
                const int64_t i = (int64_t)(q * (kEpiThreads / 64) + w) * 64 + l;
                if (i < I) {
#pragma unroll
                    for (int s = 0; s < RE; ++s) {
                        if (s < R) {
                            const TC v = (TC)xc[q][s];
                            if (A) A[i * R + s] = v;
                            sF[i * RT + s] = (double)v;   // the stored (rounded) factor, for its Gram
                        }
                    }
                }
            }
        }
        if (tid == 0) *sFlag = ok ? 1 : 0;
    }
    __syncthreads();
    return *sFlag != 0;
}

// Block (ca, cb) of the Gram of the stored factor (rows of stride RT in sF) on
// the float64 matrix core, one wave: D += F_a^T F_b over blocks of four rows
// (rows past I read as zero), F_a = columns ca..ca+15; lane l supplies
// F(i0 + l / 16, ca + l mod 16) as the first operand and F(i0 + l / 16,
// cb + l mod 16) as the second.  With `mirror` the transposed block is
// written too (the Gram is then exactly symmetric).
template <int RT>
__device__ __forceinline__ void wave_gram_block(const double* sF, int64_t I, int R, int ca, int cb, bool mirror,
                                                double* gout) {
    const int l = threadIdx.x & 63;
    v4d acc = {0.0, 0.0, 0.0, 0.0};
    // four blocks per round: their LDS reads go out together, then the
    // products run in row order
    for (int64_t i0 = 0; i0 < I; i0 += 16) {
        double va[4], vb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t i = i0 + 4 * u + (l >> 4);
            const double* row = sF + min(i, I - 1) * RT + (l & 15);
            const double xa = row[ca], xb = row[cb];
            va[u] = i < I ? xa : 0.0;
            vb[u] = i < I ? xb : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[u], vb[u], acc, 0, 0, 0);
    }
    // output of the float64 16x16x4 product: lane l, item j holds D[(l >> 4) + 4 j][l & 15]
    const int c = cb + (l & 15);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int r = ca + (l >> 4) + 4 * j;
        if (r < R && c < R) {
            gout[r * R + c] = acc[j];
            if (mirror) gout[c * R + r] = acc[j];
        }
    }
}

// Gram of a factor with at most 16 ranks (rows of stride 16), wave 0.
__device__ __forceinline__ void wave_gram16(const double* sF, int64_t I, int R, double* gout) {
    wave_gram_block<16>(sF, I, R, 0, 0, false, gout);
}

// Gram of a factor with 17..32 ranks (rows of stride 32): waves 0, 1, 2 take
// the blocks (0, 0), (0, 1) (also written transposed) and (1, 1).
__device__ __forceinline__ void waves_gram32(const double* sF, int64_t I, int R, double* gout) {
    const int w = threadIdx.x >> 6;
    if (w < 3) wave_gram_block<32>(sF, I, R, w == 2 ? 16 : 0, w == 0 ? 0 : 16, w == 1, gout);
}

// eq. 2.14 for mode n (0-based): A^(n) <- G Gamma^{-1}, Gamma symmetric positive
// definite.  Gauss-Jordan elimination without pivoting on the augmented
// system [Gamma | G^T] (float64): step k scales row k by 1/Gamma'_kk and
// removes column k from every other row, so after R steps the right part is
// Gamma^{-1} G^T = (A^(n))^T.  The pivots are those of Gamma = L D L^T, all
// positive for an SPD matrix; a pivot that is not positive and finite ends
// the attempt (the caller retries once with `jitter`: Gamma formed again and
// shifted by 1e-12 tr(Gamma)/R I).  Without `jitter`, sGam already holds Gamma
// (the caller forms it while the chain step's loads are in flight).  Rank tiles up to 32
// use the register elimination of single waves above; for a tile of 64 every thread keeps its entries of the
// system in registers (G^T entries (s, i) with s = tid mod RT, so one
// multiplier per step); a step needs only the pivot row and column, which
// their owners publish to LDS (two alternating copies, one barrier per step).
// Then the factor is stored (rounded to TC) and the Gram of the stored values
// formed.  G in sG is only read, so a retry and the cost can use it again.
// Returns false, leaving A^(n) and grams[n] untouched, if Gamma is not
// positive definite.
template <typename TC, int RT, int RE = RT>
__device__ __forceinline__ bool block_solve(const EpiArgs<TC>& a, int n, double* sG, double* sGam, double* sPub,
                                            double* spart, int* sFlag, bool jitter) {
    static_assert(kEpiThreads % RT == 0, "a thread's entries of G^T share one row of the system");
    constexpr int kPerX = kEpiGCap / kEpiThreads;                      // G^T entries per thread
    constexpr int kPerG = (RT * RT + kEpiThreads - 1) / kEpiThreads;   // Gamma entries per thread
    const int tid = threadIdx.x;
    const int R = a.fs.R;
    const int64_t I = a.fs.dims[n];
    const int nx = (int)(I * RT);          // <= kEpiGCap
    const int srow = tid & (RT - 1);
    // publication copies c = 0, 1: pivot row of Gamma' (RT), its pivot column (RT), pivot row of G^T (I)
    const int pub = 2 * RT + (int)I;
    auto prow = [&](int c) { return sPub + c * pub; };
    auto pcol = [&](int c) { return sPub + c * pub + RT; };
    auto px = [&](int c) { return sPub + c * pub + 2 * RT; };

    if (jitter) {
        // the retry: Gamma formed again, then the diagonal shifted
        __syncthreads();
        block_gamma<TC, RT>(a, n, sGam);
        __syncthreads();
        double tr = 0.0;
        for (int c = 0; c < R; ++c) tr += sGam[c * RT + c];
        __syncthreads();
        if (tid < R) sGam[tid * RT + tid] += 1e-12 * tr / R;
        __syncthreads();
    }
    if constexpr (RT <= 32) {
        // register columns: within a tile of 16 the rank rounded up to 8, 12 or 16;
        // within the tile of 32 a kernel instance of its own per choice (RE: 20 or
        // 32), since a run-time choice there costs the kernel register spills
        TC* An = (TC*)a.fs.A[n];
        bool ok;
        if constexpr (RT == 16) {
            ok = R <= 8    ? wave_eliminate<TC, RT, 8>(R, I, sG, sGam, An, sPub, sFlag)
                 : R <= 12 ? wave_eliminate<TC, RT, 12>(R, I, sG, sGam, An, sPub, sFlag)
                           : wave_eliminate<TC, RT, 16>(R, I, sG, sGam, An, sPub, sFlag);
        } else {
            ok = wave_eliminate<TC, RT, RE>(R, I, sG, sGam, An, sPub, sFlag);
        }
        if (!ok) return false;
        CPG_EPI_MARK(22);
        if constexpr (RT == 16) {
            if (tid < 64) wave_gram16(sPub, I, R, a.grams + (int64_t)n * R * R);
            __syncthreads();
        } else if constexpr (RT == 32) {
            waves_gram32(sPub, I, R, a.grams + (int64_t)n * R * R);
            __syncthreads();
        } else {
            block_gram_rows<RT>(sPub, I, R, a.grams + (int64_t)n * R * R, spart);
        }
        CPG_EPI_MARK(23);
        return true;
    }
    double g[kPerG], x[kPerX];
#pragma unroll
    for (int v = 0; v < kPerG; ++v) {
        const int e = tid + v * kEpiThreads;
        const int r = e / RT, j = e & (RT - 1);
        g[v] = (e < RT * RT && r < R && j < R) ? sGam[r * RT + j] : 0.0;
        if (e < RT * RT && r == 0) prow(0)[j] = g[v];
        if (e < RT * RT && j == 0) pcol(0)[r] = g[v];
    }
#pragma unroll
    for (int u = 0; u < kPerX; ++u) {
        const int e = tid + u * kEpiThreads;
        x[u] = (e < nx && srow < R) ? sG[e] : 0.0;
        if (e < nx && srow == 0) px(0)[e / RT] = x[u];
    }
    __syncthreads();
    for (int k = 0; k < R; ++k) {
        const int c = k & 1;
        // every read of the step first (entries past the system read nothing), then the pivot test
        const double piv = prow(c)[k];   // the same value in every thread
        const double m = pcol(c)[srow];
        double rk[kPerG], cr[kPerG], xk[kPerX];
#pragma unroll
        for (int v = 0; v < kPerG; ++v) {
            rk[v] = cr[v] = 0.0;
            if (v * kEpiThreads < RT * RT) {   // uniform over the block
                const int e = min(tid + v * kEpiThreads, RT * RT - 1);
                rk[v] = prow(c)[e & (RT - 1)];
                cr[v] = pcol(c)[e / RT];
            }
        }
#pragma unroll
        for (int u = 0; u < kPerX; ++u) {
            xk[u] = 0.0;
            if (u * kEpiThreads < nx) xk[u] = px(c)[min(tid + u * kEpiThreads, nx - 1) / RT];
        }
        if (!(piv > 0.0) || !isfinite(piv)) return false;
        const double rp = rcp_d(piv);
        const int cn = c ^ 1;
#pragma unroll
        for (int v = 0; v < kPerG; ++v) {
            if (v * kEpiThreads >= RT * RT) break;
            const int e = tid + v * kEpiThreads;
            const int r = e / RT, j = e & (RT - 1);
            const double t = rk[v] * rp;
            if (j > k) g[v] = r == k ? t : g[v] - cr[v] * t;   // columns <= k are not read again
            if (e < RT * RT && r == k + 1) prow(cn)[j] = g[v];
            if (e < RT * RT && j == k + 1) pcol(cn)[r] = g[v];
        }
#pragma unroll
        for (int u = 0; u < kPerX; ++u) {
            if (u * kEpiThreads >= nx) break;
            const int e = tid + u * kEpiThreads;
            const double t = xk[u] * rp;
            x[u] = srow == k ? t : x[u] - m * t;
            if (e < nx && srow == k + 1) px(cn)[e / RT] = x[u];
        }
        __syncthreads();
    }
    CPG_EPI_MARK(21);
    // the publication copies are no longer read (barrier above): the stored
    // (rounded) factor goes there, rows i of stride RT, for its Gram
    TC* A = (TC*)a.fs.A[n];
#pragma unroll
    for (int u = 0; u < kPerX; ++u) {
        const int e = tid + u * kEpiThreads;
        if (e < nx && srow < R) {
            const TC v = (TC)x[u];
            A[(int64_t)(e / RT) * R + srow] = v;
            sPub[e] = (double)v;
        }
    }
    __syncthreads();
    CPG_EPI_MARK(22);
    block_gram_rows<RT>(sPub, I, R, a.grams + (int64_t)n * R * R, spart);
    CPG_EPI_MARK(23);
    return true;
}

template <typename TC, int RT, int RE>
__device__ __forceinline__ void epilogue_body(const EpiArgs<TC>& a, double* sG, double* sGam,
                                              double* spart, double* sKR, d4* spart4, int* sFlag) {
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
        // Gamma of this mode's update (the Grams it reads are final by now); its
        // loads go out together with the chain step's
        if (a.update) block_gamma<TC, RT>(a, n - 1, sGam);
        if (step > 0) {
            // next right chain tensor: the previous one contracted over its last mode
            // with that mode's (updated) rank columns (eq. 3.20); next left chain
            // tensor: contracted over its first mode (eq. 3.22)
            const TC* fa = a.side == 0 ? a.fs.A[n] : a.fs.A[n - 2];
            const int64_t lo_n = a.side == 0 ? a.Jn[n] : 1;
            const int64_t tI = a.side == 0 ? a.fs.dims[n] : a.fs.dims[n - 2];
            const int64_t hi_n = a.side == 0 ? 1 : a.Kn[n - 1];
            block_ttv<TC>(cur, a.buf[buf], fa, lo_n, tI, hi_n, R, a.ld, sKR, spart4);
            cur = a.buf[buf];
            buf ^= 1;
        }
        CPG_EPI_MARK(2 + 3 * step);
        if (step == 0 && a.Gpre) {
            for (int64_t o = tid; o < I * R; o += kEpiThreads) {
                const int64_t i = o / R;
                sG[i * RT + (o - i * R)] = (double)a.Gpre[o];
            }
            block_lds_sync();
        } else if (a.side == 0) {
            // gradient of mode n: the chain tensor's leading modes contracted with their
            // Khatri-Rao rows   (eq. 3.12)
            block_grad<TC, RT>(cur, a.ld, a.fs, I, a.Jn[n - 1], a.Jn[n - 1], 1, 0, n - 1, sG, sKR, spart4);
        } else {
            // gradient of mode n: the chain tensor's trailing modes contracted with their
            // Khatri-Rao rows   (eq. 3.16)
            block_grad<TC, RT>(cur, a.ld, a.fs, I, a.Kn[n], 1, I, n, N - n, sG, sKR, spart4);
        }
        CPG_EPI_MARK(3 + 3 * step);
        if (a.update) {
            // one jittered retry if Gamma is not positive definite
            bool solved = false;
            for (int attempt = 0; attempt < 2 && !solved; ++attempt) {
                if (attempt > 0) __syncthreads();
                solved = block_solve<TC, RT, RE>(a, n - 1, sG, sGam, sKR, spart, sFlag, attempt == 1);
            }
            if (!solved && tid == 0) atomicOr(a.flags, 1);
        } else if (!(step == 0 && a.Gpre == a.Gout[n - 1])) {
            TC* G = a.Gout[n - 1];
            for (int64_t o = tid; o < I * R; o += kEpiThreads) {
                const int64_t i = o / R;
                G[o] = (TC)sG[i * RT + (o - i * R)];
            }
        }
        // an update wrote the factor and its Gram to global memory, which the
        // next step reads; a stored gradient is not read again
        if (a.update)
            __syncthreads();
        else
            block_lds_sync();
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

template <typename TC, int RT, int RE = RT>
__global__ __launch_bounds__(kEpiThreads) void k_epilogue(EpiArgs<TC> a0, EpiArgs<TC> a1) {
    __shared__ double sG[kEpiGCap];
    __shared__ double sGam[RT * RT];
    __shared__ double spart[kEpiThreads];
    __shared__ double sKR[kEpiKRCap];
    __shared__ d4 spart4[kEpiThreads];
    __shared__ int sFlag;
    // two inlined copies so that each reads its own kernel argument directly
    if (blockIdx.x == 0)
        epilogue_body<TC, RT, RE>(a0, sG, sGam, spart, sKR, spart4, &sFlag);
    else
        epilogue_body<TC, RT, RE>(a1, sG, sGam, spart, sKR, spart4, &sFlag);
}

// ---------------------------------------------------------------------------
// ALS update of a two-mode side on many blocks (eq. 2.14, Section 4 order).
// Every block solves the side's first mode n1 from its precomputed gradient
// (a small R x R system; all blocks reach identical results, block 0 stores
// the factor and its Gram).  With the new A^(n1) the chain step of eq. 3.20 /
// 3.22 is already the gradient of the last mode n2 (no Khatri-Rao block is
// left), one row per output row, and the rows of A^(n2) = G^(n2) Gamma^{-1} are
// independent: each block forms its slice of G^(n2) from the chain tensor,
// solves it and stores it, with its partials of the cost when the pass ends
// the sweep (k_epi_rows_cost then adds them up).  The Gram of A^(n2) is left
// to the next pass's reduction, which recomputes every Gram.
// ---------------------------------------------------------------------------
constexpr int kRowsTerms = 8;   // chain-tensor loads in flight per thread

template <int RT>
__global__ __launch_bounds__(kEpiThreads) void k_epi_rows(EpiRows a) {
    __shared__ double sG[kEpiGCap];        // G^(n1), rows of stride RT
    __shared__ double sF[kEpiGCap];        // new A^(n1) (rounded), later the new A^(n2)
    __shared__ double sGam[RT * RT];
    __shared__ double sGram1[RT * RT];     // Gram of the new A^(n1) (R x R)
    __shared__ double sGram2[RT * RT];     // Gram of the new A^(n2) (last block)
    __shared__ double sP[RT * RT];         // Hadamard product of the Grams of the other modes (R x R)
    static_assert(kEpiRowsCells <= kEpiThreads, "a slice's reduction fits the block");
    __shared__ double sX[kEpiRowsCells];   // this block's rows of G^(n2), stride RT
    __shared__ double sA2[kEpiRowsCells];  // ... and of the new A^(n2)
    __shared__ d4 spart4[kEpiThreads];
    __shared__ double spart[kEpiThreads];
    __shared__ int sFlag;
    const int tid = threadIdx.x;
    const int R = a.fs.R, N = a.fs.N, ld = a.ld, nq = ld >> 2;
    const int m1 = a.n1 - 1, m2 = a.n2 - 1;   // 0-based
    const int64_t I1 = a.fs.dims[m1], I2 = a.fs.dims[m2];
    float* A1 = (float*)a.fs.A[m1];
    float* A2 = (float*)a.fs.A[m2];
    CPG_ROWS_MARK(0);
    // the first batch of this block's chain-tensor loads (below) goes out now:
    // the addresses do not depend on the solve of the first mode
    const int64_t r0 = (int64_t)blockIdx.x * a.rows;
    const int nrows = (int)min((int64_t)a.rows, I2 - r0);
    const int nout = nrows * nq;
    const int parts = kEpiThreads / nout;
    const int o_t = tid % nout, part_t = tid / nout;
    const int64_t i_t = r0 + o_t / nq;
    const int q_t = o_t - (o_t / nq) * nq;
    const int64_t rs = a.side == 0 ? I2 : 1;              // row stride of term j
    const float* zsrc = a.Z + (a.side == 0 ? i_t : I1 * i_t) * ld + 4 * q_t;
    float4 zv[kRowsTerms];
    if (tid < parts * nout) {
#pragma unroll
        for (int u = 0; u < kRowsTerms; ++u) {
            const int64_t j = min((int64_t)part_t + (int64_t)u * parts, I1 - 1);
            zv[u] = *(const float4*)(zsrc + j * rs * ld);
        }
    }
    // Gamma of a mode of this side = sP .* (the other mode's Gram), eq. 2.14;
    // `jitter` adds 1e-12 tr(Gamma)/R to the diagonal (the retry)
    auto form_gamma = [&](const double* g, bool jitter) {
        __syncthreads();
        for (int e = tid; e < R * R; e += kEpiThreads) {
            const int i = e / R;
            sGam[i * RT + (e - i * R)] = sP[e] * g[e];
        }
        __syncthreads();
        if (jitter) {
            double tr = 0.0;
            for (int c = 0; c < R; ++c) tr += sGam[c * RT + c];
            __syncthreads();
            if (tid < R) sGam[tid * RT + tid] += 1e-12 * tr / R;
            __syncthreads();
        }
    };

    // first mode: G^(n1) and the Grams in one round of loads, then the solve
    // (one jittered retry)
    {
        constexpr int kGPer = kEpiGCap / kEpiThreads;   // I1 * R <= kEpiGCap
        static_assert(RT * RT <= kEpiThreads, "one Gram entry per thread");
        const int64_t nG = I1 * R;
        // loads without branches (clamped indices, values selected after),
        // so they all go out before the first wait
        float gp[kGPer];
#pragma unroll
        for (int u = 0; u < kGPer; ++u) {
            const int64_t o = tid + (int64_t)u * kEpiThreads;
            gp[u] = a.Gpre[min(o, nG - 1)];
        }
        const bool has_e = tid < R * R;
        const int e_c = min(tid, R * R - 1);
        double gv[CPG_MAX_MODES];
#pragma unroll
        for (int k = 0; k < CPG_MAX_MODES; ++k) gv[k] = a.grams[(int64_t)min(k, N - 1) * R * R + e_c];
#pragma unroll
        for (int u = 0; u < kGPer; ++u) {
            const int64_t o = tid + (int64_t)u * kEpiThreads;
            if (o < nG) {
                const int64_t i = o / R;
                sG[i * RT + (o - i * R)] = (double)gp[u];
            }
        }
        if (has_e) {
            double v = 1.0, g2 = 0.0;
#pragma unroll
            for (int k = 0; k < CPG_MAX_MODES; ++k) {
                if (k < N && k != m1 && k != m2) v *= gv[k];
                if (k == m2) g2 = gv[k];
            }
            sP[tid] = v;
            sGram2[tid] = g2;   // Gram of A^(n2) before its update
        }
    }
    form_gamma(sGram2, false);
    bool ok1 = wave_eliminate<float, RT>(R, I1, sG, sGam, blockIdx.x == 0 ? A1 : nullptr, sF, &sFlag);
    CPG_ROWS_MARK(1);
    if (!ok1) {
        form_gamma(sGram2, true);
        ok1 = wave_eliminate<float, RT>(R, I1, sG, sGam, blockIdx.x == 0 ? A1 : nullptr, sF, &sFlag);
    }
    if (!ok1) {
        // A^(n1) is kept: the chain step below uses it as it is
        if (blockIdx.x == 0 && tid == 0) atomicOr(a.flags, 1);
        for (int64_t o = tid; o < I1 * R; o += kEpiThreads) {
            const int64_t i = o / R;
            sF[i * RT + (o - i * R)] = (double)A1[o];
        }
        __syncthreads();
    }
    // Gram of A^(n1) as stored; block 0 publishes it
    if constexpr (RT == 16) {
        if (tid < 64) wave_gram16(sF, I1, R, sGram1);
        __syncthreads();
    } else {
        block_gram_rows<RT>(sF, I1, R, sGram1, spart);
    }
    if (blockIdx.x == 0 && ok1)
        for (int e = tid; e < R * R; e += kEpiThreads) a.grams[(int64_t)m1 * R * R + e] = sGram1[e];
    form_gamma(sGram1, false);
    CPG_ROWS_MARK(2);

    // this block's rows of G^(n2): G(i, r) = sum_j Z(row(i, j), r) A^(n1)(j, r),
    // right: row = i + I2 j, left: row = j + I1 i; float64 sums rounded to float
    // (as a stored chain tensor), terms j in order per thread, thread parts in order
    {
        d4 acc{0.0, 0.0, 0.0, 0.0};
        if (tid < parts * nout) {
            for (int64_t j0 = part_t; j0 < I1; j0 += (int64_t)kRowsTerms * parts) {
                if (j0 != part_t) {   // batches after the preloaded one
#pragma unroll
                    for (int u = 0; u < kRowsTerms; ++u) {
                        const int64_t j = min(j0 + (int64_t)u * parts, I1 - 1);
                        zv[u] = *(const float4*)(zsrc + j * rs * ld);
                    }
                }
#pragma unroll
                for (int u = 0; u < kRowsTerms; ++u) {
                    const int64_t j = j0 + (int64_t)u * parts;
                    if (j < I1) {
                        const double* w = sF + j * RT + 4 * q_t;
                        acc = acc + d4{(double)zv[u].x * w[0], (double)zv[u].y * w[1], (double)zv[u].z * w[2],
                                       (double)zv[u].w * w[3]};
                    }
                }
            }
        }
        spart4[tid] = acc;
        __syncthreads();
        if (tid < nout) {
            // the parts in order, eight LDS reads in flight
            d4 t{0.0, 0.0, 0.0, 0.0};
            int pp = 0;
            for (; pp + 8 <= parts; pp += 8) {
                d4 u[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) u[k] = spart4[(pp + k) * nout + tid];
#pragma unroll
                for (int k = 0; k < 8; ++k) t = t + u[k];
            }
            for (; pp < parts; ++pp) t = t + spart4[pp * nout + tid];
            const int il = tid / nq, q = tid - (tid / nq) * nq;
            const double tv[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) sX[il * RT + 4 * q + u] = (double)(float)tv[u];
        }
        __syncthreads();
    }
    CPG_ROWS_MARK(3);

    // solve the slice: A^(n2) rows = G^(n2) rows Gamma^{-1} (the same pivots in every block)
    bool ok2 = wave_eliminate<float, RT>(R, nrows, sX, sGam, A2 + r0 * R, sA2, &sFlag);
    if (!ok2) {
        form_gamma(sGram1, true);
        ok2 = wave_eliminate<float, RT>(R, nrows, sX, sGam, A2 + r0 * R, sA2, &sFlag);
    }
    if (!ok2 && tid == 0) atomicOr(a.flags, 1);
    CPG_ROWS_MARK(4);
    // cost partials of this slice (eq. 2.12), with A^(n2) as stored (the factor
    // kept on a failed solve): <Y, Yhat> part = sum G^(n2) .* A^(n2), and the
    // ||Yhat||^2 part = sum over its rows a of a^T S a, S = Hadamard product of
    // the other modes' Grams (that of A^(n1) new), since Gram(A^(n2)) is the sum
    // of a a^T over the rows
    if (a.cost) {
        if (!ok2) {
            for (int e = tid; e < nrows * R; e += kEpiThreads) {
                const int il = e / R, c = e - (e / R) * R;
                sA2[il * RT + c] = (double)A2[(r0 + il) * R + c];
            }
            __syncthreads();
        }
        // one (row, rank) entry per thread (nrows * RT <= kEpiRowsCells <= kEpiThreads)
        double acc = 0.0, quad = 0.0;
        if (tid < nrows * R) {
            const int il = tid / R, r = tid - (tid / R) * R;
            const double ar = sA2[il * RT + r];
            acc = sX[il * RT + r] * ar;
            double t = 0.0;
#pragma unroll
            for (int c = 0; c < RT; ++c)
                if (c < R) t += sP[r * R + c] * sGram1[r * R + c] * sA2[il * RT + c];
            quad = ar * t;
        }
        // fixed-order sums: a butterfly in each wave (every lane ends with the
        // same value), then the waves in order
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            acc += __shfl_xor(acc, o);
            quad += __shfl_xor(quad, o);
        }
        if ((tid & 63) == 0) {
            spart[2 * (tid >> 6)] = acc;
            spart[2 * (tid >> 6) + 1] = quad;
        }
        __syncthreads();
        if (tid == 0) {
            double inner = 0.0, h = 0.0;
            for (int w = 0; w < kEpiThreads / 64; ++w) {
                inner += spart[2 * w];
                h += spart[2 * w + 1];
            }
            a.part[2 * blockIdx.x] = inner;
            a.part[2 * blockIdx.x + 1] = h;
        }
    }
    CPG_ROWS_MARK(5);
}

// The end of the pass that closes a sweep, one small kernel after k_epi_rows:
// the cost of eq. 2.12 and the fit from the per-block partials (block order).
// The Gram of the new A^(n2) is left to the next pass's reduction.
__global__ void k_epi_rows_cost(EpiRows a, int nblocks) {
    // lane b loads block b's pair (all loads in flight at once); lane 0 adds
    // them in block order
    const int l = threadIdx.x;
    const int b = min(l, nblocks - 1);
    const double pi = a.part[2 * b], pn = a.part[2 * b + 1];
    const double y2 = a.scal[0];
    double inner = 0.0, nrm = 0.0;
    for (int k = 0; k < nblocks; ++k) {
        inner += readlane_d(pi, k);
        nrm += readlane_d(pn, k);
    }
    if (l != 0) return;
    // D = ||Y||^2 - 2 <Y, Yhat> + ||Yhat||^2
    const double D = y2 - 2.0 * inner + nrm;
    a.scal[2] = D;
    a.scal[3] = 1.0 - sqrt(D > 0.0 ? D : 0.0) / sqrt(y2);
    a.scal[4] = inner;
    a.scal[5] = nrm;
    if (!isfinite(D)) atomicOr(a.flags, 2);
}

hipError_t launch_epi_rows(const EpiRows& a, hipStream_t s) {
    const int64_t I2 = a.fs.dims[a.n2 - 1];
    const int64_t nb = (I2 + a.rows - 1) / a.rows;
    const int rt = a.fs.R <= 4 ? 4 : 16;
    if (a.fs.R > 16 || nb < 1 || nb > kEpiRowsMaxBlocks || (int64_t)a.rows * rt > kEpiRowsCells ||
        a.fs.dims[a.n1 - 1] * rt > kEpiGCap || I2 * rt > kEpiGCap || (a.ld & 3) != 0)
        return hipErrorInvalidValue;
    if (rt == 4) {
        hipLaunchKernelGGL(k_epi_rows<4>, dim3((unsigned)nb), dim3(kEpiThreads), 0, s, a);
        if (a.cost) hipLaunchKernelGGL(k_epi_rows_cost, dim3(1), dim3(64), 0, s, a, (int)nb);
    } else {
        hipLaunchKernelGGL(k_epi_rows<16>, dim3((unsigned)nb), dim3(kEpiThreads), 0, s, a);
        if (a.cost) hipLaunchKernelGGL(k_epi_rows_cost, dim3(1), dim3(64), 0, s, a, (int)nb);
    }
    return hipGetLastError();
}

template <typename TC>
static hipError_t epi_dispatch(int R, const EpiArgs<TC>* args, int nsides, hipStream_t s) {
    const EpiArgs<TC>& a0 = args[0];
    const EpiArgs<TC>& a1 = args[nsides > 1 ? 1 : 0];
    if (R <= 4)
        hipLaunchKernelGGL((k_epilogue<TC, 4>), dim3(nsides), dim3(kEpiThreads), 0, s, a0, a1);
    else if (R <= 16)
        hipLaunchKernelGGL((k_epilogue<TC, 16>), dim3(nsides), dim3(kEpiThreads), 0, s, a0, a1);
    else if (R <= 20)
        hipLaunchKernelGGL((k_epilogue<TC, 32, 20>), dim3(nsides), dim3(kEpiThreads), 0, s, a0, a1);
    else if (R <= 32)
        hipLaunchKernelGGL((k_epilogue<TC, 32, 32>), dim3(nsides), dim3(kEpiThreads), 0, s, a0, a1);
    else
        hipLaunchKernelGGL((k_epilogue<TC, 64>), dim3(nsides), dim3(kEpiThreads), 0, s, a0, a1);
    return hipGetLastError();
}

hipError_t launch_epilogue(int fdt, int R, const void* args, int nsides, hipStream_t stream) {
    if (fdt == CPG_F64) return epi_dispatch<double>(R, (const EpiArgs<double>*)args, nsides, stream);
    return epi_dispatch<float>(R, (const EpiArgs<float>*)args, nsides, stream);
}

}  // namespace cpg
