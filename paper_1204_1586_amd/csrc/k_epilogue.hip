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

// four consecutive entries of a chain row (16-byte aligned: rows have stride ld = 4k)
__device__ __forceinline__ d4 load4(const float* p) {
    const float4 v = *(const float4*)p;
    return d4{(double)v.x, (double)v.y, (double)v.z, (double)v.w};
}
__device__ __forceinline__ d4 load4(const double* p) {
    const double2 a = *(const double2*)p, b = *(const double2*)(p + 2);
    return d4{a.x, a.y, b.x, b.y};
}
__device__ __forceinline__ d4 mul4(d4 v, const double* w) { return d4{v.x * w[0], v.y * w[1], v.z * w[2], v.w * w[3]}; }

// For O outputs (each four consecutive ranks) sum T weighted terms, term(o, t)
// returning a d4; store(o, d4).  Few outputs: the terms of one output are split
// over several threads and the parts summed in fixed order.
template <typename Term, typename Store>
__device__ __forceinline__ void block_sum_terms(int64_t O, int64_t T, Term term, Store store, d4* spart) {
    const int tid = threadIdx.x;
    if (O >= kEpiThreads) {
        for (int64_t o = tid; o < O; o += kEpiThreads) {
            d4 a0{0, 0, 0, 0}, a1{0, 0, 0, 0};
            int64_t t = 0;
            for (; t + 8 <= T; t += 8) {
                const d4 v0 = term(o, t), v1 = term(o, t + 1), v2 = term(o, t + 2), v3 = term(o, t + 3);
                const d4 v4 = term(o, t + 4), v5 = term(o, t + 5), v6 = term(o, t + 6), v7 = term(o, t + 7);
                a0 = a0 + ((v0 + v1) + (v2 + v3));
                a1 = a1 + ((v4 + v5) + (v6 + v7));
            }
            for (; t < T; ++t) a0 = a0 + term(o, t);
            store(o, a0 + a1);
        }
        __syncthreads();
    } else {
        const int g = kEpiThreads / (int)O;
        d4 a0{0, 0, 0, 0}, a1{0, 0, 0, 0};
        if (tid < g * O) {
            const int64_t o = tid % O;
            const int part = tid / (int)O;
            int64_t t = part;
            for (; t + 7 * g < T; t += 8 * g) {
                const d4 v0 = term(o, t), v1 = term(o, t + g), v2 = term(o, t + 2 * g), v3 = term(o, t + 3 * g);
                const d4 v4 = term(o, t + 4 * g), v5 = term(o, t + 5 * g), v6 = term(o, t + 6 * g),
                         v7 = term(o, t + 7 * g);
                a0 = a0 + ((v0 + v1) + (v2 + v3));
                a1 = a1 + ((v4 + v5) + (v6 + v7));
            }
            for (; t < T; t += g) a0 = a0 + term(o, t);
        }
        spart[tid] = a0 + a1;
        __syncthreads();
        if (tid < O) {
            d4 acc{0, 0, 0, 0};
            for (int p = 0; p < g; ++p) acc = acc + spart[p * O + tid];
            store(tid, acc);
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
        for (int64_t e = threadIdx.x; e < T * ld; e += kEpiThreads) {
            const int64_t t = e / ld;
            const int r = (int)(e - t * ld);
            sKR[e] = r < R ? kr_entry_d(fs, kr_first, kr_count, t, r) : 0.0;
        }
        __syncthreads();
        block_sum_terms(
            I * nq, T,
            [&](int64_t o, int64_t t) {
                const int64_t i = o / nq;
                const int q4 = 4 * (int)(o - i * nq);
                return mul4(load4(Z + (i * si + t * st) * ld + q4), sKR + t * ld + q4);
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
    for (int64_t e = threadIdx.x; e < I * ld; e += kEpiThreads) {
        const int64_t i = e / ld;
        const int r = (int)(e - i * ld);
        sA[e] = r < R ? (double)a[i * R + r] : 0.0;
    }
    __syncthreads();
    block_sum_terms(
        lo_n * hi_n * nq, I,
        [&](int64_t o, int64_t i) {
            const int64_t row = o / nq;
            const int q4 = 4 * (int)(o - row * nq);
            const int64_t hi = row / lo_n, lo = row - (row / lo_n) * lo_n;
            return mul4(load4(in + (lo + lo_n * (i + I * hi)) * ld + q4), sA + i * ld + q4);
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
            for (int64_t e = threadIdx.x; e < I[m] * R; e += kEpiThreads) sA[off[m] + e] = (double)A[e];
        }
        __syncthreads();
        block_gram_staged(sA, off, I, m0, m1, R, grams, spart);
        m0 = m1;
    }
}

// eq. 2.14 for mode n (0-based) with G^(n) in sG: A^(n) <- G Gamma^{-1} by a
// float64 Cholesky factorisation Gamma = L L^T (right-looking, one block
// barrier per column; one retry with Gamma + 1e-12 tr(Gamma)/R I) and, for
// every row g of G, the two triangular solves L z = g^T, L^T x = z.  Returns
// false (leaving A^(n) and grams[n] untouched) if Gamma is not SPD.
template <typename TC, int RT>
__device__ __forceinline__ bool block_solve(const EpiArgs<TC>& a, int n, const double* sG, double* sGam, double* sL,
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
        block_grams_all(a.fs, a.grams, sKR, spart);
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
        } else {
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
