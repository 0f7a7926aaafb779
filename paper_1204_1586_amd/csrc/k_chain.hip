// Small kernels of Algorithm 2 and of the ALS sweep (Section 4):
//  * fixed-order float64 reduction of the split partial contractions;
//  * the peel-off chain steps of eqs. 3.20 / 3.22 (one mode product);
//  * the per-mode gradient of cp_gradient 'right' / 'left' (eqs. 3.12, 3.16);
//  * float64 Gram matrices, the Cholesky solve of eq. 2.14 (generic path), ||Y||^2, and the
//    cost of eq. 2.12 with fit = 1 - ||Y - Yhat|| / ||Y||.
// All reductions run in a fixed order, so results are bitwise reproducible.
#include "cpg_device.h"

#include <algorithm>

namespace cpg {

struct d4s {
    double x, y, z, w;
};

__device__ __forceinline__ double block_sum_256(double v, double* sbuf) {
    // sbuf: >= 256 doubles; returns the total in every thread
    const int tid = threadIdx.x;
    sbuf[tid] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) sbuf[tid] += sbuf[tid + s];
        __syncthreads();
    }
    const double t = sbuf[0];
    __syncthreads();
    return t;
}

// ---------------------------------------------------------------------------
// partial reduction
// ---------------------------------------------------------------------------
template <typename TC>
__global__ __launch_bounds__(256) void k_reduce_parts(const TC* __restrict__ parts, int64_t nparts, int64_t n,
                                                      TC* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    double acc = 0.0;
    int64_t p = 0;
    for (; p + 8 <= nparts; p += 8) {
        TC v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = parts[(p + u) * n + e];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += (double)v[u];
    }
    for (; p < nparts; ++p) acc += (double)parts[p * n + e];
    out[e] = (TC)acc;
}

hipError_t launch_reduce_parts(int fdt, const void* parts, int64_t nparts, int64_t rows, int ld, void* out,
                               hipStream_t s) {
    const int64_t n = rows * ld;
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (fdt == CPG_F64)
        hipLaunchKernelGGL(k_reduce_parts<double>, dim3(nb), dim3(256), 0, s, (const double*)parts, nparts, n,
                           (double*)out);
    else
        hipLaunchKernelGGL(k_reduce_parts<float>, dim3(nb), dim3(256), 0, s, (const float*)parts, nparts, n,
                           (float*)out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused partial reduction.  Block i of a side reduces the chain-tensor rows of
// its output row i over the split partials (float64, fixed order p = 0, 1, ...),
// rounds them to float32 (stored as P_R / P_L when Z is set) and forms from
// the rounded values
//   G(i, r) = sum_t Z(row(i, t), r) KR(t, r)
// with KR the float64 Khatri-Rao rows of the side's weighting modes, formed
// from the factors in place.  Weighted by the side's remaining modes this is
// its first gradient (right: eq. 3.12, rows t + T i; left: eq. 3.16, rows
// i + I t); weighted by one mode it is the side's first chain step (eqs. 3.20 /
// 3.22), read straight from the partials so that it needs no launch of its
// own after the reduction.  Extra blocks (one per mode) compute the float64
// Grams when `grams` is set.
// ---------------------------------------------------------------------------
constexpr int kRfBatch = 16;   // partial loads in flight per thread
constexpr int kRfThreads = 512;  // one term per thread at 64 terms x 4 float4 x 2 rows

// Khatri-Rao weights of term t for ranks 4q..4q+3 (zero past R): the product of
// the factor entries of modes first, first + 1, ... (Notation 2.1 order).
// Without sFac the factors are read from memory, one mode at a time.  With
// sFac they come from LDS (rows of stride ld, mode after mode, zero past R),
// one 16-byte read per mode; NM >= 0 (= count) unrolls the modes so that all
// the reads are issued before the first product.
template <int NM>
__device__ __forceinline__ void kr_weights_rf(const KrGen& kg, int first, int count, uint32_t t, int q, int R,
                                              int ld, const float* sFac, double (&w)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = 4 * q + u < R ? 1.0 : 0.0;
    uint32_t idx = t;
    if (sFac) {
        int64_t off = 4 * q;
        if constexpr (NM >= 0) {
            float4 x[NM > 0 ? NM : 1];
#pragma unroll
            for (int mm = 0; mm < NM; ++mm) {
                const FastDiv f = kg.fd[first + mm];
                const uint32_t qd = fast_div(idx, f);
                x[mm] = *(const float4*)(sFac + off + (int64_t)(idx - qd * f.d) * ld);
                off += (int64_t)f.d * ld;
                idx = qd;
            }
#pragma unroll
            for (int mm = 0; mm < NM; ++mm) {
                w[0] *= (double)x[mm].x;
                w[1] *= (double)x[mm].y;
                w[2] *= (double)x[mm].z;
                w[3] *= (double)x[mm].w;
            }
        } else {
            for (int m = first; m < first + count; ++m) {
                const FastDiv f = kg.fd[m];
                const uint32_t qd = fast_div(idx, f);
                const float4 y = *(const float4*)(sFac + off + (int64_t)(idx - qd * f.d) * ld);
                off += (int64_t)f.d * ld;
                idx = qd;
                w[0] *= (double)y.x;
                w[1] *= (double)y.y;
                w[2] *= (double)y.z;
                w[3] *= (double)y.w;
            }
        }
        return;
    }
    for (int m = first; m < first + count; ++m) {
        const FastDiv f = kg.fd[m];
        const uint32_t qd = fast_div(idx, f);
        const float* Am = kg.A[m] + (int64_t)(idx - qd * f.d) * R;
        idx = qd;
        float x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = Am[min(4 * q + u, R - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u) w[u] *= (double)x[u];
    }
}

constexpr int kRfFacCap = 4096;   // floats of LDS-staged weighting factors

template <int NM, bool STAGE>
__device__ __forceinline__ void reduce_first_rows(const ReduceFirst& a, int64_t blk, const KrGen& kg, d4s* spart,
                                                  float* sFac, bool stage_fac) {
    const int R = kg.R;
    const int tid = threadIdx.x;
    const int ld = a.ld;
    const int nq = ld >> 2;                 // float4 columns of a row
    int nqp = 1;
    while (nqp < nq) nqp <<= 1;             // threads per term (a power of two <= 16)
    const int rpb = rf_rows_per_block(a.side, ld);
    const int q = tid & (nqp - 1);
    const int sub = (tid / nqp) & (rpb - 1);  // output row of the block this thread serves
    const int tslot = tid / (nqp * rpb);
    const int tstep = kRfThreads / (nqp * rpb);
    const int64_t i = blk * rpb + sub;
    const int64_t rstride = a.side == 0 ? 1 : a.I;            // row of term t: rbase + t * rstride
    const int64_t rbase = a.side == 0 ? a.T * i : i;
    const int64_t pstride = a.rows * ld;                      // floats per partial
    const int np = (int)a.nparts;
    d4s g{0.0, 0.0, 0.0, 0.0};
    // With several terms per thread, the weighting modes' factors are first
    // staged in LDS (when they fit; the launch decides, see rf_stage_fac), so
    // that a term's weights cost LDS reads instead of scattered 4-byte loads;
    // with fewer, that round trip would not pay for itself.
    const float* fac = nullptr;
    if (STAGE && stage_fac) {
        int64_t tot = 0;
        for (int m = a.kr_first; m < a.kr_first + a.kr_count; ++m) tot += (int64_t)kg.fd[m].d * ld;
        {
            for (int64_t e = tid; e < tot; e += kRfThreads) {
                int m = a.kr_first;
                int64_t o = e;
                while (o >= (int64_t)kg.fd[m].d * ld) {
                    o -= (int64_t)kg.fd[m].d * ld;
                    ++m;
                }
                const int64_t ii = o / ld;
                const int r = (int)(o - ii * ld);
                sFac[e] = r < R ? kg.A[m][ii * R + r] : 0.f;
            }
            __syncthreads();
            fac = sFac;
        }
    }
    // float64 Khatri-Rao row t of modes kr_first.. (Notation 2.1 order), zero past R
    auto weights = [&](int64_t t, double (&w)[4]) {
        kr_weights_rf<NM>(kg, a.kr_first, a.kr_count, (uint32_t)t, q, R, ld, fac, w);
    };
    // the reduced row (partials summed in order p = 0, 1, ...), rounded to
    // float32, stored when Z is kept, and its weighted contribution
    auto finish = [&](int64_t row, const d4s& acc, const double (&w)[4]) {
        const float4 z{(float)acc.x, (float)acc.y, (float)acc.z, (float)acc.w};
        if (a.Z) *(float4*)(a.Z + row * ld + 4 * q) = z;
        g.x += (double)z.x * w[0];
        g.y += (double)z.y * w[1];
        g.z += (double)z.z * w[2];
        g.w += (double)z.w * w[3];
    };
    auto add = [](d4s& acc, const float4& v) {
        acc.x += (double)v.x;
        acc.y += (double)v.y;
        acc.z += (double)v.z;
        acc.w += (double)v.w;
    };
    if (q < nq && i < a.I) {
        if (np <= kRfBatch / 4) {
            // few partials: four terms per round trip (their partial loads and
            // weight loads all issued before any is used)
            int64_t t = tslot;
            for (; t + 3 * tstep < a.T; t += 4 * tstep) {
                float4 v[kRfBatch];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float* src = a.parts + (rbase + (t + k * tstep) * rstride) * ld + 4 * q;
#pragma unroll
                    for (int u = 0; u < kRfBatch / 4; ++u)
                        v[4 * k + u] = *(const float4*)(src + (int64_t)min(u, np - 1) * pstride);
                }
                double w[4][4];
#pragma unroll
                for (int k = 0; k < 4; ++k) weights(t + k * tstep, w[k]);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    d4s acc{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int u = 0; u < kRfBatch / 4; ++u)
                        if (u < np) add(acc, v[4 * k + u]);
                    finish(rbase + (t + k * tstep) * rstride, acc, w[k]);
                }
            }
            for (; t < a.T; t += tstep) {
                const int64_t row = rbase + t * rstride;
                const float* src = a.parts + row * ld + 4 * q;
                float4 v[kRfBatch / 4];
#pragma unroll
                for (int u = 0; u < kRfBatch / 4; ++u) v[u] = *(const float4*)(src + (int64_t)min(u, np - 1) * pstride);
                double w[4];
                weights(t, w);
                d4s acc{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int u = 0; u < kRfBatch / 4; ++u)
                    if (u < np) add(acc, v[u]);
                finish(row, acc, w);
            }
        } else {
            for (int64_t t = tslot; t < a.T; t += tstep) {
                const int64_t row = rbase + t * rstride;
                const float* src = a.parts + row * ld + 4 * q;
                // The first batch of partials goes out before the factor loads of the
                // weights (it does not depend on them), so both arrive in one round
                // trip; slots past nparts re-read the last partial and are not added.
                float4 v[kRfBatch];
#pragma unroll
                for (int u = 0; u < kRfBatch; ++u) v[u] = *(const float4*)(src + (int64_t)min(u, np - 1) * pstride);
                double w[4];
                weights(t, w);
                d4s acc{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int u = 0; u < kRfBatch; ++u)
                    if (u < np) add(acc, v[u]);
                // further full batches without branches, then the tail
                int p = kRfBatch;
                for (; p + kRfBatch <= np; p += kRfBatch) {
#pragma unroll
                    for (int u = 0; u < kRfBatch; ++u) v[u] = *(const float4*)(src + (p + u) * pstride);
#pragma unroll
                    for (int u = 0; u < kRfBatch; ++u) add(acc, v[u]);
                }
                for (; p < np; ++p) add(acc, *(const float4*)(src + p * pstride));
                finish(row, acc, w);
            }
        }
    }
    // sum over the term slots in a fixed order: a butterfly over the slots of
    // each wave, then the waves' sums in wave order
    const int grp = nqp * rpb;   // threads of one term slot (a power of two <= 64)
    for (int off = grp; off < 64; off <<= 1) {
        g.x += __shfl_xor(g.x, off);
        g.y += __shfl_xor(g.y, off);
        g.z += __shfl_xor(g.z, off);
        g.w += __shfl_xor(g.w, off);
    }
    if ((tid & 63) < grp) spart[(tid >> 6) * grp + (tid & 63)] = g;
    __syncthreads();
    if (tid < grp && q < nq && i < a.I) {
        d4s v = spart[tid];
        for (int wv = 1; wv < kRfThreads / 64; ++wv) {
            const d4s u = spart[wv * grp + tid];
            v.x += u.x;
            v.y += u.y;
            v.z += u.z;
            v.w += u.w;
        }
        const double vv[4] = {v.x, v.y, v.z, v.w};
        float* out = a.G + i * a.out_ld + 4 * q;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int r = 4 * q + u;
            if (r < R)
                out[u] = (float)vv[u];
            else if (r < a.out_ld)
                out[u] = 0.f;   // padding columns of a chain buffer
        }
    }
}

struct RfSides {
    ReduceFirst s[kMaxReduceSides];
    int stage[kMaxReduceSides];           // side k stages its weighting factors in LDS (rf_stage_fac)
    int64_t first[kMaxReduceSides + 1];   // first block of each side; first[n]: blocks of all sides
    int n;
    int* clear_flags;                     // zeroed by block 0 when set
};

template <bool STAGE>
__global__ __launch_bounds__(kRfThreads) void k_reduce_first(RfSides sd, KrGen kg, double* __restrict__ grams) {
    __shared__ d4s spart[kRfThreads];
    // kRfFacCap floats when a side stages its factors (STAGE), else none: the
    // LDS a block holds decides whether it can start beside the blocks of the
    // contraction still running before it
    extern __shared__ __align__(16) float sFac[];
    const int64_t b = blockIdx.x;
    if (b == 0 && sd.clear_flags && threadIdx.x < 8) sd.clear_flags[threadIdx.x] = 0;
    if (b < sd.first[sd.n]) {
        int k = 0;
        while (k + 1 < sd.n && b >= sd.first[k + 1]) ++k;
        const ReduceFirst& a = sd.s[k];
        const bool st = sd.stage[k] != 0;
        if constexpr (STAGE) {
            // the weights' mode count as a constant where it is small (uniform per side)
            switch (a.kr_count) {
                case 1: reduce_first_rows<1, true>(a, b - sd.first[k], kg, spart, sFac, st); break;
                case 2: reduce_first_rows<2, true>(a, b - sd.first[k], kg, spart, sFac, st); break;
                case 3: reduce_first_rows<3, true>(a, b - sd.first[k], kg, spart, sFac, st); break;
                default: reduce_first_rows<-1, true>(a, b - sd.first[k], kg, spart, sFac, st); break;
            }
        } else {
            reduce_first_rows<-1, false>(a, b - sd.first[k], kg, spart, nullptr, false);
        }
    } else {
        // float64 Gram of mode m, terms in index order; the factor is staged
        // through LDS in chunks of whole rows (one round trip per chunk)
        const int m = (int)(b - sd.first[sd.n]);
        if (grams == nullptr || m >= kg.N) return;
        const int R = kg.R;
        const int tid = threadIdx.x;
        const float* A = kg.A[m];
        const int64_t I = kg.fd[m].d;
        constexpr int kChunk = 4 * kRfThreads;       // floats: the float4 of spart
        constexpr int kPer = kChunk / kRfThreads;
        constexpr int kGrp = 4;                      // Gram entries per thread and pass
        float* sA = reinterpret_cast<float*>(spart);
        const int64_t rows_per = kChunk / R;
        for (int e0 = 0; e0 < R * R; e0 += kRfThreads * kGrp) {
            double acc[kGrp];
#pragma unroll
            for (int k = 0; k < kGrp; ++k) acc[k] = 0.0;
            for (int64_t i0 = 0; i0 < I; i0 += rows_per) {
                const int nf = (int)(min(rows_per, I - i0) * R);
                float v[kPer];
#pragma unroll
                for (int u = 0; u < kPer; ++u) v[u] = A[i0 * R + min(tid + kRfThreads * u, nf - 1)];
                __syncthreads();   // the previous chunk is consumed
#pragma unroll
                for (int u = 0; u < kPer; ++u)
                    if (tid + kRfThreads * u < nf) sA[tid + kRfThreads * u] = v[u];
                __syncthreads();
                const int nr = nf / R;
#pragma unroll
                for (int k = 0; k < kGrp; ++k) {
                    const int e = e0 + tid + kRfThreads * k;
                    if (e < R * R) {
                        const int r = e / R, c = e - (e / R) * R;
                        int ii = 0;
                        for (; ii + 8 <= nr; ii += 8) {   // eight rows of LDS reads in flight
                            float xr[8], xc[8];
#pragma unroll
                            for (int u = 0; u < 8; ++u) {
                                xr[u] = sA[(ii + u) * R + r];
                                xc[u] = sA[(ii + u) * R + c];
                            }
#pragma unroll
                            for (int u = 0; u < 8; ++u) acc[k] += (double)xr[u] * (double)xc[u];
                        }
                        for (; ii < nr; ++ii) acc[k] += (double)sA[ii * R + r] * (double)sA[ii * R + c];
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < kGrp; ++k) {
                const int e = e0 + tid + kRfThreads * k;
                if (e < R * R) grams[(int64_t)m * R * R + e] = acc[k];
            }
        }
    }
}

// Does a side stage its weighting factors in LDS?  Only with several terms
// per thread (T at least four times the term slots of a block) and factors
// that fit kRfFacCap.
static bool rf_stage_fac(const ReduceFirst& a, const KrGen& kg) {
    if (a.kr_count <= 0) return false;
    const int nq = a.ld >> 2;
    int nqp = 1;
    while (nqp < nq) nqp <<= 1;
    const int tstep = kRfThreads / (nqp * rf_rows_per_block(a.side, a.ld));
    if (a.T < 4 * (int64_t)tstep) return false;
    int64_t tot = 0;
    for (int m = a.kr_first; m < a.kr_first + a.kr_count; ++m) tot += (int64_t)kg.fd[m].d * a.ld;
    return tot <= kRfFacCap;
}

hipError_t launch_reduce_first(const ReduceFirst* sides, int nsides, const KrGen& kg, double* grams,
                               hipStream_t s, int* clear_flags) {
    if (nsides < 1 || nsides > kMaxReduceSides) return hipErrorInvalidValue;
    RfSides sd{};
    sd.n = nsides;
    sd.clear_flags = clear_flags;
    int64_t nb = 0;
    bool any_stage = false;
    for (int k = 0; k < nsides; ++k) {
        const ReduceFirst& a = sides[k];
        if ((a.ld & 3) != 0 || a.ld > 64 || a.nparts < 1 || (a.out_ld != kg.R && a.out_ld != a.ld))
            return hipErrorInvalidValue;
        sd.s[k] = a;
        sd.stage[k] = rf_stage_fac(a, kg) ? 1 : 0;
        any_stage = any_stage || sd.stage[k];
        sd.first[k] = nb;
        const int rpb = rf_rows_per_block(a.side, a.ld);
        nb += (a.I + rpb - 1) / rpb;
    }
    sd.first[nsides] = nb;
    const int64_t total = nb + (grams ? kg.N : 0);
    if (total == 0) return hipSuccess;
    if (any_stage)
        hipLaunchKernelGGL(k_reduce_first<true>, dim3((unsigned)total), dim3(kRfThreads), kRfFacCap * sizeof(float),
                           s, sd, kg, grams);
    else
        hipLaunchKernelGGL(k_reduce_first<false>, dim3((unsigned)total), dim3(kRfThreads), 0, s, sd, kg, grams);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// one chain step: out[lo + lo_n*hi][r] = sum_i in[lo + lo_n*(i + I*hi)][r] a[i][r]
//   right chain (eq. 3.20): lo_n = J_n, I = I_{n+1}, hi_n = 1
//   left chain  (eq. 3.22): lo_n = 1,   I = I_{n-1}, hi_n = K_{n-1}
// ---------------------------------------------------------------------------
template <typename TC>
__global__ __launch_bounds__(256) void k_ttv(const TC* __restrict__ in, TC* __restrict__ out,
                                             const TC* __restrict__ a, int64_t lo_n, int64_t I, int64_t hi_n,
                                             int R, int ld) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= lo_n * hi_n * R) return;
    const int64_t row = e / R;
    const int r = (int)(e - row * R);
    const int64_t hi = row / lo_n;
    const int64_t lo = row - hi * lo_n;
    const TC* src = in + (lo + lo_n * I * hi) * ld + r;
    const int64_t step = lo_n * ld;
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    int64_t i = 0;
    for (; i + 4 <= I; i += 4) {
        acc0 += (double)src[(i + 0) * step] * (double)a[(i + 0) * R + r];
        acc1 += (double)src[(i + 1) * step] * (double)a[(i + 1) * R + r];
        acc2 += (double)src[(i + 2) * step] * (double)a[(i + 2) * R + r];
        acc3 += (double)src[(i + 3) * step] * (double)a[(i + 3) * R + r];
    }
    for (; i < I; ++i) acc0 += (double)src[i * step] * (double)a[i * R + r];
    out[row * ld + r] = (TC)((acc0 + acc1) + (acc2 + acc3));
}

hipError_t launch_ttv(int fdt, const void* in, void* out, const void* a, int64_t lo_n, int64_t I, int64_t hi_n,
                      int R, int ld, hipStream_t s) {
    const int64_t n = lo_n * hi_n * R;
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (fdt == CPG_F64)
        hipLaunchKernelGGL(k_ttv<double>, dim3(nb), dim3(256), 0, s, (const double*)in, (double*)out,
                           (const double*)a, lo_n, I, hi_n, R, ld);
    else
        hipLaunchKernelGGL(k_ttv<float>, dim3(nb), dim3(256), 0, s, (const float*)in, (float*)out,
                           (const float*)a, lo_n, I, hi_n, R, ld);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// gradient of one mode from a chain tensor (cp_gradient 'right' / 'left'):
// G(i, r) = sum_{lo, hi} Z[lo + lo_n*(i + I*hi)][r] * KR_lo(lo, r) * KR_hi(hi, r)
// One block per output row i.  A thread takes one four-rank column of the
// row and every nslots-th term, with a batch of chain-tensor loads in flight
// (the Khatri-Rao weights are formed from the factors meanwhile); its terms
// are summed in order, then the threads of a column in a fixed order (a
// butterfly in each wave, then the waves in order).
// ---------------------------------------------------------------------------
constexpr int kGradMaxThreads = 1024;
template <typename TC>
constexpr int grad_batch() { return sizeof(TC) == 8 ? 4 : 8; }   // within 128 registers at 1024 threads

template <typename TC>
__device__ __forceinline__ void load4_d(const TC* p, double (&x)[4]);
template <>
__device__ __forceinline__ void load4_d<float>(const float* p, double (&x)[4]) {
    const float4 v = *(const float4*)p;
    x[0] = v.x;
    x[1] = v.y;
    x[2] = v.z;
    x[3] = v.w;
}
template <>
__device__ __forceinline__ void load4_d<double>(const double* p, double (&x)[4]) {
    const double2 a = *(const double2*)p, b = *(const double2*)(p + 2);
    x[0] = a.x;
    x[1] = a.y;
    x[2] = b.x;
    x[3] = b.y;
}

// q = x / d, m = x - q d (32-bit division when both fit)
__device__ __forceinline__ void divmod64(int64_t x, int64_t d, int64_t& q, int64_t& m) {
    if (((uint64_t)x | (uint64_t)d) <= 0xffffffffull) {
        const uint32_t q32 = (uint32_t)x / (uint32_t)d;
        q = q32;
    } else {
        q = x / d;
    }
    m = x - q * d;
}

// w[u] *= KR(idx, r0 + u) over modes first..first+count-1 (Notation 2.1 order);
// ranks past R read the last rank (the caller drops them)
template <typename TC>
__device__ __forceinline__ void kr_weights4(const FacSet<TC>& fs, int first, int count, int64_t idx, int r0,
                                            double (&w)[4]) {
    const int R = fs.R;
    for (int m = 0; m < count; ++m) {
        int64_t qd, i;
        divmod64(idx, fs.dims[first + m], qd, i);
        const TC* a = fs.A[first + m] + i * R;
#pragma unroll
        for (int u = 0; u < 4; ++u) w[u] *= (double)a[min(r0 + u, R - 1)];
        idx = qd;
    }
}

// SPLIT: block (i, s) of a (I, S) grid takes terms [s chunk, (s + 1) chunk) and
// writes its float64 sums to part[(i S + s) R + r]; k_grad_sum adds the S
// parts of each entry in order.  (Used when a row has many terms and there
// are few rows: the split fills the chip.)
template <typename TC, bool SPLIT>
__global__ __launch_bounds__(kGradMaxThreads) void k_grad(const TC* __restrict__ Z, int ld, TC* __restrict__ G,
                                                          FacSet<TC> fs, int64_t lo_n, int64_t I, int64_t hi_n,
                                                          int lo_first, int lo_count, int hi_first, int hi_count,
                                                          double* __restrict__ part, int64_t chunk) {
    __shared__ double spart[(kGradMaxThreads / 64) * 16 * 4];
    const int R = fs.R;
    const int tid = threadIdx.x;
    const int nq = ld >> 2;                 // four-rank columns of a row (ld <= 64)
    int nqp = 1;
    while (nqp < nq) nqp <<= 1;
    const int q = tid & (nqp - 1);
    const int nslots = (int)blockDim.x / nqp;
    const int slot = tid / nqp;
    const int64_t i = blockIdx.x;
    const int64_t Tall = lo_n * hi_n;
    const int64_t tb = SPLIT ? (int64_t)blockIdx.y * chunk : 0;
    const int64_t T = SPLIT ? min(Tall, tb + chunk) : Tall;
    constexpr int kGradBatch = grad_batch<TC>();
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (q < nq && tb < T) {
        for (int64_t t0 = tb + slot; t0 < T; t0 += (int64_t)kGradBatch * nslots) {
            double z[kGradBatch][4];
            int64_t lo[kGradBatch], hi[kGradBatch];
#pragma unroll
            for (int u = 0; u < kGradBatch; ++u) {
                const int64_t t = min(t0 + (int64_t)u * nslots, T - 1);   // the tail re-reads the last term
                divmod64(t, lo_n, hi[u], lo[u]);
                load4_d(Z + (lo[u] + lo_n * (i + I * hi[u])) * ld + 4 * q, z[u]);
            }
#pragma unroll
            for (int u = 0; u < kGradBatch; ++u) {
                if (t0 + (int64_t)u * nslots < T) {
                    double w[4] = {1.0, 1.0, 1.0, 1.0};
                    kr_weights4(fs, lo_first, lo_count, lo[u], 4 * q, w);
                    kr_weights4(fs, hi_first, hi_count, hi[u], 4 * q, w);
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[c] += z[u][c] * w[c];
                }
            }
        }
    }
    for (int off = nqp; off < 64; off <<= 1)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += __shfl_xor(acc[c], off);
    const int w = tid >> 6, l = tid & 63;
    if (l < nqp)
#pragma unroll
        for (int c = 0; c < 4; ++c) spart[(w * 16 + l) * 4 + c] = acc[c];
    __syncthreads();
    if (tid < nq) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int ww = 0; ww < (int)blockDim.x / 64; ++ww)
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] += spart[(ww * 16 + tid) * 4 + c];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            if (4 * tid + c >= R) continue;
            if constexpr (SPLIT)
                part[(i * gridDim.y + blockIdx.y) * R + 4 * tid + c] = v[c];
            else
                G[i * R + 4 * tid + c] = (TC)v[c];
        }
    }
}

template <typename TC>
__global__ __launch_bounds__(256) void k_grad_sum(const double* __restrict__ part, int64_t I, int R, int S,
                                                  TC* __restrict__ G) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= I * R) return;
    const int64_t i = e / R;
    const int r = (int)(e - i * R);
    double v = 0.0;
    for (int s = 0; s < S; ++s) v += part[(i * S + s) * R + r];
    G[e] = (TC)v;
}

template <typename TC>
static hipError_t grad_dispatch(const void* Z, int ld, void* G, const void* facset, int64_t lo_n, int64_t I,
                                int64_t hi_n, int lo_first, int lo_count, int hi_first, int hi_count, int S,
                                double* part, hipStream_t s) {
    const FacSet<TC>& fs = *(const FacSet<TC>*)facset;
    const int64_t T = lo_n * hi_n;
    const int64_t loads = T * (ld >> 2) / S;
    // a wide block when a block's rows have many terms
    const dim3 block(loads >= 16 * kGradMaxThreads ? kGradMaxThreads : 256);
    if (S <= 1) {
        hipLaunchKernelGGL((k_grad<TC, false>), dim3((unsigned)I), block, 0, s, (const TC*)Z, ld, (TC*)G, fs, lo_n, I,
                           hi_n, lo_first, lo_count, hi_first, hi_count, nullptr, (int64_t)0);
    } else {
        const int64_t chunk = (T + S - 1) / S;
        hipLaunchKernelGGL((k_grad<TC, true>), dim3((unsigned)I, (unsigned)S), block, 0, s, (const TC*)Z, ld, (TC*)G,
                           fs, lo_n, I, hi_n, lo_first, lo_count, hi_first, hi_count, part, chunk);
        hipLaunchKernelGGL(k_grad_sum<TC>, dim3((unsigned)((I * fs.R + 255) / 256)), dim3(256), 0, s, part, I,
                           fs.R, S, (TC*)G);
    }
    return hipGetLastError();
}

hipError_t launch_grad(int fdt, const void* Z, int ld, void* G, const void* facset, int64_t lo_n, int64_t I,
                       int64_t hi_n, int lo_first, int lo_count, int hi_first, int hi_count, hipStream_t s) {
    if ((ld & 3) != 0 || ld > 64 || I < 1) return hipErrorInvalidValue;
    if (fdt == CPG_F64)
        return grad_dispatch<double>(Z, ld, G, facset, lo_n, I, hi_n, lo_first, lo_count, hi_first, hi_count, 1,
                                     nullptr, s);
    return grad_dispatch<float>(Z, ld, G, facset, lo_n, I, hi_n, lo_first, lo_count, hi_first, hi_count, 1, nullptr,
                                s);
}

// launch_grad with the terms of each row split over up to 16 blocks when the
// rows are few and long (I S >= 512 blocks, at least 64 terms a block), the
// float64 parts in `scratch` (bytes given; fewer splits when it is short).
hipError_t launch_grad_split(int fdt, const void* Z, int ld, void* G, const void* facset, int64_t lo_n, int64_t I,
                             int64_t hi_n, int lo_first, int lo_count, int hi_first, int hi_count, void* scratch,
                             size_t scratch_bytes, hipStream_t s) {
    if ((ld & 3) != 0 || ld > 64 || I < 1) return hipErrorInvalidValue;
    const int R = ((const FacSet<float>*)facset)->R;   // N, R lead both factor-set layouts
    const int64_t T = lo_n * hi_n;
    int S = (int)std::min<int64_t>(16, (512 + I - 1) / I);
    while (S > 1 && (T / S < 64 || (size_t)(I * S * R) * sizeof(double) > scratch_bytes)) --S;
    if (fdt == CPG_F64)
        return grad_dispatch<double>(Z, ld, G, facset, lo_n, I, hi_n, lo_first, lo_count, hi_first, hi_count, S,
                                     (double*)scratch, s);
    return grad_dispatch<float>(Z, ld, G, facset, lo_n, I, hi_n, lo_first, lo_count, hi_first, hi_count, S,
                                (double*)scratch, s);
}

// ---------------------------------------------------------------------------
// float64 Gram matrices: grams[n][r][s] = sum_i A^(n)(i,r) A^(n)(i,s)
// ---------------------------------------------------------------------------
template <typename TC>
__global__ __launch_bounds__(256) void k_grams(FacSet<TC> fs, double* __restrict__ grams) {
    // the factor is staged through LDS in chunks of whole rows (coalesced, one
    // round trip per chunk); each entry still sums its rows in index order
    constexpr int kChunk = 4096;
    __shared__ double sA[kChunk];
    const int n = blockIdx.x;
    const int R = fs.R;
    const TC* A = fs.A[n];
    const int64_t I = fs.dims[n];
    const int64_t rows_per = kChunk / R;
    constexpr int kE = 4;   // Gram entries per thread (R <= 64: R * R <= 4096 = 256 x 16, in passes)
    for (int e0 = 0; e0 < R * R; e0 += 256 * kE) {
        double acc[kE] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t i0 = 0; i0 < I; i0 += rows_per) {
            const int64_t nf = min(rows_per, I - i0) * R;
            __syncthreads();   // the previous chunk is consumed
#pragma unroll 8
            for (int64_t e = threadIdx.x; e < nf; e += 256) sA[e] = (double)A[i0 * R + e];
            __syncthreads();
            const int64_t nr = nf / R;
#pragma unroll
            for (int k = 0; k < kE; ++k) {
                const int e = e0 + threadIdx.x + 256 * k;
                if (e < R * R) {
                    const int r = e / R, c = e - (e / R) * R;
                    for (int64_t i = 0; i < nr; ++i) acc[k] += sA[i * R + r] * sA[i * R + c];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < kE; ++k) {
            const int e = e0 + threadIdx.x + 256 * k;
            if (e < R * R) grams[(int64_t)n * R * R + e] = acc[k];
        }
    }
}

hipError_t launch_grams(int fdt, const void* facset, double* grams, hipStream_t s) {
    if (fdt == CPG_F64) {
        const FacSet<double>& fs = *(const FacSet<double>*)facset;
        hipLaunchKernelGGL(k_grams<double>, dim3(fs.N), dim3(256), 0, s, fs, grams);
    } else {
        const FacSet<float>& fs = *(const FacSet<float>*)facset;
        hipLaunchKernelGGL(k_grams<float>, dim3(fs.N), dim3(256), 0, s, fs, grams);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// eq. 2.14 for one mode, one block:
//   Gamma = Hadamard product of the other modes' Grams (float64),
//   Gamma = L L^T (Cholesky; one retry with Gamma + 1e-12 tr(Gamma)/R I),
//   each row x of A^(n) solves x Gamma = g (forward then back substitution),
//   then grams[n] <- A^(n)^T A^(n) from the stored (rounded) factor.
// On failure flags[0] |= 1 and A^(n), grams[n] are left untouched.
// ---------------------------------------------------------------------------
template <typename TC, int RT>
__global__ __launch_bounds__(256) void k_als_update(const TC* __restrict__ G, TC* __restrict__ A,
                                                    double* __restrict__ grams, int N, int n, int64_t I, int R,
                                                    int* __restrict__ flags) {
    __shared__ double sGam[RT * RT];
    __shared__ double sL[RT * (RT + 1)];
    __shared__ int sOk;
    __shared__ double sTr;
    const int tid = threadIdx.x;
    const int LD = RT + 1;

    for (int e = tid; e < R * R; e += 256) {
        double v = 1.0;
        for (int k = 0; k < N; ++k)
            if (k != n) v *= grams[(int64_t)k * R * R + e];
        sGam[e] = v;
    }
    __syncthreads();
    if (tid == 0) {
        double tr = 0.0;
        for (int c = 0; c < R; ++c) tr += sGam[c * R + c];
        sTr = tr;
    }
    __syncthreads();

    bool ok = false;
    for (int attempt = 0; attempt < 2 && !ok; ++attempt) {
        const double jit = attempt == 0 ? 0.0 : 1e-12 * sTr / R;
        for (int e = tid; e < R * R; e += 256) {
            const int r = e / R, c = e - (e / R) * R;
            sL[r * LD + c] = sGam[e] + (r == c ? jit : 0.0);
        }
        if (tid == 0) sOk = 1;
        __syncthreads();
        // left-looking column Cholesky: L[c][c], then L[i][c] for i > c
        for (int c = 0; c < R; ++c) {
            if (tid == 0) {
                double d = sL[c * LD + c];
                for (int k = 0; k < c; ++k) d -= sL[c * LD + k] * sL[c * LD + k];
                if (!(d > 0.0) || !isfinite(d)) {
                    sOk = 0;
                    d = 1.0;
                }
                sL[c * LD + c] = sqrt(d);
            }
            __syncthreads();
            const double lcc = sL[c * LD + c];
            for (int i = c + 1 + tid; i < R; i += 256) {
                double v = sL[i * LD + c];
                for (int k = 0; k < c; ++k) v -= sL[i * LD + k] * sL[c * LD + k];
                sL[i * LD + c] = v / lcc;
            }
            __syncthreads();
        }
        ok = sOk != 0;
        __syncthreads();
    }
    if (!ok) {
        if (tid == 0) atomicOr(flags, 1);
        return;
    }

    // solve every row: z L^T = g  ->  L z^T = g^T (forward), then L^T x^T = z^T (back)
    for (int64_t i = tid; i < I; i += 256) {
        double x[RT];
#pragma unroll
        for (int c = 0; c < RT; ++c) x[c] = (c < R) ? (double)G[i * R + c] : 0.0;
#pragma unroll
        for (int c = 0; c < RT; ++c) {
            if (c < R) {
                double v = x[c];
#pragma unroll
                for (int k = 0; k < RT; ++k)
                    if (k < c) v -= sL[c * LD + k] * x[k];
                x[c] = v / sL[c * LD + c];
            }
        }
#pragma unroll
        for (int c = RT - 1; c >= 0; --c) {
            if (c < R) {
                double v = x[c];
#pragma unroll
                for (int k = 0; k < RT; ++k)
                    if (k > c && k < R) v -= sL[k * LD + c] * x[k];
                x[c] = v / sL[c * LD + c];
            }
        }
#pragma unroll
        for (int c = 0; c < RT; ++c)
            if (c < R) A[i * R + c] = (TC)x[c];
    }
    __syncthreads();
    for (int e = tid; e < R * R; e += 256) {
        const int r = e / R, c = e - (e / R) * R;
        double acc = 0.0;
        for (int64_t i = 0; i < I; ++i) acc += (double)A[i * R + r] * (double)A[i * R + c];
        grams[(int64_t)n * R * R + e] = acc;
    }
}

template <typename TC>
static hipError_t als_dispatch(const TC* G, TC* A, double* grams, int N, int n, int64_t I, int R, int* flags,
                               hipStream_t s) {
    if (R <= 4)
        hipLaunchKernelGGL((k_als_update<TC, 4>), dim3(1), dim3(256), 0, s, G, A, grams, N, n, I, R, flags);
    else if (R <= 16)
        hipLaunchKernelGGL((k_als_update<TC, 16>), dim3(1), dim3(256), 0, s, G, A, grams, N, n, I, R, flags);
    else if (R <= 32)
        hipLaunchKernelGGL((k_als_update<TC, 32>), dim3(1), dim3(256), 0, s, G, A, grams, N, n, I, R, flags);
    else
        hipLaunchKernelGGL((k_als_update<TC, 64>), dim3(1), dim3(256), 0, s, G, A, grams, N, n, I, R, flags);
    return hipGetLastError();
}

hipError_t launch_als_update(int fdt, const void* G, void* A, double* grams, int N, int n, int64_t I, int R,
                             int* flags, hipStream_t s) {
    if (fdt == CPG_F64) return als_dispatch<double>((const double*)G, (double*)A, grams, N, n, I, R, flags, s);
    return als_dispatch<float>((const float*)G, (float*)A, grams, N, n, I, R, flags, s);
}

// ---------------------------------------------------------------------------
// ||Y||^2 in float64 (two stages, fixed order)
// ---------------------------------------------------------------------------
constexpr int kRedBlocks = 1024;

template <typename TY>
__device__ __forceinline__ double yval(const TY* p, int64_t e) { return (double)p[e]; }
template <>
__device__ __forceinline__ double yval<uint16_t>(const uint16_t* p, int64_t e) {   // bf16 bits
    return (double)__uint_as_float(((uint32_t)p[e]) << 16);
}
template <>
__device__ __forceinline__ double yval<_Float16>(const _Float16* p, int64_t e) {
    return (double)(float)p[e];
}

// Y is read in 16-byte chunks (Y is 16-byte aligned), four chunks in flight
// per thread; the entries past the last whole chunk go to block 0.  Each
// thread sums its chunks in order, the block in a fixed tree, the blocks in
// the second stage: the result does not depend on timing.
template <typename TY>
__global__ __launch_bounds__(256) void k_norm2_stage1(const TY* __restrict__ Y, int64_t n,
                                                      double* __restrict__ scratch) {
    __shared__ double sbuf[256];
    constexpr int kPer = 16 / (int)sizeof(TY);   // entries per chunk
    constexpr int kIn = 4;                      // chunks in flight
    const int64_t nch = n / kPer;
    const int64_t stride = (int64_t)gridDim.x * 256;
    double acc = 0.0;
    int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; c + (kIn - 1) * stride < nch; c += kIn * stride) {
        uint4 v[kIn];
#pragma unroll
        for (int u = 0; u < kIn; ++u) v[u] = *(const uint4*)(Y + (c + u * stride) * kPer);
#pragma unroll
        for (int u = 0; u < kIn; ++u) {
            const TY* x = reinterpret_cast<const TY*>(&v[u]);
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const double d = yval(x, k);
                acc += d * d;
            }
        }
    }
    for (; c < nch; c += stride) {
        const uint4 v = *(const uint4*)(Y + c * kPer);
        const TY* x = reinterpret_cast<const TY*>(&v);
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const double d = yval(x, k);
            acc += d * d;
        }
    }
    if (blockIdx.x == 0)
        for (int64_t e = nch * kPer + threadIdx.x; e < n; e += 256) {
            const double d = yval(Y, e);
            acc += d * d;
        }
    const double t = block_sum_256(acc, sbuf);
    if (threadIdx.x == 0) scratch[blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_sum_stage2(const double* __restrict__ scratch, int nparts,
                                                    double* __restrict__ out) {
    __shared__ double sbuf[256];
    double acc = 0.0;
    for (int p = threadIdx.x; p < nparts; p += 256) acc += scratch[p];
    const double t = block_sum_256(acc, sbuf);
    if (threadIdx.x == 0) *out = t;
}

hipError_t launch_norm2(int ydt, const void* Y, int64_t n, double* scratch, double* out, hipStream_t s) {
    if (ydt == CPG_F64)
        hipLaunchKernelGGL(k_norm2_stage1<double>, dim3(kRedBlocks), dim3(256), 0, s, (const double*)Y, n, scratch);
    else if (ydt == CPG_F32)
        hipLaunchKernelGGL(k_norm2_stage1<float>, dim3(kRedBlocks), dim3(256), 0, s, (const float*)Y, n, scratch);
    else if (ydt == CPG_F16)
        hipLaunchKernelGGL(k_norm2_stage1<_Float16>, dim3(kRedBlocks), dim3(256), 0, s, (const _Float16*)Y, n,
                           scratch);
    else
        hipLaunchKernelGGL(k_norm2_stage1<uint16_t>, dim3(kRedBlocks), dim3(256), 0, s, (const uint16_t*)Y, n,
                           scratch);
    hipLaunchKernelGGL(k_sum_stage2, dim3(1), dim3(256), 0, s, scratch, kRedBlocks, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// <Y, Yhat> = sum_{j, r} P_R(j, r) * (A^(n*) (.) ... (.) A^(1))(j, r)
// ---------------------------------------------------------------------------
template <typename TC>
__global__ __launch_bounds__(256) void k_inner_kr_stage1(const TC* __restrict__ PR, int ld, int64_t J,
                                                         FacSet<TC> fs, int nstar, double* __restrict__ scratch) {
    __shared__ double sbuf[256];
    const int R = fs.R;
    const int64_t n = J * R;
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
        const int64_t j = e / R;
        const int r = (int)(e - j * R);
        acc += (double)PR[j * ld + r] * kr_entry_d(fs, 0, nstar, j, r);
    }
    const double t = block_sum_256(acc, sbuf);
    if (threadIdx.x == 0) scratch[blockIdx.x] = t;
}

hipError_t launch_inner_kr(int fdt, const void* PR, int ld, int64_t J, const void* facset, int nstar,
                           double* scratch, double* out, hipStream_t s) {
    if (fdt == CPG_F64)
        hipLaunchKernelGGL(k_inner_kr_stage1<double>, dim3(kRedBlocks), dim3(256), 0, s, (const double*)PR, ld, J,
                           *(const FacSet<double>*)facset, nstar, scratch);
    else
        hipLaunchKernelGGL(k_inner_kr_stage1<float>, dim3(kRedBlocks), dim3(256), 0, s, (const float*)PR, ld, J,
                           *(const FacSet<float>*)facset, nstar, scratch);
    hipLaunchKernelGGL(k_sum_stage2, dim3(1), dim3(256), 0, s, scratch, kRedBlocks, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// cost (eq. 2.12) = ||Y||^2 - 2 <Y,Yhat> + ||Yhat||^2, fit = 1 - sqrt(cost)/||Y||
// ---------------------------------------------------------------------------
template <typename TC>
__global__ __launch_bounds__(256) void k_cost_fit(const TC* __restrict__ G, const TC* __restrict__ A, int64_t I,
                                                  int R, const double* __restrict__ inner_in,
                                                  const double* __restrict__ grams, int N, double* __restrict__ scal,
                                                  int* __restrict__ flags, int out) {
    __shared__ double sbuf[256];
    double acc = 0.0;
    if (G != nullptr)
        for (int64_t e = threadIdx.x; e < I * R; e += 256) acc += (double)G[e] * (double)A[e];
    const double inner = (G != nullptr) ? block_sum_256(acc, sbuf) : *inner_in;
    double h = 0.0;
    for (int e = threadIdx.x; e < R * R; e += 256) {
        double v = 1.0;
        for (int k = 0; k < N; ++k) v *= grams[(int64_t)k * R * R + e];
        h += v;
    }
    const double nrm = block_sum_256(h, sbuf);
    if (threadIdx.x == 0) {
        const double y2 = scal[0];
        const double D = y2 - 2.0 * inner + nrm;
        const double fit = 1.0 - sqrt(D > 0.0 ? D : 0.0) / sqrt(y2);
        scal[out] = D;
        scal[out + 1] = fit;
        if (out == 2) {
            scal[4] = inner;
            scal[5] = nrm;
        }
        if (out == 2 && (!isfinite(D) || !isfinite(fit))) atomicOr(flags, 2);
    }
}

hipError_t launch_cost_fit(int fdt, const void* G, const void* A, int64_t I, int R, const double* inner_in,
                           const double* grams, int N, double* scal, int* flags, hipStream_t s, int out_slot) {
    if (fdt == CPG_F64)
        hipLaunchKernelGGL(k_cost_fit<double>, dim3(1), dim3(256), 0, s, (const double*)G, (const double*)A, I, R,
                           inner_in, grams, N, scal, flags, out_slot);
    else
        hipLaunchKernelGGL(k_cost_fit<float>, dim3(1), dim3(256), 0, s, (const float*)G, (const float*)A, I, R,
                           inner_in, grams, N, scal, flags, out_slot);
    return hipGetLastError();
}

}  // namespace cpg
