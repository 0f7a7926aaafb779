// Reduced-precision forms of the big contraction of Algorithm 2 (steps 4 and
// 7): both partial products of Y_(1:n*) against Khatri-Rao blocks on 16-bit
// matrix cores (v_mfma_f32_16x16x32_bf16 / _f16) with float32 accumulation.
//
//   BF16          : P = bf16(Y) * bf16(KR)
//   BF16_REFINED  : Y stored as bf16 (exact):  P = Y*KR_hi + Y*KR_lo
//                   Y stored as float32:       P = Y_hi*KR_hi + Y_hi*KR_lo + Y_lo*KR_hi
// with x_hi = bf16(x) and x_lo = bf16(x - x_hi) (round to nearest even); the
// refinement terms are formed in the same pass over Y, so the bytes moved do
// not change.  bf16 keeps float32's exponent range, so no scaling is needed.
//
//   F16_SCALED(_REFINED): the same products in fp16 (11-bit significand, so
//   hi + lo carries 22 bits) with power-of-two scaling, since fp16's range is
//   narrow.  Each wave scales its 64 x 32 tile of Y in a step by 2^e so that
//   the tile's largest magnitude lands in [2^14, 2^15) (the max is taken over
//   the loaded tile, so no extra pass over Y is needed and any split works);
//   each Khatri-Rao column r is scaled by 2^f_r so that its largest magnitude
//   lands in the same range: that maximum is exactly the product over the
//   side's modes of max_i |A^(m)(i, r)| (the column is a Kronecker product of
//   the factor columns), taken by every block from the factors.  Products
//   accumulate in float32 and are unscaled exactly (powers of two): per step
//   for the Y scale, at the store for the Khatri-Rao scale.  Y stored as bf16
//   or fp16 converts to scaled fp16 exactly (over 29 binades below the
//   tile's maximum), so only float32 Y has a Y_lo term.
//
// Block = 4 waves x 64 rows of Y, steps of 32 columns dealt round-robin over
// the block columns (the grid sweeps Y as one moving window).  Each lane
// loads, per step, four chunks of 8 consecutive rows of one column (16 bytes
// of bf16 or 32 bytes of float32) through buffer loads that read zero past
// the edges; two steps are in flight ahead of the MFMAs and the hi / lo split
// of float32 data happens when a step is used.  A chunk is directly the
// 8-element operand of the left contraction (reduction over rows, columns as
// output rows); the right contraction reduces over columns, so each wave
// writes its 64 x 32 sub-tile into a private LDS tile row-major and reads 8
// consecutive columns of a row per operand.  The KR_R rows of all of the
// block's steps are generated into LDS before the loop and the KR_L rows into
// registers (split into hi / lo), from the factors by multiply-shift index
// unravelling.  Partials and the cross-wave reduction of the left product are
// as in the float32 MFMA kernel.
#include "cpg_device.h"
#include "cpg_fastdiv.h"

#include <algorithm>

#include <hip/hip_ext.h>

namespace cpg {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short v8us __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

constexpr int kB16Rows = 256;
constexpr int kB16Step = 32;
constexpr int kB16Depth = 2;   // steps of Y loads in flight ahead of the MFMAs
constexpr int kTrLd = 40;      // bf16 elements per row of the transposed LDS tile (80 bytes)

// float -> bf16 bits, round to nearest even
__device__ __forceinline__ unsigned short bf16_rne(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

__device__ __forceinline__ void lds_wave_sync_b() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}
__device__ __forceinline__ void lds_block_sync_b() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

__device__ __forceinline__ v8bf as_bf(v8us u) { return __builtin_bit_cast(v8bf, u); }
__device__ __forceinline__ v8h as_h(v8us u) { return __builtin_bit_cast(v8h, u); }

// float <-> fp16 bits (hardware conversion, round to nearest even)
__device__ __forceinline__ unsigned short f16_bits(float x) { return __builtin_bit_cast(unsigned short, (_Float16)x); }
__device__ __forceinline__ float f16_to_f(unsigned short b) { return (float)__builtin_bit_cast(_Float16, b); }

// Scaled fp16 operands: a magnitude m is scaled by 2^(kF16Target - floor(log2 m)),
// landing in [2^14, 2^15) (one binade below fp16's largest finite value).
constexpr int kF16Target = 14;
__device__ __forceinline__ int ilog2f(float m) { return (int)((__float_as_uint(m) >> 23) & 0xff) - 127; }
__device__ __forceinline__ int clamp_exp(int e) { return e < -126 ? -126 : (e > 126 ? 126 : e); }
__device__ __forceinline__ float pow2f(int e) { return __uint_as_float((uint32_t)(e + 127) << 23); }   // |e| <= 126

// Largest value over the wave (unsigned compare; the callers pass |x| bits).
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    v = max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true));    // quad [1,0,3,2]
    v = max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true));    // quad [2,3,0,1]
    v = max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x141, 0xF, 0xF, true));   // half-row mirror
    v = max(v, (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x140, 0xF, 0xF, true));   // row mirror
    const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 0), b = (uint32_t)__builtin_amdgcn_readlane((int)v, 16);
    const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 32), d = (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
    return max(max(a, b), max(c, d));
}

// 16 x 16 x 32 matrix-core product of 8-element operands (bf16 or fp16 bits).
template <bool F16>
__device__ __forceinline__ v4f mma16(v8us a, v8us b, v4f c) {
    if constexpr (F16) return __builtin_amdgcn_mfma_f32_16x16x32_f16(as_h(a), as_h(b), c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(a), as_bf(b), c, 0, 0, 0);
}

// 16-bit split of a float32 value: hi = round(x), lo = round(x - hi)
template <bool F16>
__device__ __forceinline__ unsigned short to16(float x) { return F16 ? f16_bits(x) : bf16_rne(x); }
template <bool F16>
__device__ __forceinline__ float from16(unsigned short b) { return F16 ? f16_to_f(b) : bf16_to_f(b); }

// one step of Y as loaded: float32 storage (two float4 per chunk) or bf16 storage
struct RawF {
    v4f a[4], b[4];
};
struct RawB {
    v8us c[4];
};
template <bool TYF>
struct RawSel {
    typedef RawF T;
};
template <>
struct RawSel<false> {
    typedef RawB T;
};

// LDS row stride (bf16 elements) of the KR_R tile for kcols columns
__host__ __device__ constexpr int64_t krr_stride(int64_t kcols) { return kcols + 8; }

// YK: storage of Y, 0 = float32 (hi/lo split in registers), 1 = bf16, 2 = fp16.
// F16: fp16 matrix cores with the power-of-two scaling, else bf16.
template <int YK, int NRT, bool DO_R, bool DO_L, bool REFINE, bool F16>
__global__ __launch_bounds__(256) void k_contract_bf16(const void* __restrict__ Yv, int64_t J, int64_t K,
                                                        int64_t kcols, int ld, KrGen kg, float* __restrict__ PRpart,
                                                        float* __restrict__ PLpart) {
    constexpr bool TYF = YK == 0;
    constexpr int RT = NRT * 16;
    constexpr bool YLO = TYF && REFINE;   // a Y_lo term exists
    constexpr bool KLO = REFINE;          // a KR_lo term exists
    constexpr uint32_t ES = TYF ? 4 : 2;  // bytes per element of Y
    typedef typename RawSel<TYF>::T Raw;
    // dynamic LDS: KR_R hi (and lo) tiles [RT][krr_stride(kcols)] bf16
    extern __shared__ __attribute__((aligned(16))) unsigned short sKRdyn[];
    __shared__ __attribute__((aligned(16))) unsigned short sTr[DO_R ? 4 : 1][YLO ? 2 : 1][DO_R ? 64 * kTrLd : 8];
    __shared__ v4f sRed[DO_L ? 2 : 1][DO_L ? 4 * 2 * NRT * 64 : 1];
    // fp16 scaling: factor column maxima (|x| bits) and the Khatri-Rao column
    // scales: [0] left side, [1] right side, [2] / [3] their inverses
    __shared__ unsigned int sCm[F16 ? CPG_MAX_MODES : 1][F16 ? RT : 1];
    __shared__ float sKs[F16 ? 4 : 1][F16 ? RT : 1];
    const int KRS = (int)krr_stride(kcols);
    unsigned short* sKRh = sKRdyn;
    unsigned short* sKRl = sKRdyn + RT * KRS;

    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int l = tid & 63;
    const int q = l >> 4;
    const int c16 = l & 15;
    const int R = kg.R;
    const int64_t jb = (int64_t)blockIdx.x * kB16Rows;
    const int64_t jw = jb + 64 * w;
    const int64_t n_kc = gridDim.y;
    const int64_t gsteps = (K + kB16Step - 1) / kB16Step;
    const int64_t nsteps = (gsteps - blockIdx.y + n_kc - 1) / n_kc;
    auto step_col = [&](int64_t st) { return (st * n_kc + blockIdx.y) * kB16Step; };
    auto fac_rsrc = [&](int m) { return buf_rsrc(kg.A[m], (uint32_t)(kg.fd[m].d * (uint32_t)R * 4)); };

    // chunk s of a step: column step_col(st) + 16*(s&1) + c16, rows jw + 32*(s>>1) + 8q .. +7
    auto load_step = [&](Raw& dst, int64_t st) {
        const int64_t k0 = step_col(st);
        const int64_t ncol = st < nsteps ? max((int64_t)0, min((int64_t)kB16Step, K - k0)) : 0;
        const auto rs = buf_rsrc((const char*)Yv + (st < nsteps ? k0 : 0) * J * ES, (uint32_t)(ncol * J * ES));
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int64_t row = jw + 32 * (s >> 1) + 8 * q;   // J % 8 == 0: a chunk is all in or all out
            const uint32_t off =
                row < J ? (uint32_t)(((int64_t)(16 * (s & 1) + c16) * J + row) * ES) : kOOB;
            if constexpr (TYF) {
                dst.a[s] = __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0));
                dst.b[s] = __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(off + 16), 0, 0));
            } else {
                dst.c[s] = __builtin_bit_cast(v8us, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0));
            }
        }
    };
    // hi / lo split with the hardware conversion (round to nearest even).
    // fp16: the wave's tile is first scaled by 2^e from its largest magnitude;
    // returns the inverse scale (1 for bf16).
    auto split = [&](const Raw& r, v8us (&hi)[4], v8us (&lo)[4]) -> float {
        if constexpr (!F16) {
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                if constexpr (TYF) {
                    const float x[8] = {r.a[s][0], r.a[s][1], r.a[s][2], r.a[s][3],
                                        r.b[s][0], r.b[s][1], r.b[s][2], r.b[s][3]};
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const __bf16 h = (__bf16)x[t];
                        hi[s][t] = __builtin_bit_cast(unsigned short, h);
                        if (YLO) lo[s][t] = __builtin_bit_cast(unsigned short, (__bf16)(x[t] - (float)h));
                    }
                } else {
                    hi[s] = r.c[s];
                }
            }
            return 1.f;
        } else {
            float x[4][8];
            uint32_t m = 0;
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    if constexpr (TYF) x[s][t] = t < 4 ? r.a[s][t] : r.b[s][t - 4];
                    else if constexpr (YK == 1) x[s][t] = bf16_to_f(r.c[s][t]);
                    else x[s][t] = f16_to_f(r.c[s][t]);
                    m = max(m, __float_as_uint(x[s][t]) & 0x7fffffffu);
                }
            m = wave_max_u32(m);
            // an all-zero tile keeps scale 1; a non-finite one too (its products stay non-finite)
            const int e = (m == 0u || m >= 0x7f800000u) ? 0 : clamp_exp(kF16Target - ilog2f(__uint_as_float(m)));
            const float sc = pow2f(e);
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const float v = x[s][t] * sc;
                    const unsigned short h = f16_bits(v);
                    hi[s][t] = h;
                    if (YLO) lo[s][t] = f16_bits(v - f16_to_f(h));
                }
            return pow2f(-e);
        }
    };

    // Khatri-Rao rows (eq. 3.3, Notation 2.1 order), products in float32 in mode
    // order, split into hi / lo.  KR_L: rows jw + 32*jc + 8q + t, rank rt*16 + c16.
    // KR_R: LDS column st*32 + kk <- Y column step_col(st) + kk.  Round j loads
    // mode j of the left product and mode n*+j of the right one.
    v8us krl_hi[DO_L ? 2 : 1][DO_L ? NRT : 1], krl_lo[DO_L && KLO ? 2 : 1][DO_L && KLO ? NRT : 1];
    constexpr int kKrBatch = 8;
    constexpr int kPeel = NRT <= 2 ? 2 : 1;   // Khatri-Rao rounds whose loads precede the first Y loads
    const int n4 = (int)(nsteps * kB16Step) * (RT / 4);
    auto gen_kr = [&](int base, bool with_left, auto&& mid) {
        float fl[DO_L ? NRT : 1][16];
        uint32_t idxL[16], idxR[kKrBatch];
        int r4[kKrBatch];
        v4f t[kKrBatch];
        if (DO_L && with_left) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t j = jw + 32 * (e >> 3) + 8 * q + (e & 7);
                idxL[e] = j < J ? (uint32_t)j : 0u;
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) fl[rt][e] = j < J ? 1.f : 0.f;
            }
        }
        if (DO_R) {
#pragma unroll
            for (int u = 0; u < kKrBatch; ++u) {
                const int e = base + u * 256 + tid;
                const int kk = e / (RT / 4);
                r4[u] = (e - kk * (RT / 4)) * 4;
                const int64_t k = step_col(kk / kB16Step) + (kk & (kB16Step - 1));
                const bool ok = e < n4 && k < K;
                idxR[u] = ok ? (uint32_t)k : 0u;
                const float one = ok ? 1.f : 0.f;
                t[u] = v4f{one, one, one, one};
            }
        }
        const int nL = (DO_L && with_left) ? kg.nstar : 0;
        const int nR = DO_R ? kg.N - kg.nstar : 0;
        const int rounds = nL > nR ? nL : nR;
        // factor loads of round j (a mode past a side's count reads zero here and
        // multiplies by one below)
        auto issue = [&](int j, float (&vl)[DO_L ? NRT : 1][16], float (&vr)[DO_R ? kKrBatch : 1][4]) {
            const bool aL = j < nL, aR = j < nR;
            if (DO_L && with_left) {
                const int m = aL ? j : 0;
                const FastDiv f = kg.fd[m];
                const auto rs = fac_rsrc(m);
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const uint32_t qd = fast_div(idxL[e], f);
                    const uint32_t i = idxL[e] - qd * f.d;
                    idxL[e] = qd;
#pragma unroll
                    for (int rt = 0; rt < NRT; ++rt) {
                        const int r = rt * 16 + c16;
                        const uint32_t off = (aL && r < R) ? (i * (uint32_t)R + (uint32_t)r) * 4 : kOOB;
                        vl[rt][e] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
                    }
                }
            }
            if (DO_R) {
                const int m = kg.nstar + (aR ? j : 0);
                const FastDiv f = kg.fd[m];
                const auto rs = fac_rsrc(m);
#pragma unroll
                for (int u = 0; u < kKrBatch; ++u) {
                    const uint32_t qd = fast_div(idxR[u], f);
                    const uint32_t i = idxR[u] - qd * f.d;
                    idxR[u] = qd;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const int r = r4[u] + c;
                        const uint32_t off = (aR && r < R) ? (i * (uint32_t)R + (uint32_t)r) * 4 : kOOB;
                        vr[u][c] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
                    }
                }
            }
        };
        auto consume = [&](int j, const float (&vl)[DO_L ? NRT : 1][16], const float (&vr)[DO_R ? kKrBatch : 1][4]) {
            const bool aL = j < nL, aR = j < nR;
            if (DO_L && with_left) {
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
                    for (int e = 0; e < 16; ++e) fl[rt][e] *= aL ? vl[rt][e] : 1.f;
            }
            if (DO_R) {
#pragma unroll
                for (int u = 0; u < kKrBatch; ++u)
#pragma unroll
                    for (int c = 0; c < 4; ++c) t[u][c] *= aR ? vr[u][c] : 1.f;
            }
        };
        // The first kPeel rounds are issued before `mid` (the first steps of Y
        // on the first chunk), so that waiting for them does not wait for Y as
        // well (loads complete in order for the wait counter); later rounds, if
        // any, load and multiply in turn.
        float vlp[kPeel][DO_L ? NRT : 1][16], vrp[kPeel][DO_R ? kKrBatch : 1][4];
#pragma unroll
        for (int j = 0; j < kPeel; ++j) issue(j, vlp[j], vrp[j]);
        __builtin_amdgcn_sched_barrier(0);
        mid();
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < kPeel; ++j) consume(j, vlp[j], vrp[j]);
        for (int j = kPeel; j < rounds; ++j) {
            float vl[DO_L ? NRT : 1][16], vr[DO_R ? kKrBatch : 1][4];
            issue(j, vl, vr);
            consume(j, vl, vr);
        }
        if (DO_L && with_left) {
#pragma unroll
            for (int jc = 0; jc < 2; ++jc)
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
                    for (int tt = 0; tt < 8; ++tt) {
                        const float v = fl[rt][8 * jc + tt] * (F16 ? sKs[0][F16 ? rt * 16 + c16 : 0] : 1.f);
                        const unsigned short h = to16<F16>(v);
                        krl_hi[jc][rt][tt] = h;
                        if (KLO)
                            krl_lo[DO_L && KLO ? jc : 0][DO_L && KLO ? rt : 0][tt] = to16<F16>(v - from16<F16>(h));
                    }
        }
        if (DO_R) {
#pragma unroll
            for (int u = 0; u < kKrBatch; ++u) {
                const int e = base + u * 256 + tid;
                if (e < n4) {
                    const int kk = e / (RT / 4);
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const float v = t[u][c] * (F16 ? sKs[1][F16 ? r4[u] + c : 0] : 1.f);
                        const unsigned short h = to16<F16>(v);
                        sKRh[(r4[u] + c) * KRS + kk] = h;
                        if (KLO) sKRl[(r4[u] + c) * KRS + kk] = to16<F16>(v - from16<F16>(h));
                    }
                }
            }
        }
    };

    v4f accR[DO_R ? 4 : 1][DO_R ? NRT : 1];
#pragma unroll
    for (int e = 0; e < (DO_R ? 4 : 1); ++e)
#pragma unroll
        for (int rt = 0; rt < (DO_R ? NRT : 1); ++rt) accR[e][rt] = v4f{0.f, 0.f, 0.f, 0.f};

    auto step = [&](Raw& curRaw, Raw& nxtRaw, int64_t st) {
        const int buf = (int)(st & 1);
        load_step(nxtRaw, st + kB16Depth);
        __builtin_amdgcn_sched_barrier(0);   // keep the prefetch ahead of the step's MFMAs
        v8us cur_hi[4], cur_lo[4];
        const float inv_s = split(curRaw, cur_hi, cur_lo);
        (void)inv_s;
        if (DO_R) {
            // transpose through this wave's LDS tile: row (32*jc + 8q + t), column (16*kt + c16)
            // Lanes of adjacent columns (c16 even / odd) swap half of their eight
            // rows (one DPP exchange of two 32-bit words), so each lane writes four
            // 32-bit words holding both columns of a row: the even lane rows 0..3,
            // the odd lane rows 4..7.
            const bool odd = (c16 & 1) != 0;
#pragma unroll
            for (int part = 0; part < (YLO ? 2 : 1); ++part) {
                unsigned int* T = (unsigned int*)sTr[w][YLO ? part : 0];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const v8us v = part == 0 ? cur_hi[s] : cur_lo[s];
                    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
                    const v4u own = __builtin_bit_cast(v4u, v);   // word k = rows 2k (low) and 2k+1 (high)
                    const unsigned int snd0 = odd ? own[0] : own[2], snd1 = odd ? own[1] : own[3];
                    const unsigned int rcv0 = (unsigned int)__builtin_amdgcn_mov_dpp((int)snd0, 0xB1, 0xF, 0xF, true);
                    const unsigned int rcv1 = (unsigned int)__builtin_amdgcn_mov_dpp((int)snd1, 0xB1, 0xF, 0xF, true);
                    // this lane's four rows of its own column and of the neighbour's
                    const unsigned int mw0 = odd ? own[2] : own[0], mw1 = odd ? own[3] : own[1];
                    const unsigned int mine[4] = {mw0 & 0xffffu, mw0 >> 16, mw1 & 0xffffu, mw1 >> 16};
                    const unsigned int nb[4] = {rcv0 & 0xffffu, rcv0 >> 16, rcv1 & 0xffffu, rcv1 >> 16};
                    const int col2 = (16 * (s & 1) + (c16 & ~1)) >> 1;   // 32-bit column of the pair
                    const int row0 = 32 * (s >> 1) + 8 * q + (odd ? 4 : 0);
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const unsigned int word = odd ? (nb[k] | (mine[k] << 16)) : (mine[k] | (nb[k] << 16));
                        T[(row0 + k) * (kTrLd / 2) + col2] = word;
                    }
                }
            }
            lds_wave_sync_b();
            // right product: rows 16*rr + c16 (output), columns 8q .. 8q+7 (reduced)
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt) {
                const v8us bh = *(const v8us*)(&sKRh[(rt * 16 + c16) * KRS + st * kB16Step + 8 * q]);
                v8us bl;
                if (KLO) bl = *(const v8us*)(&sKRl[(rt * 16 + c16) * KRS + st * kB16Step + 8 * q]);
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const v8us ah = *(const v8us*)(&sTr[w][0][(16 * rr + c16) * kTrLd + 8 * q]);
                    // fp16: the step's products in their own accumulator, unscaled by the tile's scale
                    v4f a = F16 ? v4f{0.f, 0.f, 0.f, 0.f} : accR[rr][rt];
                    a = mma16<F16>(ah, bh, a);
                    if (KLO) a = mma16<F16>(ah, bl, a);
                    if (YLO) {
                        const v8us al = *(const v8us*)(&sTr[w][YLO ? 1 : 0][(16 * rr + c16) * kTrLd + 8 * q]);
                        a = mma16<F16>(al, bh, a);
                    }
                    if constexpr (F16) accR[rr][rt] += a * inv_s;
                    else accR[rr][rt] = a;
                }
            }
        }
        if (DO_L) {
            // left product: columns step_col(st) + 16*kt + c16 are the output rows, rows are reduced
            v4f accL[2][NRT];
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) {
                    v4f a = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int jc = 0; jc < 2; ++jc) {
                        const int s = 2 * jc + kt;
                        a = mma16<F16>(cur_hi[s], krl_hi[jc][rt], a);
                        if (KLO) a = mma16<F16>(cur_hi[s], krl_lo[DO_L && KLO ? jc : 0][DO_L && KLO ? rt : 0], a);
                        if (YLO) a = mma16<F16>(cur_lo[s], krl_hi[jc][rt], a);
                    }
                    // fp16: unscale by the tile's and this rank column's scales before the cross-wave sum
                    if constexpr (F16) a *= inv_s * sKs[2][F16 ? rt * 16 + c16 : 0];
                    accL[kt][rt] = a;
                }
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) sRed[buf][((w * 2 + kt) * NRT + rt) * 64 + l] = accL[kt][rt];
            lds_block_sync_b();
            // P_L partial stores of this block row over the step's columns (past K: dropped);
            // every thread stores 2*NRT values (uniform count, exact load counters)
            const int64_t k0 = step_col(st);
            const auto lrs = buf_rsrc(PLpart + ((int64_t)blockIdx.x * K + k0) * ld,
                                      (uint32_t)(max((int64_t)0, min((int64_t)kB16Step, K - k0)) * ld * 4));
#pragma unroll
            for (int jj = 0; jj < NRT; ++jj) {
                const int item = jj * 128 + (tid >> 1);   // (kt, rt, lane) of the wave partials
                const int lane = item & 63;
                const int rt = (item >> 6) % NRT;
                const int kt = (item >> 6) / NRT;
                const int v0 = 2 * (tid & 1);
                const float* src = (const float*)sRed[buf];
                float s0 = 0.f, s1 = 0.f;
#pragma unroll
                for (int ww = 0; ww < 4; ++ww) {
                    const float* e = src + (((ww * 2 + kt) * NRT + rt) * 64 + lane) * 4 + v0;
                    s0 += e[0];
                    s1 += e[1];
                }
                const int r = rt * 16 + (lane & 15);
                const uint32_t off = r < ld ? (uint32_t)(((kt * 16 + 4 * (lane >> 4) + v0) * ld + r) * 4) : kOOB;
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(s0), lrs, (int)off, 0, kStoreThrough);
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(s1), lrs, (int)(off + (uint32_t)(ld * 4)), 0, kStoreThrough);
            }
        }
    };

    // fp16 scaling of the Khatri-Rao columns: max_i |A^(m)(i, r)| of every factor
    // (LDS atomics on the |x| bits), then per side 2^f_r from the product of its
    // modes' maxima (exponents summed, so no float overflow on the way).
    if constexpr (F16) {
        const int N = kg.N;
        for (int e = tid; e < N * RT; e += 256) sCm[F16 ? e / RT : 0][F16 ? e % RT : 0] = 0u;
        __syncthreads();
        for (int m = 0; m < N; ++m) {
            const int tot = (int)kg.fd[m].d * R;
            for (int e = tid; e < tot; e += 256)
                atomicMax(&sCm[F16 ? m : 0][F16 ? e % R : 0], __float_as_uint(kg.A[m][e]) & 0x7fffffffu);
        }
        __syncthreads();
        if (tid < 2 * RT) {
            const int side = tid / RT, r = tid % RT;
            const int m0 = side == 0 ? 0 : kg.nstar, m1 = side == 0 ? kg.nstar : N;
            bool zero = r >= R;
            int ex = 0;
            float mant = 1.f;
            for (int m = m0; m < m1 && !zero; ++m) {
                const unsigned int b = sCm[F16 ? m : 0][F16 ? r : 0];
                if (b == 0u || b >= 0x7f800000u) {
                    zero = true;   // an all-zero (or non-finite) column: scale 1
                } else {
                    int em = 0;
                    mant *= frexpf(__uint_as_float(b), &em);   // mantissa in [0.5, 1)
                    ex += em;
                }
            }
            const int e = zero ? 0 : clamp_exp(kF16Target - (ex + ilog2f(mant)));
            sKs[F16 ? side : 0][F16 ? r : 0] = pow2f(e);
            sKs[F16 ? 2 + side : 0][F16 ? r : 0] = pow2f(-e);
        }
        __syncthreads();
    }

    // Prologue: the first steps of Y go out first, then the Khatri-Rao rows.
    constexpr int NB = kB16Depth + 1;
    Raw rbuf[NB];
    gen_kr(0, true, [&] {
#pragma unroll
        for (int d = 0; d < kB16Depth; ++d) load_step(rbuf[d], d);
    });
    for (int base = kKrBatch * 256; DO_R && base < n4; base += kKrBatch * 256)   // wide chunks
        gen_kr(base, false, [] {});
    lds_block_sync_b();

    for (int64_t st = 0; st < nsteps; st += NB) {
#pragma unroll
        for (int ph = 0; ph < NB; ++ph)
            if (ph == 0 || st + ph < nsteps) step(rbuf[ph], rbuf[(ph + kB16Depth) % NB], st + ph);
    }

    if (DO_R) {
        // lane holds rows jw + 16*rr + 4q + v, rank rt*16 + c16
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt) {
                const int r = rt * 16 + c16;
                if (r < ld) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int64_t j = jw + 16 * rr + 4 * q + v;
                        const float x = accR[rr][rt][v] * (F16 ? sKs[3][F16 ? r : 0] : 1.f);
                        if (j < J) store_through(&PRpart[((int64_t)blockIdx.y * J + j) * ld + r], x);
                    }
                }
            }
    }
}

// LDS of one block: static transpose / reduction tiles (and the fp16 scale
// tables) plus the dynamic KR_R tiles.
static constexpr int64_t b16_static_lds(int nrt, bool do_r, bool do_l, bool ylo, bool f16) {
    return (do_r ? (int64_t)4 * (ylo ? 2 : 1) * 64 * kTrLd * 2 : 0) + (do_l ? (int64_t)2 * 4 * 2 * nrt * 64 * 16 : 0) +
           (f16 ? (int64_t)(CPG_MAX_MODES + 4) * nrt * 16 * 4 : 0);
}
constexpr int64_t kB16LdsPerCu = 160 * 1024;

// Widest column chunk whose KR_R rows fit the LDS of a CU shared by
// `blocks_per_cu` blocks.
int64_t mfma_bf16_max_cols_shared(int rt, int roles, bool ylo, bool klo, bool f16, int blocks_per_cu) {
    const int nrt = rt / 16;
    const int64_t st = b16_static_lds(nrt, (roles & 1) != 0, (roles & 2) != 0, ylo, f16);
    if (!(roles & 1)) return int64_t(1) << 30;   // no KR_R tile
    const int64_t per_col = (int64_t)(klo ? 2 : 1) * rt * 2;
    const int64_t cols = (kB16LdsPerCu / blocks_per_cu - st - (int64_t)(klo ? 2 : 1) * rt * 2 * 8) / per_col;
    return std::max<int64_t>(kB16Step, cols / kB16Step * kB16Step);
}

int64_t mfma_bf16_max_cols(int rt, int roles, bool ylo, bool klo, bool f16) {
    return mfma_bf16_max_cols_shared(rt, roles, ylo, klo, f16, 1);
}

template <int YK, int NRT, bool DO_R, bool DO_L, bool REFINE, bool F16>
static hipError_t launch_b16_one(dim3 grid, const void* Y, int64_t J, int64_t K, int64_t kcols, const MfmaBufs& o,
                                 hipStream_t s) {
    constexpr bool TYF = YK == 0;
    auto kern = k_contract_bf16<YK, NRT, DO_R, DO_L, REFINE, F16>;
    const size_t dyn = DO_R ? (size_t)(REFINE ? 2 : 1) * NRT * 16 * krr_stride(kcols) * 2 : 0;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(kB16LdsPerCu - b16_static_lds(NRT, DO_R, DO_L, TYF && REFINE, F16)));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    if (o.ev0)
        hipExtLaunchKernelGGL(kern, grid, dim3(256), (uint32_t)dyn, s, o.ev0, o.ev1, 0u, Y, J, K, kcols, o.ld, o.kg,
                              o.PRpart, o.PLpart);
    else
        hipLaunchKernelGGL(kern, grid, dim3(256), dyn, s, Y, J, K, kcols, o.ld, o.kg, o.PRpart, o.PLpart);
    return hipGetLastError();
}

template <int YK, int NRT, bool REFINE, bool F16>
static hipError_t launch_b16_roles(const void* Y, int64_t J, int64_t K, const Tiling& t, int roles,
                                   const MfmaBufs& o, hipStream_t s) {
    dim3 grid((unsigned)t.n_jr, (unsigned)t.n_kc);
    const int64_t kcols = t.ktb * kB16Step;
    if (kcols > mfma_bf16_max_cols(NRT * 16, roles, YK == 0 && REFINE, REFINE, F16)) return hipErrorInvalidValue;
    if (roles == 3) return launch_b16_one<YK, NRT, true, true, REFINE, F16>(grid, Y, J, K, kcols, o, s);
    if (roles == 1) return launch_b16_one<YK, NRT, true, false, REFINE, F16>(grid, Y, J, K, kcols, o, s);
    if (roles == 2) return launch_b16_one<YK, NRT, false, true, REFINE, F16>(grid, Y, J, K, kcols, o, s);
    return hipErrorInvalidValue;
}

template <int YK, bool REFINE, bool F16>
static hipError_t launch_b16_nrt(const void* Y, int64_t J, int64_t K, const Tiling& t, int roles, const MfmaBufs& o,
                                 hipStream_t s) {
    switch (t.rt) {
        case 16: return launch_b16_roles<YK, 1, REFINE, F16>(Y, J, K, t, roles, o, s);
        case 32: return launch_b16_roles<YK, 2, REFINE, F16>(Y, J, K, t, roles, o, s);
        case 48: return launch_b16_roles<YK, 3, REFINE, F16>(Y, J, K, t, roles, o, s);
        case 64: return launch_b16_roles<YK, 4, REFINE, F16>(Y, J, K, t, roles, o, s);
        default: return hipErrorInvalidValue;
    }
}

template <int YK, bool F16>
static hipError_t launch_b16_mode(bool refine, const void* Y, int64_t J, int64_t K, const Tiling& t, int roles,
                                  const MfmaBufs& o, hipStream_t s) {
    return refine ? launch_b16_nrt<YK, true, F16>(Y, J, K, t, roles, o, s)
                  : launch_b16_nrt<YK, false, F16>(Y, J, K, t, roles, o, s);
}

hipError_t launch_contract_bf16(int ydt, int mode, const void* Y, int64_t J, int64_t K, const Tiling& t, int roles,
                                const MfmaBufs& o, hipStream_t stream) {
    if ((J % 8) != 0) return hipErrorInvalidValue;
    const bool f16 = mode == CPG_MODE_F16_SCALED || mode == CPG_MODE_F16_SCALED_REFINED;
    const bool refine = mode == CPG_MODE_BF16_REFINED || mode == CPG_MODE_F16_SCALED_REFINED;
    if (f16) {
        if (ydt == CPG_F32) return launch_b16_mode<0, true>(refine, Y, J, K, t, roles, o, stream);
        if (ydt == CPG_BF16) return launch_b16_mode<1, true>(refine, Y, J, K, t, roles, o, stream);
        if (ydt == CPG_F16) return launch_b16_mode<2, true>(refine, Y, J, K, t, roles, o, stream);
        return hipErrorInvalidValue;
    }
    if (ydt == CPG_F32) return launch_b16_mode<0, false>(refine, Y, J, K, t, roles, o, stream);
    if (ydt == CPG_BF16) return launch_b16_mode<1, false>(refine, Y, J, K, t, roles, o, stream);
    return hipErrorInvalidValue;
}

}  // namespace cpg
