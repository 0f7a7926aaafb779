// Reduced-precision form of the big contraction of Algorithm 2 (steps 4 and
// 7): both partial products of Y_(1:n*) against Khatri-Rao blocks on bf16
// matrix cores (v_mfma_f32_16x16x32_bf16) with float32 accumulation.
//
//   BF16          : P = bf16(Y) * bf16(KR)
//   BF16_REFINED  : Y stored as bf16 (exact):  P = Y*KR_hi + Y*KR_lo
//                   Y stored as float32:       P = Y_hi*KR_hi + Y_hi*KR_lo + Y_lo*KR_hi
// with x_hi = bf16(x) and x_lo = bf16(x - x_hi) (round to nearest even); the
// refinement terms are formed in the same pass over Y, so the bytes moved do
// not change.  bf16 keeps float32's exponent range, so no scaling is needed.
//
// Block = 4 waves x 64 rows of Y, steps of 32 columns.  Each lane loads, per
// step, four chunks of 8 consecutive rows of one column (16 bytes of bf16 or
// 32 bytes of float32).  A chunk is directly the 8-element operand of the
// left contraction (reduction over rows, columns as output rows); the right
// contraction reduces over columns, so each wave writes its 64 x 32 sub-tile
// into a private LDS tile row-major and reads 8 consecutive columns of a row
// per operand.  KR_R rows of the next step are built cooperatively in LDS
// (split into hi / lo); KR_L rows of the block are built once into
// registers.  Partials and the cross-wave reduction of the left product are
// as in the float32 MFMA kernel.
#include "cpg_internal.h"

namespace cpg {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned short v8us __attribute__((ext_vector_type(8)));

constexpr int kB16Rows = 256;
constexpr int kB16Step = 32;
constexpr int kTrLd = 40;   // bf16 elements per row of the transposed LDS tile (80 bytes)
constexpr int kKrLd = 40;   // bf16 elements per rank row of the KR_R tile

// float -> bf16 bits, round to nearest even
__device__ __forceinline__ unsigned short bf16_rne(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short b) { return __uint_as_float(((unsigned int)b) << 16); }

__device__ __forceinline__ float kr_prod_f(const FacSet<float>& fs, int first, int count, int64_t idx, int r) {
    float v = 1.f;
    for (int m = 0; m < count; ++m) {
        const int64_t d = fs.dims[first + m];
        const int64_t q = idx / d;
        const int64_t i = idx - q * d;
        idx = q;
        v *= fs.A[first + m][i * fs.R + r];
    }
    return v;
}

__device__ __forceinline__ void lds_wave_sync_b() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ v8bf as_bf(v8us u) { return __builtin_bit_cast(v8bf, u); }

// TYF: true if Y is stored as float32 (hi/lo split in registers), false for bf16 storage.
template <bool TYF, int NRT, bool DO_R, bool DO_L, bool REFINE>
__global__ __launch_bounds__(256) void k_contract_bf16(const void* __restrict__ Yv, int64_t J, int64_t K,
                                                        FacSet<float> fs, int nstar, int64_t kcols, int ld,
                                                        float* __restrict__ PRpart, float* __restrict__ PLpart) {
    constexpr int RT = NRT * 16;
    constexpr bool YLO = TYF && REFINE;   // a Y_lo term exists
    constexpr bool KLO = REFINE;          // a KR_lo term exists
    __shared__ __attribute__((aligned(16))) unsigned short sKR[DO_R ? 2 : 1][KLO ? 2 : 1][DO_R ? RT * kKrLd : 8];
    __shared__ __attribute__((aligned(16))) unsigned short sTr[DO_R ? 4 : 1][YLO ? 2 : 1][DO_R ? 64 * kTrLd : 8];
    __shared__ v4f sRed[DO_L ? 2 : 1][DO_L ? 4 * 2 * NRT * 64 : 1];

    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int l = tid & 63;
    const int q = l >> 4;
    const int c16 = l & 15;
    const int R = fs.R;
    const int N = fs.N;
    const int64_t jb = (int64_t)blockIdx.x * kB16Rows;
    const int64_t jw = jb + 64 * w;
    const int64_t k_begin = (int64_t)blockIdx.y * kcols;
    const int64_t k_end = min(K, k_begin + kcols);
    const int64_t nsteps = (k_end - k_begin + kB16Step - 1) / kB16Step;

    // KR_L operand of the left product: rows jw + 32*jc + 8q + t, rank rt*16 + c16
    v8us krl_hi[DO_L ? 2 : 1][DO_L ? NRT : 1], krl_lo[DO_L && KLO ? 2 : 1][DO_L && KLO ? NRT : 1];
    if (DO_L) {
#pragma unroll
        for (int jc = 0; jc < 2; ++jc)
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt) {
                const int r = rt * 16 + c16;
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int64_t j = jw + 32 * jc + 8 * q + t;
                    const float v = (j < J && r < R) ? kr_prod_f(fs, 0, nstar, j, r) : 0.f;
                    const unsigned short h = bf16_rne(v);
                    krl_hi[jc][rt][t] = h;
                    if (KLO) krl_lo[DO_L && KLO ? jc : 0][DO_L && KLO ? rt : 0][t] = bf16_rne(v - bf16_to_f(h));
                }
            }
    }

    auto build_krr = [&](int buf, int64_t k0) {
        for (int e = tid; e < kB16Step * RT; e += 256) {
            const int r = e / kB16Step, kk = e - (e / kB16Step) * kB16Step;
            const int64_t k = k0 + kk;
            const float v = (k < k_end && r < R) ? kr_prod_f(fs, nstar, N - nstar, k, r) : 0.f;
            const unsigned short h = bf16_rne(v);
            sKR[buf][0][r * kKrLd + kk] = h;
            if (KLO) sKR[buf][KLO ? 1 : 0][r * kKrLd + kk] = bf16_rne(v - bf16_to_f(h));
        }
    };

    // chunk s of a step: column k0 + 16*(s&1) + c16, rows jw + 32*(s>>1) + 8q .. +7
    const int64_t rbase = jw + 8 * q;
    auto load_step = [&](v8us* hi, v8us* lo, int64_t k0) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int64_t k = k0 + 16 * (s & 1) + c16;
            const int64_t row = rbase + 32 * (s >> 1);
            const bool ok = row < J && k < k_end;   // J % 8 == 0: a chunk is all in or all out
            if (TYF) {
                const float* Y = (const float*)Yv;
                v4f a = v4f{0.f, 0.f, 0.f, 0.f}, b = a;
                if (ok) {
                    a = *(const v4f*)(Y + k * J + row);
                    b = *(const v4f*)(Y + k * J + row + 4);
                }
                const float x[8] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const unsigned short h = bf16_rne(x[t]);
                    hi[s][t] = h;
                    if (YLO) lo[s][t] = bf16_rne(x[t] - bf16_to_f(h));
                }
            } else {
                const unsigned short* Y = (const unsigned short*)Yv;
                hi[s] = ok ? *(const v8us*)(Y + k * J + row) : v8us{0, 0, 0, 0, 0, 0, 0, 0};
            }
        }
    };

    v4f accR[DO_R ? 4 : 1][DO_R ? NRT : 1];
#pragma unroll
    for (int e = 0; e < (DO_R ? 4 : 1); ++e)
#pragma unroll
        for (int rt = 0; rt < (DO_R ? NRT : 1); ++rt) accR[e][rt] = v4f{0.f, 0.f, 0.f, 0.f};

    if (DO_R) build_krr(0, k_begin);
    v8us cur_hi[4], cur_lo[4], nxt_hi[4], nxt_lo[4];
    load_step(cur_hi, cur_lo, k_begin);
    __syncthreads();

    for (int64_t st = 0; st < nsteps; ++st) {
        const int64_t k0 = k_begin + st * kB16Step;
        const int buf = (int)(st & 1);
        if (st + 1 < nsteps) load_step(nxt_hi, nxt_lo, k0 + kB16Step);

        if (DO_L) {
            // left product: columns k0 + 16*kt + c16 are the output rows, rows are reduced
            v4f accL[2][NRT];
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) {
                    v4f a = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int jc = 0; jc < 2; ++jc) {
                        const int s = 2 * jc + kt;
                        a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(cur_hi[s]), as_bf(krl_hi[jc][rt]), a, 0, 0, 0);
                        if (KLO)
                            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                as_bf(cur_hi[s]), as_bf(krl_lo[DO_L && KLO ? jc : 0][DO_L && KLO ? rt : 0]), a, 0, 0, 0);
                        if (YLO)
                            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(cur_lo[s]), as_bf(krl_hi[jc][rt]), a, 0, 0, 0);
                    }
                    accL[kt][rt] = a;
                }
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) sRed[buf][((w * 2 + kt) * NRT + rt) * 64 + l] = accL[kt][rt];
        }
        if (DO_R) {
            // transpose through this wave's LDS tile: row (32*jc + 8q + t), column (16*kt + c16)
#pragma unroll
            for (int part = 0; part < (YLO ? 2 : 1); ++part) {
                unsigned short* T = sTr[w][YLO ? part : 0];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const v8us v = part == 0 ? cur_hi[s] : cur_lo[s];
                    const int col = 16 * (s & 1) + c16;
                    const int row0 = 32 * (s >> 1) + 8 * q;
#pragma unroll
                    for (int t = 0; t < 8; ++t) T[(row0 + t) * kTrLd + col] = v[t];
                }
            }
            lds_wave_sync_b();
            // right product: rows 16*rr + c16 (output), columns 8q .. 8q+7 (reduced)
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt) {
                const v8us bh = *(const v8us*)(&sKR[buf][0][(rt * 16 + c16) * kKrLd + 8 * q]);
                v8us bl;
                if (KLO) bl = *(const v8us*)(&sKR[buf][KLO ? 1 : 0][(rt * 16 + c16) * kKrLd + 8 * q]);
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const v8us ah = *(const v8us*)(&sTr[w][0][(16 * rr + c16) * kTrLd + 8 * q]);
                    accR[rr][rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ah), as_bf(bh), accR[rr][rt], 0, 0, 0);
                    if (KLO)
                        accR[rr][rt] =
                            __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(ah), as_bf(bl), accR[rr][rt], 0, 0, 0);
                    if (YLO) {
                        const v8us al = *(const v8us*)(&sTr[w][YLO ? 1 : 0][(16 * rr + c16) * kTrLd + 8 * q]);
                        accR[rr][rt] =
                            __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(al), as_bf(bh), accR[rr][rt], 0, 0, 0);
                    }
                }
            }
        }
        if (DO_R && st + 1 < nsteps) build_krr(buf ^ 1, k0 + kB16Step);
        __syncthreads();
        if (DO_L) {
            for (int e = tid; e < 2 * NRT * 64; e += 256) {
                const int lane = e & 63;
                const int rt = (e >> 6) % NRT;
                const int kt = (e >> 6) / NRT;
                v4f s = sRed[buf][((0 * 2 + kt) * NRT + rt) * 64 + lane];
#pragma unroll
                for (int ww = 1; ww < 4; ++ww) s += sRed[buf][((ww * 2 + kt) * NRT + rt) * 64 + lane];
                const int r = rt * 16 + (lane & 15);
                if (r < ld) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int64_t k = k0 + kt * 16 + 4 * (lane >> 4) + v;
                        if (k < k_end) PLpart[((int64_t)blockIdx.x * K + k) * ld + r] = s[v];
                    }
                }
            }
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            cur_hi[s] = nxt_hi[s];
            if (YLO) cur_lo[s] = nxt_lo[s];
        }
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
                        if (j < J) PRpart[((int64_t)blockIdx.y * J + j) * ld + r] = accR[rr][rt][v];
                    }
                }
            }
    }
}

template <bool TYF, int NRT, bool REFINE>
static hipError_t launch_b16_roles(const void* Y, int64_t J, int64_t K, const FacSet<float>& fs, int nstar,
                                   const Tiling& t, int roles, const MfmaBufs& o, hipStream_t s) {
    dim3 grid((unsigned)t.n_jr, (unsigned)t.n_kc);
    const int64_t kcols = t.ktb * kB16Step;
    if (roles == 3)
        hipLaunchKernelGGL((k_contract_bf16<TYF, NRT, true, true, REFINE>), grid, dim3(256), 0, s, Y, J, K, fs, nstar,
                           kcols, o.ld, o.PRpart, o.PLpart);
    else if (roles == 1)
        hipLaunchKernelGGL((k_contract_bf16<TYF, NRT, true, false, REFINE>), grid, dim3(256), 0, s, Y, J, K, fs,
                           nstar, kcols, o.ld, o.PRpart, o.PLpart);
    else if (roles == 2)
        hipLaunchKernelGGL((k_contract_bf16<TYF, NRT, false, true, REFINE>), grid, dim3(256), 0, s, Y, J, K, fs,
                           nstar, kcols, o.ld, o.PRpart, o.PLpart);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <bool TYF, bool REFINE>
static hipError_t launch_b16_nrt(const void* Y, int64_t J, int64_t K, const FacSet<float>& fs, int nstar,
                                 const Tiling& t, int roles, const MfmaBufs& o, hipStream_t s) {
    switch (t.rt) {
        case 16: return launch_b16_roles<TYF, 1, REFINE>(Y, J, K, fs, nstar, t, roles, o, s);
        case 32: return launch_b16_roles<TYF, 2, REFINE>(Y, J, K, fs, nstar, t, roles, o, s);
        case 48: return launch_b16_roles<TYF, 3, REFINE>(Y, J, K, fs, nstar, t, roles, o, s);
        case 64: return launch_b16_roles<TYF, 4, REFINE>(Y, J, K, fs, nstar, t, roles, o, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_contract_bf16(int ydt, int mode, const void* Y, int64_t J, int64_t K, const FacSet<float>& fs,
                                int nstar, const Tiling& t, int roles, const MfmaBufs& o, hipStream_t stream) {
    if ((J % 8) != 0) return hipErrorInvalidValue;
    const bool refine = mode == CPG_MODE_BF16_REFINED;
    if (ydt == CPG_F32)
        return refine ? launch_b16_nrt<true, true>(Y, J, K, fs, nstar, t, roles, o, stream)
                      : launch_b16_nrt<true, false>(Y, J, K, fs, nstar, t, roles, o, stream);
    if (ydt == CPG_BF16)
        return refine ? launch_b16_nrt<false, true>(Y, J, K, fs, nstar, t, roles, o, stream)
                      : launch_b16_nrt<false, false>(Y, J, K, fs, nstar, t, roles, o, stream);
    return hipErrorInvalidValue;
}

}  // namespace cpg
