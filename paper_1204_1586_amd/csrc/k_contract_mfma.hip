// Matrix-core (MFMA) big contraction of Algorithm 2, steps 4 and 7, for
// float32 tensors: both partial products of the free J x K view Y_(1:n*)
// (eq. 2.3) against Khatri-Rao blocks (eq. 3.3, Notation 2.1):
//   right: P_R(j, r) = sum_k Y(j, k) KR_R(k, r)      (eq. 3.10)
//   left : P_L(r, k) = sum_j KR_L(j, r) Y(j, k)      (eq. 3.9)
//
// Block = 4 waves, 256 rows of Y (64 per wave) x a chunk of columns, walked in
// steps of 32 columns.  Per step each lane loads eight float4 of Y (each 16
// lanes read 256 contiguous bytes of one column).  Element e of those float4
// is directly the A operand of a 16x16x4 f32 MFMA whose 16 output rows are
// {4i + e}: the right contraction needs no LDS for Y.  The left contraction
// reduces over rows, so each wave transposes its own 64 x 32 sub-tile
// through a private LDS region and runs 16x16x4 MFMAs with the columns as
// output rows; the four waves' partial sums meet in LDS and one partial row
// block of P_L is written per step.  KR_R rows for the next step are built
// cooperatively in LDS (double buffer, one block barrier per step); KR_L
// rows of the block are built once into registers.  Partials go to
// PRpart[block column][J][R] and PLpart[block row][K][R], reduced later in a
// fixed order.
#include "cpg_internal.h"

namespace cpg {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kMfmaRows = 256;  // rows of Y per block (64 per wave)
constexpr int kStep = 32;       // columns of Y per step
constexpr int kTLd = 68;        // LDS leading dimension of the transposed sub-tile

__device__ __forceinline__ float kr_prod(const FacSet<float>& fs, int first, int count, int64_t idx, int r) {
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

__device__ __forceinline__ void lds_wave_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

template <int NRT, bool DO_R, bool DO_L>
__global__ __launch_bounds__(256) void k_contract_mfma_f32(const float* __restrict__ Y, int64_t J, int64_t K,
                                                            FacSet<float> fs, int nstar, int64_t kcols, int ld,
                                                            float* __restrict__ PRpart, float* __restrict__ PLpart) {
    constexpr int RT = NRT * 16;
    constexpr int KRLD = RT + 4;  // LDS row stride of the KR_R tile
    __shared__ float sKRR[DO_R ? 2 : 1][DO_R ? kStep * KRLD : 1];
    __shared__ float sT[DO_L ? 4 : 1][DO_L ? kStep * kTLd : 1];
    __shared__ v4f sRed[DO_L ? 2 : 1][DO_L ? 4 * 2 * NRT * 64 : 1];

    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int l = tid & 63;
    const int q = l >> 4;
    const int c16 = l & 15;
    const int R = fs.R;
    const int N = fs.N;
    const int64_t jb = (int64_t)blockIdx.x * kMfmaRows;
    const int64_t jw = jb + 64 * w;                 // first row of this wave
    const int64_t k_begin = (int64_t)blockIdx.y * kcols;
    const int64_t k_end = min(K, k_begin + kcols);
    const int64_t nsteps = (k_end - k_begin + kStep - 1) / kStep;

    // KR_L operand of the left contraction: rows jw + 16q + s, columns rt*16 + c16
    float krl[DO_L ? NRT : 1][16];
    if (DO_L) {
#pragma unroll
        for (int rt = 0; rt < NRT; ++rt) {
            const int r = rt * 16 + c16;
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const int64_t j = jw + 16 * q + s;
                krl[rt][s] = (j < J && r < R) ? kr_prod(fs, 0, nstar, j, r) : 0.f;
            }
        }
    }

    auto build_krr = [&](int buf, int64_t k0) {
        for (int e = tid; e < kStep * RT; e += 256) {
            const int kk = e / RT, r = e - (e / RT) * RT;
            const int64_t k = k0 + kk;
            sKRR[buf][kk * KRLD + r] = (k < k_end && r < R) ? kr_prod(fs, nstar, N - nstar, k, r) : 0.f;
        }
    };

    // Y loads: lane (q, c16), slot c -> rows jw + 4*c16 .. +3 of column k0 + 4c + q
    const bool row_ok = (jw + 4 * c16) < J;  // J % 4 == 0: a float4 is all in or all out
    auto load_step = [&](v4f* dst, int64_t k0) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int64_t k = k0 + 4 * c + q;
            if (row_ok && k < k_end)
                dst[c] = *(const v4f*)(Y + k * J + jw + 4 * c16);
            else
                dst[c] = v4f{0.f, 0.f, 0.f, 0.f};
        }
    };

    v4f accR[DO_R ? 4 : 1][DO_R ? NRT : 1];
#pragma unroll
    for (int e = 0; e < (DO_R ? 4 : 1); ++e)
#pragma unroll
        for (int rt = 0; rt < (DO_R ? NRT : 1); ++rt) accR[e][rt] = v4f{0.f, 0.f, 0.f, 0.f};

    if (DO_R) build_krr(0, k_begin);
    v4f cur[8], nxt[8];
    load_step(cur, k_begin);
    __syncthreads();

    for (int64_t st = 0; st < nsteps; ++st) {
        const int64_t k0 = k_begin + st * kStep;
        const int buf = (int)(st & 1);
        if (st + 1 < nsteps) load_step(nxt, k0 + kStep);

        if (DO_R) {
            // P_R rows {4i + e} += Y(rows, k0 .. k0+31) KR_R(k0 .. k0+31, :)
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                float b[NRT];
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) b[rt] = sKRR[buf][(4 * c + q) * KRLD + rt * 16 + c16];
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int rt = 0; rt < NRT; ++rt)
                        accR[e][rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur[c][e], b[rt], accR[e][rt], 0, 0, 0);
            }
        }
        if (DO_L) {
            // transpose this wave's 64 x 32 sub-tile through its private LDS region
            float* T = sT[w];
#pragma unroll
            for (int c = 0; c < 8; ++c) *(v4f*)(T + (4 * c + q) * kTLd + 4 * c16) = cur[c];
            lds_wave_sync();
            v4f accL[2][NRT];
#pragma unroll
            for (int kt = 0; kt < 2; ++kt) {
                v4f tl[4];
#pragma unroll
                for (int sg = 0; sg < 4; ++sg) tl[sg] = *(const v4f*)(T + (kt * 16 + c16) * kTLd + 16 * q + 4 * sg);
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) {
                    v4f a = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int s = 0; s < 16; ++s)
                        a = __builtin_amdgcn_mfma_f32_16x16x4f32(tl[s >> 2][s & 3], krl[rt][s], a, 0, 0, 0);
                    accL[kt][rt] = a;
                }
            }
            // this wave's partial: lane holds columns k0 + kt*16 + 4q + v, rank rt*16 + c16
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) sRed[buf][((w * 2 + kt) * NRT + rt) * 64 + l] = accL[kt][rt];
        }
        if (DO_R && st + 1 < nsteps) build_krr(buf ^ 1, k0 + kStep);
        __syncthreads();
        if (DO_L) {
            // sum the four waves and write this block row's partial of P_L
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
        for (int c = 0; c < 8; ++c) cur[c] = nxt[c];
    }

    if (DO_R) {
        // lane holds rows jw + 4*(4q + v) + e, rank rt*16 + c16
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int rt = 0; rt < NRT; ++rt) {
                const int r = rt * 16 + c16;
                if (r < ld) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int64_t j = jw + 4 * (4 * q + v) + e;
                        if (j < J) PRpart[((int64_t)blockIdx.y * J + j) * ld + r] = accR[e][rt][v];
                    }
                }
            }
    }

}

bool mfma_supported(int ydt, int fdt, int mode, int R) {
    (void)R;
    return ydt == CPG_F32 && fdt == CPG_F32 && mode == CPG_MODE_NATIVE;
}

template <int NRT>
static hipError_t launch_nrt(const float* Y, int64_t J, int64_t K, const FacSet<float>& fs, int nstar,
                             const Tiling& t, int roles, const MfmaOut& o, hipStream_t s) {
    dim3 grid((unsigned)t.n_jr, (unsigned)t.n_kc);
    const int64_t kcols = t.ktb * kStep;
    if (roles == 3)
        hipLaunchKernelGGL((k_contract_mfma_f32<NRT, true, true>), grid, dim3(256), 0, s, Y, J, K, fs, nstar, kcols, o.ld,
                           o.PRpart, o.PLpart);
    else if (roles == 1)
        hipLaunchKernelGGL((k_contract_mfma_f32<NRT, true, false>), grid, dim3(256), 0, s, Y, J, K, fs, nstar,
                           kcols, o.ld, o.PRpart, o.PLpart);
    else if (roles == 2)
        hipLaunchKernelGGL((k_contract_mfma_f32<NRT, false, true>), grid, dim3(256), 0, s, Y, J, K, fs, nstar,
                           kcols, o.ld, o.PRpart, o.PLpart);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_contract_mfma(int ydt, int mode, const void* Y, int64_t J, int64_t K, const FacSet<float>& fs,
                                int nstar, const Tiling& t, int roles, const MfmaOut& o, hipStream_t stream) {
    if (ydt != CPG_F32 || mode != CPG_MODE_NATIVE || (J % 4) != 0) return hipErrorInvalidValue;
    switch (t.rt) {
        case 16: return launch_nrt<1>((const float*)Y, J, K, fs, nstar, t, roles, o, stream);
        case 32: return launch_nrt<2>((const float*)Y, J, K, fs, nstar, t, roles, o, stream);
        case 48: return launch_nrt<3>((const float*)Y, J, K, fs, nstar, t, roles, o, stream);
        case 64: return launch_nrt<4>((const float*)Y, J, K, fs, nstar, t, roles, o, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace cpg
