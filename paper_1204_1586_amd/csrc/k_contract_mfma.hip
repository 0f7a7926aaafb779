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
// block of P_L is written per step.  The KR_R rows of all of the block's
// column steps are generated once into LDS before the loop and the KR_L rows
// of the block once into registers, so the only global loads inside the loop
// are the Y loads of the steps ahead, which stay in flight across the step's
// MFMAs.  Steps of 32 columns are dealt round-robin over the block columns.
// Partials go to PRpart[block column][J][R] and PLpart[block row][K][R],
// reduced later in a fixed order.
#include "cpg_device.h"
#include "cpg_fastdiv.h"

#include <algorithm>

#include <hip/hip_ext.h>

// Optional timestamps for profiling builds; compiled out by default.
#ifndef CPG_CONTRACT_MARK
#define CPG_CONTRACT_MARK(k)
#endif
#ifndef CPG_CONTRACT_WAVE_MARK
#define CPG_CONTRACT_WAVE_MARK(k)
#endif

namespace cpg {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kMfmaRows = 256;  // rows of Y per block (64 per wave)
constexpr int kStep = 32;       // columns of Y per step
constexpr int kTLd = 68;        // LDS leading dimension of the transposed sub-tile
constexpr int kDepth = 2;       // steps of Y loads in flight ahead of the MFMAs


__device__ __forceinline__ void lds_wave_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

// Block barrier that orders LDS only: it does not wait for global loads in
// flight (the next step's Y), unlike a full __syncthreads() fence.
__device__ __forceinline__ void lds_block_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int NRT, bool DO_R, bool DO_L>
__global__ __launch_bounds__(256) void k_contract_mfma_f32(const float* __restrict__ Y, int64_t J, int64_t K,
                                                            int64_t kcols, int ld, KrGen kg,
                                                            float* __restrict__ PRpart, float* __restrict__ PLpart,
                                                            int fstage) {
    constexpr int RT = NRT * 16;
    constexpr int KRLD = RT + 4;  // LDS row stride of the KR_R tile
    extern __shared__ float sKRR[];  // kcols x KRLD: KR_R rows of this block's column steps, then
                                     // fstage floats of staged factors
    (void)kcols;                     // sizes sKRR (at least 32 x the block's step count)
    __shared__ float sT[DO_L ? 4 : 1][DO_L ? kStep * kTLd : 1];
    __shared__ v4f sRed[DO_L ? 2 : 1][DO_L ? 4 * 2 * NRT * 64 : 1];

    CPG_CONTRACT_MARK(0);
    CPG_CONTRACT_WAVE_MARK(50);
    const int tid = threadIdx.x;
    const int w = tid >> 6;
    const int l = tid & 63;
    const int q = l >> 4;
    const int c16 = l & 15;
    const int64_t jb = (int64_t)blockIdx.x * kMfmaRows;
    const int64_t jw = jb + 64 * w;                 // first row of this wave
    // Steps of 32 columns are dealt round-robin over the block columns: block
    // column by takes global steps by, by + n_kc, by + 2 n_kc, ... (at most
    // kcols / 32 of them), so at any time the grid reads one contiguous window
    // of Y that moves through memory (measured: about 1.4x the bandwidth of
    // giving each block a contiguous chunk of columns).
    const int64_t n_kc = gridDim.y;
    const int64_t gsteps = (K + kStep - 1) / kStep;
    const int64_t nsteps = (gsteps - blockIdx.y + n_kc - 1) / n_kc;
    auto step_col = [&](int64_t st) { return (st * n_kc + blockIdx.y) * kStep; };   // first column of step st

    // Prologue.  The block's Khatri-Rao rows (eq. 3.3, Notation 2.1 order: the
    // first mode of a product fastest) are generated from the factors: row
    // indices unravel into per-mode indices by multiply-shift division, one
    // round of factor loads per mode; factor entries past R read as zero
    // (buffer loads, no branches).  Products are formed in float32 in mode
    // order.  The first steps of Y are issued right after the factor loads of
    // the first rounds, so they are in flight while the rows are formed.
    const int R = kg.R;
    auto fac_rsrc = [&](int m) { return buf_rsrc(kg.A[m], (uint32_t)(kg.fd[m].d * (uint32_t)R * 4)); };
    //
    // KR_L operand of the left contraction: rows jw + 16q + s, columns rt*16 + c16
    float krl[DO_L ? NRT : 1][16];
    // KR_R rows of the block's steps (LDS row st*32 + kk <- column step_col(st) + kk),
    // four ranks per entry; rows past K and ranks past R are zero
    constexpr int kKrBatch = 8;
    constexpr int kPeel = NRT <= 2 ? 2 : 1;   // Khatri-Rao rounds whose loads precede the first Y loads
    const int n4 = (int)(nsteps * kStep) * (RT / 4);
    auto load_krr = [&](v4f (&t)[kKrBatch], int base) {
        uint32_t idx[kKrBatch];
        int r4[kKrBatch];
#pragma unroll
        for (int u = 0; u < kKrBatch; ++u) {
            const int e = base + u * 256 + tid;
            const int kk = e / (RT / 4);
            r4[u] = (e - kk * (RT / 4)) * 4;
            const int64_t k = step_col(kk / kStep) + (kk & (kStep - 1));
            const bool ok = e < n4 && k < K;
            idx[u] = ok ? (uint32_t)k : 0u;
            const float one = ok ? 1.f : 0.f;
            t[u] = v4f{one, one, one, one};
        }
        for (int m = kg.nstar; m < kg.N; ++m) {
            const FastDiv f = kg.fd[m];
            const auto rs = fac_rsrc(m);
#pragma unroll
            for (int u = 0; u < kKrBatch; ++u) {
                const uint32_t qd = fast_div(idx[u], f);
                const uint32_t i = idx[u] - qd * f.d;
                idx[u] = qd;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const int r = r4[u] + c;
                    const uint32_t off = r < R ? (i * (uint32_t)R + (uint32_t)r) * 4 : kOOB;
                    t[u][c] *= __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
                }
            }
        }
    };
    // First batch of KR_R rows and the KR_L rows together: round j loads mode j
    // of the left product and mode n*+j of the right one, so the rounds are
    // max(n*, N-n*) (a mode past a side's count multiplies by one).
    auto gen_first = [&](v4f (&t)[kKrBatch], auto&& mid) {
        uint32_t idxL[16], idxR[kKrBatch];
        int r4[kKrBatch];
        if (DO_L) {
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const int64_t j = jw + 16 * q + s;
                idxL[s] = j < J ? (uint32_t)j : 0u;
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) krl[rt][s] = j < J ? 1.f : 0.f;
            }
        }
        if (DO_R) {
#pragma unroll
            for (int u = 0; u < kKrBatch; ++u) {
                const int e = u * 256 + tid;
                const int kk = e / (RT / 4);
                r4[u] = (e - kk * (RT / 4)) * 4;
                const int64_t k = step_col(kk / kStep) + (kk & (kStep - 1));
                const bool ok = e < n4 && k < K;
                idxR[u] = ok ? (uint32_t)k : 0u;
                const float one = ok ? 1.f : 0.f;
                t[u] = v4f{one, one, one, one};
            }
        }
        const int nL = DO_L ? kg.nstar : 0;
        const int nR = DO_R ? kg.N - kg.nstar : 0;
        const int rounds = nL > nR ? nL : nR;
        // factor loads of round j (a mode past a side's count reads zero here and
        // multiplies by one below)
        auto issue = [&](int j, float (&vl)[DO_L ? NRT : 1][16], float (&vr)[DO_R ? kKrBatch : 1][4]) {
            const bool aL = j < nL, aR = j < nR;
            if (DO_L) {
                const int m = aL ? j : 0;
                const FastDiv f = kg.fd[m];
                const auto rs = fac_rsrc(m);
#pragma unroll
                for (int s = 0; s < 16; ++s) {
                    const uint32_t qd = fast_div(idxL[s], f);
                    const uint32_t i = idxL[s] - qd * f.d;
                    idxL[s] = qd;
#pragma unroll
                    for (int rt = 0; rt < NRT; ++rt) {
                        const int r = rt * 16 + c16;
                        const uint32_t off = (aL && r < R) ? (i * (uint32_t)R + (uint32_t)r) * 4 : kOOB;
                        vl[rt][s] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
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
            if (DO_L) {
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt)
#pragma unroll
                    for (int s = 0; s < 16; ++s) krl[rt][s] *= aL ? vl[rt][s] : 1.f;
            }
            if (DO_R) {
#pragma unroll
                for (int u = 0; u < kKrBatch; ++u)
#pragma unroll
                    for (int c = 0; c < 4; ++c) t[u][c] *= aR ? vr[u][c] : 1.f;
            }
        };
        // The first kPeel rounds are issued before the first steps of Y, so that
        // waiting for them does not wait for Y as well (loads complete in order
        // for the wait counter); later rounds, if any, load and multiply in turn.
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
    };
    auto store_krr = [&](const v4f (&t)[kKrBatch], int base) {
#pragma unroll
        for (int u = 0; u < kKrBatch; ++u) {
            const int e = base + u * 256 + tid;
            const int kk = e / (RT / 4), r4 = (e - kk * (RT / 4)) * 4;
            if (e < n4) *(v4f*)(sKRR + kk * KRLD + r4) = t[u];
        }
    };

    // The same rows from factors staged in LDS (fstage > 0): every factor is
    // copied by LDS-DMA loads of 64 floats per wave instruction (each factor's
    // region rounded up to 64 floats), so the rows need no scattered global
    // loads.  Mode m's factor sits at the sum of the rounded sizes before it.
    float* sFac = sKRR + (DO_R ? kcols * KRLD : 0);
    auto stage_factors = [&]() {
        int fb = 0;
        for (int m = 0; m < kg.N; ++m) {
            const int sz = (int)kg.fd[m].d * R;
            const int nch = (sz + 63) >> 6;
            const float* Am = kg.A[m];
            for (int c = w; c < nch; c += 4) {
                const int e = min(c * 64 + l, sz - 1);
                __builtin_amdgcn_global_load_lds((const void*)(Am + e),
                                                 (__attribute__((address_space(3))) void*)(sFac + fb + c * 64), 4, 0, 0);
            }
            fb += nch * 64;
        }
    };
    // One Khatri-Rao row from the staged factors, formed by one thread: its
    // index unravels into the indices of modes m0 .. m1-1 with one division per
    // mode, and the RT products (float32, mode order) read whole factor rows
    // from LDS.  Ranks past R and a row index past `lim` give zeros.
    auto kr_row_lds = [&](float (&v)[RT], int64_t row, int64_t lim, int m0, int m1) {
        const bool ok = row < lim;
#pragma unroll
        for (int r = 0; r < RT; ++r) v[r] = ok && r < R ? 1.f : 0.f;
        uint32_t idx = ok ? (uint32_t)row : 0u;
        int fb = 0;
        for (int m = 0; m < m0; ++m) fb += (((int)kg.fd[m].d * R + 63) >> 6) << 6;
        for (int m = m0; m < m1; ++m) {
            const FastDiv f = kg.fd[m];
            const uint32_t qd = fast_div(idx, f);
            const float* Fr = sFac + fb + (int)(idx - qd * f.d) * R;
            idx = qd;
            // all RT entries read (past R: the next row, or the slack after
            // the staged factors), those past R replaced by zero
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const float x = Fr[r];
                v[r] *= r < R ? x : 0.f;
            }
            fb += (((int)f.d * R + 63) >> 6) << 6;
        }
    };
    // A KR_L row and a KR_R row formed together: round j reads mode j of the
    // left product and mode n*+j of the right one before multiplying either,
    // so the LDS round trips of the two rows overlap (both divisors are read
    // before either row's LDS reads, whose wait would otherwise include them).
    // The products are those of kr_row_lds, in the same order.
    auto rows_paired = [&](float (&vl)[RT], int64_t rowL, float (&vr)[RT], int64_t rowR, bool doL) {
        const bool okL = rowL < J, okR = rowR < K;
#pragma unroll
        for (int r = 0; r < RT; ++r) {
            vl[r] = okL && r < R ? 1.f : 0.f;
            vr[r] = okR && r < R ? 1.f : 0.f;
        }
        uint32_t iL = okL ? (uint32_t)rowL : 0u, iR = okR ? (uint32_t)rowR : 0u;
        int fbL = 0, fbR = 0;
        for (int m = 0; m < kg.nstar; ++m) fbR += (((int)kg.fd[m].d * R + 63) >> 6) << 6;
        const int nL = doL ? kg.nstar : 0, nR = kg.N - kg.nstar;
        const int rounds = nL > nR ? nL : nR;
        // one path for every R (a branch here makes the compiler wait for all
        // LDS reads where the paths join): all RT entries, past R zero
        auto read_row = [&](float (&x)[RT], const float* Fr) {
#pragma unroll
            for (int r = 0; r < RT; ++r) {
                const float y = Fr[r];
                x[r] = r < R ? y : 0.f;
            }
        };
        for (int j = 0; j < rounds; ++j) {
            const bool aL = j < nL, aR = j < nR;
            const FastDiv fL = kg.fd[aL ? j : 0], fR = kg.fd[kg.nstar + (aR ? j : 0)];
            const uint32_t qL = fast_div(iL, fL), qR = fast_div(iR, fR);
            int oL = fbL + (int)(iL - qL * fL.d) * R, oR = fbR + (int)(iR - qR * fR.d) * R;
            // both offsets formed here, before the first LDS read of the round
            asm volatile("" : "+v"(oL), "+v"(oR));
            float xl[RT], xr[RT];
            if (aL) {
                read_row(xl, sFac + oL);
                iL = qL;
            }
            if (aR) {
                read_row(xr, sFac + oR);
                iR = qR;
            }
            if (aL) {
#pragma unroll
                for (int r = 0; r < RT; ++r) vl[r] *= xl[r];
                fbL += (((int)fL.d * R + 63) >> 6) << 6;
            }
            if (aR) {
#pragma unroll
                for (int r = 0; r < RT; ++r) vr[r] *= xr[r];
                fbR += (((int)fR.d * R + 63) >> 6) << 6;
            }
        }
    };
    auto store_krr_row = [&](const float (&v)[RT], int kk) {
#pragma unroll
        for (int g = 0; g < RT / 4; ++g)
            *(v4f*)(sKRR + kk * KRLD + 4 * g) = v4f{v[4 * g], v[4 * g + 1], v[4 * g + 2], v[4 * g + 3]};
    };
    // The block's Khatri-Rao rows from the staged factors, one row per thread
    // and pass: KR_R rows of the block's steps into LDS; up to 32 ranks, lane l
    // also forms its wave's KR_L row jw + l (paired with its first KR_R row)
    // into the wave's transpose area (free until the first step), and every
    // lane then reads its MFMA operand from there.  Wider tiles: each lane
    // forms its own KR_L operand entries, one division per row, mode and entry.
    auto form_rows = [&]() {
        constexpr bool kLRow = DO_L && NRT <= 2;
        constexpr int LD = RT + 1;   // odd stride: the operand reads hit distinct banks
        static_assert(!kLRow || 64 * LD <= kStep * kTLd, "a wave's Khatri-Rao rows fit its transpose area");
        const int nrow = DO_R ? (int)(nsteps * kStep) : 0;
        int kk = tid;
        if constexpr (DO_R) {
            float vl[RT], vr[RT];
            rows_paired(vl, kLRow ? jw + l : J, vr, kk < nrow ? step_col(kk / kStep) + (kk & (kStep - 1)) : K,
                        kLRow);
            if (kk < nrow) store_krr_row(vr, kk);
            if constexpr (kLRow) {
#pragma unroll
                for (int r = 0; r < RT; ++r) sT[w][l * LD + r] = vl[r];
            }
            kk += 256;
        } else if constexpr (kLRow) {
            float v[RT];
            kr_row_lds(v, jw + l, J, 0, kg.nstar);
#pragma unroll
            for (int r = 0; r < RT; ++r) sT[w][l * LD + r] = v[r];
        }
        for (; kk < nrow; kk += 256) {
            float v[RT];
            kr_row_lds(v, step_col(kk / kStep) + (kk & (kStep - 1)), K, kg.nstar, kg.N);
            store_krr_row(v, kk);
        }
        if constexpr (kLRow) {
            lds_wave_sync();
#pragma unroll
            for (int s = 0; s < 16; ++s)
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) krl[rt][s] = sT[w][(16 * q + s) * LD + rt * 16 + c16];
        } else if constexpr (DO_L) {
            uint32_t idxL[16];
#pragma unroll
            for (int s = 0; s < 16; ++s) {
                const int64_t j = jw + 16 * q + s;
                idxL[s] = j < J ? (uint32_t)j : 0u;
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) krl[rt][s] = j < J ? 1.f : 0.f;
            }
            int fb = 0;
            for (int m = 0; m < kg.nstar; ++m) {
                const FastDiv f = kg.fd[m];
                const float* Fm = sFac + fb;
#pragma unroll
                for (int s = 0; s < 16; ++s) {
                    const uint32_t qd = fast_div(idxL[s], f);
                    const uint32_t i = idxL[s] - qd * f.d;
                    idxL[s] = qd;
#pragma unroll
                    for (int rt = 0; rt < NRT; ++rt) {
                        const int r = rt * 16 + c16;
                        const float x = Fm[i * R + min(r, R - 1)];
                        krl[rt][s] *= r < R ? x : 0.f;
                    }
                }
                fb += (((int)f.d * R + 63) >> 6) << 6;
            }
        }
    };

    // Y loads: lane (q, c16), slot c -> rows jw + 4*c16 .. +3 of column
    // step_col(st) + 4c + q, through a buffer resource over the step's 32
    // columns: columns past K, steps past the block's last one and rows past
    // J (lane offset kOOB) read as zero.
    const uint32_t lane_off = (jw + 4 * c16) < J ? (uint32_t)((jw + 4 * c16) * 4) : kOOB;
    const uint32_t col_bytes = (uint32_t)(J * 4);
    auto load_step = [&](v4f (&dst)[8], int64_t st) {
        const int64_t k0 = step_col(st);
        const int64_t ncol = st < nsteps ? max((int64_t)0, min((int64_t)kStep, K - k0)) : 0;
        const auto yrs = buf_rsrc(Y + (st < nsteps ? k0 : 0) * J, (uint32_t)(ncol * J * 4));
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint32_t off = lane_off + (uint32_t)(4 * c + q) * col_bytes;
            dst[c] = __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(yrs, (int)off, 0, 0));
        }
    };

    v4f accR[DO_R ? 4 : 1][DO_R ? NRT : 1];
#pragma unroll
    for (int e = 0; e < (DO_R ? 4 : 1); ++e)
#pragma unroll
        for (int rt = 0; rt < (DO_R ? NRT : 1); ++rt) accR[e][rt] = v4f{0.f, 0.f, 0.f, 0.f};

    // one step: MFMAs on `cur` (columns st*32 ..) while `nxt` receives step
    // st + kDepth; steps st + 1 .. st + kDepth - 1 are already in flight
    auto step = [&](v4f (&cur)[8], v4f (&nxt)[8], int64_t st) {
        const int buf = (int)(st & 1);
        CPG_CONTRACT_MARK(2 + 4 * st);
        load_step(nxt, st + kDepth);
        __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the step's MFMAs
        if (DO_R) {
            // P_R rows {4i + e} += Y(rows, k0 .. k0+31) KR_R(k0 .. k0+31, :)
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                float b[NRT];
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) b[rt] = sKRR[(st * kStep + 4 * c + q) * KRLD + rt * 16 + c16];
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int rt = 0; rt < NRT; ++rt)
                        accR[e][rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(cur[c][e], b[rt], accR[e][rt], 0, 0, 0);
            }
        }
        CPG_CONTRACT_MARK(3 + 4 * st);
        if (DO_L) {
            // transpose this wave's 64 x 32 sub-tile through its private LDS region
            float* T = sT[w];
#pragma unroll
            for (int c = 0; c < 8; ++c) *(v4f*)(T + (4 * c + q) * kTLd + 4 * c16) = cur[c];
            lds_wave_sync();
            // both 16-column halves of the step at once, so the two dependent
            // MFMA chains interleave
            v4f tl[2][4];
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
#pragma unroll
                for (int sg = 0; sg < 4; ++sg) tl[kt][sg] = *(const v4f*)(T + (kt * 16 + c16) * kTLd + 16 * q + 4 * sg);
            v4f accL[2][NRT];
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) accL[kt][rt] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 16; ++s)
#pragma unroll
                for (int kt = 0; kt < 2; ++kt)
#pragma unroll
                    for (int rt = 0; rt < NRT; ++rt)
                        accL[kt][rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(tl[kt][s >> 2][s & 3], krl[rt][s],
                                                                           accL[kt][rt], 0, 0, 0);
            // this wave's partial: lane holds columns k0 + kt*16 + 4q + v, rank rt*16 + c16
#pragma unroll
            for (int kt = 0; kt < 2; ++kt)
#pragma unroll
                for (int rt = 0; rt < NRT; ++rt) sRed[buf][((w * 2 + kt) * NRT + rt) * 64 + l] = accL[kt][rt];
            CPG_CONTRACT_MARK(4 + 4 * st);
            lds_block_sync();
            // P_L partial stores of this block row over the step's columns (past K: dropped)
            const int64_t k0 = step_col(st);
            const auto lrs = buf_rsrc(PLpart + ((int64_t)blockIdx.x * K + k0) * ld,
                                      (uint32_t)(max((int64_t)0, min((int64_t)kStep, K - k0)) * ld * 4));
            // sum the four waves and write this block row's partial of P_L: every
            // thread stores 2*NRT values (uniform count, so the wait for the next
            // step's Y loads stays exact)
#pragma unroll
            for (int j = 0; j < NRT; ++j) {
                const int item = j * 128 + (tid >> 1);  // (kt, rt, lane) of the wave partials
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
            CPG_CONTRACT_MARK(5 + 4 * st);
        }
    };

    // kDepth + 1 register buffers rotate through the unrolled loop (no copies,
    // so the loads of the kDepth steps ahead stay in flight)
    constexpr int NB = kDepth + 1;
    v4f buf[NB][8];
    if (fstage > 0) {
        // staged factors first (their wait must not include Y), then the first
        // steps of Y, which stay in flight while the rows are formed
        stage_factors();
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the staging loads
        CPG_CONTRACT_WAVE_MARK(54);
        __syncthreads();
        CPG_CONTRACT_MARK(40);
#pragma unroll
        for (int d = 0; d < kDepth; ++d) load_step(buf[d], d);
        CPG_CONTRACT_MARK(41);
        form_rows();
        CPG_CONTRACT_MARK(42);
    } else {
        v4f krt[kKrBatch];
        gen_first(krt, [&] {
#pragma unroll
            for (int d = 0; d < kDepth; ++d) load_step(buf[d], d);
        });
        if (DO_R) store_krr(krt, 0);
        for (int base = kKrBatch * 256; DO_R && base < n4; base += kKrBatch * 256) {  // wide chunks only
            load_krr(krt, base);
            store_krr(krt, base);
        }
    }
    lds_block_sync();
    CPG_CONTRACT_MARK(1);
    for (int64_t st = 0; st < nsteps; st += NB) {
#pragma unroll
        for (int ph = 0; ph < NB; ++ph)
            if (ph == 0 || st + ph < nsteps) step(buf[ph], buf[(ph + kDepth) % NB], st + ph);
    }

    CPG_CONTRACT_MARK(60);
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
                        if (j < J) store_through(&PRpart[((int64_t)blockIdx.y * J + j) * ld + r], accR[e][rt][v]);
                    }
                }
            }
    }

}

bool mfma_supported(int ydt, int fdt, int mode, int R) {
    (void)R;
    return ydt == CPG_F32 && fdt == CPG_F32 && mode == CPG_MODE_NATIVE;
}

// LDS of one block: static transpose/reduction buffers plus the dynamic KR_R
// chunk (kcols rows of RT + 4 floats) and the staged factors.
static constexpr int64_t static_lds(int nrt, bool do_l) {
    return do_l ? (int64_t)4 * kStep * kTLd * 4 + (int64_t)2 * 4 * 2 * nrt * 64 * 16 : 0;
}
constexpr int64_t kLdsPerCu = 160 * 1024;

int64_t mfma_f32_max_cols(int rt, int roles, int64_t fac_stage) {
    const int nrt = rt / 16;
    const int64_t row = (int64_t)(rt + 4) * 4;
    // staged factors plus one rank tile of slack after them (rows are read
    // whole, up to RT floats past a factor's last row)
    const int64_t st = static_lds(nrt, (roles & 2) != 0) + (fac_stage > 0 ? (fac_stage + rt) * 4 : 0);
    // one block per CU (the tiling targets one long-running block per CU)
    const int64_t budget = kLdsPerCu - st;
    return std::max<int64_t>(kStep, (budget / row) / kStep * kStep);
}

template <int NRT, bool DO_R, bool DO_L>
static hipError_t launch_one(dim3 grid, const float* Y, int64_t J, int64_t K, int64_t kcols, const MfmaBufs& o,
                             hipStream_t s) {
    auto kern = k_contract_mfma_f32<NRT, DO_R, DO_L>;
    const size_t dyn = (DO_R ? (size_t)kcols * (NRT * 16 + 4) * sizeof(float) : 0) +
                       (o.fac_stage > 0 ? (size_t)(o.fac_stage + NRT * 16) * 4 : 0);
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(kLdsPerCu - static_lds(NRT, DO_L)));
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    if (o.ev0)
        hipExtLaunchKernelGGL(kern, grid, dim3(256), (uint32_t)dyn, s, o.ev0, o.ev1, 0u, Y, J, K, kcols, o.ld, o.kg,
                              o.PRpart, o.PLpart, o.fac_stage);
    else
        hipLaunchKernelGGL(kern, grid, dim3(256), dyn, s, Y, J, K, kcols, o.ld, o.kg, o.PRpart, o.PLpart, o.fac_stage);
    return hipGetLastError();
}

template <int NRT>
static hipError_t launch_nrt(const float* Y, int64_t J, int64_t K, const Tiling& t, int roles, const MfmaBufs& o,
                             hipStream_t s) {
    dim3 grid((unsigned)t.n_jr, (unsigned)t.n_kc);
    const int64_t kcols = t.ktb * kStep;
    if (kcols > mfma_f32_max_cols(NRT * 16, roles, o.fac_stage) || o.fac_stage < 0 || o.fac_stage > kFacStageMax)
        return hipErrorInvalidValue;
    if (roles == 3) return launch_one<NRT, true, true>(grid, Y, J, K, kcols, o, s);
    if (roles == 1) return launch_one<NRT, true, false>(grid, Y, J, K, kcols, o, s);
    if (roles == 2) return launch_one<NRT, false, true>(grid, Y, J, K, kcols, o, s);
    return hipErrorInvalidValue;
}

hipError_t launch_contract_mfma(int ydt, int mode, const void* Y, int64_t J, int64_t K, const Tiling& t, int roles,
                                const MfmaBufs& o, hipStream_t stream) {
    if (ydt != CPG_F32 || mode != CPG_MODE_NATIVE || (J % 4) != 0) return hipErrorInvalidValue;
    switch (t.rt) {
        case 16: return launch_nrt<1>((const float*)Y, J, K, t, roles, o, stream);
        case 32: return launch_nrt<2>((const float*)Y, J, K, t, roles, o, stream);
        case 48: return launch_nrt<3>((const float*)Y, J, K, t, roles, o, stream);
        case 64: return launch_nrt<4>((const float*)Y, J, K, t, roles, o, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace cpg
