// Generic (vector-ALU) big contraction of Algorithm 2, steps 4 and 7:
//   right: P_R = Y_(1:n*) (A^(N) (.) ... (.) A^(n*+1))        (J x R, eq. 3.10)
//   left : P_L = (A^(n*) (.) ... (.) A^(1))^T Y_(1:n*)          (R x K, eq. 3.9)
// over the free J x K matrix view of vec(Y) (eq. 2.3, Remark 2.1.4).  Used for
// float64 tensors and as the fallback for every other type; the float32 / bf16
// fast path is the MFMA kernel in k_contract_mfma.hip.
//
// One block (256 threads = 4 waves) owns a region of jtiles x 64 rows and
// ktiles x 64 columns.  Each 64x64 tile of Y is loaded once, coalesced along
// the contiguous j direction, into LDS and used by both contractions: the
// right one accumulates the block's rows of P_R over all its columns in
// registers, the left one accumulates each column tile of P_L over the
// block's rows.  Khatri-Rao rows (eq. 3.3) are generated on the fly into LDS
// from the factors and never stored in HBM.  Partial results go to
// PRpart[block column][J][R] and PLpart[block row][K][R]; a fixed-order
// float64 reduction (k_chain.hip) finishes them, so results are deterministic.
#include "cpg_internal.h"

namespace cpg {

template <typename T> __device__ __forceinline__ T load_y(const T* p) { return *p; }
__device__ __forceinline__ float load_bf16(const uint16_t* p) {
    return __uint_as_float(((uint32_t)(*p)) << 16);
}

template <typename TY, typename TC> struct YLoad;
template <> struct YLoad<double, double> {
    static __device__ __forceinline__ double get(const double* p) { return *p; }
};
template <> struct YLoad<float, float> {
    static __device__ __forceinline__ float get(const float* p) { return *p; }
};
template <> struct YLoad<uint16_t, float> {
    static __device__ __forceinline__ float get(const uint16_t* p) { return load_bf16(p); }
};

// Khatri-Rao entry: prod over modes m in [first, first+count) of A^(m)(i_m, r),
// where (i_first, ...) = unravel(idx) with the first listed mode fastest.
template <typename TC>
__device__ __forceinline__ TC kr_entry(const FacSet<TC>& fs, int first, int count, int64_t idx, int r) {
    TC v = (TC)1;
    for (int m = 0; m < count; ++m) {
        const int64_t d = fs.dims[first + m];
        const int64_t q = idx / d;
        const int64_t i = idx - q * d;
        idx = q;
        v *= fs.A[first + m][i * fs.R + r];
    }
    return v;
}

template <typename TY, typename TC, int RT, int JTB, bool DO_R, bool DO_L>
__global__ __launch_bounds__(256) void k_contract_valu(const TY* __restrict__ Y, int64_t J, int64_t K,
                                                        FacSet<TC> fs, int nstar, int jtiles,
                                                        int64_t ktiles, int ld, TC* __restrict__ PRpart,
                                                        TC* __restrict__ PLpart) {
    constexpr int RC = RT < 16 ? RT : 16;   // rank chunk of the cross-wave reduction
    __shared__ TC sY[64][65];
    __shared__ TC sKRR[DO_R ? 64 * RT : 1];
    __shared__ TC sKRL[DO_L ? JTB * 64 * RT : 1];
    __shared__ TC sRed[3][64][RC];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int grp = tid >> 6;
    const int R = fs.R;
    const int N = fs.N;
    const int64_t j_base = (int64_t)blockIdx.x * jtiles * 64;
    const int64_t k_base = (int64_t)blockIdx.y * ktiles * 64;

    if (DO_L) {
        for (int idx = tid; idx < jtiles * 64 * RT; idx += 256) {
            const int jj = idx / RT, r = idx - (idx / RT) * RT;
            const int64_t j = j_base + jj;
            sKRL[idx] = (j < J && r < R) ? kr_entry(fs, 0, nstar, j, r) : (TC)0;
        }
    }

    TC accR[DO_R ? JTB : 1][RT];
#pragma unroll
    for (int a = 0; a < (DO_R ? JTB : 1); ++a)
#pragma unroll
        for (int r = 0; r < RT; ++r) accR[a][r] = (TC)0;

    for (int64_t kt = 0; kt < ktiles; ++kt) {
        const int64_t k0 = k_base + kt * 64;
        if (k0 >= K) break;
        __syncthreads();
        if (DO_R) {
            for (int idx = tid; idx < 64 * RT; idx += 256) {
                const int kk = idx / RT, r = idx - (idx / RT) * RT;
                const int64_t k = k0 + kk;
                sKRR[idx] = (k < K && r < R) ? kr_entry(fs, nstar, N - nstar, k, r) : (TC)0;
            }
        }
        TC accL[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) accL[r] = (TC)0;

#pragma unroll
        for (int jt = 0; jt < JTB; ++jt) {
            if (jt < jtiles) {
                const int64_t j0 = j_base + (int64_t)jt * 64;
                if (j0 < J) {
                    __syncthreads();
                    const int64_t j = j0 + lane;
#pragma unroll 4
                    for (int s = 0; s < 16; ++s) {
                        const int kk = grp + 4 * s;
                        const int64_t k = k0 + kk;
                        sY[kk][lane] = (j < J && k < K) ? (TC)YLoad<TY, TC>::get(Y + k * J + j) : (TC)0;
                    }
                    __syncthreads();
                    if (DO_R) {
#pragma unroll 4
                        for (int s = 0; s < 16; ++s) {
                            const int kk = grp * 16 + s;
                            const TC y = sY[kk][lane];
#pragma unroll
                            for (int r = 0; r < RT; ++r) accR[DO_R ? jt : 0][r] += y * sKRR[kk * RT + r];
                        }
                    }
                    if (DO_L) {
#pragma unroll 4
                        for (int s = 0; s < 16; ++s) {
                            const int jj = grp * 16 + s;
                            const TC y = sY[lane][jj];
#pragma unroll
                            for (int r = 0; r < RT; ++r) accL[r] += sKRL[(jt * 64 + jj) * RT + r] * y;
                        }
                    }
                }
            }
        }
        if (DO_L) {
            // sum the four row groups; group 0 writes this column tile of P_L
            const int64_t k = k0 + lane;
#pragma unroll
            for (int rc = 0; rc < RT; rc += RC) {
                __syncthreads();
                if (grp > 0) {
#pragma unroll
                    for (int q = 0; q < RC; ++q) sRed[grp - 1][lane][q] = accL[rc + q];
                }
                __syncthreads();
                if (grp == 0 && k < K) {
#pragma unroll
                    for (int q = 0; q < RC; ++q) {
                        const int r = rc + q;
                        if (r < ld) {
                            TC v = accL[r] + sRed[0][lane][q] + sRed[1][lane][q] + sRed[2][lane][q];
                            PLpart[((int64_t)blockIdx.x * K + k) * ld + r] = v;
                        }
                    }
                }
            }
        }
    }

    if (DO_R) {
#pragma unroll
        for (int jt = 0; jt < JTB; ++jt) {
            if (jt < jtiles) {
                const int64_t j = j_base + (int64_t)jt * 64 + lane;
#pragma unroll
                for (int rc = 0; rc < RT; rc += RC) {
                    __syncthreads();
                    if (grp > 0) {
#pragma unroll
                        for (int q = 0; q < RC; ++q) sRed[grp - 1][lane][q] = accR[DO_R ? jt : 0][rc + q];
                    }
                    __syncthreads();
                    if (grp == 0 && j < J) {
#pragma unroll
                        for (int q = 0; q < RC; ++q) {
                            const int r = rc + q;
                            if (r < ld) {
                                TC v = accR[DO_R ? jt : 0][r] + sRed[0][lane][q] + sRed[1][lane][q] +
                                       sRed[2][lane][q];
                                PRpart[((int64_t)blockIdx.y * J + j) * ld + r] = v;
                            }
                        }
                    }
                }
            }
        }
    }
}

// JTB: j-tiles per block the kernel is compiled for (register budget of the
// right accumulators / LDS budget of the left Khatri-Rao rows).
template <typename TC, int RT>
constexpr int valu_jtb() {
    return (RT * (int)sizeof(TC) <= 64) ? 4 : ((RT * (int)sizeof(TC) <= 128) ? 2 : 1);
}

template <typename TY, typename TC, int RT>
static hipError_t dispatch_roles(const TY* Y, int64_t J, int64_t K, const FacSet<TC>& fs, int nstar,
                                 const Tiling& t, int roles, int ld, TC* PRpart, TC* PLpart, hipStream_t s) {
    constexpr int JTB = valu_jtb<TC, RT>();
    if (t.jtb > JTB) return hipErrorInvalidValue;
    dim3 grid((unsigned)t.n_jr, (unsigned)t.n_kc);
    if (roles == 3)
        hipLaunchKernelGGL((k_contract_valu<TY, TC, RT, JTB, true, true>), grid, dim3(256), 0, s, Y, J, K, fs,
                           nstar, t.jtb, t.ktb, ld, PRpart, PLpart);
    else if (roles == 1)
        hipLaunchKernelGGL((k_contract_valu<TY, TC, RT, JTB, true, false>), grid, dim3(256), 0, s, Y, J, K, fs,
                           nstar, t.jtb, t.ktb, ld, PRpart, PLpart);
    else if (roles == 2)
        hipLaunchKernelGGL((k_contract_valu<TY, TC, RT, JTB, false, true>), grid, dim3(256), 0, s, Y, J, K, fs,
                           nstar, t.jtb, t.ktb, ld, PRpart, PLpart);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename TY, typename TC>
static hipError_t dispatch_rt(const TY* Y, int64_t J, int64_t K, const FacSet<TC>& fs, int nstar,
                              const Tiling& t, int roles, int ld, TC* PRpart, TC* PLpart, hipStream_t s) {
    switch (t.rt) {
        case 4: return dispatch_roles<TY, TC, 4>(Y, J, K, fs, nstar, t, roles, ld, PRpart, PLpart, s);
        case 16: return dispatch_roles<TY, TC, 16>(Y, J, K, fs, nstar, t, roles, ld, PRpart, PLpart, s);
        case 32: return dispatch_roles<TY, TC, 32>(Y, J, K, fs, nstar, t, roles, ld, PRpart, PLpart, s);
        case 64: return dispatch_roles<TY, TC, 64>(Y, J, K, fs, nstar, t, roles, ld, PRpart, PLpart, s);
        default: return hipErrorInvalidValue;
    }
}

int valu_max_jtb(int fdt, int rt) {
    const int sz = (fdt == CPG_F64) ? 8 : 4;
    return (rt * sz <= 64) ? 4 : ((rt * sz <= 128) ? 2 : 1);
}

hipError_t launch_contract_valu(int ydt, int fdt, const void* Y, int64_t J, int64_t K, const void* facset,
                                int nstar, const Tiling& t, int roles, int ld, void* PRpart, void* PLpart,
                                hipStream_t stream) {
    if (fdt == CPG_F64 && ydt == CPG_F64)
        return dispatch_rt<double, double>((const double*)Y, J, K, *(const FacSet<double>*)facset, nstar, t,
                                           roles, ld, (double*)PRpart, (double*)PLpart, stream);
    if (fdt == CPG_F32 && ydt == CPG_F32)
        return dispatch_rt<float, float>((const float*)Y, J, K, *(const FacSet<float>*)facset, nstar, t, roles, ld,
                                         (float*)PRpart, (float*)PLpart, stream);
    if (fdt == CPG_F32 && ydt == CPG_BF16)
        return dispatch_rt<uint16_t, float>((const uint16_t*)Y, J, K, *(const FacSet<float>*)facset, nstar, t,
                                            roles, ld, (float*)PRpart, (float*)PLpart, stream);
    return hipErrorInvalidValue;
}

}  // namespace cpg
