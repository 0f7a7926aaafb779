// Step-size proposer of the learned extrapolation step: a small float32 MLP
//   h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  z = w3 . h2 + b3,
//   sigma = sigma_max * sigmoid(z)
// with hand-written inference, gradient and Adam kernels.  Training loss:
// mean over the batch of (log(1 + sigma) - log(1 + target))^2.
// Parameters are one flat float32 vector: [W1 (H x F, row-major), b1 (H),
// W2 (H x H), b2 (H), w3 (H), b3].  The batch gradient is formed as
// per-block partial sums reduced in a fixed order, so it is deterministic.
#include <new>

#include "cpg_internal.h"
#include "cpmlp.h"

namespace cpg {

constexpr int kMlpMaxIn = 32;
constexpr int kMlpMaxHidden = 32;
constexpr int kMlpSamples = 64;    // samples per block of the gradient kernel (LDS stays under 64 KB)

struct MlpDims {
    int F, H;
    float smax;
};

__host__ __device__ inline int64_t mlp_nparams(int F, int H) { return (int64_t)H * F + H + (int64_t)H * H + H + H + 1; }

__device__ __forceinline__ float sigmoidf_(float z) { return 1.f / (1.f + expf(-z)); }

// forward of one sample from parameters in LDS; keeps the activations
__device__ __forceinline__ float mlp_forward_one(const float* P, const MlpDims& d, const float* x, float* h1, float* h2,
                                                 float* zout) {
    const int F = d.F, H = d.H;
    const float* W1 = P;
    const float* b1 = W1 + H * F;
    const float* W2 = b1 + H;
    const float* b2 = W2 + H * H;
    const float* w3 = b2 + H;
    const float b3 = w3[H];
    for (int i = 0; i < H; ++i) {
        float a = b1[i];
        for (int f = 0; f < F; ++f) a += W1[i * F + f] * x[f];
        h1[i] = tanhf(a);
    }
    for (int i = 0; i < H; ++i) {
        float a = b2[i];
        for (int j = 0; j < H; ++j) a += W2[i * H + j] * h1[j];
        h2[i] = tanhf(a);
    }
    float z = b3;
    for (int i = 0; i < H; ++i) z += w3[i] * h2[i];
    *zout = z;
    return d.smax * sigmoidf_(z);
}

// Inference: eight samples per 256-thread block, one lane per hidden unit, so
// a layer costs one pass over its inputs instead of one per unit (each unit's
// sums run in the order of mlp_forward_one, so the results are the same).
constexpr int kFwdSamples = 256 / kMlpMaxHidden;
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ params, MlpDims d,
                                                     const float* __restrict__ X, int batch,
                                                     float* __restrict__ sigma) {
    extern __shared__ float sP[];
    __shared__ float sX[kFwdSamples][kMlpMaxIn], sH1[kFwdSamples][kMlpMaxHidden], sH2[kFwdSamples][kMlpMaxHidden];
    const int F = d.F, H = d.H;
    const int64_t np = mlp_nparams(F, H);
    for (int64_t e = threadIdx.x; e < np; e += blockDim.x) sP[e] = params[e];
    const int sl = threadIdx.x / kMlpMaxHidden, i = threadIdx.x % kMlpMaxHidden;
    const int s = blockIdx.x * kFwdSamples + sl;
    if (s < batch && i < F) sX[sl][i] = X[(int64_t)s * F + i];
    __syncthreads();
    const float* W1 = sP;
    const float* b1 = W1 + H * F;
    const float* W2 = b1 + H;
    const float* b2 = W2 + H * H;
    const float* w3 = b2 + H;
    const bool on = s < batch && i < H;
    if (on) {
        float a = b1[i];
        for (int f = 0; f < F; ++f) a += W1[i * F + f] * sX[sl][f];
        sH1[sl][i] = tanhf(a);
    }
    __syncthreads();
    if (on) {
        float a = b2[i];
        for (int j = 0; j < H; ++j) a += W2[i * H + j] * sH1[sl][j];
        sH2[sl][i] = tanhf(a);
    }
    __syncthreads();
    if (s < batch && i == 0) {
        float z = w3[H];
        for (int k = 0; k < H; ++k) z += w3[k] * sH2[sl][k];
        sigma[s] = d.smax * sigmoidf_(z);
    }
}

// Per-block partial gradient over up to kMlpSamples samples.
// parts[block][np], lossp[block] (sum of squared errors of the block)
__global__ __launch_bounds__(256) void k_mlp_grad_part(const float* __restrict__ params, MlpDims d,
                                                       const float* __restrict__ X, const float* __restrict__ target,
                                                       int batch, float* __restrict__ parts,
                                                       double* __restrict__ lossp) {
    extern __shared__ float smem[];
    const int F = d.F, H = d.H;
    const int64_t np = mlp_nparams(F, H);
    float* sP = smem;                                   // np
    float* sX = sP + np;                                // S x F
    float* sH1 = sX + kMlpSamples * F;                  // S x H
    float* sD1 = sH1 + kMlpSamples * H;                 // S x H   (delta at layer 1 pre-activation)
    float* sH2 = sD1 + kMlpSamples * H;                 // S x H
    float* sD2 = sH2 + kMlpSamples * H;                 // S x H   (delta at layer 2 pre-activation)
    float* sDz = sD2 + kMlpSamples * H;                 // S
    __shared__ double sLoss[256];
    for (int64_t e = threadIdx.x; e < np; e += blockDim.x) sP[e] = params[e];
    __syncthreads();
    const int s0 = blockIdx.x * kMlpSamples;
    const int ns = min(kMlpSamples, batch - s0);
    const float* W2 = sP + H * F + H;
    const float* w3 = W2 + H * H + H;
    double lsum = 0.0;
    const int t = threadIdx.x;
    if (t < kMlpSamples) {
        if (t < ns) {
            float x[kMlpMaxIn], h1[kMlpMaxHidden], h2[kMlpMaxHidden], z;
            for (int f = 0; f < F; ++f) x[f] = X[(int64_t)(s0 + t) * F + f];
            const float sig = mlp_forward_one(sP, d, x, h1, h2, &z);
            const float u = log1pf(sig), tg = log1pf(target[s0 + t]);
            const float err = u - tg;
            lsum = (double)err * (double)err;
            // dL/du = 2 err / batch; du/dsigma = 1/(1+sigma); dsigma/dz = sigma (1 - sigma/smax)
            const float dz = 2.f * err / (float)batch / (1.f + sig) * sig * (1.f - sig / d.smax);
            for (int f = 0; f < F; ++f) sX[t * F + f] = x[f];
            float d2[kMlpMaxHidden];
            for (int i = 0; i < H; ++i) {
                sH1[t * H + i] = h1[i];
                sH2[t * H + i] = h2[i];
                d2[i] = dz * w3[i] * (1.f - h2[i] * h2[i]);
                sD2[t * H + i] = d2[i];
            }
            for (int j = 0; j < H; ++j) {
                float a = 0.f;
                for (int i = 0; i < H; ++i) a += W2[i * H + j] * d2[i];
                sD1[t * H + j] = a * (1.f - h1[j] * h1[j]);
            }
            sDz[t] = dz;
        }
    }
    sLoss[t] = lsum;
    __syncthreads();
    // parameter gradients: one thread per parameter, samples in fixed order
    for (int64_t e = t; e < np; e += blockDim.x) {
        float g = 0.f;
        int64_t r = e;
        if (r < (int64_t)H * F) {                      // W1[i][f]
            const int i = (int)(r / F), f = (int)(r % F);
            for (int s = 0; s < ns; ++s) g += sD1[s * H + i] * sX[s * F + f];
        } else if ((r -= (int64_t)H * F) < H) {         // b1[i]
            for (int s = 0; s < ns; ++s) g += sD1[s * H + r];
        } else if ((r -= H) < (int64_t)H * H) {         // W2[i][j]
            const int i = (int)(r / H), j = (int)(r % H);
            for (int s = 0; s < ns; ++s) g += sD2[s * H + i] * sH1[s * H + j];
        } else if ((r -= (int64_t)H * H) < H) {         // b2[i]
            for (int s = 0; s < ns; ++s) g += sD2[s * H + r];
        } else if ((r -= H) < H) {                      // w3[i]
            for (int s = 0; s < ns; ++s) g += sDz[s] * sH2[s * H + r];
        } else {                                        // b3
            for (int s = 0; s < ns; ++s) g += sDz[s];
        }
        parts[(int64_t)blockIdx.x * np + e] = g;
    }
    // block loss (fixed tree order)
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st) sLoss[t] += sLoss[t + st];
        __syncthreads();
    }
    if (t == 0) lossp[blockIdx.x] = sLoss[0];
}

// grad[e] = sum_b parts[b][e]; optionally one Adam step on params.
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ parts, int nparts, int64_t np,
                                                    float* __restrict__ grad, float* __restrict__ params,
                                                    float* __restrict__ m, float* __restrict__ v, int adam_t,
                                                    float lr) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= np) return;
    float g = 0.f;
    for (int b = 0; b < nparts; ++b) g += parts[(int64_t)b * np + e];
    if (grad) grad[e] = g;
    if (adam_t > 0) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float mm = b1 * m[e] + (1.f - b1) * g;
        const float vv = b2 * v[e] + (1.f - b2) * g * g;
        m[e] = mm;
        v[e] = vv;
        const float mh = mm / (1.f - powf(b1, (float)adam_t));
        const float vh = vv / (1.f - powf(b2, (float)adam_t));
        params[e] -= lr * mh / (sqrtf(vh) + eps);
    }
}

__global__ void k_mlp_loss(const double* __restrict__ lossp, int nparts, int batch, double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nparts; ++b) s += lossp[b];
    *out = s / batch;
}

}  // namespace cpg

using namespace cpg;

struct cpmlp_s {
    MlpDims d{};
    int64_t np = 0;
    hipStream_t stream = nullptr;
    float* params = nullptr;   // device
    float* m = nullptr;
    float* v = nullptr;
    float* parts = nullptr;
    double* lossp = nullptr;
    double* loss = nullptr;
    int parts_cap = 0;         // blocks the partial buffers hold
    int adam_t = 0;
    double* host = nullptr;
};

static size_t grad_smem(const MlpDims& d, int64_t np) {
    return (size_t)(np + (int64_t)kMlpSamples * (d.F + 4 * d.H) + kMlpSamples) * sizeof(float);
}

static int ensure_parts(cpmlp_s* q, int nblocks) {
    if (nblocks <= q->parts_cap) return CPG_OK;
    if (q->parts) (void)hipFree(q->parts);
    if (q->lossp) (void)hipFree(q->lossp);
    q->parts = nullptr;
    q->lossp = nullptr;
    if (hipMalloc(&q->parts, (size_t)nblocks * q->np * sizeof(float)) != hipSuccess) return CPG_ERR_NOMEM;
    if (hipMalloc(&q->lossp, (size_t)nblocks * sizeof(double)) != hipSuccess) return CPG_ERR_NOMEM;
    q->parts_cap = nblocks;
    return CPG_OK;
}

static int mlp_grad(cpmlp_s* q, const float* X, const float* target, int batch, float* grad, int adam, float lr,
                    double* loss_out) {
    if (!q || !X || !target || batch < 1) return CPG_ERR_INVALID;
    const int nb = (batch + kMlpSamples - 1) / kMlpSamples;
    int st = ensure_parts(q, nb);
    if (st) return st;
    hipLaunchKernelGGL(k_mlp_grad_part, dim3(nb), dim3(256), grad_smem(q->d, q->np), q->stream, q->params, q->d, X,
                       target, batch, q->parts, q->lossp);
    if (hipGetLastError() != hipSuccess) return CPG_ERR_HIP;
    if (adam) ++q->adam_t;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)((q->np + 255) / 256)), dim3(256), 0, q->stream, q->parts, nb,
                       q->np, grad, q->params, q->m, q->v, adam ? q->adam_t : 0, lr);
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(64), 0, q->stream, q->lossp, nb, batch, q->loss);
    if (hipGetLastError() != hipSuccess) return CPG_ERR_HIP;
    if (loss_out) {
        if (hipMemcpyAsync(q->host, q->loss, sizeof(double), hipMemcpyDeviceToHost, q->stream) != hipSuccess)
            return CPG_ERR_HIP;
        if (hipStreamSynchronize(q->stream) != hipSuccess) return CPG_ERR_HIP;
        *loss_out = q->host[0];
    }
    return CPG_OK;
}

extern "C" {

int cpmlp_create(cpmlp_t* out, int n_in, int n_hidden, float sigma_max, void* stream) {
    if (!out) return CPG_ERR_INVALID;
    *out = nullptr;
    if (n_in < 1 || n_in > kMlpMaxIn || n_hidden < 1 || n_hidden > kMlpMaxHidden || !(sigma_max > 0.f))
        return CPG_ERR_INVALID;
    cpmlp_s* q = new (std::nothrow) cpmlp_s();
    if (!q) return CPG_ERR_NOMEM;
    q->d = MlpDims{n_in, n_hidden, sigma_max};
    q->np = mlp_nparams(n_in, n_hidden);
    q->stream = (hipStream_t)stream;
    bool ok = hipMalloc(&q->params, q->np * sizeof(float)) == hipSuccess &&
              hipMalloc(&q->m, q->np * sizeof(float)) == hipSuccess &&
              hipMalloc(&q->v, q->np * sizeof(float)) == hipSuccess &&
              hipMalloc(&q->loss, sizeof(double)) == hipSuccess &&
              hipHostMalloc((void**)&q->host, 8 * sizeof(double), hipHostMallocDefault) == hipSuccess;
    if (ok) {
        ok = hipMemsetAsync(q->params, 0, q->np * sizeof(float), q->stream) == hipSuccess &&
             hipMemsetAsync(q->m, 0, q->np * sizeof(float), q->stream) == hipSuccess &&
             hipMemsetAsync(q->v, 0, q->np * sizeof(float), q->stream) == hipSuccess;
    }
    if (!ok) {
        cpmlp_destroy(q);
        return CPG_ERR_NOMEM;
    }
    *out = q;
    return CPG_OK;
}

int cpmlp_num_params(cpmlp_t q, int64_t* n) {
    if (!q || !n) return CPG_ERR_INVALID;
    *n = q->np;
    return CPG_OK;
}

int cpmlp_set_params(cpmlp_t q, const float* host, int64_t n) {
    if (!q || !host || n != q->np) return CPG_ERR_INVALID;
    if (hipMemcpyAsync(q->params, host, n * sizeof(float), hipMemcpyHostToDevice, q->stream) != hipSuccess)
        return CPG_ERR_HIP;
    if (hipMemsetAsync(q->m, 0, n * sizeof(float), q->stream) != hipSuccess) return CPG_ERR_HIP;
    if (hipMemsetAsync(q->v, 0, n * sizeof(float), q->stream) != hipSuccess) return CPG_ERR_HIP;
    q->adam_t = 0;
    return hipStreamSynchronize(q->stream) == hipSuccess ? CPG_OK : CPG_ERR_HIP;
}

int cpmlp_get_params(cpmlp_t q, float* host, int64_t n) {
    if (!q || !host || n != q->np) return CPG_ERR_INVALID;
    if (hipMemcpyAsync(host, q->params, n * sizeof(float), hipMemcpyDeviceToHost, q->stream) != hipSuccess)
        return CPG_ERR_HIP;
    return hipStreamSynchronize(q->stream) == hipSuccess ? CPG_OK : CPG_ERR_HIP;
}

int cpmlp_forward(cpmlp_t q, const float* X, int batch, float* sigma) {
    if (!q || !X || !sigma || batch < 1) return CPG_ERR_INVALID;
    hipLaunchKernelGGL(k_mlp_forward, dim3((batch + kFwdSamples - 1) / kFwdSamples), dim3(256),
                       q->np * sizeof(float), q->stream, q->params, q->d, X, batch, sigma);
    return hipGetLastError() == hipSuccess ? CPG_OK : CPG_ERR_HIP;
}

int cpmlp_gradients(cpmlp_t q, const float* X, const float* target, int batch, float* grad, double* loss_out) {
    if (!grad) return CPG_ERR_INVALID;
    return mlp_grad(q, X, target, batch, grad, 0, 0.f, loss_out);
}

int cpmlp_train_step(cpmlp_t q, const float* X, const float* target, int batch, float lr, double* loss_out) {
    if (!(lr >= 0.f)) return CPG_ERR_INVALID;
    return mlp_grad(q, X, target, batch, nullptr, 1, lr, loss_out);
}

int cpmlp_destroy(cpmlp_t q) {
    if (!q) return CPG_OK;
    if (q->stream) (void)hipStreamSynchronize(q->stream);
    else (void)hipDeviceSynchronize();
    if (q->params) (void)hipFree(q->params);
    if (q->m) (void)hipFree(q->m);
    if (q->v) (void)hipFree(q->v);
    if (q->parts) (void)hipFree(q->parts);
    if (q->lossp) (void)hipFree(q->lossp);
    if (q->loss) (void)hipFree(q->loss);
    if (q->host) (void)hipHostFree(q->host);
    delete q;
    return CPG_OK;
}

}  // extern "C"

namespace cpg {
hipError_t launch_mlp_forward(cpmlp_t q, const float* X, int batch, float* sigma, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_forward, dim3((batch + kFwdSamples - 1) / kFwdSamples), dim3(256),
                       q->np * sizeof(float), s, q->params, q->d, X, batch, sigma);
    return hipGetLastError();
}
int mlp_num_inputs(cpmlp_t q) { return q->d.F; }
}  // namespace cpg
