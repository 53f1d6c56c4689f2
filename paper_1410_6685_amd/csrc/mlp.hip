// Cost model of the plan selector: a 24-64-64-1 float32 MLP with ReLU, trained on measured
// plan timings (mean squared error, Adam after Kingma and Ba, ICLR 2015) and evaluated for
// every candidate plan of a chain.
//
// Training runs in one workgroup: the whole network (5825 parameters) and a batch of 128
// samples' activations fit in LDS, so a step is forward, backward and update with only
// barriers between phases, and every gradient is a sum over the batch in sample order
// (identical results from run to run).  Inference runs one sample per thread over a grid.
//
// Parameter layout (floats): W1[24][64] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "sg_runtime.h"

namespace sg {

constexpr int MI = 24, MH = 64, MB = 128;
constexpr int OW1 = 0, OB1 = OW1 + MI * MH, OW2 = OB1 + MH, OB2 = OW2 + MH * MH, OW3 = OB2 + MH, OB3 = OW3 + MH;
constexpr int MP = OB3 + 1;  // 5825
constexpr int HP = MH + 1;   // padded activation row (no LDS bank conflicts)

struct MlpLds {
    float w[MP];
    float x[MB][MI + 1];
    float h1[MB][HP];
    float h2[MB][HP];   // reused for dH1 after the output layer's gradient
    float d2[MB][HP];
    float dy[MB];
    float loss[MB];
};

struct AdamArgs {
    float lr, b1, b2, eps;
};

// One optimisation step over samples [s0, s0 + B) of X (n x 24) / T (n).  With update == 0
// it only writes the gradient (for checks); loss_out receives the batch loss.
__device__ void mlp_step(MlpLds& L, float* __restrict__ P, float* __restrict__ G, float* __restrict__ M1,
                         float* __restrict__ M2, const float* __restrict__ X, const float* __restrict__ T, int64_t s0,
                         int B, int step, AdamArgs ad, bool update, double* loss_out) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < MP; i += nt) L.w[i] = P[i];
    for (int i = tid; i < B * MI; i += nt) L.x[i / MI][i % MI] = X[(s0 + i / MI) * MI + i % MI];
    __syncthreads();
    // forward: one sample per thread
    for (int s = tid; s < B; s += nt) {
        for (int j = 0; j < MH; ++j) {
            float a = L.w[OB1 + j];
            for (int i = 0; i < MI; ++i) a += L.x[s][i] * L.w[OW1 + i * MH + j];
            L.h1[s][j] = a > 0.f ? a : 0.f;
        }
        for (int j = 0; j < MH; ++j) {
            float a = L.w[OB2 + j];
            for (int i = 0; i < MH; ++i) a += L.h1[s][i] * L.w[OW2 + i * MH + j];
            L.h2[s][j] = a > 0.f ? a : 0.f;
        }
        float y = L.w[OB3];
        for (int j = 0; j < MH; ++j) y += L.h2[s][j] * L.w[OW3 + j];
        const float e = y - T[s0 + s];
        L.loss[s] = e * e;
        L.dy[s] = 2.f * e / (float)B;
        for (int j = 0; j < MH; ++j) L.d2[s][j] = L.h2[s][j] > 0.f ? L.dy[s] * L.w[OW3 + j] : 0.f;
    }
    __syncthreads();
    // output layer gradient (needs h2), then dH1 overwrites h2
    for (int j = tid; j < MH + 1; j += nt) {
        float g = 0.f;
        for (int s = 0; s < B; ++s) g += (j < MH ? L.h2[s][j] : 1.f) * L.dy[s];
        G[j < MH ? OW3 + j : OB3] = g;
    }
    __syncthreads();
    for (int s = tid; s < B; s += nt) {
        for (int i = 0; i < MH; ++i) {
            float a = 0.f;
            for (int j = 0; j < MH; ++j) a += L.d2[s][j] * L.w[OW2 + i * MH + j];
            L.h2[s][i] = L.h1[s][i] > 0.f ? a : 0.f;  // dH1
        }
    }
    __syncthreads();
    for (int k = tid; k < MH * MH + MH; k += nt) {
        float g = 0.f;
        if (k < MH * MH) {
            const int i = k / MH, j = k % MH;
            for (int s = 0; s < B; ++s) g += L.h1[s][i] * L.d2[s][j];
            G[OW2 + k] = g;
        } else {
            const int j = k - MH * MH;
            for (int s = 0; s < B; ++s) g += L.d2[s][j];
            G[OB2 + j] = g;
        }
    }
    for (int k = tid; k < MI * MH + MH; k += nt) {
        float g = 0.f;
        if (k < MI * MH) {
            const int i = k / MH, j = k % MH;
            for (int s = 0; s < B; ++s) g += L.x[s][i] * L.h2[s][j];
            G[OW1 + k] = g;
        } else {
            const int j = k - MI * MH;
            for (int s = 0; s < B; ++s) g += L.h2[s][j];
            G[OB1 + j] = g;
        }
    }
    if (tid == 0) {
        double l = 0.0;
        for (int s = 0; s < B; ++s) l += L.loss[s];
        *loss_out = l / B;
    }
    __syncthreads();
    if (!update) return;
    __threadfence_block();
    const float c1 = 1.f - powf(ad.b1, (float)step), c2 = 1.f - powf(ad.b2, (float)step);
    for (int i = tid; i < MP; i += nt) {
        const float g = G[i];
        const float m = ad.b1 * M1[i] + (1.f - ad.b1) * g;
        const float v = ad.b2 * M2[i] + (1.f - ad.b2) * (g * g);
        M1[i] = m;
        M2[i] = v;
        P[i] = L.w[i] - ad.lr * (m / c1) / (sqrtf(v / c2) + ad.eps);
    }
    __syncthreads();
}

// Train for `epochs` passes over n samples in batches of B (the last partial batch included).
__global__ __launch_bounds__(256) void mlp_train_kernel(float* P, float* G, float* M1, float* M2, const float* X,
                                                       const float* T, int64_t n, int B, int epochs, int step0,
                                                       AdamArgs ad, double* epoch_loss) {
    extern __shared__ char smem[];
    MlpLds& L = *reinterpret_cast<MlpLds*>(smem);
    int step = step0;
    for (int e = 0; e < epochs; ++e) {
        double tot = 0.0;
        int64_t cnt = 0;
        for (int64_t s0 = 0; s0 < n; s0 += B) {
            const int b = (int)(n - s0 < B ? n - s0 : B);
            double l = 0.0;
            mlp_step(L, P, G, M1, M2, X, T, s0, b, ++step, ad, true, epoch_loss + epochs);
            l = epoch_loss[epochs];
            tot += l * b;
            cnt += b;
            __syncthreads();
        }
        if (threadIdx.x == 0) epoch_loss[e] = tot / (double)(cnt ? cnt : 1);
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void mlp_grad_kernel(float* P, float* G, const float* X, const float* T, int B,
                                                      double* loss) {
    extern __shared__ char smem[];
    MlpLds& L = *reinterpret_cast<MlpLds*>(smem);
    mlp_step(L, P, G, nullptr, nullptr, X, T, 0, B, 1, AdamArgs{0.f, 0.f, 0.f, 0.f}, false, loss);
}

__global__ __launch_bounds__(256) void mlp_predict_kernel(const float* __restrict__ P, const float* __restrict__ X,
                                                         int64_t n, float* __restrict__ Y) {
    __shared__ float w[MP];
    for (int i = threadIdx.x; i < MP; i += blockDim.x) w[i] = P[i];
    __syncthreads();
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= n) return;
    float x[MI], h1[MH];
    for (int i = 0; i < MI; ++i) x[i] = X[s * MI + i];
    for (int j = 0; j < MH; ++j) {
        float a = w[OB1 + j];
        for (int i = 0; i < MI; ++i) a += x[i] * w[OW1 + i * MH + j];
        h1[j] = a > 0.f ? a : 0.f;
    }
    float y = w[OB3];
    for (int j = 0; j < MH; ++j) {
        float a = w[OB2 + j];
        for (int i = 0; i < MH; ++i) a += h1[i] * w[OW2 + i * MH + j];
        y += (a > 0.f ? a : 0.f) * w[OW3 + j];
    }
    Y[s] = y;
}


// Training data of the cost model.  One block per feature column: the column's mean and
// population standard deviation (two passes, float64, each thread's strided partial sums
// added lanes-then-waves in a fixed order), minimum and maximum.  stats[k] = {mean, std, lo,
// hi} as doubles.
__global__ __launch_bounds__(256) void mlp_colstats_kernel(const float* __restrict__ X, int64_t n,
                                                           double* __restrict__ stats) {
    __shared__ double red[4];
    __shared__ float rmin[4], rmax[4];
    const int k = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    auto block_sum = [&](double v) -> double {
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) red[wave] = v;
        __syncthreads();
        const double t = (red[0] + red[1]) + (red[2] + red[3]);
        __syncthreads();
        return t;
    };
    double s = 0.0;
    float lo = __builtin_inff(), hi = -__builtin_inff();
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const float x = X[i * MI + k];
        s += (double)x;
        lo = fminf(lo, x);
        hi = fmaxf(hi, x);
    }
    const double mean = block_sum(s) / (double)n;
    double q = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
        const double d = (double)X[i * MI + k] - mean;
        q += d * d;
    }
    const double var = block_sum(q) / (double)n;
    for (int o = 32; o > 0; o >>= 1) {
        lo = fminf(lo, __shfl_xor(lo, o));
        hi = fmaxf(hi, __shfl_xor(hi, o));
    }
    if (lane == 0) { rmin[wave] = lo; rmax[wave] = hi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        stats[4 * k + 0] = mean;
        stats[4 * k + 1] = __builtin_sqrt(var);
        stats[4 * k + 2] = fminf(fminf(rmin[0], rmin[1]), fminf(rmin[2], rmin[3]));
        stats[4 * k + 3] = fmaxf(fmaxf(rmax[0], rmax[1]), fmaxf(rmax[2], rmax[3]));
    }
}

// Xn = (X - mean) / scale per feature (float32 operations), T = log(1000 ms) (microseconds,
// computed in float64 and rounded to float32).
__global__ __launch_bounds__(256) void mlp_standardize_kernel(const float* __restrict__ X, const double* __restrict__ ms,
                                                              int64_t n, const float* __restrict__ mean,
                                                              const float* __restrict__ scale, float* __restrict__ Xn,
                                                              float* __restrict__ T) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n * MI) {
        const int k = (int)(i % MI);
        Xn[i] = (X[i] - mean[k]) / scale[k];
    }
    if (ms && i < n) T[i] = (float)log(ms[i] * 1000.0);
}

}  // namespace sg

using namespace sgrt;


extern "C" {

sg_status sg_mlp_create(sg_ctx ctx, const float* params, int64_t nparams, sg_mlp* out) {
    if (!ctx || !out || !params || nparams != sg::MP) return fail(ctx, SG_E_INVALID, "mlp_create: need 5825 initial parameters");
    auto* m = new sg_mlp_s();
    m->ctx = ctx;
    ctx_retain(ctx);
    if (hipMalloc(&m->P, 4 * sg::MP * sizeof(float)) != hipSuccess || hipMalloc(&m->loss, 1024 * sizeof(double)) != hipSuccess) {
        (void)sg_mlp_release(m);
        return fail(ctx, SG_E_OOM, "mlp_create: allocation");
    }
    hipError_t e = hipMemsetAsync(m->P, 0, 4 * sg::MP * sizeof(float), ctx->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(m->P, params, sg::MP * sizeof(float), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        (void)sg_mlp_release(m);
        return hip_fail(ctx, e, "mlp_create: upload");
    }
    *out = m;
    return SG_OK;
}

sg_status sg_mlp_release(sg_mlp m) {
    if (!m) return SG_E_INVALID;
    sg_ctx_s* ctx = m->ctx;
    (void)hipStreamSynchronize(ctx->stream);
    if (m->P) (void)hipFree(m->P);
    if (m->loss) (void)hipFree(m->loss);
    delete m;
    ctx_release(ctx);
    return SG_OK;
}

sg_status sg_mlp_get_params(sg_mlp m, float* params, int64_t nparams) {
    if (!m || !params || nparams != sg::MP) return fail(m ? m->ctx : nullptr, SG_E_INVALID, "mlp_get_params: bad buffer");
    SG_HIP(m->ctx, hipMemcpyAsync(params, m->P, sg::MP * sizeof(float), hipMemcpyDeviceToHost, m->ctx->stream));
    SG_HIP(m->ctx, hipStreamSynchronize(m->ctx->stream));
    return SG_OK;
}

// Loss and gradient of one batch (no update): X_dev is B x 24, T_dev B floats (device).
sg_status sg_mlp_grad(sg_mlp m, const float* X_dev, const float* T_dev, int32_t B, float* grad_host, double* loss) {
    if (!m || !X_dev || !T_dev || B < 1 || B > sg::MB || !grad_host) return fail(m ? m->ctx : nullptr, SG_E_INVALID, "mlp_grad: bad argument (1 <= B <= 128)");
    sg_ctx_s* ctx = m->ctx;
    if (sg_status st = check_device_range(ctx, X_dev, (size_t)B * sg::MI * 4, "mlp_grad X")) return st;
    if (sg_status st = check_device_range(ctx, T_dev, (size_t)B * 4, "mlp_grad T")) return st;
    SG_HIP(ctx, hipFuncSetAttribute((const void*)sg::mlp_grad_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)sizeof(sg::MlpLds)));
    hipLaunchKernelGGL(sg::mlp_grad_kernel, dim3(1), dim3(256), sizeof(sg::MlpLds), ctx->stream, m->P, m->P + sg::MP,
                       X_dev, T_dev, (int)B, m->loss);
    SG_HIP(ctx, hipGetLastError());
    SG_HIP(ctx, hipMemcpyAsync(grad_host, m->P + sg::MP, sg::MP * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    double l = 0;
    SG_HIP(ctx, hipMemcpyAsync(&l, m->loss, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    SG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (loss) *loss = l;
    return SG_OK;
}

// Train on n samples (device X n x 24, T n) for `epochs` epochs in batches of `batch` (<= 128),
// in the given sample order.  epoch_loss (host, `epochs` doubles) receives the mean loss.
sg_status sg_mlp_train(sg_mlp m, const float* X_dev, const float* T_dev, int64_t n, int32_t batch, int32_t epochs,
                       float lr, double* epoch_loss) {
    if (!m || !X_dev || !T_dev || n < 1 || batch < 1 || batch > sg::MB || epochs < 1 || epochs > 1000)
        return fail(m ? m->ctx : nullptr, SG_E_INVALID, "mlp_train: bad argument");
    sg_ctx_s* ctx = m->ctx;
    if (sg_status st = check_device_range(ctx, X_dev, (size_t)n * sg::MI * 4, "mlp_train X")) return st;
    if (sg_status st = check_device_range(ctx, T_dev, (size_t)n * 4, "mlp_train T")) return st;
    sg::AdamArgs ad{lr, 0.9f, 0.999f, 1e-8f};
    const char* name = "mlp_train";
    static bool attr_set = false;
    if (!attr_set) {
        SG_HIP(ctx, hipFuncSetAttribute((const void*)sg::mlp_train_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)sizeof(sg::MlpLds)));
        SG_HIP(ctx, hipFuncSetAttribute((const void*)sg::mlp_grad_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)sizeof(sg::MlpLds)));
        attr_set = true;
    }
    hipEvent_t a = nullptr, b = nullptr;
    if (ctx->timing) {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        (void)hipEventRecord(a, ctx->stream);
    }
    hipLaunchKernelGGL(sg::mlp_train_kernel, dim3(1), dim3(256), sizeof(sg::MlpLds), ctx->stream, m->P,
                       m->P + sg::MP, m->P + 2 * sg::MP, m->P + 3 * sg::MP, X_dev, T_dev, n, (int)batch, (int)epochs,
                       m->step, ad, m->loss);
    SG_HIP(ctx, hipGetLastError());
    if (ctx->timing) (void)hipEventRecord(b, ctx->stream);
    m->step += (int)(epochs * ((n + batch - 1) / batch));
    std::vector<double> el(epochs);
    SG_HIP(ctx, hipMemcpyAsync(el.data(), m->loss, epochs * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    SG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->timing) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, a, b) == hipSuccess) { ctx->times[name].ms += ms; ctx->times[name].n += 1; }
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    if (epoch_loss) std::memcpy(epoch_loss, el.data(), epochs * sizeof(double));
    return SG_OK;
}

// Predictions for n samples (device X n x 24 -> device Y n).
sg_status sg_mlp_predict(sg_mlp m, const float* X_dev, int64_t n, float* Y_dev) {
    if (!m || !X_dev || !Y_dev || n < 0) return fail(m ? m->ctx : nullptr, SG_E_INVALID, "mlp_predict: bad argument");
    if (n == 0) return SG_OK;
    sg_ctx_s* ctx = m->ctx;
    if (sg_status st = check_device_range(ctx, X_dev, (size_t)n * sg::MI * 4, "mlp_predict X")) return st;
    if (sg_status st = check_device_range(ctx, Y_dev, (size_t)n * 4, "mlp_predict Y")) return st;
    const unsigned grid = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(sg::mlp_predict_kernel, dim3(grid), dim3(256), 0, ctx->stream, m->P, X_dev, n, Y_dev);
    SG_HIP(ctx, hipGetLastError());
    return SG_OK;
}

// Training data of the cost model, prepared on the device: fit the standardization on the
// raw features X (n x 24), then write the standardized features Xn and, when ms is given, the
// targets log(run time in microseconds).
sg_status sg_mlp_fit_data(sg_mlp m, const float* X_dev, const double* ms_dev, int64_t n, float* Xn_dev, float* T_dev) {
    if (!m || !X_dev || !Xn_dev || n < 1 || (ms_dev && !T_dev))
        return fail(m ? m->ctx : nullptr, SG_E_INVALID, "mlp_fit_data: bad argument");
    sg_ctx_s* ctx = m->ctx;
    if (sg_status st = check_device_range(ctx, X_dev, (size_t)n * sg::MI * 4, "mlp_fit_data X")) return st;
    if (sg_status st = check_device_range(ctx, Xn_dev, (size_t)n * sg::MI * 4, "mlp_fit_data Xn")) return st;
    if (ms_dev) {
        if (sg_status st = check_device_range(ctx, ms_dev, (size_t)n * 8, "mlp_fit_data ms")) return st;
        if (sg_status st = check_device_range(ctx, T_dev, (size_t)n * 4, "mlp_fit_data T")) return st;
    }
    // statistics (24 x 4 doubles), then the float32 mean and scale the kernels and the
    // selector use
    void* w = dev_alloc(ctx, sg::MI * 4 * sizeof(double) + 2 * sg::MI * sizeof(float));
    if (!w) return fail(ctx, SG_E_OOM, "mlp_fit_data: workspace");
    double* stats = (double*)w;
    float* msd = (float*)(stats + sg::MI * 4);
    double h[sg::MI * 4];
    hipLaunchKernelGGL(sg::mlp_colstats_kernel, dim3(sg::MI), dim3(256), 0, ctx->stream, X_dev, n, stats);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h, stats, sizeof(h), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        dev_free(ctx, w);
        return hip_fail(ctx, e, "mlp_fit_data: statistics");
    }
    float mean[sg::MI], scale[sg::MI], lo[sg::MI], hi[sg::MI], both[2 * sg::MI];
    for (int k = 0; k < sg::MI; ++k) {
        mean[k] = (float)h[4 * k];
        // a constant feature keeps scale 1 (it standardizes to 0)
        scale[k] = h[4 * k + 1] > 1e-6 ? (float)h[4 * k + 1] : 1.0f;
        lo[k] = (float)h[4 * k + 2];
        hi[k] = (float)h[4 * k + 3];
        both[k] = mean[k];
        both[sg::MI + k] = scale[k];
    }
    (void)sg_mlp_set_norm(m, mean, scale, lo, hi);
    e = hipMemcpyAsync(msd, both, sizeof(both), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) {
        const int64_t tot = n * sg::MI;
        hipLaunchKernelGGL(sg::mlp_standardize_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx->stream,
                           X_dev, ms_dev, n, msd, msd + sg::MI, Xn_dev, T_dev);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    dev_free(ctx, w);
    if (e != hipSuccess) return hip_fail(ctx, e, "mlp_fit_data: standardize");
    return SG_OK;
}

// Standardized features of n samples with the model's fitted standardization (and targets).
sg_status sg_mlp_standardize(sg_mlp m, const float* X_dev, const double* ms_dev, int64_t n, float* Xn_dev, float* T_dev) {
    if (!m || !X_dev || !Xn_dev || n < 0 || (ms_dev && !T_dev))
        return fail(m ? m->ctx : nullptr, SG_E_INVALID, "mlp_standardize: bad argument");
    sg_ctx_s* ctx = m->ctx;
    if (!m->norm_set) return fail(ctx, SG_E_STATE, "mlp_standardize: the model has no standardization");
    if (n == 0) return SG_OK;
    if (sg_status st = check_device_range(ctx, X_dev, (size_t)n * sg::MI * 4, "mlp_standardize X")) return st;
    if (sg_status st = check_device_range(ctx, Xn_dev, (size_t)n * sg::MI * 4, "mlp_standardize Xn")) return st;
    if (ms_dev) {
        if (sg_status st = check_device_range(ctx, ms_dev, (size_t)n * 8, "mlp_standardize ms")) return st;
        if (sg_status st = check_device_range(ctx, T_dev, (size_t)n * 4, "mlp_standardize T")) return st;
    }
    float* msd = (float*)dev_alloc(ctx, 2 * sg::MI * sizeof(float));
    if (!msd) return fail(ctx, SG_E_OOM, "mlp_standardize: workspace");
    float both[2 * sg::MI];
    std::memcpy(both, m->mean, sizeof(m->mean));
    std::memcpy(both + sg::MI, m->scale, sizeof(m->scale));
    hipError_t e = hipMemcpyAsync(msd, both, sizeof(both), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) {
        const int64_t tot = n * sg::MI;
        hipLaunchKernelGGL(sg::mlp_standardize_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, ctx->stream,
                           X_dev, ms_dev, n, msd, msd + sg::MI, Xn_dev, T_dev);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    dev_free(ctx, msd);
    if (e != hipSuccess) return hip_fail(ctx, e, "mlp_standardize");
    return SG_OK;
}

}  // extern "C"
