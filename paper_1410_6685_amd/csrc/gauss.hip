// Determinant by Gaussian elimination (Section 5, Listing 5): a loop of fused row updates,
// captured once into a HIP graph and replayed.
//
// The listing's inner loop is the row update of the optimizer's example: every row below the
// pivot row loses a multiple of it, fused into one expression per element.  The elimination
// here is the textbook one (partial pivoting; a zero pivot means the matrix is singular), in
// float64 on the float32 input widened exactly.  Per column k: one block finds the pivot row
// (largest |W[i][k]|, the first on ties, NaN largest) and multiplies it into the determinant;
// a swap kernel exchanges the pivot row with row k; the update kernel computes
// W[i][j] = W[i][j] - (W[i][k] / W[k][k]) * W[k][j] for the trailing block, the multiplier once
// per row in LDS, the product and the difference rounded separately (no fused multiply-add).
// The determinant is kept as sign, mantissa in [0.5, 1) and binary exponent, so it is exact to
// the last rounding even where it leaves the float64 range.  The 3n + 1 kernels of an n x n
// matrix are captured into one graph per node (and per buffer address), replayed by every
// later execution.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "sg_runtime.h"

namespace sgg {

constexpr int GB = 256;  // threads per block
constexpr int GR = 8;    // rows per update block

struct DetState {
    int32_t sign;      // -1, 1; 0 once singular
    int32_t singular;
    int64_t expo;      // det = sign * mant * 2^expo
    double mant;       // in [0.5, 1)
    int64_t piv;       // pivot row of the current column
};

__global__ void g_init(const float* __restrict__ A, double* __restrict__ W, int64_t nn, DetState* st) {
    const int64_t i = (int64_t)blockIdx.x * GB + threadIdx.x;
    if (i < nn) W[i] = (double)A[i];
    if (i == 0) {
        st->sign = 1;
        st->singular = 0;
        st->expo = 1;  // the empty product: 1 = 0.5 * 2^1
        st->mant = 0.5;
        st->piv = 0;
    }
}

// order of |x| as an unsigned key: |x| bit patterns are monotone, NaN above infinity
__device__ __forceinline__ uint64_t abs_key(double x) {
    return __builtin_bit_cast(uint64_t, x) & 0x7FFFFFFFFFFFFFFFull;
}

__global__ __launch_bounds__(GB) void g_pivot(double* __restrict__ W, int64_t n, int64_t k, DetState* st) {
    __shared__ uint64_t skey[GB / 64];
    __shared__ int64_t sidx[GB / 64];
    if (st->singular) return;
    uint64_t best = 0;
    int64_t bi = k;
    for (int64_t i = k + threadIdx.x; i < n; i += GB) {
        const uint64_t key = abs_key(W[i * n + k]);
        if (key > best) { best = key; bi = i; }  // rows in increasing order: ties keep the first
    }
    if (best == 0) bi = n;  // no nonzero entry seen by this thread
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t kb = __shfl_xor(best, o);
        const int64_t ib = __shfl_xor(bi, o);
        if (kb > best || (kb == best && ib < bi)) { best = kb; bi = ib; }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { skey[wave] = best; sidx[wave] = bi; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < GB / 64; ++w)
            if (skey[w] > best || (skey[w] == best && sidx[w] < bi)) { best = skey[w]; bi = sidx[w]; }
        if (best == 0) {  // the column is zero from row k down: singular
            st->singular = 1;
            st->sign = 0;
            st->mant = 0.0;
            st->expo = 0;
            return;
        }
        const double piv = W[bi * n + k];
        int pe = 0;
        double pm = frexp(piv, &pe);
        int32_t sg = st->sign * (bi != k ? -1 : 1);
        if (pm < 0) { pm = -pm; sg = -sg; }
        int e2 = 0;
        const double m = frexp(st->mant * pm, &e2);
        st->mant = m;
        st->expo += (int64_t)pe + e2;
        st->sign = sg;
        st->piv = bi;
    }
}

__global__ __launch_bounds__(GB) void g_swap(double* __restrict__ W, int64_t n, int64_t k, const DetState* st) {
    if (st->singular) return;
    const int64_t p = st->piv;
    if (p == k) return;
    const int64_t j = k + (int64_t)blockIdx.x * GB + threadIdx.x;
    if (j < n) {
        const double a = W[k * n + j], b = W[p * n + j];
        W[k * n + j] = b;
        W[p * n + j] = a;
    }
}

__global__ __launch_bounds__(GB) void g_update(double* __restrict__ W, int64_t n, int64_t k, const DetState* st) {
    __shared__ double l[GR];
    if (st->singular) return;
    const int64_t i0 = k + 1 + (int64_t)blockIdx.y * GR;
    const int64_t j = k + 1 + (int64_t)blockIdx.x * GB + threadIdx.x;
    if (threadIdx.x < GR) {
        const int64_t i = i0 + threadIdx.x;
        l[threadIdx.x] = i < n ? W[i * n + k] / W[k * n + k] : 0.0;
    }
    __syncthreads();
    if (j >= n) return;
    const double pk = W[k * n + j];
#pragma unroll
    for (int r = 0; r < GR; ++r) {
        const int64_t i = i0 + r;
        if (i < n) {
            const double prod = l[r] * pk;
            W[i * n + j] = W[i * n + j] - prod;
        }
    }
}

}  // namespace sgg

namespace sgrt {

// Workspace and captured graph of one determinant node (owned by the node).
struct GaussCache {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    const void* a = nullptr;  // input address the graph was captured for
    void* w = nullptr;        // W (n x n doubles) then the determinant state
    int64_t n = -1;
};

void gauss_cache_free(sg_ctx_s* ctx, void* p) {
    auto* c = (GaussCache*)p;
    if (!c) return;
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->w) dev_free(ctx, c->w);
    delete c;
}

sg_status run_gauss(sg_ctx_s* ctx, sg_node_s* node) {
    using namespace sgg;
    sg_node_s* A = node->src[0];
    const int64_t n = A->rows;
    if (A->rows != A->cols) return fail(ctx, SG_E_SHAPE, "determinant: the matrix must be square (rows = columns)");
    if (n > 0 && !A->dev) return fail(ctx, SG_E_STATE, "determinant: matrix has no storage");
    auto* c = (GaussCache*)node->aux;
    if (!c) {
        c = new GaussCache();
        node->aux = c;
    }
    if (c->n != n) {
        if (c->exec) (void)hipGraphExecDestroy(c->exec);
        if (c->graph) (void)hipGraphDestroy(c->graph);
        c->exec = nullptr;
        c->graph = nullptr;
        if (c->w) dev_free(ctx, c->w);
        c->w = dev_alloc(ctx, (size_t)std::max<int64_t>(n * n, 1) * 8 + 256);
        if (!c->w) return fail(ctx, SG_E_OOM, "determinant: workspace");
        c->n = n;
    }
    double* W = (double*)c->w;
    DetState* st = (DetState*)((char*)c->w + (((size_t)std::max<int64_t>(n * n, 1) * 8 + 255) & ~(size_t)255));
    if (!c->exec || c->a != A->dev) {
        if (c->exec) (void)hipGraphExecDestroy(c->exec);
        if (c->graph) (void)hipGraphDestroy(c->graph);
        c->exec = nullptr;
        c->graph = nullptr;
        hipStream_t cs = ctx->stream;
        bool own = false;
        if (!cs) {
            SG_HIP(ctx, hipStreamCreate(&cs));
            own = true;
        }
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const int64_t nn = n * n;
            hipLaunchKernelGGL(g_init, dim3((unsigned)std::max<int64_t>((nn + GB - 1) / GB, 1)), dim3(GB), 0, cs,
                               (const float*)A->dev, W, nn, st);
            for (int64_t k = 0; k < n && e == hipSuccess; ++k) {
                hipLaunchKernelGGL(g_pivot, dim3(1), dim3(GB), 0, cs, W, n, k, st);
                hipLaunchKernelGGL(g_swap, dim3((unsigned)((n - k + GB - 1) / GB)), dim3(GB), 0, cs, W, n, k, st);
                const int64_t m = n - k - 1;
                if (m > 0)
                    hipLaunchKernelGGL(g_update, dim3((unsigned)((m + GB - 1) / GB), (unsigned)((m + GR - 1) / GR)),
                                       dim3(GB), 0, cs, W, n, k, st);
                e = hipGetLastError();
            }
        }
        hipError_t e2 = hipStreamEndCapture(cs, &c->graph);
        if (own) (void)hipStreamDestroy(cs);
        if (e != hipSuccess || e2 != hipSuccess) return hip_fail(ctx, e != hipSuccess ? e : e2, "determinant: graph capture");
        SG_HIP(ctx, hipGraphInstantiate(&c->exec, c->graph, nullptr, nullptr, 0));
        c->a = A->dev;
    }
    SG_HIP(ctx, hipGraphLaunch(c->exec, ctx->stream));
    DetState h;
    SG_HIP(ctx, hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    SG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    node->det_sign = h.sign;
    node->det_mant = h.mant;
    node->det_expo = h.expo;
    const double v = h.mant == 0.0 ? 0.0 : std::ldexp(h.mant, (int)std::max<int64_t>(std::min<int64_t>(h.expo, 4096), -4096));
    node->fval = h.sign < 0 ? -v : v;
    node->f64 = node->fval;
    node->ival = h.sign;
    return SG_OK;
}

}  // namespace sgrt
