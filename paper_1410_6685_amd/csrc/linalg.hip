// Matrix transposition and matrix-vector products (Section 3.4: transpose, right_multiply,
// left_multiply; Listing 1).  Both read and write HBM once per element, so they are built for
// bandwidth: the transpose moves 64 x 64 tiles through LDS (coalesced 16-byte reads of rows,
// coalesced 16-byte writes of the transposed rows, 4-byte accesses in tiles at the matrix's
// edge or with unaligned rows, a padded tile against bank conflicts); the right
// product gives each row one wave (16-byte loads along the row, float64 lane sums reduced in a
// fixed order); the left product has blocks of 256 columns walk a chunk of rows each (coalesced
// row reads) and adds the chunks' float64 partial sums in chunk order.  Results are the float64
// sums of exact float32 products, rounded to float32, identical from run to run.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sg_runtime.h"

namespace sgl {

constexpr int TT = 64;  // transpose tile

__global__ __launch_bounds__(256) void t_transpose(const uint32_t* __restrict__ a, uint32_t* __restrict__ b,
                                                   int64_t rows, int64_t cols) {
    __shared__ uint32_t tile[TT][TT + 1];
    const int64_t r0 = (int64_t)blockIdx.y * TT, c0 = (int64_t)blockIdx.x * TT;
    // a tile inside the matrix with 16-byte aligned rows: 16-byte reads of 16 rows and 16-byte
    // writes of 16 transposed rows per step (the same for the whole block)
    if (r0 + TT <= rows && c0 + TT <= cols && rows % 4 == 0 && cols % 4 == 0 &&
        ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15) == 0) {
        const int tr = threadIdx.x >> 4, tc = (threadIdx.x & 15) * 4;
        uint4 v[TT / 16];
#pragma unroll
        for (int k = 0; k < TT / 16; ++k) v[k] = *reinterpret_cast<const uint4*>(a + (r0 + tr + 16 * k) * cols + c0 + tc);
#pragma unroll
        for (int k = 0; k < TT / 16; ++k) {
            uint32_t* t = &tile[tr + 16 * k][tc];
            t[0] = v[k].x; t[1] = v[k].y; t[2] = v[k].z; t[3] = v[k].w;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < TT / 16; ++k) {
            const int c = tr + 16 * k;  // output row c0 + c, columns r0 + tc .. + 3
            uint4 o;
            o.x = tile[tc + 0][c]; o.y = tile[tc + 1][c]; o.z = tile[tc + 2][c]; o.w = tile[tc + 3][c];
            *reinterpret_cast<uint4*>(b + (c0 + c) * rows + r0 + tc) = o;
        }
        return;
    }
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4 threads
#pragma unroll
    for (int k = 0; k < TT / 4; ++k) {
        const int64_t r = r0 + ty + 4 * k, c = c0 + tx;
        if (r < rows && c < cols) tile[ty + 4 * k][tx] = a[r * cols + c];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < TT / 4; ++k) {
        const int64_t c = c0 + ty + 4 * k, r = r0 + tx;  // output row c, column r
        if (r < rows && c < cols) b[c * rows + r] = tile[tx][ty + 4 * k];
    }
}

// y = M v: one wave per row
__global__ __launch_bounds__(256) void mv_right(const float* __restrict__ M, const float* __restrict__ v,
                                                float* __restrict__ y, int64_t rows, int64_t cols) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= rows) return;
    const float* m = M + row * cols;
    double acc = 0.0;
    const bool vec = ((reinterpret_cast<uintptr_t>(m) | reinterpret_cast<uintptr_t>(v)) & 15) == 0;
    int64_t k0 = 0;
    if (vec) {
        const int64_t c4 = cols & ~(int64_t)3;
        for (int64_t k = (int64_t)lane * 4; k < c4; k += 256) {
            const float4 a = *reinterpret_cast<const float4*>(m + k);
            const float4 b = *reinterpret_cast<const float4*>(v + k);
            acc += (double)a.x * (double)b.x;
            acc += (double)a.y * (double)b.y;
            acc += (double)a.z * (double)b.z;
            acc += (double)a.w * (double)b.w;
        }
        k0 = c4;
    }
    for (int64_t k = k0 + lane; k < cols; k += 64) acc += (double)m[k] * (double)v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) y[row] = (float)acc;
}

// partial[chunk][j] = sum over the chunk's rows of v_i M[i][j]
__global__ __launch_bounds__(256) void mv_left_part(const float* __restrict__ M, const float* __restrict__ v,
                                                    double* __restrict__ part, int64_t rows, int64_t cols,
                                                    int64_t rows_per_chunk) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.y * rows_per_chunk, i1 = std::min<int64_t>(rows, i0 + rows_per_chunk);
    if (j >= cols) return;
    double acc = 0.0;
    for (int64_t i = i0; i < i1; ++i) acc += (double)v[i] * (double)M[i * cols + j];
    part[(int64_t)blockIdx.y * cols + j] = acc;
}

__global__ __launch_bounds__(256) void mv_left_sum(const double* __restrict__ part, float* __restrict__ y,
                                                   int64_t cols, int64_t chunks) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= cols) return;
    double acc = 0.0;
    for (int64_t c = 0; c < chunks; ++c) acc += part[c * cols + j];
    y[j] = (float)acc;
}

}  // namespace sgl

namespace sgrt {

sg_status run_linalg(sg_ctx_s* ctx, sg_node_s* n) {
    using namespace sgl;
    hipStream_t st = ctx->stream;
    if (n->op == OPN_TRANSPOSE) {
        const sg_node_s* a = n->src[0];
        const int64_t rows = a->rows, cols = a->cols;
        if (rows > 0 && cols > 0) {
            const dim3 grid((unsigned)((cols + TT - 1) / TT), (unsigned)((rows + TT - 1) / TT));
            hipLaunchKernelGGL(t_transpose, grid, dim3(256), 0, st, (const uint32_t*)a->dev, (uint32_t*)n->dev, rows, cols);
            SG_HIP(ctx, hipGetLastError());
        }
        n->count = n->n;
        return SG_OK;
    }
    if (n->op != OPN_MATVEC) return fail(ctx, SG_E_INVALID, "run_linalg: not a transpose or matrix-vector product");
    const sg_node_s* M = n->src[0];
    const sg_node_s* v = n->src[1];
    const int64_t rows = M->rows, cols = M->cols;
    n->count = n->n;
    if (n->binop == 0) {  // right: y = M v
        if (rows == 0) return SG_OK;
        hipLaunchKernelGGL(mv_right, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, (const float*)M->dev,
                           (const float*)v->dev, (float*)n->dev, rows, cols);
        SG_HIP(ctx, hipGetLastError());
        return SG_OK;
    }
    // left: y = v M, rows split into chunks so that the grid fills the device
    if (cols == 0) return SG_OK;
    const int64_t cblocks = (cols + 255) / 256;
    const int64_t chunks = std::max<int64_t>(1, std::min<int64_t>(rows, (2048 + cblocks - 1) / cblocks));
    const int64_t rpc = std::max<int64_t>(1, (rows + chunks - 1) / chunks);
    const int64_t nch = std::max<int64_t>(1, (rows + rpc - 1) / rpc);
    double* part = (double*)dev_alloc(ctx, (size_t)nch * cols * sizeof(double));
    if (!part) return fail(ctx, SG_E_OOM, "left_multiply: workspace");
    if (rows > 0) {
        hipLaunchKernelGGL(mv_left_part, dim3((unsigned)cblocks, (unsigned)nch), dim3(256), 0, st, (const float*)M->dev,
                           (const float*)v->dev, part, rows, cols, rpc);
    } else {
        (void)hipMemsetAsync(part, 0, (size_t)cols * sizeof(double), st);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(mv_left_sum, dim3((unsigned)cblocks), dim3(256), 0, st, part, (float*)n->dev, cols,
                           rows > 0 ? nch : 1);
        e = hipGetLastError();
    }
    // the workspace returns to the pool once the kernels that read it are done
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    dev_free(ctx, part);
    if (e != hipSuccess) return hip_fail(ctx, e, "left_multiply");
    return SG_OK;
}

}  // namespace sgrt
