// Product postcondition of the matrix product: a Freivalds-style check in float64.
//
// For probe vectors r_v (rows of R), with e = C r - A (B r) and b = |A| (|B| |r|), the check
// holds when |e_i| <= tol * b_i for every probe and row; tol = gamma_2K + 2^-40 is the
// a-priori rounding bound of a K-term float32 dot product (doubled because the matrix
// cores' summation order is unspecified) plus slack for this float64 evaluation.  The
// reported index is the first violating row of the first probe that has one, and the measure
// is max |e_i| / b_i.  Three streaming passes read B, A and C once each:
//   1. BW = [B r_v | |B| |r_v|]          (K x 8)
//   2. AW = [A BW_v | |A| BW_(4+v)]       (M x 8)
//   3. C r_v, compared row by row with AW.
// Each pass is a row-by-matrix product with an 8-column right-hand side staged in LDS;
// a wave works on two rows at a time, reading 16 bytes per lane.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sg_kernels.h"

namespace sg {

constexpr int PCH = 1024;  // right-hand-side rows staged per LDS chunk
constexpr int PRW = 2;     // rows per wave

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// out[i][c] = sum_j f_c(X[i][j]) W[j][c], f_c(x) = x for c < 4 and |x| for c >= 4 (NW = 8).
// W comes from R (nvec x cols floats; column c is r_c for c < 4, |r_(c-4)| for c >= 4) or from
// a cols x 8 double matrix Wd.  With cmp != null (NW = 4) the rows are compared with cmp.
template <int NW>
__global__ __launch_bounds__(256) void rowdot_kernel(const float* __restrict__ X, int64_t rows, int64_t cols,
                                                     const float* __restrict__ R, int nvec,
                                                     const double* __restrict__ Wd, double* __restrict__ out,
                                                     const double* __restrict__ cmp, double tol,
                                                     InstResult* res, int zero_res) {
    __shared__ double Ws[PCH][NW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (zero_res && blockIdx.x == 0 && tid == 0) {
        res->slot[0] = 0;
        res->sum[0] = 0.0;
        res->err = 0;
    }
    const int64_t row0 = ((int64_t)blockIdx.x * 4 + wave) * PRW;
    double acc[PRW][NW];
#pragma unroll
    for (int r = 0; r < PRW; ++r)
#pragma unroll
        for (int c = 0; c < NW; ++c) acc[r][c] = 0.0;
    const bool vec = (cols % 4 == 0) && ((uintptr_t)X % 16 == 0);

    for (int64_t c0 = 0; c0 < cols; c0 += PCH) {
        __syncthreads();
        for (int idx = tid; idx < PCH * NW; idx += 256) {
            const int j = idx / NW, c = idx % NW;
            const int64_t gj = c0 + j;
            double w = 0.0;
            if (gj < cols) {
                if (Wd) {
                    w = Wd[gj * 8 + c];
                } else {
                    const int v = c & 3;
                    if (v < nvec) {
                        const float rv = R[(int64_t)v * cols + gj];
                        w = c < 4 ? (double)rv : (double)__builtin_fabsf(rv);
                    }
                }
            }
            Ws[j][c] = w;
        }
        __syncthreads();
        const int64_t lim = cols - c0 < PCH ? cols - c0 : PCH;
        for (int64_t j = 4 * lane; j < lim; j += 256) {
            float x[PRW][4];
#pragma unroll
            for (int r = 0; r < PRW; ++r) {
                const int64_t row = row0 + r;
                const float* xp = X + row * cols + c0 + j;
                if (row < rows && vec && j + 3 < lim) {
                    const float4 v = *(const float4*)xp;
                    x[r][0] = v.x; x[r][1] = v.y; x[r][2] = v.z; x[r][3] = v.w;
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) x[r][q] = (row < rows && j + q < lim) ? xp[q] : 0.f;
                }
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (j + q >= lim) break;
                double w[NW];
#pragma unroll
                for (int c = 0; c < NW; ++c) w[c] = Ws[j + q][c];
#pragma unroll
                for (int r = 0; r < PRW; ++r) {
                    const double xv = (double)x[r][q];
                    const double ax = xv < 0 ? -xv : xv;
#pragma unroll
                    for (int c = 0; c < NW; ++c) acc[r][c] += (c < 4 ? xv : ax) * w[c];
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < PRW; ++r) {
        const int64_t row = row0 + r;
        double tot[NW];
#pragma unroll
        for (int c = 0; c < NW; ++c) tot[c] = wsum(acc[r][c]);
        if (lane != 0 || row >= rows) continue;
        if (!cmp) {
#pragma unroll
            for (int c = 0; c < NW; ++c) out[row * 8 + c] = tot[c];
        } else {
            for (int v = 0; v < nvec; ++v) {
                const double e = tot[v] - cmp[row * 8 + v];
                const double b = cmp[row * 8 + 4 + v];
                const double ae = e < 0 ? -e : e;
                const bool ok = ae <= tol * b;
                double ratio = b > 0 ? ae / b : (ae == 0 ? 0.0 : __builtin_inf());
                if (ratio != ratio) ratio = __builtin_inf();
                if (!ok) atomicMax((unsigned long long*)&res->slot[0], (unsigned long long)~(((uint64_t)v << 40) | (uint64_t)row));
                atomicMax((unsigned long long*)&res->sum[0], (unsigned long long)__builtin_bit_cast(uint64_t, ratio));
            }
        }
    }
}

}  // namespace sg

hipError_t sg_launch_product_check(const float* C, const float* A, const float* B, const float* R, int64_t M,
                                   int64_t N, int64_t K, int64_t nvec, double tol, double* work,
                                   sg::InstResult* res, hipStream_t s) {
    using namespace sg;
    if (nvec < 1 || nvec > 4) return hipErrorInvalidValue;
    double* BW = work;           // K x 8
    double* AW = work + K * 8;   // M x 8
    const int rows_per_block = 4 * PRW;
    auto blocks = [&](int64_t rows) { return (unsigned)((rows + rows_per_block - 1) / rows_per_block > 0 ? (rows + rows_per_block - 1) / rows_per_block : 1); };
    hipLaunchKernelGGL(rowdot_kernel<8>, dim3(blocks(K)), dim3(256), 0, s, B, K, N, R, (int)nvec, (const double*)nullptr,
                       BW, (const double*)nullptr, tol, res, 1);
    hipLaunchKernelGGL(rowdot_kernel<8>, dim3(blocks(M)), dim3(256), 0, s, A, M, K, (const float*)nullptr, (int)nvec,
                       (const double*)BW, AW, (const double*)nullptr, tol, res, 0);
    hipLaunchKernelGGL(rowdot_kernel<4>, dim3(blocks(M)), dim3(256), 0, s, C, M, N, R, (int)nvec, (const double*)nullptr,
                       (double*)nullptr, (const double*)AW, tol, res, 0);
    return hipGetLastError();
}
