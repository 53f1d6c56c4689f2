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
// Each pass is a row-by-matrix product with an 8-column right-hand side read through the
// caches; a wave works on two rows at a time, reading 16 bytes per lane.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sg_kernels.h"

namespace sg {

constexpr int PRW = 2;     // rows per wave

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// out[i][c] = sum_j f_c(X[i][j]) W[j][c], f_c(x) = x for c < 4 and |x| for c >= 4 (NW = 8).
// W comes from R (nvec x cols floats; column c is r_c for c < 4, |r_(c-4)| for c >= 4) or from
// a cols x 8 double matrix Wd.  With cmp != null (NW = 4) the rows are compared with cmp.
// W (at most cols x 8 doubles) is read directly and stays in the caches; each lane owns the
// columns 4 lane + 256 k, taken in increasing order, and two of its column groups are loaded
// before either is used, so a wave keeps several loads of X and W in flight.
template <int NW>
__global__ __launch_bounds__(256) void rowdot_kernel(const float* __restrict__ X, int64_t rows, int64_t cols,
                                                     const float* __restrict__ R, int nvec,
                                                     const double* __restrict__ Wd, double* __restrict__ out,
                                                     const double* __restrict__ cmp, double tol,
                                                     InstResult* res, int zero_res) {
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
    const bool vec = (cols % 4 == 0) && ((uintptr_t)X % 16 == 0) && (R == nullptr || (uintptr_t)R % 16 == 0);

    // one group: columns j..j+3 of this lane's rows, and the matching rows of W
    struct Group {
        float x[PRW][4];
        double w[4][NW];
    };
    auto load = [&](int64_t j, Group& g) {
        const bool full = vec && j + 3 < cols;
#pragma unroll
        for (int r = 0; r < PRW; ++r) {
            const int64_t row = row0 + r;
            const float* xp = X + row * cols + j;
            if (row < rows && full) {
                const float4 v = *(const float4*)xp;
                g.x[r][0] = v.x; g.x[r][1] = v.y; g.x[r][2] = v.z; g.x[r][3] = v.w;
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) g.x[r][q] = (row < rows && j + q < cols) ? xp[q] : 0.f;
            }
        }
        if (Wd) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int c = 0; c < NW; ++c) g.w[q][c] = j + q < cols ? Wd[(j + q) * 8 + c] : 0.0;
        } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float rv[4] = {0.f, 0.f, 0.f, 0.f};
                if (v < nvec) {
                    const float* rp = R + (int64_t)v * cols + j;
                    if (full) {
                        const float4 t = *(const float4*)rp;
                        rv[0] = t.x; rv[1] = t.y; rv[2] = t.z; rv[3] = t.w;
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) rv[q] = j + q < cols ? rp[q] : 0.f;
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    g.w[q][v] = (double)rv[q];
                    if (NW == 8) g.w[q][(v + 4) % NW] = (double)__builtin_fabsf(rv[q]);
                }
            }
        }
    };
    auto use = [&](int64_t j, const Group& g) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (j + q >= cols) break;
#pragma unroll
            for (int r = 0; r < PRW; ++r) {
                const double xv = (double)g.x[r][q];
                const double ax = xv < 0 ? -xv : xv;
#pragma unroll
                for (int c = 0; c < NW; ++c) acc[r][c] += (c < 4 ? xv : ax) * g.w[q][c];
            }
        }
    };
    int64_t j = 4 * lane;
    for (; j + 256 < cols; j += 512) {
        Group g0, g1;
        load(j, g0);
        load(j + 256, g1);
        use(j, g0);
        use(j + 256, g1);
    }
    if (j < cols) {
        Group g0;
        load(j, g0);
        use(j, g0);
    }
    // the largest ratio |e| / b of the block goes out with one atomic (nonnegative doubles
    // order as their bit patterns); violations, rare, each with their own
    uint64_t worst = 0;
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
                const uint64_t rb = __builtin_bit_cast(uint64_t, ratio);
                worst = rb > worst ? rb : worst;
            }
        }
    }
    if (cmp) {
        __shared__ uint64_t wmax[4];
        if (lane == 0) wmax[wave] = worst;
        __syncthreads();
        if (tid == 0) {
            uint64_t m = 0;
            for (int w = 0; w < 4; ++w) m = wmax[w] > m ? wmax[w] : m;
            if (m) atomicMax((unsigned long long*)&res->sum[0], (unsigned long long)m);
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
