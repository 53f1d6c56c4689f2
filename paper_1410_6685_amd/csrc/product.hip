// Product postcondition of the matrix product: a Freivalds-style check in float64.
//
// For probe vectors r_v (rows of R), with e = C r - A (B r) and b = |A| (|B| |r|), the check
// holds when |e_i| <= tol * b_i for every probe and row; tol = gamma_2K + 2^-40 is the
// a-priori rounding bound of a K-term float32 dot product (doubled because the matrix
// cores' summation order is unspecified) plus slack for this float64 evaluation.  The
// reported index is the first violating row of the first probe that has one, and the measure
// is max |e_i| / b_i.  After RW = [r_v | |r_v|] (N x 8, float64) is written, three streaming
// passes read B, A and C once each:
//   1. BW = [B RW_v | |B| RW_(4+v)]       (K x 8)   } one launch: both need only RW
//      C RW_v                             (M x 4)   }
//   2. AW = [A BW_v | |A| BW_(4+v)]       (M x 8), compared row by row with C RW_v.
// RW and BW are padded with zero rows to a whole number of LDS chunks, so a pass loads its
// right-hand side with no bounds conditions.
// Each pass is a row-by-matrix product with a narrow right-hand side.  The columns are split
// into slices so that a 4096-row pass still has thousands of workgroups: a workgroup stages
// its slice of the right-hand side in LDS (float64, 512 columns at a time), each of its four
// waves reads four rows with 16-byte loads per lane and keeps 4 x 8 float64 sums per lane; a
// second small kernel adds B's slices in slice order into BW, and the comparison adds the
// slices of C and A in the same order itself.  Every sum is taken in a fixed order, so results
// repeat from run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "sg_kernels.h"

namespace sg {

constexpr int PC_RPW = 4;                 // rows per wave
constexpr int PC_RPB = 4 * PC_RPW;        // rows per workgroup (4 waves)
constexpr int PC_CH = 512;                // columns staged in LDS at a time
constexpr int PC_TARGET_BLOCKS = 512;     // workgroups a pass aims for (two per CU)

// rows of a padded right-hand side: cols rounded up to a whole number of LDS chunks
__host__ __device__ inline int64_t pc_pad(int64_t cols) { return (cols + PC_CH - 1) / PC_CH * PC_CH; }

// RW[j] = [r_0..r_3, |r_0|..|r_3|][j] for j < cols (missing probes zero), zero rows up to
// pc_pad(cols); also clears the verdict the passes accumulate into.
__global__ __launch_bounds__(256) void pc_prep(const float* __restrict__ R, int nvec, int64_t cols,
                                               double* __restrict__ RW, InstResult* res) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j == 0) {
        res->slot[0] = 0;
        res->sum[0] = 0.0;
        res->err = 0;
    }
    if (j >= pc_pad(cols)) return;
    double r[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) r[v] = (j < cols && v < nvec) ? (double)R[(int64_t)v * cols + j] : 0.0;
    double4* o = (double4*)(RW + j * 8);
    o[0] = make_double4(r[0], r[1], r[2], r[3]);
    o[1] = make_double4(__builtin_fabs(r[0]), __builtin_fabs(r[1]), __builtin_fabs(r[2]), __builtin_fabs(r[3]));
}

// One wave's sums over the columns [s0, s1) of its PC_RPW rows from row0, chunk by chunk: acc[r][c] +=
// f_c(X[row0 + r][j]) W[j][c].  FULL: every row and every chunk of the range lies inside the
// matrix and X rows are 16-byte aligned, so the loads take no condition (a divergent branch
// around each load would make every load wait for the one before it).
template <int NW, bool FULL>
__device__ __forceinline__ void pc_chunks(const float* __restrict__ X, int64_t rows, int64_t cols,
                                          const double* __restrict__ Wd, int64_t s0, int64_t s1, int64_t row0,
                                          double (&acc)[PC_RPW][NW], double (&w)[NW][PC_CH]) {
    const int tid = threadIdx.x, lane = tid & 63;
    static_assert(PC_CH == 512, "two right-hand side rows per thread, two float4 per row and lane");
    for (int64_t c0 = s0; c0 < s1; c0 += PC_CH) {
        const int cw = FULL ? PC_CH : (int)std::min<int64_t>(PC_CH, s1 - c0);
        // this thread's rows of the right-hand side (j = tid, tid + 256), issued before the
        // rows of X so that both are in flight together; the padding makes them all present
        double4 wa[2], wb[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double* wp = Wd + (c0 + tid + 256 * h) * 8;
            wa[h] = *(const double4*)wp;
            if (NW == 8) wb[h] = *(const double4*)(wp + 4);
        }
        // this chunk's rows of X: columns c0 + 4 lane + 256 g (+0..3), g = 0, 1
        float x[2][PC_RPW][4];
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const int jl = 4 * lane + 256 * g;
#pragma unroll
            for (int r = 0; r < PC_RPW; ++r) {
                const float* xp = X + (row0 + r) * cols + c0 + jl;
                if (FULL) {
                    const float4 v = *(const float4*)xp;
                    x[g][r][0] = v.x; x[g][r][1] = v.y; x[g][r][2] = v.z; x[g][r][3] = v.w;
                } else {
#pragma unroll
                    for (int q = 0; q < 4; ++q) x[g][r][q] = (row0 + r < rows && jl + q < cw) ? xp[q] : 0.f;
                }
            }
        }
        __syncthreads();  // the previous chunk's right-hand side is no longer read
        // stored transposed (w[c][j]): a lane's four consecutive columns are one contiguous
        // 32-byte run, and a wave's reads of one c cover 2 KiB contiguously (no bank conflicts)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = tid + 256 * h;
            w[0][j] = wa[h].x; w[1][j] = wa[h].y; w[2][j] = wa[h].z; w[3][j] = wa[h].w;
            if (NW == 8) { w[4 % NW][j] = wb[h].x; w[5 % NW][j] = wb[h].y; w[6 % NW][j] = wb[h].z; w[7 % NW][j] = wb[h].w; }
        }
        __syncthreads();
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const int jl = 4 * lane + 256 * g;
            double xv[PC_RPW][4];
#pragma unroll
            for (int r = 0; r < PC_RPW; ++r)
#pragma unroll
                for (int q = 0; q < 4; ++q) xv[r][q] = (double)x[g][r][q];
#pragma unroll
            for (int c = 0; c < NW; ++c) {
                // columns past the matrix hold zeros in w (padding) and in x
                const double4 wv = *(const double4*)&w[c][jl];
                const double wq[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int r = 0; r < PC_RPW; ++r) acc[r][c] += (c < 4 ? xv[r][q] : __builtin_fabs(xv[r][q])) * wq[q];
            }
        }
    }
}

// The same sums for a workgroup whose rows and chunks all lie inside the matrix, software
// pipelined: the next chunk's right-hand side rows and X rows are loaded while the current
// chunk is computed, and its right-hand side is staged in the other of two LDS buffers, so a
// chunk costs one barrier and the loads of one chunk are always in flight.  The loads are
// unconditional (the last chunk loads itself again, from the caches) so that nothing waits
// for them before the compute that follows.
template <int NW>
__device__ __forceinline__ void pc_chunks_pipe(const float* __restrict__ X, int64_t cols,
                                               const double* __restrict__ Wd, int64_t s0, int64_t s1, int64_t row0,
                                               double (&acc)[PC_RPW][NW], double (&w2)[2][NW][PC_CH]) {
    const int tid = threadIdx.x, lane = tid & 63;
    double4 wa[2], wb[2];
    float x[2][PC_RPW][4];
    auto load = [&](int64_t c0) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double* wp = Wd + (c0 + tid + 256 * h) * 8;
            wa[h] = *(const double4*)wp;
            if (NW == 8) wb[h] = *(const double4*)(wp + 4);
        }
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int r = 0; r < PC_RPW; ++r) {
                const float4 v = *(const float4*)(X + (row0 + r) * cols + c0 + 4 * lane + 256 * g);
                x[g][r][0] = v.x; x[g][r][1] = v.y; x[g][r][2] = v.z; x[g][r][3] = v.w;
            }
    };
    auto stage = [&](int buf) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = tid + 256 * h;
            w2[buf][0][j] = wa[h].x; w2[buf][1][j] = wa[h].y; w2[buf][2][j] = wa[h].z; w2[buf][3][j] = wa[h].w;
            if (NW == 8) {
                w2[buf][4 % NW][j] = wb[h].x; w2[buf][5 % NW][j] = wb[h].y;
                w2[buf][6 % NW][j] = wb[h].z; w2[buf][7 % NW][j] = wb[h].w;
            }
        }
    };
    load(s0);
    stage(0);
    __syncthreads();
    int buf = 0;
    for (int64_t c0 = s0; c0 < s1; c0 += PC_CH) {
        float xc[2][PC_RPW][4];
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int r = 0; r < PC_RPW; ++r)
#pragma unroll
                for (int q = 0; q < 4; ++q) xc[g][r][q] = x[g][r][q];
        load(c0 + PC_CH < s1 ? c0 + PC_CH : c0);
#pragma unroll
        for (int g = 0; g < 2; ++g) {
            const int jl = 4 * lane + 256 * g;
            double xv[PC_RPW][4];
#pragma unroll
            for (int r = 0; r < PC_RPW; ++r)
#pragma unroll
                for (int q = 0; q < 4; ++q) xv[r][q] = (double)xc[g][r][q];
#pragma unroll
            for (int c = 0; c < NW; ++c) {
                const double4 wv = *(const double4*)&w2[buf][c][jl];
                const double wq[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int r = 0; r < PC_RPW; ++r) acc[r][c] += (c < 4 ? xv[r][q] : __builtin_fabs(xv[r][q])) * wq[q];
            }
        }
        // the other buffer was last read before the previous barrier
        stage(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
}

// part[slice][row][c] = sum over the slice's columns j of f_c(X[row][j]) W[j][c], with
// f_c(x) = x for c < 4 and |x| for c >= 4, W a padded float64 right-hand side with 8 columns
// (pc_pad(cols) rows, 32-byte aligned).  NW = 4 computes the first four columns only.
// One workgroup: row block rb, column slice sl.
template <int NW>
__device__ __forceinline__ void pc_part_body(const float* __restrict__ X, int64_t rows, int64_t cols,
                                             const double* __restrict__ Wd, int64_t slice_w,
                                             double* __restrict__ part, int64_t rb, int64_t sl,
                                             double (&w2)[2][NW][PC_CH]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t row0 = rb * PC_RPB + wave * PC_RPW;
    const int64_t s0 = sl * slice_w, s1 = std::min<int64_t>(cols, s0 + slice_w);
    double acc[PC_RPW][NW];
#pragma unroll
    for (int r = 0; r < PC_RPW; ++r)
#pragma unroll
        for (int c = 0; c < NW; ++c) acc[r][c] = 0.0;
    // the same for the whole workgroup (it depends on the block indices only)
    const bool full = (cols % 4 == 0) && ((uintptr_t)X % 16 == 0) && (rb + 1) * PC_RPB <= rows &&
                      (s1 - s0) % PC_CH == 0;
    if (full)
        pc_chunks_pipe<NW>(X, cols, Wd, s0, s1, row0, acc, w2);
    else
        pc_chunks<NW, false>(X, rows, cols, Wd, s0, s1, row0, acc, w2[0]);
    // Sums over the wave of the PC_RPW x NW per-lane values by halving: at each step a lane
    // keeps half of its values and adds its partner's matching half, so after log2(NV) steps
    // lane l holds one value whole or in part, and the remaining steps add across the lanes
    // that share it.  32 exchanges instead of one six-step butterfly per value.
    constexpr int NV = PC_RPW * NW;
    double v[NV];
#pragma unroll
    for (int r = 0; r < PC_RPW; ++r)
#pragma unroll
        for (int c = 0; c < NW; ++c) v[r * NW + c] = acc[r][c];
    int idx = 0;  // index of the first value this lane still holds
#pragma unroll
    for (int m = NV, o = 32; m > 1; m >>= 1, o >>= 1) {
        const bool upper = (lane & o) != 0;
#pragma unroll
        for (int i = 0; i < m / 2; ++i) {
            const double mine = upper ? v[m / 2 + i] : v[i];
            const double other = upper ? v[i] : v[m / 2 + i];
            v[i] = mine + __shfl_xor(other, o);
        }
        idx += upper ? m / 2 : 0;
    }
    // lanes that hold the same value (they differ only in the offsets below 64 / NV) add up
    static_assert(NV == 16 || NV == 32, "values per lane");
#pragma unroll
    for (int o = 64 / NV / 2; o > 0; o >>= 1) v[0] += __shfl_xor(v[0], o);
    if ((lane & (64 / NV - 1)) == 0) {
        const int r = idx / NW, c = idx % NW;
        const int64_t row = row0 + r;
        if (row < rows) part[(sl * rows + row) * 8 + c] = v[0];
    }
}

// A pass: grid (row blocks, slices).
__global__ __launch_bounds__(256, 2) void pc_part8(const float* __restrict__ X, int64_t rows, int64_t cols,
                                                   const double* __restrict__ Wd, int64_t slice_w,
                                                   double* __restrict__ part) {
    __shared__ __align__(16) double w2[2][8][PC_CH];
    pc_part_body<8>(X, rows, cols, Wd, slice_w, part, blockIdx.x, blockIdx.y, w2);
}

// Two passes over the same right-hand side in one launch (they depend on nothing but it):
// workgroups [0, nb) run the 8-column pass over X8, the rest the 4-column pass over X4; each
// pass's workgroups are numbered row block fastest, then slice.
struct PcPass {
    const float* X;
    int64_t rows, cols, slice_w, row_blocks;
    double* part;
};
__global__ __launch_bounds__(256, 2) void pc_part_pair(const double* __restrict__ Wd, PcPass p8, PcPass p4, int64_t nb) {
    __shared__ __align__(16) double w2[2][8][PC_CH];
    const int64_t i = blockIdx.x;
    if (i < nb) {
        pc_part_body<8>(p8.X, p8.rows, p8.cols, Wd, p8.slice_w, p8.part, i % p8.row_blocks, i / p8.row_blocks, w2);
    } else {
        const int64_t j = i - nb;
        pc_part_body<4>(p4.X, p4.rows, p4.cols, Wd, p4.slice_w, p4.part, j % p4.row_blocks, j / p4.row_blocks,
                        *reinterpret_cast<double(*)[2][4][PC_CH]>(&w2[0][0][0]));
    }
}

// out[row][c] = sum over slices s (in order) of part[s][row][c], c < 8, for row < rows; zero
// rows after that up to out_rows
__global__ __launch_bounds__(256) void pc_combine(const double* __restrict__ part, int64_t slices, int64_t rows,
                                                  int64_t out_rows, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= out_rows * 8) return;
    double s = 0.0;
    if (i < rows * 8)
        for (int64_t k = 0; k < slices; ++k) s += part[k * rows * 8 + i];
    out[i] = s;
}

// The comparison: C r_v and AW = [A BW_v | |A| BW_(4+v)], each the sum of its pass's slices in
// slice order (the order the combine uses), row by row; violations and the largest ratio.
__global__ __launch_bounds__(256) void pc_compare(const double* __restrict__ part, int64_t slices,
                                                  const double* __restrict__ apart, int64_t aslices, int64_t rows,
                                                  int nvec, double tol, InstResult* res) {
    __shared__ uint64_t wmax[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t row = (int64_t)blockIdx.x * 256 + tid;
    uint64_t worst = 0;
    if (row < rows) {
        for (int v = 0; v < nvec; ++v) {
            double cr = 0.0, aw = 0.0, b = 0.0;
            for (int64_t k = 0; k < slices; ++k) cr += part[(k * rows + row) * 8 + v];
            for (int64_t k = 0; k < aslices; ++k) {
                aw += apart[(k * rows + row) * 8 + v];
                b += apart[(k * rows + row) * 8 + 4 + v];
            }
            const double e = cr - aw;
            const double ae = e < 0 ? -e : e;
            const bool ok = ae <= tol * b;
            double ratio = b > 0 ? ae / b : (ae == 0 ? 0.0 : __builtin_inf());
            if (ratio != ratio) ratio = __builtin_inf();
            if (!ok) atomicMax((unsigned long long*)&res->slot[0], (unsigned long long)~(((uint64_t)v << 40) | (uint64_t)row));
            const uint64_t rb = __builtin_bit_cast(uint64_t, ratio);
            worst = rb > worst ? rb : worst;
        }
    }
    // nonnegative doubles order as their bit patterns: one atomic per workgroup
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t y = __shfl_xor(worst, o);
        worst = y > worst ? y : worst;
    }
    if (lane == 0) wmax[wave] = worst;
    __syncthreads();
    if (tid == 0) {
        uint64_t m = 0;
        for (int w = 0; w < 4; ++w) m = wmax[w] > m ? wmax[w] : m;
        if (m) atomicMax((unsigned long long*)&res->sum[0], (unsigned long long)m);
    }
}

// column slices of one pass: enough workgroups to fill the device, slices a multiple of the
// LDS chunk
struct PcSplit {
    int64_t slices, width, row_blocks;
};
inline PcSplit pc_split(int64_t rows, int64_t cols) {
    PcSplit s;
    s.row_blocks = std::max<int64_t>(1, (rows + PC_RPB - 1) / PC_RPB);
    const int64_t chunks = std::max<int64_t>(1, (cols + PC_CH - 1) / PC_CH);
    const int64_t want = std::min<int64_t>(chunks, std::max<int64_t>(1, (PC_TARGET_BLOCKS + s.row_blocks - 1) / s.row_blocks));
    s.width = ((chunks + want - 1) / want) * PC_CH;
    s.slices = std::max<int64_t>(1, (cols + s.width - 1) / s.width);
    return s;
}

}  // namespace sg

// Workspace (bytes) of a product check with C (M x N) = A (M x K) B (K x N).
size_t sg_product_check_work_bytes(int64_t M, int64_t N, int64_t K) {
    using namespace sg;
    const PcSplit p1 = pc_split(K, N), p2 = pc_split(M, K), p3 = pc_split(M, N);
    const int64_t part = std::max(p1.slices * K, p2.slices * M);  // B's partial sums, later A's
    return (size_t)(pc_pad(N) * 8 + pc_pad(K) * 8 + p3.slices * M * 8 + part * 8) * sizeof(double);
}

hipError_t sg_launch_product_check(const float* C, const float* A, const float* B, const float* R, int64_t M,
                                   int64_t N, int64_t K, int64_t nvec, double tol, double* work,
                                   sg::InstResult* res, hipStream_t s) {
    using namespace sg;
    if (nvec < 1 || nvec > 4) return hipErrorInvalidValue;
    if ((uintptr_t)work % 32 != 0) return hipErrorInvalidValue;
    double* RW = work;                      // pc_pad(N) x 8
    double* BW = RW + pc_pad(N) * 8;        // pc_pad(K) x 8
    double* cpart = BW + pc_pad(K) * 8;     // C's slices x M x 8
    const PcSplit p1 = pc_split(K, N), p2 = pc_split(M, K), p3 = pc_split(M, N);
    double* part = cpart + p3.slices * M * 8;  // B's slices x K x 8, then A's slices x M x 8
    auto grid1 = [](int64_t n) { return dim3((unsigned)std::max<int64_t>(1, (n + 255) / 256)); };
    hipLaunchKernelGGL(pc_prep, grid1(pc_pad(N)), dim3(256), 0, s, R, (int)nvec, N, RW, res);
    // B and C against the probes together, then BW, then A against BW, then the comparison
    const PcPass pb{B, K, N, p1.width, p1.row_blocks, part};
    const PcPass pcp{C, M, N, p3.width, p3.row_blocks, cpart};
    const int64_t nb = p1.row_blocks * p1.slices, nc = p3.row_blocks * p3.slices;
    hipLaunchKernelGGL(pc_part_pair, dim3((unsigned)(nb + nc)), dim3(256), 0, s, (const double*)RW, pb, pcp, nb);
    hipLaunchKernelGGL(pc_combine, grid1(pc_pad(K) * 8), dim3(256), 0, s, (const double*)part, p1.slices, K,
                       pc_pad(K), BW);
    hipLaunchKernelGGL(pc_part8, dim3((unsigned)p2.row_blocks, (unsigned)p2.slices), dim3(256), 0, s, A, M, K,
                       (const double*)BW, p2.width, part);
    hipLaunchKernelGGL(pc_compare, grid1(M), dim3(256), 0, s, (const double*)cpart, p3.slices, (const double*)part,
                       p2.slices, M, (int)nvec, tol, res);
    return hipGetLastError();
}
