// Matrix product C = A B on the FP32 matrix cores (Section 3.4: the matrix class multiplies
// row-major matrices using on-chip shared memory).
//
// v_mfma_f32_32x32x2f32: each wave multiplies a 32x2 by a 2x32 block per instruction and
// accumulates a 32x32 fp32 tile.  A 256-thread block computes a 128x128 tile of C (each wave
// 64x64 = 2x2 MFMA tiles), streaming K slices of A and B through LDS; registers hold the next
// slice while the current one is consumed.  Blocks are reordered so that the tiles of C one
// XCD holds at a time form a square patch whose panels its L2 shares.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace sg {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int GBM = 128, GBN = 128;
constexpr int APAD = 1, BPAD = 4;
// launched shape: 16-deep K slices, one LDS buffer (measured fastest of 16/32 x 1/2 buffers)
constexpr int GBK_RUN = 16, NBUF_RUN = 1;

// GBK: depth of a K slice (16 or 32); NBUF: LDS buffers (2: the next slice is stored while
// the current one is consumed, one barrier per slice; 1: two barriers per slice, half the LDS)
template <bool VEC, int GBK, int NBUF>
__global__ __launch_bounds__(256) void gemm_f32_kernel(const float* __restrict__ A, const float* __restrict__ B,
                                                       float* __restrict__ C, int M, int N, int K) {
    static_assert(GBK == 16 || GBK == 32, "K slice");
    constexpr int P = GBK / 8;      // float4 loads per thread for each of A and B
    constexpr int AQ = GBK / 4;     // float4 per row of an A slice
    __shared__ float As[NBUF][GBM][GBK + APAD];
    __shared__ float Bs[NBUF][GBK][GBN + BPAD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_m = (M + GBM - 1) / GBM, tiles_n = (N + GBN - 1) / GBN;
    const int nb = gridDim.x;
    int tile = blockIdx.x;
    if ((nb & 7) == 0) tile = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);  // XCD-contiguous
    // tiles in groups of 8 tile rows, column by column within a group: the blocks resident on
    // one XCD at a time cover an 8 x 8 patch of C, so they share 8 slices of A and 8 of B
    // (a row-major order would need 2 of A and 32 of B)
    constexpr int G = 8;
    const int width = G * tiles_n;
    const int first = (tile / width) * G;
    const int gs = tiles_m - first < G ? tiles_m - first : G;
    const int m0 = (first + (tile % width) % gs) * GBM, n0 = ((tile % width) / gs) * GBN;
    const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

    floatx16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    float ra[P][4], rb[P][4];
    auto load = [&](int k0) {
        // a slice inside the matrices (every slice of a multiple-of-tile product) loads with
        // no per-lane condition: a lane-divergent bounds branch around the 16-byte loads makes
        // the compiler wait for all loads in flight before issuing the next, which would
        // expose the memory latency the register prefetch is meant to hide
        const bool inside = VEC && m0 + GBM <= M && n0 + GBN <= N && k0 + GBK <= K;
        if (inside) {
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int idx = tid + 256 * p;
                const int row = idx / AQ, kq = (idx % AQ) * 4;
                const float4 va = *(const float4*)(A + (int64_t)(m0 + row) * K + k0 + kq);
                ra[p][0] = va.x; ra[p][1] = va.y; ra[p][2] = va.z; ra[p][3] = va.w;
                const int krow = idx >> 5, nq = (idx & 31) * 4;
                const float4 vb = *(const float4*)(B + (int64_t)(k0 + krow) * N + n0 + nq);
                rb[p][0] = vb.x; rb[p][1] = vb.y; rb[p][2] = vb.z; rb[p][3] = vb.w;
            }
            return;
        }
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int idx = tid + 256 * p;
            // A: 128 rows x GBK columns, 4 floats per thread-load
            {
                const int row = idx / AQ, kq = (idx % AQ) * 4;
                const int gm = m0 + row, gk = k0 + kq;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    ra[p][q] = (gm < M && gk + q < K) ? A[(int64_t)gm * K + gk + q] : 0.f;
            }
            // B: GBK rows x 128 columns
            {
                const int krow = idx >> 5, nq = (idx & 31) * 4;
                const int gk = k0 + krow, gn = n0 + nq;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    rb[p][q] = (gk < K && gn + q < N) ? B[(int64_t)gk * N + gn + q] : 0.f;
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const int idx = tid + 256 * p;
            const int row = idx / AQ, kq = (idx % AQ) * 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) As[buf][row][kq + q] = ra[p][q];
            const int krow = idx >> 5, nq = (idx & 31) * 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) Bs[buf][krow][nq + q] = rb[p][q];
        }
    };

    const int nk = (K + GBK - 1) / GBK;
    load(0);
    store(0);
    __syncthreads();
    const int li = lane & 31, lk = lane >> 5;
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = NBUF == 2 ? (kt & 1) : 0;
        if (kt + 1 < nk) load((kt + 1) * GBK);
#pragma unroll
        for (int kk = 0; kk < GBK; kk += 2) {
            float a[2], b[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                a[t] = As[buf][wm + 32 * t + li][kk + lk];
                b[t] = Bs[buf][kk + lk][wn + 32 * t + li];
            }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (NBUF == 1) __syncthreads();  // every wave is done with the buffer
        if (kt + 1 < nk) store(NBUF == 2 ? (buf ^ 1) : 0);
        __syncthreads();
    }
    // accumulator layout: register r of lane l holds row 8*(r/4) + 4*(l/32) + (r%4), column l%32
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm + 32 * i + 8 * (r >> 2) + 4 * lk + (r & 3);
                const int col = n0 + wn + 32 * j + li;
                if (row < M && col < N) C[(int64_t)row * N + col] = acc[i][j][r];
            }
}

}  // namespace sg

hipError_t sg_launch_gemm_f32(const float* A, const float* B, float* C, int64_t M, int64_t N, int64_t K,
                              hipStream_t s) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (M > (1 << 30) || N > (1 << 30) || K > (1 << 30)) return hipErrorInvalidValue;
    const int64_t tiles = ((M + sg::GBM - 1) / sg::GBM) * ((N + sg::GBN - 1) / sg::GBN);
    if (tiles > (1 << 30)) return hipErrorInvalidValue;
    const bool vec = (K % 4 == 0) && (N % 4 == 0) && ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0);
    if (vec)
        hipLaunchKernelGGL((sg::gemm_f32_kernel<true, sg::GBK_RUN, sg::NBUF_RUN>), dim3((unsigned)tiles), dim3(256), 0, s, A, B, C, (int)M, (int)N, (int)K);
    else
        hipLaunchKernelGGL((sg::gemm_f32_kernel<false, sg::GBK_RUN, sg::NBUF_RUN>), dim3((unsigned)tiles), dim3(256), 0, s, A, B, C, (int)M, (int)N, (int)K);
    return hipGetLastError();
}
