// Precompiled streaming kernels (the program interpreter) and their launchers.
#include <hip/hip_runtime.h>

#include "sg_stream_kernel.h"

// ---- launchers (host) ------------------------------------------------------------------------

extern "C++" hipError_t sg_launch_stream(const sg::StreamArgs& a, int unroll, bool inl, int grid, int block,
                                         size_t lds_bytes, hipStream_t s) {
    using namespace sg;
#define SG_LAUNCH(UU, LBB)                                                                                \
    if (inl) hipLaunchKernelGGL((stream_kernel<UU, true, LBB>), dim3(grid), dim3(block), lds_bytes, s, a); \
    else hipLaunchKernelGGL((stream_kernel<UU, false, LBB>), dim3(grid), dim3(block), lds_bytes, s, a);
#define SG_LAUNCH_U(LBB)               \
    switch (unroll) {                  \
        case 1: SG_LAUNCH(1, LBB); break; \
        case 2: SG_LAUNCH(2, LBB); break; \
        default: SG_LAUNCH(4, LBB); break; \
    }
    if (block <= 256) { SG_LAUNCH_U(256) } else { SG_LAUNCH_U(1024) }
#undef SG_LAUNCH_U
#undef SG_LAUNCH
    return hipGetLastError();
}

extern "C++" hipError_t sg_launch_zero(uint64_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = (int)((n + 255) / 256);
    hipLaunchKernelGGL(sg::zero_kernel, dim3(grid), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

extern "C++" hipError_t sg_launch_epoch_bump(uint32_t* e, hipStream_t s) {
    hipLaunchKernelGGL(sg::epoch_bump_kernel, dim3(1), dim3(1), 0, s, e);
    return hipGetLastError();
}

extern "C++" int sg_stream_occupancy(int unroll, bool inl, int block, size_t lds_bytes) {
    using namespace sg;
    int nb = 0;
#define SG_OCC(UU, LBB)                                                                                           \
    if (inl) (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stream_kernel<UU, true, LBB>, block, lds_bytes);  \
    else (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stream_kernel<UU, false, LBB>, block, lds_bytes);
#define SG_OCC_U(LBB)                   \
    switch (unroll) {                   \
        case 1: SG_OCC(1, LBB); break;  \
        case 2: SG_OCC(2, LBB); break;  \
        default: SG_OCC(4, LBB); break; \
    }
    if (block <= 256) { SG_OCC_U(256) } else { SG_OCC_U(1024) }
#undef SG_OCC_U
#undef SG_OCC
    return nb > 0 ? nb : 1;
}
