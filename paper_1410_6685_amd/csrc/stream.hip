// Precompiled streaming kernels (the program interpreter) and their launchers.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "sg_stream_kernel.h"

// ---- launchers (host) ------------------------------------------------------------------------

// With events given, they are recorded at the kernel's own start and end.
extern "C++" hipError_t sg_launch_stream(const sg::StreamArgs& a, int unroll, bool inl, int grid, int block,
                                         size_t lds_bytes, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    using namespace sg;
    void* args[] = {(void*)&a};
    auto go = [&](const void* f) -> hipError_t {
        if (e0) return hipExtLaunchKernel(f, dim3(grid), dim3(block), args, lds_bytes, s, e0, e1, 0);
        return hipLaunchKernel(f, dim3(grid), dim3(block), args, lds_bytes, s);
    };
    hipError_t err = hipSuccess;
#define SG_LAUNCH(UU, LBB)                                                       \
    if (inl) err = go(reinterpret_cast<const void*>(&stream_kernel<UU, true, LBB>)); \
    else err = go(reinterpret_cast<const void*>(&stream_kernel<UU, false, LBB>));
#define SG_LAUNCH_U(LBB)               \
    switch (unroll) {                  \
        case 1: SG_LAUNCH(1, LBB); break; \
        case 2: SG_LAUNCH(2, LBB); break; \
        default: SG_LAUNCH(4, LBB); break; \
    }
    if (block <= 256) { SG_LAUNCH_U(256) } else { SG_LAUNCH_U(1024) }
#undef SG_LAUNCH_U
#undef SG_LAUNCH
    return err != hipSuccess ? err : hipGetLastError();
}

extern "C++" hipError_t sg_launch_zero(uint64_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = (int)((n + 255) / 256);
    hipLaunchKernelGGL(sg::zero_kernel, dim3(grid), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

extern "C++" hipError_t sg_launch_set_word(uint32_t* p, uint32_t v, hipStream_t s) {
    hipLaunchKernelGGL(sg::set_word_kernel, dim3(1), dim3(1), 0, s, p, v);
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
