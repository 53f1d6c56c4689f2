// The product postcondition of a matrix product as one call that allocates nothing, for
// callers that cannot allocate device memory (code under HIP graph capture, serving loops).
//
// It runs the same kernels as the product clause of a program (sg_launch_product_check: the
// float64 check e = C r - A (B r) against b = |A| (|B| |r|)), with their work memory in a
// static device array instead of memory from the context's pool, and writes the verdict to
// device memory the caller owns.  The call only enqueues work on the caller's stream: no
// allocation, no memset node, no synchronization, so it can be captured into a graph.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "sg_runtime.h"

using namespace sg;

hipError_t sg_launch_product_check(const float* C, const float* A, const float* B, const float* R, int64_t M,
                                   int64_t N, int64_t K, int64_t nvec, double tol, double* work, InstResult* res,
                                   hipStream_t s);
size_t sg_product_check_work_bytes(int64_t M, int64_t N, int64_t K);

namespace {

// Work memory of the call, one copy per device, held until the process ends.  Every call on a
// device shares it, so calls that overlap on one device race.
constexpr size_t kScratchBytes = (size_t)SG_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void* g_scratch[kMaxDevices];  // the array's device address, per device (null until looked up)

// The verdict of the check, in the form a program's product clause reports it.
__global__ void na_verdict(const InstResult* res, sg_verdict* out) {
    const uint64_t e = (uint64_t)res->slot[0];
    sg_verdict v;
    v.contract_id = 0;
    v.kind = SG_ENSURE;
    v.holds = e ? 0 : 1;
    v.check = SG_CHECK_PRODUCT;
    v.first_index = e ? (int64_t)(~e & ((1ull << 40) - 1)) : -1;  // key = (probe << 40) | row
    v.measure = res->sum[0];
    *out = v;
}

}  // namespace

using namespace sgrt;

extern "C" sg_status sg_product_check_noalloc(const float* C, const float* A, const float* B, const float* R,
                                              int64_t M, int64_t N, int64_t K, int32_t nvec, void* hip_stream,
                                              sg_verdict* verdict_dev) {
    if (M < 0 || N < 0 || K < 0) return fail(nullptr, SG_E_INVALID, "product_check_noalloc: negative dimension");
    if (nvec < 1 || nvec > 4) return fail(nullptr, SG_E_UNSUPPORTED, "product_check_noalloc: 1 to 4 probe vectors");
    if (!verdict_dev) return fail(nullptr, SG_E_INVALID, "product_check_noalloc: NULL verdict");
    if ((M * N > 0 && !C) || (M * K > 0 && !A) || (K * N > 0 && !B) || (N > 0 && !R))
        return fail(nullptr, SG_E_INVALID, "product_check_noalloc: NULL matrix");
    const size_t need = 256 + sg_product_check_work_bytes(M, N, K);
    if (need > kScratchBytes)
        return fail(nullptr, SG_E_INVALID,
                    "product_check_noalloc: needs " + std::to_string(need) + " bytes of work memory, more than the " +
                        std::to_string(kScratchBytes) + " the call has; use a program's product clause instead");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(nullptr, e, "product_check_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, SG_E_INVALID, "product_check_noalloc: device index");
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (!g_scratch[dev]) {
            // the array's address on the current device (each device has its own copy)
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) return hip_fail(nullptr, e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                       "product_check_noalloc: hipGetSymbolAddress");
            g_scratch[dev] = p;
        }
        base = g_scratch[dev];
    }
    hipStream_t st = (hipStream_t)hip_stream;
    // the same tolerance as a program's product clause: gamma_2K + 2^-40
    const double t = 2.0 * (double)K * std::ldexp(1.0, -24);
    const double tol = t / (1.0 - t) + std::ldexp(1.0, -40);
    InstResult* res = (InstResult*)base;  // zeroed by the check's first kernel
    double* work = (double*)((char*)base + 256);
    e = sg_launch_product_check(C, A, B, R, M, N, K, nvec, tol, work, res, st);
    if (e != hipSuccess) return hip_fail(nullptr, e, "product_check_noalloc: launch");
    hipLaunchKernelGGL(na_verdict, dim3(1), dim3(1), 0, st, (const InstResult*)res, verdict_dev);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(nullptr, e, "product_check_noalloc: launch");
    return SG_OK;
}
