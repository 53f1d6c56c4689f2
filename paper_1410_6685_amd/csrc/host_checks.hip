// Host evaluation of device arithmetic, exported for CPU tests.
#include <hip/hip_runtime.h>
#include "../../include/safegpu.h"
#include "sg_exp.h"

extern "C" sg_status sg_host_exp_rn(const float* t, float* out, int64_t n, int64_t* slow) {
    if ((!t || !out) && n > 0) return SG_E_INVALID;
    int s = 0;
    for (int64_t i = 0; i < n; ++i) out[i] = sgx::exp_rn(t[i], &s);
    if (slow) *slow = s;
    return SG_OK;
}
