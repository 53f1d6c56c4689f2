// Steps of kernel nodes that are not streaming passes or matrix products: quicksort
// (Section 4, Listing 3) and concatenate (Table 2).  Both are host-driven: they need the item
// counts of their operands, which may be known on the device only (compacted collections), and
// they publish their own output's count in their result slot (a compacted collection's count
// for the passes that read it).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "sg_runtime.h"

using namespace sg;

namespace sgrt {

namespace {

__global__ void set_count_kernel(int64_t* p, int64_t v) { *p = v; }

// Items in collection `x` right now, during an execution of `plan`: an input's length; a
// kernel node's count (its step ran earlier); a pass output's count from the pass's result
// (the scan count of a compacted output, the source count of a dense output over a compacted
// source, else the capacity).
sg_status live_count(sg_ctx_s* ctx, const Plan& plan, const sg_node_s* x, InstResult* results, int64_t* out) {
    if (is_kernel_node(x)) { *out = x->op == OPN_MATMUL ? x->n : x->count; return SG_OK; }  // its step ran earlier
    for (auto& ip : plan.insts) {
        for (auto* o : ip.outs) {
            if (o != x) continue;
            const bool compacted = std::find(ip.compacted.begin(), ip.compacted.end(), x) != ip.compacted.end();
            if (!compacted && ip.base_count_slot < 0) { *out = x->n; return SG_OK; }  // dense: every position
            InstResult r;
            SG_HIP(ctx, hipMemcpyAsync(&r, results + ip.result_index, sizeof(r), hipMemcpyDeviceToHost, ctx->stream));
            SG_HIP(ctx, hipStreamSynchronize(ctx->stream));
            if (r.err) return fail(ctx, SG_E_DEVICE, "a streaming pass before this step reported a device-side failure");
            *out = compacted ? r.scan_count : r.slot[ip.base_count_slot];
            return SG_OK;
        }
    }
    if (x->op == OPN_INPUT) { *out = x->n; return SG_OK; }
    return fail(ctx, SG_E_STATE, "count of an operand that this execution does not compute");
}

}  // namespace

sg_status run_node_step(sg_ctx_s* ctx, const Plan& plan, sg_node_s* n, InstResult* results, InstResult* slot) {
    int64_t count = 0;
    if (n->op == OPN_QSORT) {
        sg_node_s* a = n->src[0];
        int64_t m = 0;
        if (sg_status st = live_count(ctx, plan, a, results, &m)) return st;
        if (m > 0 && !a->dev) return fail(ctx, SG_E_STATE, "quicksort: operand has no storage");
        if (sg_status st = run_quicksort(ctx, a->dev, n->dev, m, a->dtype == SG_F32, &count)) return st;
    } else if (n->op == OPN_CONCAT) {
        int64_t ca = 0, cb = 0;
        if (sg_status st = live_count(ctx, plan, n->src[0], results, &ca)) return st;
        if (sg_status st = live_count(ctx, plan, n->src[1], results, &cb)) return st;
        if (ca > 0) SG_HIP(ctx, hipMemcpyAsync(n->dev, n->src[0]->dev, (size_t)ca * 4, hipMemcpyDeviceToDevice, ctx->stream));
        if (cb > 0)
            SG_HIP(ctx, hipMemcpyAsync((char*)n->dev + (size_t)ca * 4, n->src[1]->dev, (size_t)cb * 4,
                                       hipMemcpyDeviceToDevice, ctx->stream));
        count = ca + cb;
    } else if (n->op == OPN_GAUSS) {
        return run_gauss(ctx, n);  // a scalar: no count
    } else if (n->op == OPN_TRANSPOSE || n->op == OPN_MATVEC) {
        return run_linalg(ctx, n);  // dense: count = capacity
    } else {
        return fail(ctx, SG_E_INVALID, "run_node_step: not a quicksort, concatenation or determinant");
    }
    n->count = count;
    hipLaunchKernelGGL(set_count_kernel, dim3(1), dim3(1), 0, ctx->stream, &slot->scan_count, count);
    SG_HIP(ctx, hipGetLastError());
    n->count_dev = &slot->scan_count;
    return SG_OK;
}

const char* node_step_name(const sg_node_s* n) {
    switch (n->op) {
        case OPN_QSORT: return "quicksort";
        case OPN_CONCAT: return "concat";
        case OPN_GAUSS: return "gauss";
        case OPN_TRANSPOSE: return "transpose";
        case OPN_MATVEC: return "matvec";
        default: return "node";
    }
}

}  // namespace sgrt

extern "C" sg_status sg_det_parts(sg_node s, int32_t* sign, double* mant, int64_t* expo) {
    if (!s) return sgrt::fail(nullptr, SG_E_INVALID, "det_parts: NULL node");
    if (s->op != sgrt::OPN_GAUSS) return sgrt::fail(s->ctx, SG_E_INVALID, "det_parts: not a determinant node");
    sg_status st = sg_scalar_get(s, nullptr, nullptr);  // executes the node if needed
    if (st != SG_OK) return st;
    if (sign) *sign = s->det_sign;
    if (mant) *mant = s->det_mant;
    if (expo) *expo = s->det_expo;
    return SG_OK;
}
