// Batched execution: many independent programs (each a chain with its own contracts) in one
// persistent launch of the streaming kernel, optionally captured into a HIP graph.
//
// Instances are laid out back to back in one tile space; a tile-to-instance table lets every
// block find its instance with one load.  Each instance keeps its own accumulators, look-back
// range and finalization, so results equal those of separate launches.  The batch owns its
// scratch, so the graph's baked addresses stay valid whatever else runs on the context; the
// graph is [advance the device epoch word, streaming kernel] and needs no memset nodes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "sg_kernels.h"
#include "sg_runtime.h"

using namespace sg;
using namespace sgrt;

hipError_t sg_launch_stream(const StreamArgs& a, int unroll, bool inl, int grid, int block, size_t lds_bytes,
                            hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t sg_launch_epoch_bump(uint32_t* e, hipStream_t s);
hipError_t sg_launch_set_word(uint32_t* p, uint32_t v, hipStream_t s);
hipError_t sg_launch_zero(uint64_t* p, int64_t n, hipStream_t s);

struct sg_batch_s {
    sg_ctx_s* ctx = nullptr;
    std::vector<sg_program_s*> progs;
    Scratch scratch;
    void* table = nullptr;           // InstDesc[] | SgOp[] | int32 tile_inst[]
    StreamArgs args;
    int grid = 1, block = 256, unroll = 2, substeps = 1;
    size_t lds = 0;
    int64_t total_tiles = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    InstResult* host = nullptr;
    uint32_t limit_set = 0;          // wait limit last written to the device word (raw form)
};

static sg_status batch_free(sg_batch_s* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->table) (void)hipFree(b->table);
    if (b->scratch.base) (void)hipFree(b->scratch.base);
    if (b->host) (void)hipHostFree(b->host);
    for (auto* p : b->progs) (void)sg_program_release(p);
    sg_ctx_s* ctx = b->ctx;
    delete b;
    ctx_release(ctx);
    return SG_OK;
}

extern "C" {

sg_status sg_batch_create(sg_ctx ctx, const sg_program* progs, int32_t n, int use_graph, sg_batch* out) {
    if (!ctx || !out || n <= 0 || !progs) return fail(ctx, SG_E_INVALID, "batch_create: bad argument");
    auto* b = new sg_batch_s();
    b->ctx = ctx;
    ctx_retain(ctx);
    b->block = ctx->block;
    b->unroll = ctx->unroll;
    b->substeps = 1;  // sub-tiles per tile: the context's batch setting, as far as LDS allows
    std::vector<InstDesc> descs;
    std::vector<SgOp> ops;
    std::vector<int32_t> tile_inst;
    int max_slots = 0, max_sums = 0, max_cemit = 0;
    bool any_scan = false;
    for (int i = 0; i < n; ++i) {
        sg_program_s* P = progs[i];
        if (!P || P->ctx != ctx) { batch_free(b); return fail(ctx, SG_E_INVALID, "batch_create: bad program"); }
        ++P->refs;
        b->progs.push_back(P);
        sg_status st = build_plan(P, &P->plan);
        if (st != SG_OK) { batch_free(b); return st; }
        Plan& plan = P->plan;
        if (plan.insts.size() != 1 || plan.steps.size() != 1)
            { batch_free(b); return fail(ctx, SG_E_UNSUPPORTED, "batch: every program must plan to exactly one streaming pass"); }
        for (auto* m : plan.mats)
            if ((st = alloc_output(ctx, m)) != SG_OK) { batch_free(b); return st; }
        InstPlan& ip = plan.insts[0];
        if (ip.n_src) { batch_free(b); return fail(ctx, SG_E_UNSUPPORTED, "batch: sources must have host-known lengths"); }
        max_slots = std::max(max_slots, (int)ip.slot_kind.size());
        max_sums = std::max(max_sums, ip.nsum);
        max_cemit = std::max(max_cemit, inst_cemit(ip));
        any_scan |= ip.scan_space != 0;
    }
    // the per-lane accumulators and staging buffers of every instance must fit in LDS
    for (;; b->unroll /= 2) {
        b->substeps = stream_substeps(ctx->batch_substeps, b->block, b->unroll, max_slots, max_sums, max_cemit,
                                      any_scan, 1);
        b->lds = stream_lds_bytes(max_slots, max_sums, max_cemit, b->substeps, b->block, b->unroll, 1);
        if (b->lds <= kMaxDynamicLds || b->unroll == 1) break;
    }
    if (b->lds > kMaxDynamicLds) {
        batch_free(b);
        return fail(ctx, SG_E_UNSUPPORTED, "batch needs more LDS than a block has; use a smaller block");
    }
    const int64_t tile_elems = (int64_t)b->block * 4 * b->unroll * b->substeps;
    for (int i = 0; i < n; ++i) {
        InstPlan& ip = b->progs[i]->plan.insts[0];
        const int64_t nt = std::max<int64_t>(1, (ip.n + tile_elems - 1) / tile_elems);
        InstDesc d;
        fill_inst(ip, d, b->total_tiles, nt, (int)ops.size());
        descs.push_back(d);
        ops.insert(ops.end(), ip.prog.begin(), ip.prog.end());
        for (int64_t t = 0; t < nt; ++t) tile_inst.push_back(i);
        b->total_tiles += nt;
    }
    sg_status st = alloc_scratch(ctx, b->scratch, b->total_tiles, b->total_tiles, n);
    if (st != SG_OK) { batch_free(b); return st; }
    const size_t db = descs.size() * sizeof(InstDesc), ob = ops.size() * sizeof(SgOp), tb = tile_inst.size() * 4;
    const size_t off_o = (db + 255) & ~(size_t)255, off_t = (off_o + ob + 255) & ~(size_t)255;
    if (hipMalloc(&b->table, off_t + tb) != hipSuccess) { batch_free(b); return fail(ctx, SG_E_OOM, "batch table"); }
    char* base = (char*)b->table;
    if (hipMemcpy(base, descs.data(), db, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(base + off_o, ops.data(), ob, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(base + off_t, tile_inst.data(), tb, hipMemcpyHostToDevice) != hipSuccess) {
        batch_free(b);
        return fail(ctx, SG_E_DEVICE, "batch table upload");
    }
    if (hipHostMalloc((void**)&b->host, (size_t)n * sizeof(InstResult), hipHostMallocDefault) != hipSuccess) {
        batch_free(b);
        return fail(ctx, SG_E_OOM, "batch host results");
    }
    StreamArgs& a = b->args;
    std::memset(&a, 0, sizeof(a));
    a.insts = (const InstDesc*)base;
    a.progs = (const SgOp*)(base + off_o);
    a.tile_inst = (const int32_t*)(base + off_t);
    a.total_tiles = b->total_tiles;
    a.acc = b->scratch.acc;
    a.tags = b->scratch.tags;
    a.lookback = b->scratch.lookback;
    a.epoch_ptr = b->scratch.epoch;
    a.limit_ptr = b->scratch.epoch + 1;  // zeroed with the scratch: the default limit
    a.results = b->scratch.results;
    a.ninst = n;
    a.substeps = b->substeps;
    a.spread = 1;
    a.lds_slots = max_slots;
    a.lds_sums = max_sums;
    a.lds_cemit = max_cemit;
    b->grid = stream_grid(ctx, b->total_tiles, false, b->unroll, b->block, b->lds, any_scan);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) { batch_free(b); return fail(ctx, SG_E_DEVICE, "batch sync"); }
    if (use_graph) {
        // the graph holds only the kernel node (no memset nodes): the kernel leaves its
        // scratch ready for the next replay
        hipStream_t cs = ctx->stream;
        bool own = false;
        if (!cs) {
            if (hipStreamCreate(&cs) != hipSuccess) { batch_free(b); return fail(ctx, SG_E_DEVICE, "capture stream"); }
            own = true;
        }
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) e = sg_launch_epoch_bump(b->scratch.epoch, cs);
        if (e == hipSuccess) e = sg_launch_stream(a, b->unroll, false, b->grid, b->block, b->lds, cs);
        hipError_t e2 = hipStreamEndCapture(cs, &b->graph);
        if (own) (void)hipStreamDestroy(cs);
        if (e != hipSuccess || e2 != hipSuccess) { batch_free(b); return fail(ctx, SG_E_DEVICE, "graph capture failed"); }
        if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess)
            { batch_free(b); return fail(ctx, SG_E_DEVICE, "graph instantiate failed"); }
    }
    *out = b;
    return SG_OK;
}

sg_status sg_batch_launch(sg_batch b) {
    if (!b) return fail(nullptr, SG_E_INVALID, "batch_launch: NULL batch");
    sg_ctx_s* ctx = b->ctx;
    // the spin limit lives in a device word that the kernel reads, so a graph replay sees a
    // changed context setting; it is written outside the graph, on the same stream
    if (ctx->wait_limit != b->limit_set) {
        SG_HIP(ctx, sg_launch_set_word(b->scratch.epoch + 1, ctx->wait_limit, ctx->stream));
        b->limit_set = ctx->wait_limit;
    }
    if (b->exec) {
        SG_HIP(ctx, hipGraphLaunch(b->exec, ctx->stream));
    } else {
        SG_HIP(ctx, sg_launch_epoch_bump(b->scratch.epoch, ctx->stream));
        SG_HIP(ctx, sg_launch_stream(b->args, b->unroll, false, b->grid, b->block, b->lds, ctx->stream));
    }
    return SG_OK;
}

sg_status sg_batch_run(sg_batch b, int32_t* status_out, sg_verdict* verdicts, int32_t cap, int32_t* nverdicts) {
    if (!b) return fail(nullptr, SG_E_INVALID, "batch_run: NULL batch");
    if (cap < 0 || (cap > 0 && !verdicts)) return fail(b->ctx, SG_E_INVALID, "batch_run: bad verdict buffer");
    sg_ctx_s* ctx = b->ctx;
    sg_status st = sg_batch_launch(b);
    if (st != SG_OK) return st;
    const int n = (int)b->progs.size();
    SG_HIP(ctx, hipMemcpyAsync(b->host, b->scratch.results, (size_t)n * sizeof(InstResult), hipMemcpyDeviceToHost,
                               ctx->stream));
    SG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < n; ++i)
        if (b->host[i].err) {
            // a wait that gave up leaves accumulators that late blocks added to after the
            // finalization read them, and tags of this epoch: clear the batch's scratch (the
            // epoch and limit words too) so that the next run starts from a clean state
            (void)sg_launch_zero((uint64_t*)b->scratch.base, (int64_t)(b->scratch.bytes / 8), ctx->stream);
            (void)hipStreamSynchronize(ctx->stream);
            b->limit_set = 0;
            return fail(ctx, SG_E_DEVICE, "batched kernel reported a device-side failure (a bounded wait timed out)");
        }
    int32_t nv = 0;
    std::vector<sg_verdict> V;
    std::vector<InstResult> one(1);
    for (int i = 0; i < n; ++i) {
        sg_program_s* P = b->progs[i];
        one[0] = b->host[i];  // the program's own plan reads its pass from result 0
        sg_status ps = assemble_verdicts(P, one.data(), V);
        publish_inst(P->plan.insts[0], one[0], ps != SG_PRE_VIOLATED);
        if (status_out) status_out[i] = ps;
        for (auto& v : V) {
            if (nv < cap) verdicts[nv] = v;
            ++nv;
        }
    }
    if (nverdicts) *nverdicts = nv;
    return SG_OK;
}

sg_status sg_batch_release(sg_batch b) {
    if (!b) return SG_E_INVALID;
    (void)hipStreamSynchronize(b->ctx->stream);
    return batch_free(b);
}

}  // extern "C"
