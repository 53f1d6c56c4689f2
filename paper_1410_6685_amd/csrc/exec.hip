// Executor: binds a plan to device memory, launches its steps on the context stream, reads
// the per-pass results back once, and publishes values and contract verdicts.
//
// Contract protocol (Section 4): requires are checked on entry and ensures on exit.  All
// active clauses of a pass are evaluated in the same pass as the body (the operations are
// pure, so evaluating a require speculatively changes nothing).  A failing require means
// the body "did not run": its outputs are not published and the ensures are reported as not
// evaluated.  The violation returned is the first failing clause in declaration order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>
#include <string>
#include <vector>

#include "sg_kernels.h"
#include "sg_runtime.h"

using namespace sg;

hipError_t sg_launch_stream(const StreamArgs& a, int unroll, bool inl, int grid, int block, size_t lds_bytes,
                            hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t sg_launch_gemm_f32(const float* A, const float* B, float* C, int64_t M, int64_t N, int64_t K, hipStream_t s);
hipError_t sg_launch_product_check(const float* C, const float* A, const float* B, const float* R, int64_t M,
                                   int64_t N, int64_t K, int64_t nvec, double tol, double* work, InstResult* res,
                                   hipStream_t s);
size_t sg_product_check_work_bytes(int64_t M, int64_t N, int64_t K);
int sg_stream_occupancy(int unroll, bool inl, int block, size_t lds_bytes);
hipError_t sg_launch_zero(uint64_t* p, int64_t n, hipStream_t s);

namespace sgrt {

namespace {

hipEvent_t get_event(std::vector<hipEvent_t>& pool, size_t i) {
    while (pool.size() <= i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        pool.push_back(e);
    }
    return pool[i];
}


float key_to_float(int32_t k) {
    const uint32_t b = k >= 0 ? (uint32_t)k : ((uint32_t)k ^ 0x7FFFFFFFu);
    float f;
    std::memcpy(&f, &b, 4);
    return f;
}

}  // namespace

// Blocks per CU a pass may count on being resident together.  A pass that compacts waits on
// other blocks' tiles, so all of its grid must be resident.  The runtime's occupancy figure
// has been seen to admit one block per CU too many (when LDS is filled exactly, and when the
// scalar registers bound a small kernel at 7 waves per SIMD).  When LDS alone binds, the
// conservative LDS count (a reserve and a bound on the static part) is used as it is;
// otherwise a waiting pass keeps one block per CU in reserve.
int coresident_blocks(int occupancy, int lds_blocks, bool waits_on_others) {
    const int occ = std::max(std::min(occupancy, lds_blocks), 1);
    if (!waits_on_others || lds_blocks < occupancy) return occ;
    return std::max(occ >= 3 ? occ - 1 : occ, 1);
}

int stream_grid(sg_ctx_s* ctx, int64_t ntiles, bool inl, int unroll, int block, size_t lds_bytes, bool waits) {
    auto key = std::make_tuple(unroll * (inl ? 1 : -1), block, lds_bytes);
    auto it = ctx->occupancy.find(key);
    int nb;
    if (it != ctx->occupancy.end()) {
        nb = it->second;
    } else {
        nb = sg_stream_occupancy(unroll, inl, block, lds_bytes);
        ctx->occupancy[key] = nb;
    }
    const int64_t cap = (int64_t)coresident_blocks(nb, lds_blocks_per_cu(lds_bytes), waits) * ctx->num_cu;
    return (int)std::max<int64_t>(1, std::min<int64_t>(ntiles, cap));
}

int inst_cemit(const InstPlan& ip) {
    int k = 0;
    for (auto& op : ip.prog) k += op.code == EMIT && op.sp != 0 && op.sp == ip.scan_space;
    return k;
}

size_t stream_lds_bytes(int slots, int sums, int cemit, int C, int block, int unroll, int nbuf) {
    return (size_t)(slots + sums) * block * 8 + (size_t)nbuf * cemit * C * block * 4 * unroll * 4;
}

// A pass with a scan space keeps one LDS region per wave and sub-tile of a tile (at most
// 64), and its staged values in at most 64 KiB, so that two blocks fit on a CU.
int stream_substeps(int C, int block, int unroll, int slots, int sums, int cemit, bool scan, int nbuf) {
    if (!scan) return C;
    int c = std::min(C, 64 / (block / 64));
    while (c > 1 && stream_lds_bytes(slots, sums, cemit, c, block, unroll, nbuf) > 65536) --c;
    return std::max(c, 1);
}

// Resident blocks per CU allowed by LDS, with a margin: the runtime's occupancy figure has
// been seen to admit one block too many when a grid fills the LDS exactly, and the
// compaction's waits need every block of the grid resident.
int lds_blocks_per_cu(size_t dyn_lds) {
    return (int)std::max<size_t>(1, (kLdsPerCu - kLdsReserve) / (dyn_lds + kStaticLdsBound));
}

sg_status alloc_output(sg_ctx_s* ctx, sg_node_s* n) {
    const size_t bytes = (size_t)std::max<int64_t>(n->n, 1) * 4;
    if (n->dev && n->owned && n->bytes >= bytes) return SG_OK;
    if (n->dev && n->owned) dev_free(ctx, n->dev);
    n->dev = dev_alloc(ctx, bytes);
    if (!n->dev) return fail(ctx, SG_E_OOM, "output allocation failed");
    n->owned = true;
    n->bytes = bytes;
    return SG_OK;
}

// Fill one pass's instance descriptor from the plan and the nodes' current storage.
void fill_inst(const InstPlan& ip, InstDesc& d, int64_t tile0, int64_t ntiles, int prog_off) {
    std::memset(&d, 0, sizeof(d));
    bool aligned = true;
    for (size_t k = 0; k < ip.sources.size(); ++k) {
        d.in[k] = ip.sources[k]->dev;
        aligned = aligned && ((uintptr_t)d.in[k] % 16 == 0);
    }
    for (size_t k = 0; k < ip.outs.size(); ++k) {
        d.out[k] = ip.outs[k]->dev;
        aligned = aligned && ((uintptr_t)d.out[k] % 16 == 0);
    }
    d.n = ip.n;
    d.n_dev = ip.n_src ? ip.n_src->count_dev : nullptr;
    d.tile0 = tile0;
    d.ntiles = ntiles;
    d.prog_off = prog_off;
    d.prog_len = (int32_t)ip.prog.size();
    d.nin = (int32_t)ip.sources.size();
    d.scan_space = ip.scan_space;
    d.nsum = ip.nsum;
    d.nslots = (int32_t)ip.slot_kind.size();
    d.count_slot = ip.count_slot;
    d.flags = aligned ? 1 : 0;
    for (size_t k = 0; k < ip.slot_kind.size(); ++k) d.slot_kind[k] = ip.slot_kind[k];
}

// Publish the results of one pass (after the read-back).
void publish_inst(const InstPlan& ip, const InstResult& r, bool publish_values) {
    for (auto& so : ip.scalars) {
        sg_node_s* n = so.node;
        const sg_node_s* src = n->src[0];
        const bool f = src->dtype == SG_F32;
        switch (n->red) {
            case SG_SUM:
                if (f) {
                    n->f64 = r.sum[so.sum];
                    n->fval = (double)(float)n->f64;
                    n->ival = 0;
                } else {
                    n->ival = r.slot[so.slot];
                    n->fval = n->f64 = (double)n->ival;
                }
                break;
            case SG_AVG: {
                const int64_t cnt = r.slot[so.count_slot];
                const double s = f ? r.sum[so.sum] : (double)r.slot[so.slot];
                n->f64 = cnt > 0 ? s / (double)cnt : NAN;
                n->fval = f ? (double)(float)n->f64 : n->f64;
                n->ival = cnt;
            } break;
            case SG_MAX: case SG_MIN: {
                const uint32_t e = (uint32_t)r.slot[so.slot];
                const bool mx = n->red == SG_MAX;
                if (e == 0) {  // empty collection: identity element
                    if (f) n->fval = mx ? -INFINITY : INFINITY;
                    n->ival = mx ? INT32_MIN : INT32_MAX;
                    if (!f) n->fval = (double)n->ival;
                } else {
                    const uint32_t u = mx ? e : ~e;
                    const int32_t k = (int32_t)(u ^ 0x80000000u);
                    if (f) {
                        const bool nan = mx ? (k == INT32_MAX) : (k == INT32_MIN);
                        n->fval = nan ? NAN : (double)key_to_float(k);
                        n->ival = 0;
                    } else {
                        n->ival = k;
                        n->fval = (double)k;
                    }
                }
                n->f64 = n->fval;
            } break;
            case SG_COUNT:
                n->ival = r.slot[so.slot];
                n->fval = n->f64 = (double)n->ival;
                break;
        }
        n->state = publish_values ? ST_COMPUTED : ST_UNPUBLISHED;
    }
    for (auto* o : ip.outs) {
        o->state = publish_values ? ST_COMPUTED : ST_UNPUBLISHED;
        o->count = ip.base_count_slot >= 0 ? r.slot[ip.base_count_slot] : o->n;
    }
    for (auto* o : ip.compacted) o->count = r.scan_count;
}

// Verdicts of every clause from the read-back results; returns the program status.
sg_status assemble_verdicts(sg_program_s* P, const InstResult* results, std::vector<sg_verdict>& V) {
    const Plan& plan = P->plan;
    const int nc = (int)P->contracts.size();
    V.assign(nc, sg_verdict{});
    for (int i = 0; i < nc; ++i) {
        V[i].contract_id = P->contracts[i].id;
        V[i].kind = P->contracts[i].kind;
        V[i].check = P->contracts[i].check;
        V[i].holds = -1;
        V[i].first_index = -1;
        V[i].measure = 0.0;
    }
    for (auto& ip : plan.insts) {
        const InstResult& r = results[ip.result_index];
        for (auto& ch : ip.checks) {
            const uint64_t e = (uint64_t)r.slot[ch.slot];
            const int check = P->contracts[ch.contract].check;
            sg_verdict& v = V[ch.contract];
            const bool found = e != 0;
            v.first_index = found ? (int64_t)~e : -1;
            v.holds = check == SG_CHECK_EXISTS ? (found ? 1 : 0) : (found ? 0 : 1);
        }
    }
    // close contracts: need the scalar's float64 shadow and |x| sum
    for (auto& ip : plan.insts) {
        const InstResult& r = results[ip.result_index];
        for (auto& so : ip.scalars) {
            for (int ci : plan.active) {
                const Contract& c = P->contracts[ci];
                if (c.check != SG_CHECK_CLOSE || c.node != so.node) continue;
                const double s64 = r.sum[so.sum];
                const double s32 = (double)(float)s64;
                double asum = 0.0;
                for (auto& a : ip.abssums)
                    if (a.contract == ci) asum = r.sum[a.sum];
                const double dev = std::fabs(s32 - s64);
                V[ci].measure = dev;
                V[ci].holds = dev <= c.abs_tol + c.rel_tol * asum ? 1 : 0;
            }
        }
    }
    // count = old count: counts after the body (operands are never changed by a program)
    auto count_of = [&](const sg_node_s* x) -> int64_t {
        if (is_kernel_node(x)) return x->op == OPN_MATMUL ? x->n : x->count;
        for (auto& ip : plan.insts)
            for (auto* o : ip.outs)
                if (o == x) {
                    const InstResult& r = results[ip.result_index];
                    if (std::find(ip.compacted.begin(), ip.compacted.end(), x) != ip.compacted.end()) return r.scan_count;
                    return ip.base_count_slot >= 0 ? r.slot[ip.base_count_slot] : x->n;
                }
        return x->op == OPN_INPUT ? x->n : x->count;
    };
    for (int ci : plan.active) {
        const Contract& c = P->contracts[ci];
        if (c.check != SG_CHECK_COUNT_EQ) continue;
        const int64_t a = count_of(c.node), b = count_of(c.a);
        V[ci].holds = a == b ? 1 : 0;
        V[ci].measure = (double)(a - b);
    }
    for (int ci = 0; ci < nc; ++ci) {
        if (plan.prod_result.size() <= (size_t)ci || plan.prod_result[ci] < 0) continue;
        const InstResult& r = results[plan.prod_result[ci]];
        const uint64_t e = (uint64_t)r.slot[0];
        V[ci].first_index = e ? (int64_t)(~e & ((1ull << 40) - 1)) : -1;  // key = (probe << 40) | row
        V[ci].holds = e ? 0 : 1;
        V[ci].measure = r.sum[0];
    }
    sg_status status = SG_OK;
    for (int i = 0; i < nc; ++i)
        if (V[i].kind == SG_REQUIRE && V[i].holds == 0) { status = SG_PRE_VIOLATED; break; }
    if (status == SG_PRE_VIOLATED) {
        for (int i = 0; i < nc; ++i)
            if (V[i].kind == SG_ENSURE) V[i].holds = -1;
    } else {
        for (int i = 0; i < nc; ++i)
            if (V[i].kind == SG_ENSURE && V[i].holds == 0) { status = SG_POST_VIOLATED; break; }
    }
    return status;
}

// Enqueue one execution: every pass, then the copy of its results into `es.host` (pinned);
// `es.done` (when set) is recorded after the copy.  The results are read by finish_program.
sg_status launch_program(sg_program_s* P, ExecSlot& es) {
    sg_ctx_s* ctx = P->ctx;
    es.timed.clear();
    if (!P->plan.valid || P->plan.generation != ctx->generation) {
        sg_status st = build_plan(P, &P->plan);
        if (st != SG_OK) { P->plan.valid = false; return st; }
    }
    Plan& plan = P->plan;
    const int block = P->block ? P->block : ctx->block;
    const int unroll = P->unroll ? P->unroll : ctx->unroll;
    const int C0 = P->substeps ? P->substeps : ctx->substeps;
    // launch shape of one pass: unroll U, tiles of C sub-tiles, a grid of G resident blocks;
    // a pass whose per-lane accumulators and staging buffers would not fit in LDS runs with
    // a smaller unroll
    struct Geo { int U, C, grid; int64_t ntiles; size_t lds; };
    std::vector<Geo> geo(plan.insts.size());
    std::vector<void*> jks(plan.insts.size(), nullptr);  // specialized kernels (compiled once, cached)
    int64_t max_tiles = 1;
    for (size_t i = 0; i < plan.insts.size(); ++i) {
        const InstPlan& ip = plan.insts[i];
        Geo& g = geo[i];
        // a specialized kernel keeps its accumulators in registers: no LDS rows for them
        const int ns = ctx->specialize ? 0 : (int)ip.slot_kind.size(), nu = ctx->specialize ? 0 : ip.nsum;
        const int ce = inst_cemit(ip);
        for (g.U = unroll;; g.U /= 2) {
            g.C = stream_substeps(C0, block, g.U, ns, nu, ce, ip.scan_space != 0, 2);
            g.lds = stream_lds_bytes(ns, nu, ce, g.C, block, g.U, 2);
            if (g.lds <= kMaxDynamicLds || g.U == 1) break;
        }
        if (g.lds > kMaxDynamicLds)
            return fail(ctx, SG_E_UNSUPPORTED, "pass needs more LDS than a block has (per-lane accumulators); use a smaller block");
        if (ctx->specialize) {
            InstPlan& mip = plan.insts[i];
            if (!mip.jit || mip.jit_unroll != g.U || mip.jit_block != block) {
                sg_status js = jit_kernel(ctx, ip, g.U, block, &mip.jit);
                if (js != SG_OK) { mip.jit = nullptr; return js; }
                mip.jit_unroll = g.U;
                mip.jit_block = block;
            }
            jks[i] = mip.jit;
        }
        const int64_t sub_elems = (int64_t)block * 4 * g.U;
        const int64_t nsub = std::max<int64_t>(1, (ip.n + sub_elems - 1) / sub_elems);
        g.ntiles = (nsub + g.C - 1) / g.C;
        const bool waits = ip.scan_space != 0;
        if (jks[i]) {
            const int occ = coresident_blocks(jit_occupancy(jks[i], block, g.lds), lds_blocks_per_cu(g.lds), waits);
            g.grid = (int)std::max<int64_t>(1, std::min<int64_t>(g.ntiles, (int64_t)occ * ctx->num_cu));
        } else {
            g.grid = stream_grid(ctx, g.ntiles, true, g.U, block, g.lds, waits);
        }
        max_tiles = std::max(max_tiles, g.ntiles);
    }
    int nprod = 0, nnode = 0;
    for (auto& st : plan.steps) {
        nprod += st.kind == Step::PRODUCT;
        nnode += st.kind == Step::NODE;
    }
    const int64_t nres = (int64_t)plan.insts.size() + nprod + nnode;
    for (auto& ip : plan.insts)
        if (ip.result_index < 0 || ip.result_index >= nres) return fail(ctx, SG_E_UNSUPPORTED, "plan result index out of range");
    // look-back words: one per tile, then one per round (round bases)
    sg_status st = ensure_scratch(ctx, max_tiles, 2 * max_tiles + 2, nres);
    if (st != SG_OK) return st;
    for (auto* m : plan.mats)
        if ((st = alloc_output(ctx, m)) != SG_OK) return st;
    Scratch& S = ctx->scratch;

    std::vector<Timed>& timed = es.timed;
    auto t_begin = [&](const char* name) {
        if (!ctx->timing) return;
        hipEvent_t a = get_event(*es.events, timed.size() * 2), b = get_event(*es.events, timed.size() * 2 + 1);
        timed.push_back({name, a, b});
        (void)hipEventRecord(a, ctx->stream);
    };
    auto t_end = [&]() {
        if (!ctx->timing) return;
        (void)hipEventRecord(timed.back().b, ctx->stream);
    };
    // a streaming launch records its own events at the kernel's start and end
    auto t_launch = [&](const char* name) -> std::pair<hipEvent_t, hipEvent_t> {
        if (!ctx->timing) return {nullptr, nullptr};
        hipEvent_t a = get_event(*es.events, timed.size() * 2), b = get_event(*es.events, timed.size() * 2 + 1);
        timed.push_back({name, a, b});
        return {a, b};
    };

    plan.prod_result.assign(P->contracts.size(), -1);
    int next_prod = (int)plan.insts.size();
    int next_node = (int)plan.insts.size() + nprod;
    for (auto& step : plan.steps) {
        if (step.kind == Step::STREAM) {
            InstPlan& ip = plan.insts[step.inst];
            void* jk = jks[step.inst];
            const Geo& g = geo[step.inst];
            StreamArgs a;
            std::memset(&a, 0, sizeof(a));
            a.total_tiles = g.ntiles;
            a.acc = S.acc + (int64_t)ip.result_index * MAX_SLOTS * MAX_SPREAD;
            a.tags = S.tags;
            a.lookback = S.lookback;
            a.results = S.results + ip.result_index;
            a.ninst = 1;
            a.substeps = g.C;
            a.spread = MAX_SPREAD;
            a.lds_slots = jk ? 0 : (int)ip.slot_kind.size();
            a.lds_sums = jk ? 0 : ip.nsum;
            a.lds_cemit = inst_cemit(ip);
            a.epoch_val = next_epoch(ctx);
            a.wait_limit = ctx->wait_limit;
            fill_inst(ip, a.inst0, 0, g.ntiles, 0);
            std::memcpy(a.prog0, ip.prog.data(), ip.prog.size() * sizeof(SgOp));
            const auto ev = t_launch(jk ? "stream_spec" : "stream");
            if (jk) SG_HIP(ctx, jit_launch(jk, a, g.grid, block, g.lds, ctx->stream, ev.first, ev.second));
            else SG_HIP(ctx, sg_launch_stream(a, g.U, true, g.grid, block, g.lds, ctx->stream, ev.first, ev.second));
            ctx->last_grid = g.grid;
            ctx->last_block = block;
            ctx->last_unroll = g.U;
            ctx->last_substeps = g.C;
            ctx->last_lds = g.lds;
            for (auto* o : ip.compacted) o->count_dev = &S.results[ip.result_index].scan_count;
        } else if (step.kind == Step::NODE) {
            sg_node_s* nd = step.node;
            if ((st = alloc_output(ctx, nd)) != SG_OK) return st;
            t_begin(node_step_name(nd));
            st = run_node_step(ctx, plan, nd, S.results, S.results + next_node++);
            t_end();
            if (st != SG_OK) return st;
        } else if (step.kind == Step::GEMM) {
            sg_node_s* C = step.C;
            if ((st = alloc_output(ctx, C)) != SG_OK) return st;
            t_begin("gemm");
            SG_HIP(ctx, sg_launch_gemm_f32((const float*)step.A->dev, (const float*)step.B->dev, (float*)C->dev,
                                           step.A->rows, step.B->cols, step.A->cols, ctx->stream));
            t_end();
            C->count = C->n;
        } else {
            const int ri = next_prod++;
            plan.prod_result[step.contract] = ri;
            const int64_t M = step.A->rows, K = step.A->cols, N = step.B->cols, nvec = step.R->rows;
            if (step.C->rows != M || step.C->cols != N || step.B->rows != K || step.R->cols != N)
                return fail(ctx, SG_E_SHAPE, "product check: dimensions disagree");
            const double u = std::ldexp(1.0, -24);
            const double t = 2.0 * (double)K * u;
            const double tol = t / (1.0 - t) + std::ldexp(1.0, -40);
            if (nvec < 1 || nvec > 4) return fail(ctx, SG_E_UNSUPPORTED, "product check: 1 to 4 probe vectors");
            void* work = dev_alloc(ctx, sg_product_check_work_bytes(M, N, K));
            if (!work) return fail(ctx, SG_E_OOM, "product check workspace");
            t_begin("product_check");
            hipError_t e = sg_launch_product_check((const float*)step.C->dev, (const float*)step.A->dev,
                                                   (const float*)step.B->dev, (const float*)step.R->dev, M, N, K,
                                                   nvec, tol, (double*)work, S.results + ri, ctx->stream);
            t_end();
            dev_free(ctx, work);
            if (e != hipSuccess) return hip_fail(ctx, e, "product check");
        }
    }
    if (!es.owned) {  // the context's results, sized with the scratch
        es.host = ctx->host_results;
        es.host_cap = S.insts;
    }
    if (es.host_cap < nres) {
        if (es.owned && es.host) (void)hipHostFree(es.host);
        es.host = nullptr;
        es.host_cap = 0;
        if (!es.owned) return fail(ctx, SG_E_STATE, "result buffer too small");
        SG_HIP(ctx, hipHostMalloc((void**)&es.host, (size_t)nres * sizeof(InstResult), hipHostMallocDefault));
        es.host_cap = nres;
    }
    es.nres = nres;
    SG_HIP(ctx, hipMemcpyAsync(es.host, S.results, (size_t)nres * sizeof(InstResult), hipMemcpyDeviceToHost,
                               ctx->stream));
    if (es.done) SG_HIP(ctx, hipEventRecord(es.done, ctx->stream));
    return SG_OK;
}

// Wait for an enqueued execution, then account its timings, check the kernels' error words,
// assemble the verdicts and publish the values.
sg_status finish_program(sg_program_s* P, ExecSlot& es, sg_verdict* verdicts, int32_t cap, int32_t* nverdicts) {
    sg_ctx_s* ctx = P->ctx;
    Plan& plan = P->plan;
    Scratch& S = ctx->scratch;
    const int64_t nres = es.nres;
    if (es.done) SG_HIP(ctx, hipEventSynchronize(es.done));
    else SG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (auto& t : es.timed) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
            ctx->times[t.name].ms += ms;
            ctx->times[t.name].n += 1;
        }
    }
    for (int64_t i = 0; i < nres; ++i) {
        if (const uint32_t err = es.host[i].err) {
            // reset the state the kernels keep between launches, then report
            (void)sg_launch_zero((uint64_t*)S.base, (int64_t)(S.bytes / 8), ctx->stream);
            (void)hipStreamSynchronize(ctx->stream);
            ctx->epoch = 0;
            return fail(ctx, SG_E_DEVICE,
                        (err & ERR_LOOKBACK_TIMEOUT) && (err & ERR_FINALIZE_TIMEOUT)
                            ? "streaming kernel: bounded waits timed out (compaction prefix and result finalization)"
                        : (err & ERR_LOOKBACK_TIMEOUT) ? "streaming kernel: a bounded wait for the compaction prefix timed out"
                                                        : "streaming kernel: the bounded wait of the result finalization timed out");
        }
    }

    const int nc = (int)P->contracts.size();
    std::vector<sg_verdict> V;
    sg_status status = assemble_verdicts(P, es.host, V);
    const bool publish = status != SG_PRE_VIOLATED;
    for (auto& ip : plan.insts) publish_inst(ip, es.host[ip.result_index], publish);
    for (auto& step : plan.steps)
        if (step.kind == Step::GEMM) step.C->state = publish ? ST_COMPUTED : ST_UNPUBLISHED;
        else if (step.kind == Step::NODE) step.node->state = publish ? ST_COMPUTED : ST_UNPUBLISHED;
    if (nverdicts) *nverdicts = nc;
    if (verdicts)
        for (int i = 0; i < nc && i < cap; ++i) verdicts[i] = V[i];
    return status;
}

sg_status execute_program(sg_program_s* P, sg_verdict* verdicts, int32_t cap, int32_t* nverdicts) {
    if (!P->pending.empty()) return fail(P->ctx, SG_E_STATE, "execute: the program has pending launches; wait for them first");
    sg_ctx_s* ctx = P->ctx;
    // the context's pinned results (sized with the scratch) and its event pool
    ExecSlot es;
    es.events = &ctx->events;
    sg_status st = launch_program(P, es);
    if (st != SG_OK) return st;
    return finish_program(P, es, verdicts, cap, nverdicts);
}

}  // namespace sgrt

using namespace sgrt;

// =============================================================================================
// C ABI: programs, triggers, results
// =============================================================================================

extern "C" {

sg_status sg_program_create(sg_ctx ctx, sg_program* out) {
    if (!ctx || !out) return fail(ctx, SG_E_INVALID, "program_create: NULL argument");
    auto* p = new sg_program_s();
    p->ctx = ctx;
    ctx_retain(ctx);
    *out = p;
    return SG_OK;
}

// a program with pending launches is not changed (their results are read against its plan)
static sg_status check_idle(sg_program p, const char* what) {
    if (!p->pending.empty()) return fail(p->ctx, SG_E_STATE, std::string(what) + ": the program has pending launches");
    return SG_OK;
}

static sg_status add_contract(sg_program p, sgrt::Contract c, int32_t* id);

sg_status sg_program_add_root(sg_program p, sg_node n) {
    if (!p || !n) return fail(p ? p->ctx : nullptr, SG_E_INVALID, "add_root: NULL argument");
    if (sg_status st = check_idle(p, "add_root")) return st;
    if (n->ctx != p->ctx) return fail(p->ctx, SG_E_INVALID, "add_root: node of another context");
    retain(n);
    p->roots.push_back(n);
    p->plan.valid = false;
    // built-in clauses of the operations the root depends on (Listing 2 for compwise_divide),
    // in node creation order, once per operation
    std::vector<sg_node_s*> divs, stack{n};
    std::set<sg_node_s*> seen;
    while (!stack.empty()) {
        sg_node_s* x = stack.back();
        stack.pop_back();
        if (!x || !seen.insert(x).second) continue;
        if (x->op == OPN_ZIP && x->binop == SG_DIV) divs.push_back(x);
        stack.push_back(x->src[0]);
        stack.push_back(x->src[1]);
    }
    std::sort(divs.begin(), divs.end(), [](sg_node_s* a, sg_node_s* b) { return a->id < b->id; });
    for (sg_node_s* d : divs) {
        if (std::find(p->builtin_done.begin(), p->builtin_done.end(), d) != p->builtin_done.end()) continue;
        p->builtin_done.push_back(d);
        sg_pred nz = nullptr;
        if (sg_status st = sg_pred_cmp(SG_NE, 0.0, &nz)) return st;
        sgrt::Contract r;
        r.kind = SG_REQUIRE;
        r.check = SG_CHECK_FOR_ALL;
        r.node = d->src[1];
        r.pred = nz;
        sg_status st = add_contract(p, r, nullptr);
        sg_pred_release(nz);  // the clause holds its own reference
        if (st != SG_OK) return st;
        sgrt::Contract q;
        q.kind = SG_ENSURE;
        q.check = SG_CHECK_QUOTIENT;
        q.node = d;
        q.a = d->src[0];
        q.b = d->src[1];
        if ((st = add_contract(p, q, nullptr)) != SG_OK) return st;
    }
    return SG_OK;
}

static sg_status add_contract(sg_program p, sgrt::Contract c, int32_t* id) {
    if (sg_status st = check_idle(p, "contract")) return st;
    if (c.kind != SG_REQUIRE && c.kind != SG_ENSURE) return fail(p->ctx, SG_E_INVALID, "contract kind must be require or ensure");
    c.id = p->next_contract++;
    for (auto* n : {c.node, c.a, c.b, c.r}) retain(n);
    retain(c.pred);
    p->contracts.push_back(c);
    p->plan.valid = false;
    if (id) *id = c.id;
    return SG_OK;
}

sg_status sg_program_quant(sg_program p, sg_clause kind, sg_quant q, sg_node n, sg_pred pred, int32_t* id) {
    if (!p || !n || !pred) return fail(p ? p->ctx : nullptr, SG_E_INVALID, "quant: NULL argument");
    if (!is_collection(n)) return fail(p->ctx, SG_E_INVALID, "quant: operand is a scalar");
    sgrt::Contract c;
    c.kind = kind;
    c.check = q == SG_EXISTS ? SG_CHECK_EXISTS : SG_CHECK_FOR_ALL;
    c.node = n;
    c.pred = pred;
    return add_contract(p, c, id);
}

sg_status sg_program_sorted(sg_program p, sg_clause kind, sg_node n, int32_t* id) {
    if (!p || !n) return fail(p ? p->ctx : nullptr, SG_E_INVALID, "sorted: NULL argument");
    if (!is_collection(n)) return fail(p->ctx, SG_E_INVALID, "sorted: operand is a scalar");
    sgrt::Contract c;
    c.kind = kind;
    c.check = SG_CHECK_SORTED;
    c.node = n;
    return add_contract(p, c, id);
}

sg_status sg_program_close(sg_program p, sg_clause kind, sg_node s, double abs_tol, double rel_tol, int32_t* id) {
    if (!p || !s) return fail(p ? p->ctx : nullptr, SG_E_INVALID, "close: NULL argument");
    if (s->op != OPN_REDUCE || s->red != SG_SUM || s->src[0]->dtype != SG_F32)
        return fail(p->ctx, SG_E_INVALID, "close: operand must be a float sum");
    if (!(abs_tol >= 0) || !(rel_tol >= 0)) return fail(p->ctx, SG_E_INVALID, "close: tolerances must be >= 0");
    sgrt::Contract c;
    c.kind = kind;
    c.check = SG_CHECK_CLOSE;
    c.node = s;
    c.abs_tol = abs_tol;
    c.rel_tol = rel_tol;
    return add_contract(p, c, id);
}

sg_status sg_program_product(sg_program p, sg_clause kind, sg_node C, sg_node A, sg_node B, sg_node R, int32_t* id) {
    if (!p || !C || !A || !B || !R) return fail(p ? p->ctx : nullptr, SG_E_INVALID, "product: NULL argument");
    if (!A->matrix || !B->matrix || !C->matrix || !R->matrix) return fail(p->ctx, SG_E_SHAPE, "product: operands must be matrices");
    if (A->cols != B->rows || C->rows != A->rows || C->cols != B->cols || R->cols != B->cols)
        return fail(p->ctx, SG_E_SHAPE, "product: dimensions disagree");
    for (auto* n : {A, B, C, R})
        if (n->dtype != SG_F32) return fail(p->ctx, SG_E_DTYPE, "product: f32 matrices only");
    sgrt::Contract c;
    c.kind = kind;
    c.check = SG_CHECK_PRODUCT;
    c.node = C;
    c.a = A;
    c.b = B;
    c.r = R;
    return add_contract(p, c, id);
}

sg_status sg_program_count_eq(sg_program p, sg_clause kind, sg_node n, sg_node other, int32_t* id) {
    if (!p || !n || !other) return fail(p ? p->ctx : nullptr, SG_E_INVALID, "count_eq: NULL argument");
    if (!is_collection(n) || !is_collection(other)) return fail(p->ctx, SG_E_INVALID, "count_eq: operands must be collections");
    if (n->ctx != p->ctx || other->ctx != p->ctx) return fail(p->ctx, SG_E_INVALID, "count_eq: node of another context");
    sgrt::Contract c;
    c.kind = kind;
    c.check = SG_CHECK_COUNT_EQ;
    c.node = n;
    c.a = other;
    return add_contract(p, c, id);
}

sg_status sg_program_split(sg_program p, sg_node n) {
    if (!p || !n) return fail(p ? p->ctx : nullptr, SG_E_INVALID, "split: NULL argument");
    if (sg_status st = check_idle(p, "split")) return st;
    retain(n);
    p->splits.push_back(n);
    p->plan.valid = false;
    return SG_OK;
}

sg_status sg_program_execute(sg_program p, sg_verdict* verdicts, int32_t cap, int32_t* nverdicts) {
    if (!p) return fail(nullptr, SG_E_INVALID, "execute: NULL program");
    if (cap < 0 || (cap > 0 && !verdicts)) return fail(p->ctx, SG_E_INVALID, "execute: bad verdict buffer");
    const sg_status ps = apply_plan_source(p);
    if (ps != SG_OK) return ps;
    return execute_program(p, verdicts, cap, nverdicts);
}

sg_status sg_program_launch(sg_program p) {
    if (!p) return fail(nullptr, SG_E_INVALID, "launch: NULL program");
    if ((int)p->pending.size() >= sg_program_s::kMaxPending)
        return fail(p->ctx, SG_E_STATE, "launch: too many pending launches; wait for one first");
    const sg_status ps = apply_plan_source(p);  // only before the first pending launch
    if (ps != SG_OK) return ps;
    // a plan that needs rebuilding would no longer match the pending launches' results
    if (!p->pending.empty() && (!p->plan.valid || p->plan.generation != p->ctx->generation))
        return fail(p->ctx, SG_E_STATE, "launch: the program or its context changed while launches are pending");
    int slot = 0;
    for (int i = 0; i < sg_program_s::kMaxPending; ++i) {
        bool used = false;
        for (int q : p->pending) used |= q == i;
        if (!used) { slot = i; break; }
    }
    ExecSlot& es = p->slots[slot];
    es.owned = true;
    es.events = &es.own_events;
    if (!es.done && hipEventCreateWithFlags(&es.done, hipEventDisableTiming) != hipSuccess) {
        es.done = nullptr;
        return fail(p->ctx, SG_E_DEVICE, "launch: event creation failed");
    }
    sg_status st = launch_program(p, es);
    if (st != SG_OK) return st;
    p->pending.push_back(slot);
    return SG_OK;
}

sg_status sg_program_wait(sg_program p, sg_verdict* verdicts, int32_t cap, int32_t* nverdicts) {
    if (!p) return fail(nullptr, SG_E_INVALID, "wait: NULL program");
    if (cap < 0 || (cap > 0 && !verdicts)) return fail(p->ctx, SG_E_INVALID, "wait: bad verdict buffer");
    if (p->pending.empty()) return fail(p->ctx, SG_E_STATE, "wait: no pending launch");
    const int slot = p->pending.front();
    p->pending.pop_front();
    return finish_program(p, p->slots[slot], verdicts, cap, nverdicts);
}

sg_status sg_program_release(sg_program p) {
    if (!p) return SG_E_INVALID;
    if (--p->refs > 0) return SG_OK;
    if (!p->pending.empty()) (void)hipStreamSynchronize(p->ctx->stream);  // copies into the slots end first
    for (auto& es : p->slots) {
        if (es.owned && es.host) (void)hipHostFree(es.host);
        if (es.done) (void)hipEventDestroy(es.done);
        for (hipEvent_t e : es.own_events) (void)hipEventDestroy(e);
    }
    for (auto* r : p->roots) release(r);
    for (auto& c : p->contracts) {
        for (auto* n : {c.node, c.a, c.b, c.r}) release(n);
        release(c.pred);
    }
    for (auto* s : p->splits) release(s);
    sg_ctx_s* ctx = p->ctx;
    delete p;
    ctx_release(ctx);
    return SG_OK;
}

sg_status sg_execute(sg_ctx ctx, const sg_node* roots, int32_t nroots) {
    if (!ctx || nroots < 0 || (nroots > 0 && !roots)) return fail(ctx, SG_E_INVALID, "execute: bad roots");
    sg_program p;
    sg_status st = sg_program_create(ctx, &p);
    if (st != SG_OK) return st;
    for (int i = 0; i < nroots; ++i)
        if ((st = sg_program_add_root(p, roots[i])) != SG_OK) { sg_program_release(p); return st; }
    st = execute_program(p, nullptr, 0, nullptr);
    sg_program_release(p);
    return st;
}

static sg_status trigger(sg_node n) {
    if (n->state == ST_COMPUTED) return SG_OK;
    if (n->state == ST_UNPUBLISHED) return fail(n->ctx, SG_E_STATE, "value not published: a require clause failed");
    sg_node_s* r = n;
    return sg_execute(n->ctx, &r, 1);
}

sg_status sg_scalar_get(sg_node s, double* f, int64_t* i) {
    if (!s) return fail(nullptr, SG_E_INVALID, "scalar_get: NULL node");
    if (s->op != OPN_REDUCE && s->op != OPN_GAUSS) return fail(s->ctx, SG_E_INVALID, "scalar_get: not a scalar node");
    sg_status st = trigger(s);
    if (st != SG_OK) return st;
    if (f) *f = s->fval;
    if (i) *i = s->ival;
    return SG_OK;
}

sg_status sg_scalar_shadow(sg_node s, double* f64) {
    if (!s || !f64) return fail(s ? s->ctx : nullptr, SG_E_INVALID, "scalar_shadow: NULL argument");
    if (s->op != OPN_REDUCE) return fail(s->ctx, SG_E_INVALID, "scalar_shadow: not a scalar node");
    sg_status st = trigger(s);
    if (st != SG_OK) return st;
    *f64 = s->f64;
    return SG_OK;
}

sg_status sg_count(sg_node c, int64_t* n) {
    if (!c || !n) return fail(c ? c->ctx : nullptr, SG_E_INVALID, "count: NULL argument");
    if (!is_collection(c)) return fail(c->ctx, SG_E_INVALID, "count: not a collection");
    sg_status st = trigger(c);
    if (st != SG_OK) return st;
    *n = c->count;
    return SG_OK;
}

sg_status sg_to_host(sg_node c, void* dst, int64_t cap, int64_t* n) {
    if (!c || cap < 0 || (cap > 0 && !dst)) return fail(c ? c->ctx : nullptr, SG_E_INVALID, "to_host: bad argument");
    if (!is_collection(c)) return fail(c->ctx, SG_E_INVALID, "to_host: not a collection");
    sg_status st = trigger(c);
    if (st != SG_OK) return st;
    if (!c->dev && c->count > 0) return fail(c->ctx, SG_E_STATE, "to_host: collection has no storage");
    const int64_t m = std::min(cap, c->count);
    if (m > 0) {
        SG_HIP(c->ctx, hipMemcpyAsync(dst, c->dev, (size_t)m * 4, hipMemcpyDeviceToHost, c->ctx->stream));
        SG_HIP(c->ctx, hipStreamSynchronize(c->ctx->stream));
    }
    if (n) *n = c->count;
    return SG_OK;
}

sg_status sg_item(sg_node c, int64_t i, double* f, int64_t* iv) {
    if (!c) return fail(nullptr, SG_E_INVALID, "item: NULL node");
    if (!is_collection(c)) return fail(c->ctx, SG_E_INVALID, "item: not a collection");
    sg_status st = trigger(c);
    if (st != SG_OK) return st;
    if (i < 0 || i >= c->count) return fail(c->ctx, SG_E_INVALID, "item: index out of range (0 <= i < count)");
    if (!c->dev) return fail(c->ctx, SG_E_STATE, "item: collection has no storage");
    uint32_t bits = 0;
    SG_HIP(c->ctx, hipMemcpyAsync(&bits, (const char*)c->dev + (size_t)i * 4, 4, hipMemcpyDeviceToHost, c->ctx->stream));
    SG_HIP(c->ctx, hipStreamSynchronize(c->ctx->stream));
    if (c->dtype == SG_F32) {
        float v;
        std::memcpy(&v, &bits, 4);
        if (f) *f = (double)v;
        if (iv) *iv = 0;
    } else {
        const int32_t v = (int32_t)bits;
        if (f) *f = (double)v;
        if (iv) *iv = v;
    }
    return SG_OK;
}

sg_status sg_device_ptr(sg_node c, void** dev, int64_t* n) {
    if (!c || !dev) return fail(c ? c->ctx : nullptr, SG_E_INVALID, "device_ptr: NULL argument");
    if (!is_collection(c)) return fail(c->ctx, SG_E_INVALID, "device_ptr: not a collection");
    sg_status st = trigger(c);
    if (st != SG_OK) return st;
    *dev = c->dev;
    if (n) *n = c->count;
    return SG_OK;
}

}  // extern "C"
