// Plan choice for a program: the autotuner (measure every candidate plan, keep the fastest)
// and the learned selector (predict the log run time of every candidate with the cost-model
// MLP and keep the argmin, falling back to the autotuner when the chain lies outside the
// training range or the two best predictions are too close to call).
//
// A plan is a launch configuration of the streaming kernel (block size, values per lane,
// sub-tiles per tile) plus an optional fusion split point: the paper's optimizer merges
// kernel vertices greedily (Section 5); the split lets a plan end a fused pass early.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <set>
#include <vector>

#include "sg_kernels.h"
#include "sg_runtime.h"

using namespace sg;
using namespace sgrt;

extern "C" sg_status sg_mlp_predict(sg_mlp_s* m, const float* X_dev, int64_t n, float* Y_dev);
int sg_stream_occupancy(int unroll, bool inl, int block, size_t lds_bytes);

namespace {

constexpr int NF = 24;

std::vector<sg_node_s*> split_candidates(sg_program_s* P) {
    std::set<sg_node_s*> seen;
    std::vector<sg_node_s*> out;
    std::function<void(sg_node_s*)> walk = [&](sg_node_s* n) {
        if (!n || seen.count(n)) return;
        seen.insert(n);
        walk(n->src[0]);
        walk(n->src[1]);
        if ((n->op == OPN_MAP || n->op == OPN_ZIP || n->op == OPN_FILTER)) out.push_back(n);
    };
    for (auto* r : P->roots) walk(r);
    for (auto& c : P->contracts) walk(c.node);
    std::sort(out.begin(), out.end(), [](sg_node_s* a, sg_node_s* b) { return a->id < b->id; });
    return out;
}

int fn_count(const sg_fn_s* f, int kind_group) {
    if (!f) return 0;
    if (f->kind == FK_COMPOSE) return fn_count(f->f, kind_group) + fn_count(f->g, kind_group);
    if (f->kind == FK_EXPR) {  // each operation of the expression in its group
        int c = 0;
        for (const ExprNode& e : *f->expr) {
            const int g = e.kind == EX_SQRT ? 1 : e.kind == EX_EXP ? 2
                        : (e.kind == EX_NEG || e.kind == EX_ABS) ? 3
                        : (e.kind >= EX_ADD) ? 0 : -1;
            c += g == kind_group;
        }
        return c;
    }
    int g;
    if (f->kind == FK_AFFINE || f->kind == FK_ADDC || f->kind == FK_MULC) {
        g = 0;
    } else {
        const int k = (int)f->a;
        g = (k == SG_FN_SQRT || k == SG_FN_SQRT_ABS) ? 1 : (k == SG_FN_EXP || k == SG_FN_EXP_NEG_SQ) ? 2 : 3;
    }
    return g == kind_group ? 1 : 0;
}

struct ApplyPlan {
    sg_program_s* P;
    int block, unroll, substeps;
    sg_node_s* split;
    ApplyPlan(sg_program_s* p, const sg_plan* plan, const std::vector<sg_node_s*>& cands) : P(p) {
        block = P->block; unroll = P->unroll; substeps = P->substeps; split = P->plan_split;
        P->block = plan->block; P->unroll = plan->unroll; P->substeps = plan->substeps;
        P->plan_split = (plan->split >= 0 && plan->split < (int)cands.size()) ? cands[plan->split] : nullptr;
        P->plan.valid = false;
    }
    void keep() { block = P->block; unroll = P->unroll; substeps = P->substeps; split = P->plan_split; }
    ~ApplyPlan() {
        P->block = block; P->unroll = unroll; P->substeps = substeps;
        if (P->plan_split != split) { P->plan_split = split; P->plan.valid = false; }
    }
};

bool valid_plan(const sg_plan* p) {
    return p && p->block >= 64 && p->block <= 1024 && p->block % 64 == 0 &&
           (p->unroll == 1 || p->unroll == 2 || p->unroll == 4) && p->substeps >= 1 && p->substeps <= 64;
}

// 16 chain features and 8 plan features (see the header for the list).
sg_status features(sg_program_s* P, const sg_plan* plan, const std::vector<sg_node_s*>& cands, float* f) {
    std::memset(f, 0, NF * sizeof(float));
    std::set<sg_node_s*> seen;
    std::map<sg_node_s*, int> depth;
    std::set<sg_node_s*> inputs;
    int64_t n = 0;
    bool f32 = true;
    std::function<int(sg_node_s*)> walk = [&](sg_node_s* x) -> int {
        if (!x) return 0;
        auto it = depth.find(x);
        if (it != depth.end()) return it->second;
        int d = 0;
        if (x->op == OPN_INPUT) {
            inputs.insert(x);
            n = std::max(n, x->n);
            f32 = f32 && x->dtype == SG_F32;
        } else {
            d = 1 + std::max(walk(x->src[0]), walk(x->src[1]));
        }
        depth[x] = d;
        if (seen.insert(x).second) {
            switch (x->op) {
                case OPN_MAP:
                    for (int g = 0; g < 4; ++g) f[g] += (float)fn_count(x->fn, g);
                    break;
                case OPN_ZIP: f[x->binop == SG_MUL ? 5 : 4] += 1; break;
                case OPN_FILTER: f[6] += 1; break;
                case OPN_REDUCE:
                    f[x->red == SG_SUM || x->red == SG_AVG ? 7 : x->red == SG_COUNT ? 9 : 8] += 1;
                    break;
                default: break;
            }
        }
        return d;
    };
    int dmax = 0;
    for (auto* r : P->roots) dmax = std::max(dmax, walk(r));
    for (auto& c : P->contracts) {
        dmax = std::max(dmax, walk(c.node));
        if (c.check == SG_CHECK_FOR_ALL || c.check == SG_CHECK_EXISTS) f[10] += 1;
        else f[11] += 1;
    }
    f[12] = (float)dmax;
    f[13] = n > 0 ? (float)std::log2((double)n) : 0.f;
    f[14] = f32 ? 1.f : 0.f;
    f[15] = (float)inputs.size();
    // plan features
    f[16] = (float)std::log2((double)plan->block);
    f[17] = (float)std::log2((double)plan->unroll);
    f[18] = (float)std::log2((double)plan->substeps);
    f[19] = plan->split >= 0 ? 1.f : 0.f;
    f[20] = plan->split >= 0 && !cands.empty() ? (float)(plan->split + 1) / (float)cands.size() : 0.f;
    ApplyPlan ap(P, plan, cands);
    Plan tmp;
    sg_status st = build_plan(P, &tmp);
    if (st != SG_OK) return st;
    double bytes = 0;
    for (auto& ip : tmp.insts) bytes += 4.0 * (double)(ip.sources.size() + ip.outs.size());
    f[21] = (float)tmp.insts.size();
    f[22] = (float)bytes;
    int occ = 0;
    for (auto& ip : tmp.insts) {
        // the same LDS rows as the execution: none for the accumulators of a specialized kernel
        const bool spec = P->ctx->specialize;
        const int ns = spec ? 0 : (int)ip.slot_kind.size(), nu = spec ? 0 : ip.nsum, ce = inst_cemit(ip);
        const int C = stream_substeps(plan->substeps, plan->block, plan->unroll, ns, nu, ce, ip.scan_space != 0, 2);
        const size_t lds = stream_lds_bytes(ns, nu, ce, C, plan->block, plan->unroll, 2);
        const int o = std::min(sg_stream_occupancy(plan->unroll, true, plan->block, lds), lds_blocks_per_cu(lds));
        occ = occ == 0 ? o : std::min(occ, o);
    }
    f[23] = (float)occ;  // resident blocks per CU of the tightest pass
    return SG_OK;
}

}  // namespace

extern "C" {

sg_status sg_program_split_candidates(sg_program p, int32_t* n) {
    if (!p || !n) return fail(p ? p->ctx : nullptr, SG_E_INVALID, "split_candidates: NULL argument");
    *n = (int32_t)split_candidates(p).size();
    return SG_OK;
}

sg_status sg_program_set_plan(sg_program p, const sg_plan* plan) {
    if (!p) return fail(nullptr, SG_E_INVALID, "set_plan: NULL program");
    if (!p->pending.empty()) return fail(p->ctx, SG_E_STATE, "set_plan: the program has pending launches");
    if (!plan) {
        p->block = p->unroll = p->substeps = 0;
        p->plan_split = nullptr;
        p->plan.valid = false;
        p->plan_from = SG_PLAN_DEFAULT;
        p->plan_auto_tried = false;  // the context's plan source applies again
        return SG_OK;
    }
    if (!valid_plan(plan)) return fail(p->ctx, SG_E_INVALID, "set_plan: block 64..1024 (x64), unroll 1/2/4, substeps 1..64");
    auto cands = split_candidates(p);
    ApplyPlan ap(p, plan, cands);
    ap.keep();
    p->plan_from = SG_PLAN_SET;
    return SG_OK;
}

sg_status sg_program_features(sg_program p, const sg_plan* plan, float* f24) {
    if (!p || !f24 || !valid_plan(plan)) return fail(p ? p->ctx : nullptr, SG_E_INVALID, "features: bad argument");
    if (!p->pending.empty()) return fail(p->ctx, SG_E_STATE, "features: the program has pending launches");
    return features(p, plan, split_candidates(p), f24);
}

// Device time (ms, median of `reps` executions after one warm-up) of each plan.
sg_status sg_program_time_plans(sg_program p, const sg_plan* plans, int32_t n, int32_t reps, double* ms_out) {
    if (!p || !plans || n < 1 || reps < 1 || !ms_out) return fail(p ? p->ctx : nullptr, SG_E_INVALID, "time_plans: bad argument");
    if (!p->pending.empty()) return fail(p->ctx, SG_E_STATE, "time_plans: the program has pending launches");
    sg_ctx_s* ctx = p->ctx;
    auto cands = split_candidates(p);
    const bool timing = ctx->timing;
    ctx->timing = true;
    sg_status result = SG_OK;
    for (int i = 0; i < n && result == SG_OK; ++i) {
        if (!valid_plan(&plans[i])) { result = fail(ctx, SG_E_INVALID, "time_plans: invalid plan"); break; }
        ApplyPlan ap(p, &plans[i], cands);
        std::vector<double> t;
        for (int r = 0; r <= reps; ++r) {
            auto saved = ctx->times;
            ctx->times.clear();
            sg_status st = execute_program(p, nullptr, 0, nullptr);
            if (st != SG_OK && st != SG_PRE_VIOLATED && st != SG_POST_VIOLATED) { result = st; break; }
            double ms = 0;
            for (auto& kv : ctx->times) ms += kv.second.ms;
            ctx->times = saved;
            if (r > 0) t.push_back(ms);
        }
        if (result != SG_OK) break;
        std::sort(t.begin(), t.end());
        ms_out[i] = t[t.size() / 2];
    }
    ctx->timing = timing;
    return result;
}

// Time every candidate and keep the fastest as the program's plan.
sg_status sg_autotune(sg_program p, const sg_plan* plans, int32_t n, int32_t reps, int32_t* best, double* ms_out) {
    std::vector<double> ms(n > 0 ? n : 1);
    sg_status st = sg_program_time_plans(p, plans, n, reps, ms.data());
    if (st != SG_OK) return st;
    int b = (int)(std::min_element(ms.begin(), ms.begin() + n) - ms.begin());
    if (best) *best = b;
    if (ms_out) std::memcpy(ms_out, ms.data(), n * sizeof(double));
    st = sg_program_set_plan(p, &plans[b]);
    if (st == SG_OK) p->plan_from = SG_PLAN_AUTOTUNE;
    return st;
}

// The built-in candidate plans of a plan source: ten launch shapes, and two with the first
// fusion split point when the program has one.
static std::vector<sg_plan> builtin_plans(sg_program_s* p) {
    std::vector<sg_plan> c = {{64, 1, 8, -1},  {128, 2, 8, -1}, {256, 1, 8, -1}, {256, 2, 8, -1},
                              {256, 4, 8, -1}, {256, 2, 32, -1}, {512, 2, 4, -1}, {512, 4, 8, -1},
                              {1024, 1, 4, -1}, {1024, 2, 8, -1}};
    if (!split_candidates(p).empty()) {
        c.push_back({256, 2, 8, 0});
        c.push_back({256, 4, 8, 0});
    }
    return c;
}

sg_status sg_ctx_set_plan_source(sg_ctx ctx, int32_t source, const sg_plan* plans, int32_t n, int32_t reps,
                                 sg_mlp model, sg_tunedb db, float margin) {
    if (!ctx) return fail(nullptr, SG_E_INVALID, "set_plan_source: NULL context");
    if (source < SG_PLAN_DEFAULT || source > SG_PLAN_LEARNED)
        return fail(ctx, SG_E_INVALID, "set_plan_source: source must be SG_PLAN_DEFAULT, _AUTOTUNE or _LEARNED");
    if (n < 0 || (n > 0 && !plans) || reps < 1 || !(margin >= 0.0f))
        return fail(ctx, SG_E_INVALID, "set_plan_source: bad plans, repetitions or margin");
    for (int i = 0; i < n; ++i)
        if (!valid_plan(&plans[i])) return fail(ctx, SG_E_INVALID, "set_plan_source: invalid plan");
    if (source == SG_PLAN_LEARNED) {
        if (!model) return fail(ctx, SG_E_INVALID, "set_plan_source: the learned source needs a model");
        if (model->ctx != ctx) return fail(ctx, SG_E_INVALID, "set_plan_source: model of another context");
        if (!model->norm_set) return fail(ctx, SG_E_STATE, "set_plan_source: the model has no standardization");
    }
    if (db && tunedb_ctx(db) != ctx) return fail(ctx, SG_E_INVALID, "set_plan_source: database of another context");
    ctx->plan_source = source;
    ctx->plan_cands.assign(plans, plans + n);
    ctx->plan_model = source == SG_PLAN_LEARNED ? model : nullptr;
    ctx->plan_db = source == SG_PLAN_DEFAULT ? nullptr : db;
    ctx->plan_margin = margin;
    ctx->plan_reps = reps;
    return SG_OK;
}

sg_status sg_program_plan(sg_program p, sg_plan* plan, int32_t* source) {
    if (!p || !plan || !source) return fail(p ? p->ctx : nullptr, SG_E_INVALID, "program_plan: NULL argument");
    const sg_ctx_s* ctx = p->ctx;
    plan->block = p->block ? p->block : ctx->block;
    plan->unroll = p->unroll ? p->unroll : ctx->unroll;
    plan->substeps = p->substeps ? p->substeps : ctx->substeps;
    plan->split = -1;
    if (p->plan_split) {
        auto cands = split_candidates(p);
        for (size_t i = 0; i < cands.size(); ++i)
            if (cands[i] == p->plan_split) plan->split = (int32_t)i;
    }
    *source = p->plan_from;
    return SG_OK;
}

}  // extern "C"

// ---- learned selector -----------------------------------------------------------------------

extern "C" {

// Feature standardization of the cost model: x' = (x - mean) / scale; lo/hi is the range of
// each raw feature in the training set (outside it the selector falls back).
sg_status sg_mlp_set_norm(sg_mlp m, const float* mean24, const float* scale24, const float* lo24, const float* hi24) {
    if (!m || !mean24 || !scale24 || !lo24 || !hi24) return fail(nullptr, SG_E_INVALID, "mlp_set_norm: NULL argument");
    std::memcpy(m->mean, mean24, sizeof(m->mean));
    std::memcpy(m->scale, scale24, sizeof(m->scale));
    std::memcpy(m->lo, lo24, sizeof(m->lo));
    std::memcpy(m->hi, hi24, sizeof(m->hi));
    m->norm_set = true;
    return SG_OK;
}

sg_status sg_mlp_get_norm(sg_mlp m, float* mean24, float* scale24, float* lo24, float* hi24) {
    if (!m || !mean24 || !scale24 || !lo24 || !hi24) return fail(nullptr, SG_E_INVALID, "mlp_get_norm: NULL argument");
    if (!m->norm_set) return fail(m->ctx, SG_E_STATE, "mlp_get_norm: the model has no standardization");
    std::memcpy(mean24, m->mean, sizeof(m->mean));
    std::memcpy(scale24, m->scale, sizeof(m->scale));
    std::memcpy(lo24, m->lo, sizeof(m->lo));
    std::memcpy(hi24, m->hi, sizeof(m->hi));
    return SG_OK;
}

// Predict every candidate's log run time and keep the argmin.  *fallback = 1 when a raw
// feature is outside the training range or the best two predictions differ by less than
// `margin` (log units); the plan is then left unchanged for the autotuner to decide.
sg_status sg_select_plan(sg_mlp m, sg_program p, const sg_plan* plans, int32_t n, float margin, int32_t* best,
                         float* pred_out, int32_t* fallback) {
    if (!m || !p || !plans || n < 1 || !best || !fallback) return fail(p ? p->ctx : nullptr, SG_E_INVALID, "select_plan: bad argument");
    sg_ctx_s* ctx = p->ctx;
    if (!m->norm_set) return fail(ctx, SG_E_STATE, "select_plan: cost model has no normalization");
    const sg_mlp_s& N = *m;
    auto cands = split_candidates(p);
    std::vector<float> X((size_t)n * NF);
    bool ood = false;
    for (int i = 0; i < n; ++i) {
        if (!valid_plan(&plans[i])) return fail(ctx, SG_E_INVALID, "select_plan: invalid plan");
        float f[NF];
        sg_status st = features(p, &plans[i], cands, f);
        if (st != SG_OK) return st;
        for (int k = 0; k < NF; ++k) {
            if (f[k] < N.lo[k] || f[k] > N.hi[k]) ood = true;
            X[(size_t)i * NF + k] = (f[k] - N.mean[k]) / N.scale[k];
        }
    }
    void* buf = dev_alloc(ctx, X.size() * 4 + (size_t)n * 4);
    if (!buf) return fail(ctx, SG_E_OOM, "select_plan: workspace");
    float* Xd = (float*)buf;
    float* Yd = Xd + X.size();
    std::vector<float> Y(n);
    hipError_t e = hipMemcpyAsync(Xd, X.data(), X.size() * 4, hipMemcpyHostToDevice, ctx->stream);
    sg_status st = e == hipSuccess ? sg_mlp_predict(m, Xd, n, Yd) : hip_fail(ctx, e, "select_plan: upload");
    if (st == SG_OK) {
        e = hipMemcpyAsync(Y.data(), Yd, (size_t)n * 4, hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) st = hip_fail(ctx, e, "select_plan: read-back");
    }
    dev_free(ctx, buf);
    if (st != SG_OK) return st;
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return Y[a] < Y[b]; });
    *best = order[0];
    *fallback = ood || (n > 1 && Y[order[1]] - Y[order[0]] < margin) ? 1 : 0;
    if (pred_out) std::memcpy(pred_out, Y.data(), (size_t)n * 4);
    if (*fallback) return SG_OK;
    st = sg_program_set_plan(p, &plans[*best]);
    if (st == SG_OK) p->plan_from = SG_PLAN_LEARNED;
    return st;
}


}  // extern "C"

namespace sgrt {

// Before a program's first execution or launch: a program with no plan of its own gets one from
// its context's plan source (once; sg_program_set_plan(p, NULL) re-arms it).  The autotuner
// runs the program itself (through the internal execution path) on every candidate.
sg_status apply_plan_source(sg_program_s* p) {
    sg_ctx_s* ctx = p->ctx;
    if (ctx->plan_source == SG_PLAN_DEFAULT || p->plan_auto_tried || p->block != 0 || !p->pending.empty())
        return SG_OK;
    p->plan_auto_tried = true;
    const std::vector<sg_plan> c = ctx->plan_cands.empty() ? builtin_plans(p) : ctx->plan_cands;
    const int32_t n = (int32_t)c.size();
    int32_t best = 0, fallback = 1;
    if (ctx->plan_source == SG_PLAN_LEARNED) {
        sg_status st = sg_select_plan(ctx->plan_model, p, c.data(), n, ctx->plan_margin, &best, nullptr, &fallback);
        if (st != SG_OK || !fallback) return st;
    }
    // the autotuner: the source itself, or the learned source's fallback
    if (ctx->plan_db) return sg_autotune_db(p, ctx->plan_db, c.data(), n, ctx->plan_reps, &best, nullptr, nullptr);
    return sg_autotune(p, c.data(), n, ctx->plan_reps, &best, nullptr);
}

}  // namespace sgrt
