// What the plan choice keeps between processes: the autotuner's timings (an append-only file
// keyed by program and plan) and the cost model's parameters with its standardization.
//
// The optimizer of Section 5 chooses one plan per pending computation; here that choice is
// measured (the autotuner) or predicted (the cost model), and both the measurements and the
// trained model are worth keeping: a later process tunes a program it has seen before without
// timing it again, and selects plans with a model trained earlier.
//
// Timing file: text, one record per line, appended and flushed as it is measured:
//     sgtune1 <program key, 16 hex digits> <block> <unroll> <substeps> <split> <milliseconds>
// The key covers the program's operations, constants, element types and lengths, its clauses
// and the context mode, the device's architecture and compute-unit count; the last record of
// a (key, plan) pair wins.  Model file: binary little-endian, the 8 bytes "sgmlp001", then
// 5825 float32 parameters, Adam's first and second moments (5825 float32 each), the 4 x 24
// float32 standardization vectors (mean, scale, lo, hi) and the int32 Adam step count, so
// that training resumes where it stopped.
#include <hip/hip_runtime.h>

#include <cinttypes>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <functional>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "sg_runtime.h"

using namespace sgrt;

struct sg_tunedb_s {
    sg_ctx_s* ctx = nullptr;
    std::string path;
    FILE* f = nullptr;  // opened for appending
    std::map<std::tuple<uint64_t, int, int, int, int>, double> ms;
    int64_t records = 0;
};

namespace {

constexpr uint64_t kFnvOffset = 0xcbf29ce484222325ull, kFnvPrime = 0x100000001b3ull;

struct Hasher {
    uint64_t h = kFnvOffset;
    void bytes(const void* p, size_t n) {
        const unsigned char* c = (const unsigned char*)p;
        for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * kFnvPrime;
    }
    template <class T>
    void val(const T& v) { bytes(&v, sizeof(v)); }
};

void hash_fn(Hasher& H, const sg_fn_s* f) {
    if (!f) { H.val<int>(-1); return; }
    H.val(f->kind);
    H.val(f->a);
    H.val(f->b);
    if (f->kind == FK_COMPOSE) { hash_fn(H, f->f); hash_fn(H, f->g); }
    if (f->kind == FK_EXPR) {
        H.val(f->expr_root);
        for (const ExprNode& e : *f->expr) { H.val(e.kind); H.val(e.c); H.val(e.a); H.val(e.b); }
    }
}

void hash_pred(Hasher& H, const sg_pred_s* p) {
    if (!p) { H.val<int>(-1); return; }
    H.val(p->kind);
    H.val(p->cmp);
    H.val(p->c);
    H.val(p->lo);
    H.val(p->hi);
    hash_pred(H, p->p);
    hash_pred(H, p->q);
}

// Every node reachable from the program, in creation order, with its operands named by their
// position in that order (so the key does not depend on addresses or on the ids of nodes
// created elsewhere); a wrapped input contributes its type and length, not its contents.
uint64_t program_key(sg_program_s* P) {
    std::set<sg_node_s*> seen;
    std::vector<sg_node_s*> nodes;
    std::function<void(sg_node_s*)> walk = [&](sg_node_s* n) {
        if (!n || seen.count(n)) return;
        seen.insert(n);
        walk(n->src[0]);
        walk(n->src[1]);
        nodes.push_back(n);
    };
    for (auto* r : P->roots) walk(r);
    for (auto& c : P->contracts) { walk(c.node); walk(c.a); walk(c.b); walk(c.r); }
    std::sort(nodes.begin(), nodes.end(), [](sg_node_s* a, sg_node_s* b) { return a->id < b->id; });
    std::map<sg_node_s*, int> pos;
    for (size_t i = 0; i < nodes.size(); ++i) pos[nodes[i]] = (int)i;
    auto ref = [&](sg_node_s* n) { return n ? pos[n] : -1; };
    Hasher H;
    H.bytes("sgkey1", 6);
    H.bytes(P->ctx->arch.data(), P->ctx->arch.size());
    H.val(P->ctx->num_cu);
    H.val((int)P->ctx->mode);
    for (sg_node_s* n : nodes) {
        H.val(n->op);
        H.val((int)n->dtype);
        H.val(n->n);
        H.val(n->rows);
        H.val(n->cols);
        H.val(n->binop);
        H.val(n->red);
        H.val(ref(n->src[0]));
        H.val(ref(n->src[1]));
        hash_fn(H, n->fn);
        hash_pred(H, n->pred);
    }
    H.val((int)P->roots.size());
    for (auto* r : P->roots) H.val(ref(r));
    for (auto& c : P->contracts) {
        H.val(c.kind);
        H.val(c.check);
        H.val(ref(c.node));
        H.val(ref(c.a));
        H.val(ref(c.b));
        H.val(ref(c.r));
        H.val(c.abs_tol);
        H.val(c.rel_tol);
        hash_pred(H, c.pred);
    }
    for (auto* s : P->splits) H.val(ref(s));
    return H.h;
}

constexpr int64_t kParams = 5825;      // parameters of the 24-64-64-1 network
constexpr char kMlpMagic[9] = "sgmlp001";

bool plan_ok(const sg_plan& p) {
    return p.block >= 64 && p.block <= 1024 && p.block % 64 == 0 && (p.unroll == 1 || p.unroll == 2 || p.unroll == 4) &&
           p.substeps >= 1 && p.substeps <= 64;
}

}  // namespace

extern "C" {

sg_status sg_program_key(sg_program p, uint64_t* key) {
    if (!p || !key) return fail(p ? p->ctx : nullptr, SG_E_INVALID, "program_key: NULL argument");
    *key = program_key(p);
    return SG_OK;
}

sg_status sg_tunedb_open(sg_ctx ctx, const char* path, sg_tunedb* out) {
    if (!ctx || !path || !out) return fail(ctx, SG_E_INVALID, "tunedb_open: NULL argument");
    auto* db = new sg_tunedb_s();
    db->ctx = ctx;
    db->path = path;
    if (FILE* r = std::fopen(path, "r")) {
        char line[256];
        int64_t lineno = 0;
        while (std::fgets(line, sizeof(line), r)) {
            ++lineno;
            if (line[0] == '\n' || line[0] == '\0') continue;
            char tag[16];
            uint64_t key = 0;
            sg_plan pl{};
            double ms = 0;
            const int got = std::sscanf(line, "%15s %" SCNx64 " %d %d %d %d %lf", tag, &key, &pl.block, &pl.unroll,
                                        &pl.substeps, &pl.split, &ms);
            if (got != 7 || std::strcmp(tag, "sgtune1") != 0 || !plan_ok(pl) || !(ms > 0)) {
                std::fclose(r);
                delete db;
                return fail(ctx, SG_E_INVALID, "tunedb_open: malformed record at line " + std::to_string(lineno) + " of " + path);
            }
            db->ms[std::make_tuple(key, pl.block, pl.unroll, pl.substeps, pl.split)] = ms;
            ++db->records;
        }
        std::fclose(r);
    }
    db->f = std::fopen(path, "a");
    if (!db->f) {
        delete db;
        return fail(ctx, SG_E_INVALID, std::string("tunedb_open: cannot append to ") + path);
    }
    ctx_retain(ctx);
    *out = db;
    return SG_OK;
}

sg_status sg_tunedb_close(sg_tunedb db) {
    if (!db) return SG_E_INVALID;
    sg_ctx_s* ctx = db->ctx;
    if (db->f) std::fclose(db->f);
    delete db;
    ctx_release(ctx);
    return SG_OK;
}

sg_status sg_tunedb_records(sg_tunedb db, int64_t* records, int64_t* distinct) {
    if (!db) return SG_E_INVALID;
    if (records) *records = db->records;
    if (distinct) *distinct = (int64_t)db->ms.size();
    return SG_OK;
}

sg_status sg_tunedb_lookup(sg_tunedb db, uint64_t key, const sg_plan* plan, double* ms) {
    if (!db || !plan || !ms) return fail(db ? db->ctx : nullptr, SG_E_INVALID, "tunedb_lookup: NULL argument");
    auto it = db->ms.find(std::make_tuple(key, plan->block, plan->unroll, plan->substeps, plan->split));
    *ms = it == db->ms.end() ? -1.0 : it->second;
    return SG_OK;
}

sg_status sg_tunedb_record(sg_tunedb db, uint64_t key, const sg_plan* plan, double ms) {
    if (!db || !plan || !plan_ok(*plan) || !(ms > 0)) return fail(db ? db->ctx : nullptr, SG_E_INVALID, "tunedb_record: bad argument");
    if (std::fprintf(db->f, "sgtune1 %016" PRIx64 " %d %d %d %d %.9g\n", key, plan->block, plan->unroll, plan->substeps,
                     plan->split, ms) < 0 ||
        std::fflush(db->f) != 0)
        return fail(db->ctx, SG_E_INVALID, "tunedb_record: write failed on " + db->path);
    db->ms[std::make_tuple(key, plan->block, plan->unroll, plan->substeps, plan->split)] = ms;
    ++db->records;
    return SG_OK;
}

sg_status sg_autotune_db(sg_program p, sg_tunedb db, const sg_plan* plans, int32_t n, int32_t reps, int32_t* best,
                         double* ms_out, int32_t* measured) {
    if (!p || !db || !plans || n < 1 || !best) return fail(p ? p->ctx : nullptr, SG_E_INVALID, "autotune_db: bad argument");
    if (db->ctx != p->ctx) return fail(p->ctx, SG_E_INVALID, "autotune_db: database of another context");
    const uint64_t key = program_key(p);
    std::vector<double> ms(n, -1.0);
    std::vector<sg_plan> todo;
    std::vector<int> where;
    for (int i = 0; i < n; ++i) {
        if (!plan_ok(plans[i])) return fail(p->ctx, SG_E_INVALID, "autotune_db: invalid plan");
        sg_status st = sg_tunedb_lookup(db, key, &plans[i], &ms[i]);
        if (st != SG_OK) return st;
        if (ms[i] < 0) {
            todo.push_back(plans[i]);
            where.push_back(i);
        }
    }
    if (!todo.empty()) {
        std::vector<double> t(todo.size());
        sg_status st = sg_program_time_plans(p, todo.data(), (int32_t)todo.size(), reps, t.data());
        if (st != SG_OK) return st;
        for (size_t k = 0; k < todo.size(); ++k) {
            ms[where[k]] = t[k];
            st = sg_tunedb_record(db, key, &todo[k], t[k]);
            if (st != SG_OK) return st;
        }
    }
    int b = 0;
    for (int i = 1; i < n; ++i)
        if (ms[i] < ms[b]) b = i;
    sg_status st = sg_program_set_plan(p, &plans[b]);
    if (st != SG_OK) return st;
    p->plan_from = SG_PLAN_AUTOTUNE;
    *best = b;
    if (ms_out) std::memcpy(ms_out, ms.data(), sizeof(double) * n);
    if (measured) *measured = (int32_t)todo.size();
    return SG_OK;
}

sg_status sg_mlp_save(sg_mlp m, const char* path) {
    if (!m || !path) return fail(m ? m->ctx : nullptr, SG_E_INVALID, "mlp_save: NULL argument");
    if (!m->norm_set) return fail(m->ctx, SG_E_STATE, "mlp_save: the model has no standardization");
    sg_ctx_s* ctx = m->ctx;
    // parameters and Adam's two moment vectors (the gradient buffer between them is not kept)
    std::vector<float> P(3 * kParams);
    SG_HIP(ctx, hipMemcpyAsync(P.data(), m->P, kParams * 4, hipMemcpyDeviceToHost, ctx->stream));
    SG_HIP(ctx, hipMemcpyAsync(P.data() + kParams, m->P + 2 * kParams, 2 * kParams * 4, hipMemcpyDeviceToHost, ctx->stream));
    SG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fail(ctx, SG_E_INVALID, std::string("mlp_save: cannot write ") + path);
    const int32_t step = m->step;
    bool ok = std::fwrite(kMlpMagic, 1, 8, f) == 8 && std::fwrite(P.data(), 4, P.size(), f) == P.size() &&
              std::fwrite(m->mean, 4, 24, f) == 24 && std::fwrite(m->scale, 4, 24, f) == 24 &&
              std::fwrite(m->lo, 4, 24, f) == 24 && std::fwrite(m->hi, 4, 24, f) == 24 && std::fwrite(&step, 4, 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(ctx, SG_E_INVALID, std::string("mlp_save: write failed on ") + path);
    }
    return SG_OK;
}

sg_status sg_mlp_load(sg_ctx ctx, const char* path, sg_mlp* out) {
    if (!ctx || !path || !out) return fail(ctx, SG_E_INVALID, "mlp_load: NULL argument");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(ctx, SG_E_INVALID, std::string("mlp_load: cannot read ") + path);
    char magic[8];
    std::vector<float> P(3 * kParams);
    float mean[24], scale[24], lo[24], hi[24];
    int32_t step = 0;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMlpMagic, 8) == 0 &&
              std::fread(P.data(), 4, P.size(), f) == P.size() && std::fread(mean, 4, 24, f) == 24 &&
              std::fread(scale, 4, 24, f) == 24 && std::fread(lo, 4, 24, f) == 24 && std::fread(hi, 4, 24, f) == 24 &&
              std::fread(&step, 4, 1, f) == 1;
    char extra;
    ok = ok && std::fread(&extra, 1, 1, f) == 0;
    std::fclose(f);
    if (!ok || step < 0) return fail(ctx, SG_E_INVALID, std::string("mlp_load: not a cost-model file: ") + path);
    sg_mlp m = nullptr;
    sg_status st = sg_mlp_create(ctx, P.data(), kParams, &m);
    if (st != SG_OK) return st;
    st = sg_mlp_set_norm(m, mean, scale, lo, hi);
    hipError_t e = hipSuccess;
    if (st == SG_OK) {
        e = hipMemcpyAsync(m->P + 2 * kParams, P.data() + kParams, 2 * kParams * 4, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) st = hip_fail(ctx, e, "mlp_load: upload");
    }
    if (st != SG_OK) {
        (void)sg_mlp_release(m);
        return st;
    }
    m->step = step;
    *out = m;
    return SG_OK;
}

}  // extern "C"

namespace sgrt {
sg_ctx_s* tunedb_ctx(const sg_tunedb_s* db) { return db->ctx; }
}  // namespace sgrt
