// Host runtime behind the C ABI: handles, lazy graph, planner, executor.
//
// Composition calls build a DAG of nodes (Section 5: pending operations become an
// execution plan whose vertices are data and kernels).  A trigger plans the program: the
// element-wise nodes, filters and reductions that share an index space are merged into one
// pass of the streaming kernel (the merged vertices of Figures 2 and 3), range contracts
// (Section 4) are placed in the pass that streams their operand, and matrix products and
// product checks get kernels of their own.  With fusion off, every node and every contract
// is its own pass and every intermediate is materialized: the one-kernel-per-call strategy
// Section 5 describes as the naive alternative.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <set>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/safegpu.h"
#include "sg_kernels.h"
#include "sg_runtime.h"

using namespace sg;

// ---- kernels (defined in the .hip kernel files) ---------------------------------------------
hipError_t sg_launch_zero(uint64_t* p, int64_t n, hipStream_t s);
int sg_stream_occupancy(int unroll, bool inl, int block, size_t lds_bytes);

namespace sgrt {

// ---------------------------------------------------------------------------------------------
// errors

thread_local std::string g_tls_error;

sg_status fail(sg_ctx_s* ctx, sg_status st, const std::string& msg) {
    if (ctx) ctx->error = msg;
    g_tls_error = msg;
    return st;
}

sg_status hip_fail(sg_ctx_s* ctx, hipError_t e, const char* what) {
    return fail(ctx, SG_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// A kernel handed a host address or a buffer shorter than its arguments say would fault the
// GPU; the runtime knows the allocation that holds a device address, so the range is checked
// before anything is launched on it.
sg_status check_device_range(sg_ctx_s* ctx, const void* p, size_t bytes, const char* what) {
    if (bytes == 0) return SG_OK;
    if (!p) return fail(ctx, SG_E_INVALID, std::string(what) + ": NULL device pointer");
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return fail(ctx, SG_E_INVALID, std::string(what) + ": not a device address");
    }
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, SG_E_INVALID, std::string(what) + ": address is in no device allocation");
    }
    const uintptr_t b = (uintptr_t)base, a = (uintptr_t)p;
    if (a < b || a - b > size || bytes > size - (a - b))
        return fail(ctx, SG_E_INVALID, std::string(what) + ": buffer extends past its device allocation");
    return SG_OK;
}

// ---------------------------------------------------------------------------------------------
// device memory

void* dev_alloc(sg_ctx_s* ctx, size_t bytes) {
    if (bytes == 0) bytes = 16;
    bytes = (bytes + 255) & ~(size_t)255;
    if (ctx->ext.alloc) {  // the caller's allocator
        void* p = ctx->ext.alloc(bytes, (void*)ctx->stream, ctx->ext.user);
        if (p) ctx->ext_blocks[p] = ctx->ext;
        return p;
    }
    auto it = ctx->pool.find(bytes);
    if (it != ctx->pool.end() && !it->second.empty()) {
        void* p = it->second.back();
        it->second.pop_back();
        ctx->pooled_bytes -= bytes;
        return p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        // the pool keeps freed blocks by size, so blocks of sizes that do not come back pile up:
        // return them to the device (after the work that may still use them) and try again
        if (pool_trim(ctx) == 0 || hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    ctx->sizes[p] = bytes;
    return p;
}

size_t pool_trim(sg_ctx_s* ctx) {
    size_t freed = 0;
    bool synced = false;
    for (auto& kv : ctx->pool) {
        for (void* q : kv.second) {
            if (!synced) {
                (void)hipDeviceSynchronize();  // pooled blocks may still be read by queued kernels
                synced = true;
            }
            (void)hipFree(q);
            ctx->sizes.erase(q);
            freed += kv.first;
        }
        kv.second.clear();
    }
    ctx->pool.clear();
    ctx->pooled_bytes = 0;
    return freed;
}

// Pooled blocks beyond this many bytes go back to the device: blocks of sizes that do not
// come back (programs over many different lengths) would otherwise hold the device memory
// that later allocations, and the runtime's own, need.
constexpr size_t kPoolCapBytes = (size_t)16 << 30;

void dev_free(sg_ctx_s* ctx, void* p) {
    if (!p) return;
    auto xe = ctx->ext_blocks.find(p);
    if (xe != ctx->ext_blocks.end()) {  // back to the allocator it came from
        const sg_allocator a = xe->second;
        ctx->ext_blocks.erase(xe);
        a.free(p, (void*)ctx->stream, a.user);
        return;
    }
    auto it = ctx->sizes.find(p);
    if (it == ctx->sizes.end()) return;
    ctx->pool[it->second].push_back(p);
    ctx->pooled_bytes += it->second;
    if (ctx->pooled_bytes > kPoolCapBytes) (void)pool_trim(ctx);
}

// Scratch of the streaming kernel, zeroed once: the kernel leaves the accumulators zero and
// tags everything else with the launch epoch.
sg_status alloc_scratch(sg_ctx_s* ctx, Scratch& S, int64_t tiles, int64_t chunks, int64_t insts) {
    if (S.base) (void)hipFree(S.base);
    S = Scratch();
    const int64_t nt = std::max<int64_t>(tiles, 1), nc = std::max<int64_t>(chunks, 1), ni = std::max<int64_t>(insts, 1);
    // layout (bytes): acc | results | tags | lookback | epoch
    size_t acc_b = (size_t)ni * MAX_SLOTS * MAX_SPREAD * 8;
    size_t res_b = (size_t)ni * sizeof(InstResult);
    size_t tag_b = (size_t)nt * TAG_WORDS * 8;
    size_t lb_b = (size_t)nc * 8;
    size_t ep_b = 256;
    size_t total = acc_b + res_b + tag_b + lb_b + ep_b;
    void* p = nullptr;
    SG_HIP(ctx, hipMalloc(&p, total));
    S.base = p;
    char* c = (char*)p;
    S.acc = (uint64_t*)c; c += acc_b;
    S.results = (InstResult*)c; c += res_b;
    S.tags = (uint64_t*)c; c += tag_b;
    S.lookback = (uint64_t*)c; c += lb_b;
    S.epoch = (uint32_t*)c;
    S.tiles = nt;
    S.chunks = nc;
    S.insts = ni;
    S.bytes = total;
    SG_HIP(ctx, sg_launch_zero((uint64_t*)p, (int64_t)(total / 8), ctx->stream));
    return SG_OK;
}

sg_status ensure_scratch(sg_ctx_s* ctx, int64_t tiles, int64_t chunks, int64_t insts) {
    Scratch& S = ctx->scratch;
    if (tiles <= S.tiles && chunks <= S.chunks && insts <= S.insts) return SG_OK;
    SG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    sg_status st = alloc_scratch(ctx, S, std::max<int64_t>({tiles, S.tiles * 2, 1024}),
                                 std::max<int64_t>({chunks, S.chunks * 2, 16384}),
                                 std::max<int64_t>({insts, S.insts * 2, 16}));
    if (st != SG_OK) return st;
    ctx->epoch = 0;
    if (ctx->host_results) (void)hipHostFree(ctx->host_results);
    ctx->host_results = nullptr;
    SG_HIP(ctx, hipHostMalloc((void**)&ctx->host_results, (size_t)S.insts * sizeof(InstResult), hipHostMallocDefault));
    return SG_OK;
}

// Epoch of the next direct launch.  Look-back descriptors keep 30 bits of it: on wrap-around
// they are cleared so that no descriptor of an earlier launch can look current.
uint32_t next_epoch(sg_ctx_s* ctx) {
    ctx->epoch = (ctx->epoch + 1) & 0x3FFFFFFFu;
    if (ctx->epoch == 0) {
        (void)sg_launch_zero(ctx->scratch.lookback, ctx->scratch.chunks, ctx->stream);
        (void)sg_launch_zero(ctx->scratch.tags, ctx->scratch.tiles * TAG_WORDS, ctx->stream);
        ctx->epoch = 1;
    }
    return ctx->epoch;
}

// ---------------------------------------------------------------------------------------------
// refcounting

// The context lives until its creator and every object made on it have released it, so
// objects may be released in any order (e.g. by a garbage collector at interpreter exit).
void ctx_retain(sg_ctx_s* ctx) { if (ctx) ++ctx->refs; }
void ctx_release(sg_ctx_s* ctx) {
    if (!ctx || --ctx->refs > 0) return;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& kv : ctx->pool)
        for (void* p : kv.second) (void)hipFree(p);
    // blocks from a caller's allocator are all back by now: every node, program and batch that
    // held one has released the context before this point
    if (ctx->scratch.base) (void)hipFree(ctx->scratch.base);
    if (ctx->host_results) (void)hipHostFree(ctx->host_results);
    for (auto& ev : ctx->events) (void)hipEventDestroy(ev);
    delete ctx;
}

void retain(sg_node_s* n) { if (n) ++n->refs; }
void retain(sg_fn_s* f) { if (f) ++f->refs; }
void retain(sg_pred_s* p) { if (p) ++p->refs; }

void release(sg_fn_s* f) {
    if (!f || --f->refs > 0) return;
    release(f->f);
    release(f->g);
    delete f->expr;
    delete f;
}
void release(sg_pred_s* p) {
    if (!p || --p->refs > 0) return;
    release(p->p);
    release(p->q);
    delete p;
}
void release(sg_node_s* n) {
    if (!n || --n->refs > 0) return;
    if (n->owned && n->dev) dev_free(n->ctx, n->dev);
    if (n->op == OPN_GAUSS && n->aux) gauss_cache_free(n->ctx, n->aux);
    release(n->src[0]);
    release(n->src[1]);
    release(n->fn);
    release(n->pred);
    sg_ctx_s* ctx = n->ctx;
    delete n;
    ctx_release(ctx);
}

// ---------------------------------------------------------------------------------------------
// planning helpers

bool is_elementwise(const sg_node_s* n) {
    return n->op == OPN_MAP || n->op == OPN_ZIP || n->op == OPN_FILTER || n->op == OPN_REDUCE;
}
bool is_collection(const sg_node_s* n) { return n->op != OPN_REDUCE && n->op != OPN_GAUSS; }

// value dtype after applying fn to dtype
bool fn_out_dtype(const sg_fn_s* f, sg_dtype in, sg_dtype* out, std::string* why) {
    switch (f->kind) {
        case FK_COMPOSE: {
            sg_dtype mid;
            if (!fn_out_dtype(f->f, in, &mid, why)) return false;
            return fn_out_dtype(f->g, mid, out, why);
        }
        case FK_AFFINE: case FK_ADDC: case FK_MULC: *out = in; return true;
        case FK_EXPR:
            if (in != SG_F32) { *why = "expression functions are defined on f32"; return false; }
            *out = SG_F32; return true;
        case FK_UNARY:
            switch ((int)f->a) {
                case SG_FN_SQUARE: case SG_FN_NEG: case SG_FN_ABS: *out = in; return true;
                case SG_FN_SQRT: case SG_FN_SQRT_ABS: case SG_FN_EXP: case SG_FN_EXP_NEG_SQ:
                    if (in != SG_F32) { *why = "sqrt/exp are defined on f32"; return false; }
                    *out = SG_F32; return true;
                case SG_FN_I2F:
                    if (in != SG_I32) { *why = "i2f needs an i32 operand"; return false; }
                    *out = SG_F32; return true;
            }
    }
    *why = "unknown element function";
    return false;
}

inline int32_t to_i32(double c) { return (int32_t)(int64_t)c; }

int fn_temps(const sg_fn_s* f) {
    if (!f) return 0;
    if (f->kind == FK_COMPOSE) return std::max(fn_temps(f->f), fn_temps(f->g));
    if (f->kind == FK_EXPR) return expr_temps(*f->expr, f->expr_root);
    return 0;
}

// emit the in-place ops applying f to register r (element type dt)
bool emit_fn(std::vector<SgOp>& prog, const sg_fn_s* f, int r, sg_dtype dt, const std::vector<int>& temps) {
    auto op = [&](uint8_t code, float c0 = 0.f, float c1 = 0.f) {
        SgOp o{};
        o.code = code; o.a = (uint8_t)r; o.dst = (uint8_t)r; o.c0.f = c0; o.c1.f = c1;
        prog.push_back(o);
    };
    auto opi = [&](uint8_t code, int32_t c0 = 0, int32_t c1 = 0) {
        SgOp o{};
        o.code = code; o.a = (uint8_t)r; o.dst = (uint8_t)r; o.c0.i = c0; o.c1.i = c1;
        prog.push_back(o);
    };
    switch (f->kind) {
        case FK_COMPOSE: {
            if (!emit_fn(prog, f->f, r, dt, temps)) return false;
            sg_dtype mid;
            std::string why;
            fn_out_dtype(f->f, dt, &mid, &why);
            return emit_fn(prog, f->g, r, mid, temps);
        }
        case FK_EXPR:
            return emit_expr(prog, *f->expr, f->expr_root, r, temps);
        case FK_AFFINE:
            if (dt == SG_F32) op(F_AFFINE, (float)f->a, (float)f->b);
            else opi(I_AFFINE, to_i32(f->a), to_i32(f->b));
            return true;
        case FK_ADDC:
            if (dt == SG_F32) op(F_ADDC, (float)f->a);
            else opi(I_ADDC, to_i32(f->a));
            return true;
        case FK_MULC:
            if (dt == SG_F32) op(F_MULC, (float)f->a);
            else opi(I_MULC, to_i32(f->a));
            return true;
        case FK_UNARY:
            switch ((int)f->a) {
                case SG_FN_SQUARE: if (dt == SG_F32) op(F_SQUARE); else opi(I_SQUARE); return true;
                case SG_FN_NEG: if (dt == SG_F32) op(F_NEG); else opi(I_NEG); return true;
                case SG_FN_ABS: if (dt == SG_F32) op(F_ABS); else opi(I_ABS); return true;
                case SG_FN_SQRT: op(F_SQRT); return true;
                case SG_FN_SQRT_ABS: op(F_SQRT_ABS); return true;
                case SG_FN_EXP: op(F_EXP); return true;
                case SG_FN_EXP_NEG_SQ: op(F_EXP_NEG_SQ); return true;
                case SG_FN_I2F: op(I_TO_F); return true;
            }
    }
    return false;
}

// emit ops pushing predicate p evaluated on register r
void emit_pred(std::vector<SgOp>& prog, const sg_pred_s* p, int r, sg_dtype dt) {
    SgOp o{};
    o.a = (uint8_t)r;
    switch (p->kind) {
        case PK_TRUE: o.code = P_TRUE; prog.push_back(o); return;
        case PK_FINITE:
            if (dt == SG_F32) o.code = P_FINITE;
            else o.code = P_TRUE;
            prog.push_back(o);
            return;
        case PK_CMP:
            o.aux = (uint8_t)p->cmp;
            if (dt == SG_F32) { o.code = P_CMP_F; o.c0.f = (float)p->c; }
            else { o.code = P_CMP_I; o.c0.i = to_i32(p->c); }
            prog.push_back(o);
            return;
        case PK_RANGE:
            if (dt == SG_F32) { o.code = P_RANGE_F; o.c0.f = (float)p->lo; o.c1.f = (float)p->hi; }
            else { o.code = P_RANGE_I; o.c0.i = to_i32(p->lo); o.c1.i = to_i32(p->hi); }
            prog.push_back(o);
            return;
        case PK_AND: case PK_OR:
            emit_pred(prog, p->p, r, dt);
            emit_pred(prog, p->q, r, dt);
            o.code = p->kind == PK_AND ? P_AND : P_OR;
            prog.push_back(o);
            return;
        case PK_NOT:
            emit_pred(prog, p->p, r, dt);
            o.code = P_NOT;
            prog.push_back(o);
            return;
    }
}

int pred_depth(const sg_pred_s* p) {
    switch (p->kind) {
        case PK_AND: case PK_OR: return std::max(pred_depth(p->p), 1 + pred_depth(p->q));
        case PK_NOT: return pred_depth(p->p);
        default: return 1;
    }
}

}  // namespace sgrt

using namespace sgrt;

// =============================================================================================
// C ABI: context
// =============================================================================================

extern "C" {

sg_status sg_ctx_create(int device, void* hip_stream, sg_ctx* out) {
    if (!out) return fail(nullptr, SG_E_INVALID, "out is NULL");
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0) return fail(nullptr, SG_E_DEVICE, "no HIP device");
    if (device < 0 || device >= ndev) return fail(nullptr, SG_E_INVALID, "bad device index");
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(nullptr, e, "hipSetDevice");
    auto* c = new sg_ctx_s();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        c->num_cu = prop.multiProcessorCount;
        std::string arch = prop.gcnArchName;
        c->arch = arch.substr(0, arch.find(':'));  // e.g. "gfx950" from "gfx950:sramecc+:xnack-"
    }
    *out = c;
    return SG_OK;
}

sg_status sg_ctx_destroy(sg_ctx ctx) {
    if (!ctx) return SG_E_INVALID;
    ctx_release(ctx);
    return SG_OK;
}

sg_status sg_ctx_set_allocator(sg_ctx ctx, const sg_allocator* a) {
    if (!ctx) return SG_E_INVALID;
    if (!a) {
        ctx->ext = sg_allocator{};
        return SG_OK;
    }
    if (!a->alloc || !a->free) return fail(ctx, SG_E_INVALID, "set_allocator: alloc and free are both needed");
    ctx->ext = *a;
    return SG_OK;
}

sg_status sg_ctx_set_mode(sg_ctx ctx, sg_mode mode) {
    if (!ctx || mode < SG_MODE_OFF || mode > SG_MODE_PRE_POST) return fail(ctx, SG_E_INVALID, "bad mode");
    ctx->mode = mode;
    ++ctx->generation;
    return SG_OK;
}

sg_status sg_ctx_set_fusion(sg_ctx ctx, int fused) {
    if (!ctx) return SG_E_INVALID;
    ctx->fused = fused != 0;
    ++ctx->generation;
    return SG_OK;
}

sg_status sg_ctx_set_launch(sg_ctx ctx, int block, int unroll) {
    if (!ctx) return SG_E_INVALID;
    if (block != 0 && (block < 64 || block > 1024 || block % 64)) return fail(ctx, SG_E_INVALID, "block must be 64..1024, multiple of 64");
    if (unroll != 0 && unroll != 1 && unroll != 2 && unroll != 4) return fail(ctx, SG_E_INVALID, "unroll must be 1, 2 or 4");
    if (block) ctx->block = block;
    if (unroll) ctx->unroll = unroll;
    return SG_OK;
}

sg_status sg_ctx_set_batch_substeps(sg_ctx ctx, int substeps) {
    if (!ctx) return SG_E_INVALID;
    if (substeps < 1 || substeps > 16) return fail(ctx, SG_E_INVALID, "batch sub-tiles per tile must be 1..16");
    ctx->batch_substeps = substeps;
    return SG_OK;
}

sg_status sg_ctx_set_specialize(sg_ctx ctx, int on) {
    if (!ctx) return SG_E_INVALID;
    ctx->specialize = on != 0;
    return SG_OK;
}

sg_status sg_ctx_set_wait_limit(sg_ctx ctx, int64_t spins) {
    if (!ctx) return SG_E_INVALID;
    if (spins >= (int64_t)0xFFFFFFFEu) return fail(ctx, SG_E_INVALID, "wait limit: at most 2^32 - 2 spins");
    ctx->wait_limit = spins < 0 ? 0u : (uint32_t)(spins + 1);
    return SG_OK;
}

sg_status sg_ctx_set_timing(sg_ctx ctx, int on) {
    if (!ctx) return SG_E_INVALID;
    ctx->timing = on != 0;
    return SG_OK;
}

sg_status sg_ctx_timing(sg_ctx ctx, const char* kernel, double* total_ms, int64_t* launches) {
    if (!ctx || !kernel) return SG_E_INVALID;
    auto it = ctx->times.find(kernel);
    if (total_ms) *total_ms = it == ctx->times.end() ? 0.0 : it->second.ms;
    if (launches) *launches = it == ctx->times.end() ? 0 : it->second.n;
    return SG_OK;
}

sg_status sg_ctx_last_launch(sg_ctx ctx, int32_t* grid, int32_t* block, int32_t* unroll, int32_t* substeps,
                             int64_t* lds_bytes) {
    if (!ctx) return SG_E_INVALID;
    if (grid) *grid = ctx->last_grid;
    if (block) *block = ctx->last_block;
    if (unroll) *unroll = ctx->last_unroll;
    if (substeps) *substeps = ctx->last_substeps;
    if (lds_bytes) *lds_bytes = (int64_t)ctx->last_lds;
    return SG_OK;
}

sg_status sg_ctx_timing_reset(sg_ctx ctx) {
    if (!ctx) return SG_E_INVALID;
    ctx->times.clear();
    return SG_OK;
}

const char* sg_last_error(sg_ctx ctx) { return ctx ? ctx->error.c_str() : g_tls_error.c_str(); }

// =============================================================================================
// collections
// =============================================================================================

static sg_node_s* new_node(sg_ctx_s* ctx, int op, sg_dtype dt, int64_t n) {
    auto* nd = new sg_node_s();
    nd->ctx = ctx;
    ctx_retain(ctx);
    nd->op = op;
    nd->dtype = dt;
    nd->n = n;
    nd->id = ++ctx->next_id;
    return nd;
}

static bool valid_elem_dtype(sg_dtype d) { return d == SG_F32 || d == SG_I32; }

sg_status sg_vector_wrap(sg_ctx ctx, sg_dtype dtype, void* dev, int64_t n, sg_node* out) {
    if (!ctx || !out || n < 0 || (!dev && n > 0)) return fail(ctx, SG_E_INVALID, "vector_wrap: bad argument");
    if (!valid_elem_dtype(dtype)) return fail(ctx, SG_E_DTYPE, "vector_wrap: dtype must be f32 or i32");
    if (n >= (int64_t)1 << 32) return fail(ctx, SG_E_INVALID, "vector_wrap: at most 2^32-1 elements");
    if (sg_status st = check_device_range(ctx, dev, (size_t)n * 4, "vector_wrap")) return st;
    auto* nd = new_node(ctx, OPN_INPUT, dtype, n);
    nd->dev = dev;
    nd->space = 0;  // dense index space; filters open new ones
    nd->state = ST_COMPUTED;
    nd->count = n;
    *out = nd;
    return SG_OK;
}

sg_status sg_matrix_wrap(sg_ctx ctx, sg_dtype dtype, void* dev, int64_t rows, int64_t cols, sg_node* out) {
    if (rows < 0 || cols < 0) return fail(ctx, SG_E_INVALID, "matrix_wrap: negative dimension");
    sg_status st = sg_vector_wrap(ctx, dtype, dev, rows * cols, out);
    if (st != SG_OK) return st;
    (*out)->matrix = true;
    (*out)->rows = rows;
    (*out)->cols = cols;
    return SG_OK;
}

sg_status sg_vector_from_host(sg_ctx ctx, sg_dtype dtype, const void* host, int64_t n, sg_node* out) {
    if (!ctx || !out || n < 0 || (!host && n > 0)) return fail(ctx, SG_E_INVALID, "vector_from_host: bad argument");
    if (!valid_elem_dtype(dtype)) return fail(ctx, SG_E_DTYPE, "vector_from_host: dtype must be f32 or i32");
    void* d = dev_alloc(ctx, (size_t)n * 4);
    if (!d) return fail(ctx, SG_E_OOM, "vector_from_host: device allocation failed");
    if (n > 0) SG_HIP(ctx, hipMemcpyAsync(d, host, (size_t)n * 4, hipMemcpyHostToDevice, ctx->stream));
    SG_HIP(ctx, hipStreamSynchronize(ctx->stream));
    sg_status st = sg_vector_wrap(ctx, dtype, d, n, out);
    if (st != SG_OK) { dev_free(ctx, d); return st; }
    (*out)->owned = true;
    return SG_OK;
}

sg_status sg_matrix_from_host(sg_ctx ctx, sg_dtype dtype, const void* host, int64_t rows, int64_t cols, sg_node* out) {
    if (rows < 0 || cols < 0) return fail(ctx, SG_E_INVALID, "matrix_from_host: negative dimension");
    sg_status st = sg_vector_from_host(ctx, dtype, host, rows * cols, out);
    if (st != SG_OK) return st;
    (*out)->matrix = true;
    (*out)->rows = rows;
    (*out)->cols = cols;
    return SG_OK;
}

// =============================================================================================
// agents
// =============================================================================================

static sg_status new_fn(int kind, double a, double b, sg_fn_s* f, sg_fn_s* g, sg_fn* out) {
    if (!out) return fail(nullptr, SG_E_INVALID, "out is NULL");
    auto* fn = new sg_fn_s();
    fn->kind = kind; fn->a = a; fn->b = b; fn->f = f; fn->g = g;
    retain(f);
    retain(g);
    *out = fn;
    return SG_OK;
}

sg_status sg_fn_affine(double a, double b, sg_fn* out) { return new_fn(FK_AFFINE, a, b, nullptr, nullptr, out); }
sg_status sg_fn_add_c(double c, sg_fn* out) { return new_fn(FK_ADDC, c, 0, nullptr, nullptr, out); }
sg_status sg_fn_mul_c(double c, sg_fn* out) { return new_fn(FK_MULC, c, 0, nullptr, nullptr, out); }
sg_status sg_fn_unary(sg_fn_kind kind, sg_fn* out) {
    if (kind < SG_FN_SQUARE || kind > SG_FN_I2F) return fail(nullptr, SG_E_INVALID, "unknown unary function");
    return new_fn(FK_UNARY, (double)kind, 0, nullptr, nullptr, out);
}
sg_status sg_fn_compose(sg_fn f, sg_fn g, sg_fn* out) {
    if (!f || !g) return fail(nullptr, SG_E_INVALID, "compose: NULL function");
    return new_fn(FK_COMPOSE, 0, 0, f, g, out);
}
sg_status sg_fn_release(sg_fn f) {
    if (!f) return SG_E_INVALID;
    release(f);
    return SG_OK;
}

static sg_status new_pred(int kind, int cmp, double c, double lo, double hi, sg_pred_s* p, sg_pred_s* q, sg_pred* out) {
    if (!out) return fail(nullptr, SG_E_INVALID, "out is NULL");
    auto* pr = new sg_pred_s();
    pr->kind = kind; pr->cmp = cmp; pr->c = c; pr->lo = lo; pr->hi = hi; pr->p = p; pr->q = q;
    retain(p);
    retain(q);
    *out = pr;
    return SG_OK;
}

sg_status sg_pred_cmp(sg_cmp op, double c, sg_pred* out) {
    if (op < SG_LT || op > SG_NE) return fail(nullptr, SG_E_INVALID, "unknown comparison");
    return new_pred(PK_CMP, op, c, 0, 0, nullptr, nullptr, out);
}
sg_status sg_pred_isfinite(sg_pred* out) { return new_pred(PK_FINITE, 0, 0, 0, 0, nullptr, nullptr, out); }
sg_status sg_pred_in_range(double lo, double hi, sg_pred* out) { return new_pred(PK_RANGE, 0, 0, lo, hi, nullptr, nullptr, out); }
sg_status sg_pred_true(sg_pred* out) { return new_pred(PK_TRUE, 0, 0, 0, 0, nullptr, nullptr, out); }
sg_status sg_pred_and(sg_pred p, sg_pred q, sg_pred* out) {
    if (!p || !q) return fail(nullptr, SG_E_INVALID, "and: NULL predicate");
    return new_pred(PK_AND, 0, 0, 0, 0, p, q, out);
}
sg_status sg_pred_or(sg_pred p, sg_pred q, sg_pred* out) {
    if (!p || !q) return fail(nullptr, SG_E_INVALID, "or: NULL predicate");
    return new_pred(PK_OR, 0, 0, 0, 0, p, q, out);
}
sg_status sg_pred_not(sg_pred p, sg_pred* out) {
    if (!p) return fail(nullptr, SG_E_INVALID, "not: NULL predicate");
    return new_pred(PK_NOT, 0, 0, 0, 0, p, nullptr, out);
}
sg_status sg_pred_release(sg_pred p) {
    if (!p) return SG_E_INVALID;
    release(p);
    return SG_OK;
}

// =============================================================================================
// lazy operations
// =============================================================================================

sg_status sg_map(sg_node in, sg_fn f, sg_node* out) {
    if (!in || !f || !out) return fail(in ? in->ctx : nullptr, SG_E_INVALID, "map: NULL argument");
    if (!is_collection(in)) return fail(in->ctx, SG_E_INVALID, "map: operand is a scalar");
    sg_dtype dt;
    std::string why;
    if (!fn_out_dtype(f, in->dtype, &dt, &why)) return fail(in->ctx, SG_E_DTYPE, "map: " + why);
    auto* nd = new_node(in->ctx, OPN_MAP, dt, in->n);
    nd->src[0] = in; retain(in);
    nd->fn = f; retain(f);
    nd->space = in->space;
    nd->matrix = in->matrix; nd->rows = in->rows; nd->cols = in->cols;
    *out = nd;
    return SG_OK;
}

sg_status sg_zip(sg_node a, sg_node b, sg_binop op, sg_node* out) {
    sg_ctx_s* ctx = a ? a->ctx : (b ? b->ctx : nullptr);
    if (!a || !b || !out) return fail(ctx, SG_E_INVALID, "zip: NULL argument");
    if (op < SG_ADD || op > SG_DIV) return fail(ctx, SG_E_INVALID, "zip: unknown operator");
    if (!is_collection(a) || !is_collection(b)) return fail(ctx, SG_E_INVALID, "zip: operand is a scalar");
    if (a->dtype != b->dtype) return fail(ctx, SG_E_DTYPE, "zip: operands differ in element type");
    if (op == SG_DIV && a->dtype != SG_F32) return fail(ctx, SG_E_DTYPE, "zip: compwise_divide is defined on f32");
    // built-in scalar contracts of vector arithmetic: equal counts (and equal dimensions)
    if (a->n != b->n) return fail(ctx, SG_E_SHAPE, "zip: operand counts differ");
    if (a->matrix && b->matrix && (a->rows != b->rows || a->cols != b->cols))
        return fail(ctx, SG_E_SHAPE, "zip: matrix dimensions differ");
    if (a->space != b->space) return fail(ctx, SG_E_SHAPE, "zip: operands are not in the same index space (filtered differently)");
    auto* nd = new_node(ctx, OPN_ZIP, a->dtype, a->n);
    nd->src[0] = a; retain(a);
    nd->src[1] = b; retain(b);
    nd->binop = op;
    nd->space = a->space;
    nd->matrix = a->matrix; nd->rows = a->rows; nd->cols = a->cols;
    *out = nd;
    return SG_OK;
}

sg_status sg_filter(sg_node in, sg_pred p, sg_node* out) {
    if (!in || !p || !out) return fail(in ? in->ctx : nullptr, SG_E_INVALID, "filter: NULL argument");
    if (!is_collection(in)) return fail(in->ctx, SG_E_INVALID, "filter: operand is a scalar");
    if (pred_depth(p) > 4) return fail(in->ctx, SG_E_UNSUPPORTED, "filter: predicate nests deeper than 4");
    auto* nd = new_node(in->ctx, OPN_FILTER, in->dtype, in->n);
    nd->src[0] = in; retain(in);
    nd->pred = p; retain(p);
    nd->space = nd->id;
    *out = nd;
    return SG_OK;
}

sg_status sg_reduce(sg_node in, sg_red red, sg_node* out) {
    if (!in || !out) return fail(in ? in->ctx : nullptr, SG_E_INVALID, "reduce: NULL argument");
    if (!is_collection(in)) return fail(in->ctx, SG_E_INVALID, "reduce: operand is a scalar");
    if (red < SG_SUM || red > SG_COUNT) return fail(in->ctx, SG_E_INVALID, "reduce: unknown reduction");
    sg_dtype dt = in->dtype;
    if (red == SG_COUNT) dt = SG_I64;
    else if (red == SG_SUM && in->dtype == SG_I32) dt = SG_I64;
    else if (red == SG_AVG) dt = in->dtype == SG_F32 ? SG_F32 : SG_F64;
    auto* nd = new_node(in->ctx, OPN_REDUCE, dt, 1);
    nd->src[0] = in; retain(in);
    nd->red = red;
    nd->space = in->space;
    *out = nd;
    return SG_OK;
}

sg_status sg_matmul(sg_node A, sg_node B, sg_node* out) {
    sg_ctx_s* ctx = A ? A->ctx : nullptr;
    if (!A || !B || !out) return fail(ctx, SG_E_INVALID, "matmul: NULL argument");
    if (!A->matrix || !B->matrix) return fail(ctx, SG_E_SHAPE, "matmul: operands must be matrices");
    if (A->cols != B->rows) return fail(ctx, SG_E_SHAPE, "matmul: inner dimensions differ");
    if (A->dtype != SG_F32 || B->dtype != SG_F32) return fail(ctx, SG_E_DTYPE, "matmul: f32 matrices only");
    auto* nd = new_node(ctx, OPN_MATMUL, SG_F32, A->rows * B->cols);
    nd->src[0] = A; retain(A);
    nd->src[1] = B; retain(B);
    nd->matrix = true; nd->rows = A->rows; nd->cols = B->cols;
    nd->space = 0;
    *out = nd;
    return SG_OK;
}

sg_status sg_concat(sg_node a, sg_node b, sg_node* out) {
    sg_ctx_s* ctx = a ? a->ctx : (b ? b->ctx : nullptr);
    if (!a || !b || !out) return fail(ctx, SG_E_INVALID, "concat: NULL argument");
    if (a->ctx != b->ctx) return fail(ctx, SG_E_INVALID, "concat: operands of different contexts");
    if (!is_collection(a) || !is_collection(b)) return fail(ctx, SG_E_INVALID, "concat: operand is a scalar");
    if (a->dtype != b->dtype) return fail(ctx, SG_E_DTYPE, "concat: operands differ in element type");
    if (a->n + b->n >= (int64_t)1 << 32) return fail(ctx, SG_E_INVALID, "concat: at most 2^32-1 elements");
    auto* nd = new_node(ctx, OPN_CONCAT, a->dtype, a->n + b->n);
    nd->src[0] = a; retain(a);
    nd->src[1] = b; retain(b);
    nd->space = nd->id;  // its count is known on the device only: a compacted collection
    *out = nd;
    return SG_OK;
}

sg_status sg_quicksort(sg_node in, sg_node* out) {
    if (!in || !out) return fail(in ? in->ctx : nullptr, SG_E_INVALID, "quicksort: NULL argument");
    if (!is_collection(in)) return fail(in->ctx, SG_E_INVALID, "quicksort: operand is a scalar");
    if (in->dtype != SG_F32 && in->dtype != SG_I32) return fail(in->ctx, SG_E_DTYPE, "quicksort: f32 or i32 vectors");
    auto* nd = new_node(in->ctx, OPN_QSORT, in->dtype, in->n);
    nd->src[0] = in; retain(in);
    nd->space = nd->id;  // dropped items make the count device-side
    *out = nd;
    return SG_OK;
}

sg_status sg_transpose(sg_node M, sg_node* out) {
    sg_ctx_s* ctx = M ? M->ctx : nullptr;
    if (!M || !out) return fail(ctx, SG_E_INVALID, "transpose: NULL argument");
    if (!M->matrix) return fail(ctx, SG_E_SHAPE, "transpose: operand must be a matrix");
    if (M->space != 0) return fail(ctx, SG_E_SHAPE, "transpose: operand has no fixed shape (filtered)");
    auto* nd = new_node(ctx, OPN_TRANSPOSE, M->dtype, M->n);
    nd->src[0] = M; retain(M);
    nd->matrix = true; nd->rows = M->cols; nd->cols = M->rows;
    nd->space = 0;
    *out = nd;
    return SG_OK;
}

sg_status sg_matvec(sg_node M, sg_node v, int side, sg_node* out) {
    sg_ctx_s* ctx = M ? M->ctx : nullptr;
    if (!M || !v || !out) return fail(ctx, SG_E_INVALID, "matvec: NULL argument");
    if (side != 0 && side != 1) return fail(ctx, SG_E_INVALID, "matvec: side is 0 (right) or 1 (left)");
    if (!M->matrix) return fail(ctx, SG_E_SHAPE, "matvec: first operand must be a matrix");
    if (!is_collection(v) || v->space != 0) return fail(ctx, SG_E_SHAPE, "matvec: the vector must be a dense collection");
    if (M->dtype != SG_F32 || v->dtype != SG_F32) return fail(ctx, SG_E_DTYPE, "matvec: f32 operands");
    const int64_t need = side == 0 ? M->cols : M->rows;
    if (v->n != need)
        return fail(ctx, SG_E_SHAPE, side == 0 ? "right_multiply: count(v) must equal the matrix's columns"
                                               : "left_multiply: count(v) must equal the matrix's rows");
    auto* nd = new_node(ctx, OPN_MATVEC, SG_F32, side == 0 ? M->rows : M->cols);
    nd->matrix = true;
    nd->rows = side == 0 ? M->rows : 1;
    nd->cols = side == 0 ? 1 : M->cols;
    nd->space = 0;
    // M^T v = v M: read the transpose's operand in the other orientation
    sg_node_s* src = M;
    int s = side;
    if (M->op == OPN_TRANSPOSE) {
        src = M->src[0];
        s = 1 - side;
    }
    nd->src[0] = src; retain(src);
    nd->src[1] = v; retain(v);
    nd->binop = s;  // side of the product as computed
    *out = nd;
    return SG_OK;
}

sg_status sg_gauss_det(sg_node A, sg_node* out) {
    sg_ctx_s* ctx = A ? A->ctx : nullptr;
    if (!A || !out) return fail(ctx, SG_E_INVALID, "gauss_det: NULL argument");
    if (!A->matrix) return fail(ctx, SG_E_SHAPE, "gauss_det: operand must be a matrix");
    if (A->rows != A->cols) return fail(ctx, SG_E_SHAPE, "gauss_det: the matrix must be square (rows = columns)");
    if (A->dtype != SG_F32) return fail(ctx, SG_E_DTYPE, "gauss_det: f32 matrices (eliminated in float64)");
    if (A->rows > 46340) return fail(ctx, SG_E_UNSUPPORTED, "gauss_det: at most 46340 rows");
    auto* nd = new_node(ctx, OPN_GAUSS, SG_F64, 1);
    nd->src[0] = A; retain(A);
    nd->space = 0;
    *out = nd;
    return SG_OK;
}

sg_status sg_release(sg_node n) {
    if (!n) return SG_E_INVALID;
    release(n);
    return SG_OK;
}

}  // extern "C"
