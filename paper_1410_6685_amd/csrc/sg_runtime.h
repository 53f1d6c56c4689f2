// Host-side objects of the runtime: context, nodes, agents, programs and plans.
#pragma once
#include <hip/hip_runtime.h>

#include <deque>
#include <map>
#include <tuple>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/safegpu.h"
#include "sg_kernels.h"

namespace sgrt {

// OPN_MATMUL and later: "kernel nodes", computed by a step of their own (not a streaming pass)
enum NodeOp { OPN_INPUT = 0, OPN_MAP, OPN_ZIP, OPN_FILTER, OPN_REDUCE, OPN_MATMUL, OPN_QSORT, OPN_CONCAT, OPN_GAUSS,
              OPN_TRANSPOSE, OPN_MATVEC };
enum NodeState { ST_NONE = 0, ST_COMPUTED = 1, ST_UNPUBLISHED = 2 };
enum FnKind { FK_AFFINE = 0, FK_ADDC, FK_MULC, FK_UNARY, FK_COMPOSE, FK_EXPR };
// node of an expression agent: x, a binary32 constant, a unary or a binary operation
enum ExprKind : uint8_t { EX_X = 0, EX_CONST, EX_NEG, EX_ABS, EX_SQRT, EX_EXP, EX_ADD, EX_SUB, EX_MUL, EX_DIV };
struct ExprNode {
    uint8_t kind;
    float c;   // EX_CONST
    int a, b;  // operand nodes
};
enum PredKind { PK_CMP = 0, PK_FINITE, PK_RANGE, PK_TRUE, PK_AND, PK_OR, PK_NOT };

struct Scratch {
    void* base = nullptr;
    uint64_t* acc = nullptr;          // insts x MAX_SLOTS x MAX_SPREAD
    sg::InstResult* results = nullptr;
    uint64_t* tags = nullptr;         // tiles x TAG_WORDS
    uint64_t* lookback = nullptr;     // tiles x substeps x MAX_WAVES
    uint32_t* epoch = nullptr;        // device epoch word (graph replays)
    int64_t tiles = 0, insts = 0, chunks = 0;
    size_t bytes = 0;
};

struct KTime { double ms = 0; int64_t n = 0; };

struct Plan;

}  // namespace sgrt

struct sg_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    int refs = 1;  // the creator's reference plus one per node, program, batch and MLP
    int num_cu = 256;
    std::string arch = "gfx950";  // offload target of run-time compiled kernels
    bool specialize = false;       // run passes through kernels compiled for their program
    sg_mode mode = SG_MODE_PRE_POST;
    bool fused = true;
    int block = 256;
    int unroll = 2;
    int substeps = 8;
    int batch_substeps = 1;  // sub-tiles per tile of batched launches
    // where programs without a plan of their own get one (sg_ctx_set_plan_source); the model
    // and the timing database are the caller's, borrowed while they are set
    int plan_source = SG_PLAN_DEFAULT;
    std::vector<sg_plan> plan_cands;  // empty: the built-in candidates
    struct sg_mlp_s* plan_model = nullptr;
    struct sg_tunedb_s* plan_db = nullptr;
    float plan_margin = 0.01f;
    int plan_reps = 3;
    uint32_t epoch = 0;  // host epoch of direct launches
    int last_grid = 0, last_block = 0, last_unroll = 0, last_substeps = 0;  // last streaming launch
    size_t last_lds = 0;
    bool timing = false;
    uint32_t wait_limit = 0;  // spin limit of the kernels' bounded waits (raw form, 0 = default)
    uint64_t next_id = 0;
    uint64_t generation = 0;  // bumped when a setting that changes plans changes
    std::string error;
    std::map<size_t, std::vector<void*>> pool;  // freed blocks by size, reused by later allocations
    size_t pooled_bytes = 0;                     // bytes held in `pool`
    std::unordered_map<void*, size_t> sizes;
    sg_allocator ext{};                          // the caller's allocator (alloc null: none)
    std::unordered_map<void*, sg_allocator> ext_blocks;  // blocks from a caller's allocator
    sgrt::Scratch scratch;
    sg::InstResult* host_results = nullptr;
    std::map<std::string, sgrt::KTime> times;
    std::vector<hipEvent_t> events;
    std::map<std::tuple<int, int, size_t>, int> occupancy;  // (±unroll, block, LDS bytes) -> blocks per CU
};

struct sg_fn_s {
    int refs = 1;
    int kind = 0;
    double a = 0, b = 0;
    sg_fn_s* f = nullptr;
    sg_fn_s* g = nullptr;
    std::vector<sgrt::ExprNode>* expr = nullptr;  // FK_EXPR: the parsed expression (owned)
    int expr_root = -1;
};

struct sg_pred_s {
    int refs = 1;
    int kind = 0;
    int cmp = 0;
    double c = 0, lo = 0, hi = 0;
    sg_pred_s* p = nullptr;
    sg_pred_s* q = nullptr;
};

struct sg_node_s {
    int refs = 1;
    sg_ctx_s* ctx = nullptr;
    int op = 0;
    sg_dtype dtype = SG_F32;
    int64_t n = 0;  // capacity (element count of the unfiltered index space)
    bool matrix = false;
    int64_t rows = 0, cols = 0;
    sg_node_s* src[2] = {nullptr, nullptr};
    sg_fn_s* fn = nullptr;
    sg_pred_s* pred = nullptr;
    int binop = 0, red = 0;
    uint64_t space = 0;  // index-space identity (filters start a new one)
    uint64_t id = 0;     // creation order: a topological order of the DAG
    // storage of a materialized collection
    void* dev = nullptr;
    bool owned = false;
    size_t bytes = 0;
    // results
    int state = sgrt::ST_NONE;
    int64_t count = 0;     // elements of a computed collection
    double fval = 0.0;     // scalar value (float results rounded to their dtype)
    double f64 = 0.0;      // float64 shadow of float sums / averages
    int64_t ival = 0;      // integer scalar value
    const int64_t* count_dev = nullptr;  // device address of a compacted collection's count
    void* aux = nullptr;   // kernel-node state kept between executions (determinant: workspace, graph)
    int32_t det_sign = 0;  // determinant = det_sign * det_mant * 2^det_expo
    double det_mant = 0.0;
    int64_t det_expo = 0;
};

namespace sgrt {

struct Contract {
    int32_t id = 0;
    int kind = SG_REQUIRE;
    int check = SG_CHECK_FOR_ALL;
    sg_node_s* node = nullptr;
    sg_pred_s* pred = nullptr;
    sg_node_s *a = nullptr, *b = nullptr, *r = nullptr;  // product check operands
    double abs_tol = 0, rel_tol = 0;
};

// One pass of the streaming kernel.
struct InstPlan {
    std::vector<sg_node_s*> sources;   // loaded into registers 0..nin-1
    std::vector<sg::SgOp> prog;
    std::vector<sg_node_s*> outs;      // materialized outputs, out[k]
    std::vector<uint8_t> slot_kind;
    int nsum = 0;
    int scan_space = 0;
    int count_slot = -1;
    int base_count_slot = -1;          // count of space 0 when it is a compacted source's
    int64_t n = 0;                     // element count (capacity when n_src is set)
    sg_node_s* n_src = nullptr;        // compacted source whose device count is n
    struct ScalarOut { sg_node_s* node; int slot; int sum; int count_slot; };
    std::vector<ScalarOut> scalars;
    struct CheckOut { int contract; int slot; };
    std::vector<CheckOut> checks;
    struct AbsSum { int contract; int sum; };
    std::vector<AbsSum> abssums;
    std::vector<sg_node_s*> compacted;  // outputs whose count is the scan count
    int result_index = 0;               // slot in the results array
    // specialized kernel of this pass (owned by the kernel cache) and the shape it was
    // compiled for; looked up again only when the shape changes
    void* jit = nullptr;
    int jit_unroll = 0, jit_block = 0;
};

struct Step {
    enum Kind { STREAM = 0, GEMM = 1, PRODUCT = 2, NODE = 3 } kind = STREAM;
    int inst = -1;                           // STREAM
    sg_node_s *A = nullptr, *B = nullptr, *C = nullptr, *R = nullptr;  // GEMM / PRODUCT
    int contract = -1;                       // PRODUCT
    sg_node_s* node = nullptr;               // NODE: the kernel node it computes
};

struct Plan {
    std::vector<InstPlan> insts;
    std::vector<Step> steps;
    std::vector<int> active;        // contracts evaluated (indices into the program's list)
    std::vector<sg_node_s*> mats;   // nodes materialized by this plan
    std::vector<int> prod_result;   // contract -> result slot of its product check (-1)
    uint64_t generation = 0;
    bool valid = false;
};

struct Timed {
    const char* name;
    hipEvent_t a, b;
};

// Where one execution's results and timing events go: the context's pinned results and event
// pool for a synchronous execution, a slot of the program for an asynchronous launch.
struct ExecSlot {
    sg::InstResult* host = nullptr;      // results copied back (pinned host memory)
    int64_t host_cap = 0, nres = 0;
    bool owned = false;                  // host allocated for this slot (else the context's)
    hipEvent_t done = nullptr;           // recorded after the copy (asynchronous launches)
    std::vector<Timed> timed;
    std::vector<hipEvent_t>* events = nullptr;  // pool the timing events are drawn from
    std::vector<hipEvent_t> own_events;
};

sg_status fail(sg_ctx_s* ctx, sg_status st, const std::string& msg);
// the context a timing database belongs to (persist.hip)
sg_ctx_s* tunedb_ctx(const sg_tunedb_s* db);
// a program with no plan of its own gets one from its context's plan source, before its
// first execution or launch (tune.hip)
sg_status apply_plan_source(sg_program_s* p);
// SG_OK when [p, p + bytes) lies inside one device allocation of the calling process
sg_status check_device_range(sg_ctx_s* ctx, const void* p, size_t bytes, const char* what);
sg_status hip_fail(sg_ctx_s* ctx, hipError_t e, const char* what);
void* dev_alloc(sg_ctx_s* ctx, size_t bytes);
void dev_free(sg_ctx_s* ctx, void* p);
// Return every pooled (freed, unused) block to the device after the device is idle; bytes freed.
size_t pool_trim(sg_ctx_s* ctx);
sg_status ensure_scratch(sg_ctx_s* ctx, int64_t tiles, int64_t chunks, int64_t insts);
sg_status alloc_scratch(sg_ctx_s* ctx, Scratch& S, int64_t tiles, int64_t chunks, int64_t insts);
uint32_t next_epoch(sg_ctx_s* ctx);
void ctx_retain(sg_ctx_s* ctx);
// run-time specialized streaming kernels (jit.hip)
sg_status jit_kernel(sg_ctx_s* ctx, const InstPlan& ip, int unroll, int block, void** handle);
int jit_occupancy(void* handle, int block, size_t lds);
// with events given, they are recorded at the kernel's own start and end
hipError_t jit_launch(void* handle, const sg::StreamArgs& a, int grid, int block, size_t lds, hipStream_t s,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void ctx_release(sg_ctx_s* ctx);
void fill_inst(const InstPlan& ip, sg::InstDesc& d, int64_t tile0, int64_t ntiles, int prog_off);
void publish_inst(const InstPlan& ip, const sg::InstResult& r, bool publish_values);
sg_status alloc_output(sg_ctx_s* ctx, sg_node_s* n);
sg_status assemble_verdicts(sg_program_s* P, const sg::InstResult* results, std::vector<sg_verdict>& V);
int stream_grid(sg_ctx_s* ctx, int64_t ntiles, bool inl, int unroll, int block, size_t lds_bytes, bool waits);
int coresident_blocks(int occupancy, int lds_blocks, bool waits_on_others);
// Launch shape of a pass: sub-tiles per tile (clamped when values are staged for
// compaction) and the dynamic LDS bytes of its per-lane accumulators and staging regions.
int inst_cemit(const InstPlan& ip);
int stream_substeps(int C, int block, int unroll, int slots, int sums, int cemit, bool scan, int nbuf);
size_t stream_lds_bytes(int slots, int sums, int cemit, int C, int block, int unroll, int nbuf);
int lds_blocks_per_cu(size_t dyn_lds);
constexpr size_t kLdsPerCu = 160 * 1024;      // LDS of a gfx950 CU
constexpr size_t kLdsReserve = 2 * 1024;      // margin kept free when sizing a resident grid
constexpr size_t kStaticLdsBound = 10 * 1024;  // the streaming kernel's static LDS (checked there)
// dynamic LDS a streaming block may use (160 KiB per CU, less the kernel's static part)
constexpr size_t kMaxDynamicLds = 152 * 1024;
void retain(sg_node_s* n);
void retain(sg_fn_s* f);
void retain(sg_pred_s* p);
void release(sg_node_s* n);
void release(sg_fn_s* f);
void release(sg_pred_s* p);
bool is_elementwise(const sg_node_s* n);
// computed by a step of its own: matrix product, quicksort, concatenation
inline bool is_kernel_node(const sg_node_s* n) { return n->op >= OPN_MATMUL; }
bool is_collection(const sg_node_s* n);
// emit the ops applying f in place to register r; `temps` are registers free for the duration
// (expression agents need them: fn_temps).  False when there are too few.
bool emit_fn(std::vector<sg::SgOp>& prog, const sg_fn_s* f, int r, sg_dtype dt, const std::vector<int>& temps = {});
int fn_temps(const sg_fn_s* f);
// expression agents (expr.hip)
bool parse_expr(const char* text, std::vector<ExprNode>& out, int* root, std::string* why);
int expr_temps(const std::vector<ExprNode>& e, int root);
bool emit_expr(std::vector<sg::SgOp>& prog, const std::vector<ExprNode>& e, int root, int r, const std::vector<int>& temps);
void emit_pred(std::vector<sg::SgOp>& prog, const sg_pred_s* p, int r, sg_dtype dt);

}  // namespace sgrt

struct sg_program_s {
    int refs = 1;
    sg_ctx_s* ctx = nullptr;
    std::vector<sg_node_s*> roots;
    std::vector<sgrt::Contract> contracts;
    std::vector<sg_node_s*> splits;
    std::vector<sg_node_s*> builtin_done;  // operations whose built-in clauses are attached
    // launch plan chosen for this program (autotuner / selector); 0 = the context default
    int block = 0, unroll = 0, substeps = 0;
    sg_node_s* plan_split = nullptr;  // extra fusion split point of the plan
    int plan_from = SG_PLAN_DEFAULT;  // how the plan was chosen (SG_PLAN_*)
    bool plan_auto_tried = false;     // the context's plan source has been applied
    sgrt::Plan plan;
    int32_t next_contract = 0;
    // asynchronous launches: slots in use, oldest first (the program is not changed meanwhile)
    static constexpr int kMaxPending = 4;
    sgrt::ExecSlot slots[kMaxPending];
    std::deque<int> pending;
};

struct sg_batch_s;

// Cost-model MLP (24-64-64-1) of the learned plan selector.
struct sg_mlp_s {
    sg_ctx_s* ctx = nullptr;
    float* P = nullptr;    // params | grad | Adam m | Adam v (device)
    double* loss = nullptr;
    int step = 0;
    bool norm_set = false;
    float mean[24], scale[24], lo[24], hi[24];
};

#define SG_HIP(ctx, call)                                              \
    do {                                                               \
        hipError_t _e = (call);                                        \
        if (_e != hipSuccess) return sgrt::hip_fail((ctx), _e, #call); \
    } while (0)

namespace sgrt {
sg_status build_plan(sg_program_s* P, Plan* out);
// Run the step of a quicksort or concatenation node (host-driven; synchronizes the stream).
// `results` are the execution's device results (a compacted source's count is read from the
// pass that made it); `slot` is this step's result slot, which receives the output's count.
sg_status run_node_step(sg_ctx_s* ctx, const Plan& plan, sg_node_s* n, sg::InstResult* results, sg::InstResult* slot);
// sort m items into out (quicksort of Listing 3); *count = items kept
sg_status run_quicksort(sg_ctx_s* ctx, const void* in, void* out, int64_t m, bool is_f32, int64_t* count);
// determinant by Gaussian elimination (graph-captured loop); sets the node's scalar fields
sg_status run_gauss(sg_ctx_s* ctx, sg_node_s* node);
// transposition and matrix-vector products (linalg.hip)
sg_status run_linalg(sg_ctx_s* ctx, sg_node_s* node);
void gauss_cache_free(sg_ctx_s* ctx, void* cache);
const char* node_step_name(const sg_node_s* n);
sg_status execute_program(sg_program_s* P, sg_verdict* v, int32_t cap, int32_t* nv);
}  // namespace sgrt
