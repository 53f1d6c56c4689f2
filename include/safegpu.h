/*
 * safegpu.h -- C ABI of the contract-checked, fused collection library for AMD Instinct
 * MI355X (gfx950).
 *
 * The calls follow the library's problem statement: create a collection (from_array,
 * Section 3.2 / Table 2), compose operations with agents (project, filter, reductions,
 * vector and matrix arithmetic, Sections 3.2-3.4), attach require/ensure clauses built from
 * range queries (for_all, exists, is_sorted, sums; Section 4), and trigger execution
 * (scalar query, to_array, update; Section 5).  Composition is lazy: nothing runs on the GPU
 * until a trigger.  The planner then fuses element-wise operations, filters and reductions
 * over one index space into a single kernel pass (the barrier and expression fusions of
 * Figures 2 and 3), and evaluates range contracts inside the same pass.
 *
 * Conventions (all entry points):
 *   - Every call returns sg_status; results are written through out-parameters only when
 *     the call returns SG_OK (or a contract status, see sg_program_execute).
 *   - Device pointers are HIP device addresses on the context's device; host pointers are
 *     ordinary host memory.  Sizes are element counts (int64), never bytes, unless named
 *     *_bytes.
 *   - Handles (sg_ctx, sg_node, sg_fn, sg_pred, sg_program, sg_batch) are owned by the
 *     caller and released with the matching *_release / *_destroy call.  A derived node
 *     holds references to its operands, a program to its roots and contract operands, so
 *     operands may be released early.
 *   - Misuse (NULL handle, wrong element type, mismatched counts) returns an SG_E_* code
 *     and never aborts; sg_last_error() then describes it.  HIP runtime failures map to
 *     SG_E_DEVICE.
 *   - Indices reported by contracts are 0-based int64; -1 means "none".
 *   - All device work is ordered on the stream given to sg_ctx_create; calls that return
 *     host-visible results synchronize that stream.  A context is not thread-safe.
 */
#ifndef SAFEGPU_H
#define SAFEGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sg_status {
    SG_OK = 0,
    SG_E_INVALID = 1,      /* bad argument or handle */
    SG_E_SHAPE = 2,        /* built-in scalar contract: counts / dimensions disagree */
    SG_E_DTYPE = 3,        /* operation not defined on this element type */
    SG_E_OOM = 4,          /* device or host allocation failed */
    SG_E_DEVICE = 5,       /* HIP runtime error or device-side failure */
    SG_E_STATE = 6,        /* value not available (not computed, or unpublished) */
    SG_E_UNSUPPORTED = 7,  /* a chain the planner cannot place (limits exceeded) */
    SG_PRE_VIOLATED = 16,  /* a require clause failed: the body's outputs are not published */
    SG_POST_VIOLATED = 17  /* an ensure clause failed: outputs exist, the clause is flagged */
} sg_status;

typedef enum sg_dtype { SG_F32 = 1, SG_I32 = 2, SG_I64 = 3, SG_F64 = 4 } sg_dtype;

/* Monitoring modes of Section 6.3 without class invariants (this library has none). */
typedef enum sg_mode { SG_MODE_OFF = 0, SG_MODE_PRE = 1, SG_MODE_PRE_POST = 2 } sg_mode;

/* Element functions (agents of type FUNCTION, Section 3.2). */
typedef enum sg_fn_kind {
    SG_FN_SQUARE = 1, SG_FN_NEG = 2, SG_FN_ABS = 3, SG_FN_SQRT = 4, SG_FN_SQRT_ABS = 5,
    SG_FN_EXP = 6, SG_FN_EXP_NEG_SQ = 7, SG_FN_I2F = 8
} sg_fn_kind;

typedef enum sg_cmp { SG_LT = 0, SG_LE = 1, SG_GT = 2, SG_GE = 3, SG_EQ = 4, SG_NE = 5 } sg_cmp;
typedef enum sg_binop { SG_ADD = 0, SG_SUB = 1, SG_MUL = 2, SG_DIV = 3 } sg_binop;
typedef enum sg_red { SG_SUM = 0, SG_MIN = 1, SG_MAX = 2, SG_AVG = 3, SG_COUNT = 4 } sg_red;
typedef enum sg_clause { SG_REQUIRE = 0, SG_ENSURE = 1 } sg_clause;
typedef enum sg_quant { SG_FOR_ALL = 0, SG_EXISTS = 1 } sg_quant;

typedef struct sg_ctx_s* sg_ctx;
typedef struct sg_node_s* sg_node;
typedef struct sg_fn_s* sg_fn;
typedef struct sg_pred_s* sg_pred;
typedef struct sg_program_s* sg_program;
typedef struct sg_batch_s* sg_batch;

/* One verdict per contract clause of a program, in declaration order. */
typedef struct sg_verdict {
    int32_t contract_id;  /* id returned when the clause was attached */
    int32_t kind;         /* SG_REQUIRE or SG_ENSURE */
    int32_t holds;        /* 1 holds, 0 violated, -1 not evaluated (mode, or body not run) */
    int32_t check;        /* SG_CHECK_* */
    int64_t first_index;  /* first violating (for_all, sorted) / witnessing (exists) index,
                             first violating row (product); -1 if none */
    double measure;       /* product: max |e_i|/b_i; close: |s - s64|; else 0 */
} sg_verdict;

enum { SG_CHECK_FOR_ALL = 0, SG_CHECK_EXISTS = 1, SG_CHECK_SORTED = 2, SG_CHECK_CLOSE = 3,
       SG_CHECK_PRODUCT = 4, SG_CHECK_COUNT_EQ = 5, SG_CHECK_QUOTIENT = 6 };

/* Device memory for the library's outputs and work buffers from the caller's allocator (for
 * example the framework's caching allocator, so that one pool serves both).  alloc returns
 * `bytes` of device memory usable by work on `stream` (the context's hipStream_t) or NULL;
 * free releases it; the library calls free only after enqueueing the last work that uses
 * the block on that stream, so a stream-ordered allocator may reuse it at once.  `user` is
 * passed through.  Stream scratch, batch tables and the static no-alloc array stay the
 * library's own. */
typedef struct sg_allocator {
    void* (*alloc)(size_t bytes, void* stream, void* user);
    void (*free)(void* p, void* stream, void* user);
    void* user;
} sg_allocator;

/* ---- context ---------------------------------------------------------------------------- */

/* Create a context on HIP device `device` (Section 2.2: the runtime that owns device memory
 * and launches generated kernels); `hip_stream` is a hipStream_t (NULL = the null stream) on
 * which all work is enqueued.  Mode defaults to SG_MODE_PRE_POST, fusion on.  SG_E_INVALID
 * for a bad device or NULL out. */
sg_status sg_ctx_create(int device, void* hip_stream, sg_ctx* out);
/* Releases the context once every node, program and batch made from it is released. */
sg_status sg_ctx_destroy(sg_ctx ctx);
/* Use `a` (copied; both functions non-NULL) for the device memory allocated from now on, or the
 * library's own pool when a is NULL.  Blocks keep the allocator they came from.  SG_E_INVALID
 * for a NULL context or a half-filled allocator. */
sg_status sg_ctx_set_allocator(sg_ctx ctx, const sg_allocator* a);
/* Contract monitoring mode (Section 6.3: no checking, preconditions only, pre- and
 * postconditions).  SG_E_INVALID for an unknown mode. */
sg_status sg_ctx_set_mode(sg_ctx ctx, sg_mode mode);
/* fused != 0: fuse (default; Section 5, Figures 2 and 3 after optimization).  fused == 0:
 * the plan before optimization, one kernel per operation and per contract, every
 * intermediate materialized. */
sg_status sg_ctx_set_fusion(sg_ctx ctx, int fused);
/* Launch plan for the streaming kernel (the launch configuration of a generated kernel,
 * Section 5): block size (64..1024, multiple of 64) and unroll (1, 2 or 4: 16-byte loads per
 * lane per input and sub-tile).  0 keeps the default; other values give SG_E_INVALID. */
sg_status sg_ctx_set_launch(sg_ctx ctx, int block, int unroll);
/* Sub-tiles per tile (1..16) of the batched launches created afterwards (sg_batch_create):
 * a tile is the unit a block takes, publishes and finalizes, so larger tiles mean fewer such
 * steps per element; capped where the tile's compaction staging would not fit in LDS.
 * Default 1.  SG_E_INVALID outside 1..16. */
sg_status sg_ctx_set_batch_substeps(sg_ctx ctx, int substeps);
/* on != 0: run every single-program pass through a kernel compiled at run time (hiprtc) for
 * that pass's program, as the paper generates one kernel per merged plan (Section 5);
 * compiled once per device and program, then cached for the process.  on == 0 (default):
 * the precompiled interpreter kernel.  Results are identical; a compilation failure is
 * reported as SG_E_DEVICE with the compiler log in sg_last_error.  Batches always use the
 * interpreter. */
sg_status sg_ctx_set_specialize(sg_ctx ctx, int on);
/* Record the device time of every kernel launch with HIP events on the context stream (the
 * measurements of Section 6.1 without the host-side floor). */
sg_status sg_ctx_set_timing(sg_ctx ctx, int on);
/* Spin limit of the kernels' bounded waits (compaction prefixes, result finalization): a
 * wait that reaches it gives up, and the execution returns SG_E_DEVICE with the context's
 * (or the batch's) kernel state cleared, so the next execution starts clean.  spins < 0
 * restores the default (about 4 s); 0 makes every such wait give up at once, which lets the
 * error path be exercised from the host.  Applies to later launches, including replays of
 * batches created earlier. */
sg_status sg_ctx_set_wait_limit(sg_ctx ctx, int64_t spins);
/* Accumulated device time (ms) and launch count of one kernel family since the last reset:
 * "stream" (interpreter), "stream_spec" (specialized), "gemm", "product_check", "mlp_train",
 * "mlp_infer". */
sg_status sg_ctx_timing(sg_ctx ctx, const char* kernel, double* total_ms, int64_t* launches);
sg_status sg_ctx_timing_reset(sg_ctx ctx);
/* Shape of the last streaming-kernel launch on this context (single-program passes): grid
 * and block size, unroll, sub-tiles per tile and dynamic LDS bytes per block.  Any out
 * pointer may be NULL. */
sg_status sg_ctx_last_launch(sg_ctx ctx, int32_t* grid, int32_t* block, int32_t* unroll, int32_t* substeps,
                             int64_t* lds_bytes);
/* Message for the last error on this context (thread-unsafe, valid until the next call). */
const char* sg_last_error(sg_ctx ctx);

/* ---- collections (Section 3.2 from_array; Section 3.4 row-major matrices) ------------- */

/* Borrow `n` elements of device memory at `dev` (a collection of count = capacity = n,
 * Section 3.2; 16-byte alignment gives 128-bit loads).  The caller keeps the memory alive
 * and unmodified while any execution reads it.  SG_E_INVALID for a NULL address with n > 0
 * or memory the HIP runtime does not know as device memory of the context's device. */
sg_status sg_vector_wrap(sg_ctx ctx, sg_dtype dtype, void* dev, int64_t n, sg_node* out);
/* A rows x cols matrix stored row-wise in one array (Section 3.4). */
sg_status sg_matrix_wrap(sg_ctx ctx, sg_dtype dtype, void* dev, int64_t rows, int64_t cols, sg_node* out);
/* from_array (Table 2): copy `n` host elements to new device memory owned by the node, in
 * one copy (Section 3.2).  SG_E_OOM when the device memory cannot be had. */
sg_status sg_vector_from_host(sg_ctx ctx, sg_dtype dtype, const void* host, int64_t n, sg_node* out);
sg_status sg_matrix_from_host(sg_ctx ctx, sg_dtype dtype, const void* host, int64_t rows, int64_t cols, sg_node* out);

/* ---- agents ---------------------------------------------------------------------------- */

/* Agents of type FUNCTION (Section 3.2, project): side-effect free element functions.
 * f32: x -> RN(RN(a*x) + b).  i32: x -> a*x + b modulo 2^32 (a, b truncated to int32).
 * Constants are rounded to the element type when the function is applied. */
sg_status sg_fn_affine(double a, double b, sg_fn* out);
/* x + c and x * c (the scalar operations of Section 3.3 with the vector's own rounding). */
sg_status sg_fn_add_c(double c, sg_fn* out);
sg_status sg_fn_mul_c(double c, sg_fn* out);
/* One of sg_fn_kind (sqrt as in the project example of Section 3.2; exp correctly rounded).
 * SG_E_INVALID for an unknown kind. */
sg_status sg_fn_unary(sg_fn_kind kind, sg_fn* out);
/* A user element function written as an arithmetic expression in x (an agent of type
 * FUNCTION, Section 3.2, which the paper compiles into the generated kernel, Section 5):
 *     expr := term (("+" | "-") term)*     term := unary (("*" | "/") unary)*
 *     unary := "-" unary | primary
 *     primary := number | "x" | "(" expr ")" | ("sqrt" | "abs" | "exp") "(" expr ")"
 * Literals are rounded to binary32 (through their float64 value) when the function is made;
 * every operation gives the correctly rounded binary32 result on binary32 operands, along the
 * tree the grammar gives.  Defined on f32 (SG_E_DTYPE otherwise).  SG_E_INVALID with the
 * offset of the first error for text outside the grammar.  A map by an expression needs
 * registers of the streaming pass for its intermediate values; a chain that runs out of them
 * gets SG_E_UNSUPPORTED (a split point helps). */
sg_status sg_fn_expr(const char* text, sg_fn* out);
/* first f, then g (one agent made of two, evaluated as one expression, Figure 3) */
sg_status sg_fn_compose(sg_fn f, sg_fn g, sg_fn* out);
sg_status sg_fn_release(sg_fn f);

/* Agents of type PREDICATE (Section 3.2, filter / for_all / exists).  Comparisons are IEEE
 * comparisons against c rounded to the operand's element type (false with NaN). */
sg_status sg_pred_cmp(sg_cmp op, double c, sg_pred* out);
sg_status sg_pred_isfinite(sg_pred* out);
sg_status sg_pred_in_range(double lo, double hi, sg_pred* out); /* lo <= x <= hi */
sg_status sg_pred_true(sg_pred* out);
sg_status sg_pred_and(sg_pred p, sg_pred q, sg_pred* out);
sg_status sg_pred_or(sg_pred p, sg_pred q, sg_pred* out);
sg_status sg_pred_not(sg_pred p, sg_pred* out);
sg_status sg_pred_release(sg_pred p);

/* ---- lazy operations ------------------------------------------------------------------- */

/* project (Table 2): a new collection of count(in) items, item i = f(in[i]).  Lazy: nothing
 * runs until a trigger (Section 5).  SG_E_DTYPE when f is not defined on the element type. */
sg_status sg_map(sg_node in, sg_fn f, sg_node* out);
/* Vector plus / minus / compwise multiply / compwise_divide (Section 3.3).  Built-in scalar
 * contract: equal counts and dimensions, same index space (SG_E_SHAPE).  SG_DIV is defined on
 * f32 and carries the built-in clauses of Listing 2, which a program receives when a root that
 * depends on the division is added (in node creation order, after the clauses already there):
 * require for_all(divisor /= 0) over the divisor and ensure quotient (SG_CHECK_QUOTIENT):
 * RN(q * d) = n, or |RN(q * d) - n| <= 4u |n| + 2^-149 |d| with u = 2^-24, for every item
 * (the float reading of Result * other = Current).  'Current = old Current' holds by
 * construction: operations never change their operands. */
sg_status sg_zip(sg_node a, sg_node b, sg_binop op, sg_node* out);
/* filter (Table 2): the items of `in` for which p holds, in their order (stable); capacity
 * = capacity(in), count known on the device after execution (Section 3.2). */
sg_status sg_filter(sg_node in, sg_pred p, sg_node* out);
/* sum / min / max / avg (Section 3.3, device-side reductions) and count (Table 2) as a
 * scalar node.  Float sums accumulate in float64 in a fixed order; min / max of an empty
 * collection are -inf / +inf (INT_MIN / INT_MAX), avg of an empty collection is NaN. */
sg_status sg_reduce(sg_node in, sg_red red, sg_node* out);
/* multiply (Section 3.4): C = A B for f32 matrices with cols(A) = rows(B) (built-in scalar
 * contract, SG_E_SHAPE), on the FP32 matrix cores with FP32 accumulation. */
sg_status sg_matmul(sg_node A, sg_node B, sg_node* out);
/* Matrix transposition (Section 3.4 transpose): rows x cols -> cols x rows, row-major. */
sg_status sg_transpose(sg_node M, sg_node* out);
/* Matrix-vector products (Section 3.4 right_multiply / left_multiply, Listing 1) of an f32
 * matrix M (r x c) and a dense f32 vector v: side 0 (right) M v with count(v) = c -> r x 1;
 * side 1 (left) v M with count(v) = r -> 1 x c (built-in scalar contracts, SG_E_SHAPE).  Each
 * entry is a float64 sum of the exact float32 products in a fixed order, rounded to float32.
 * A right product of a transposed matrix is planned as the left product of the original
 * (the transpose is not materialized; the result keeps its c x 1 shape). */
sg_status sg_matvec(sg_node M, sg_node v, int side, sg_node* out);
/* concatenate (Table 2): the items of a followed by those of b (same element type; vectors).
 * Capacity a.capacity + b.capacity; count a.count + b.count. */
sg_status sg_concat(sg_node a, sg_node b, sg_node* out);
/* The quicksort of Section 4 (Listing 3) on an f32 or i32 vector: pivot = the item at index
 * count / 2, three stable filters (less, equal, greater), result = quicksort(less) ++ equal ++
 * quicksort(greater), run level by level on the GPU.  Items no filter keeps (NaN items, or all
 * items of a collection whose pivot is NaN) are dropped, as in the listing, so the result's
 * count can be smaller than the input's: attach sg_program_count_eq to check it.  Capacity =
 * the input's capacity. */
sg_status sg_quicksort(sg_node in, sg_node* out);
/* Determinant of a square f32 matrix by Gaussian elimination (Section 5, Listing 5, in its
 * textbook form: partial pivoting, a zero pivot column means det = 0), in float64 on the
 * widened input, as a scalar node.  Built-in precondition rows = columns (SG_E_SHAPE).  The
 * elimination loop (3n + 1 kernels) is captured into a HIP graph once per node and replayed.
 * sg_scalar_get gives f = the determinant as a double (+-inf beyond its range), i = its sign;
 * sg_det_parts the exact representation. */
sg_status sg_gauss_det(sg_node A, sg_node* out);
/* det = sign * mant * 2^expo with mant in [0.5, 1) (0, 0.0, 0 when singular). */
sg_status sg_det_parts(sg_node det, int32_t* sign, double* mant, int64_t* expo);
sg_status sg_release(sg_node n);

/* ---- programs: roots plus require/ensure clauses ---------------------------------------- */

/* A program is the routine of Section 4: roots (the body) plus require and ensure clauses
 * built from range queries, monitored per the context's mode. */
sg_status sg_program_create(sg_ctx ctx, sg_program* out);
sg_status sg_program_add_root(sg_program p, sg_node n);
/* for_all / exists (Table 2) of predicate `pred` over collection `n` as a require or ensure
 * clause (Section 4; the range preconditions of Listing 2).  The verdict's first_index is the
 * first violating (for_all) or witnessing (exists) index; an empty collection satisfies
 * for_all and fails exists, index -1.  *id receives the clause id. */
sg_status sg_program_quant(sg_program p, sg_clause kind, sg_quant q, sg_node n, sg_pred pred, int32_t* id);
/* is_sorted (Section 3.3; the postcondition of Listing 3): non-decreasing order of
 * collection `n`; first_index = the left item of the first pair out of order (a NaN breaks
 * its pairs). */
sg_status sg_program_sorted(sg_program p, sg_clause kind, sg_node n, int32_t* id);
/* A sum postcondition (the scalar contracts of Section 6.3) made robust to rounding:
 * |value(s) - shadow(s)| <= abs_tol + rel_tol * sum|x| for a float sum node s, where the
 * shadow is the same sum accumulated in float64 in the same pass. */
sg_status sg_program_close(sg_program p, sg_clause kind, sg_node s, double abs_tol, double rel_tol, int32_t* id);
/* Product check of C = A B (the product postcondition Result * other = Current of Listing 2,
 * read with a rounding bound) with the nvec x N matrix R of probe vectors (one per row):
 * |C r - A(B r)|_i <= (gamma_2K + 2^-40) (|A|(|B||r|))_i for every probe and row, in float64;
 * first_index = the first violating row of the first violating probe. */
sg_status sg_program_product(sg_program p, sg_clause kind, sg_node C, sg_node A, sg_node B, sg_node R, int32_t* id);
/* Scalar contract count(n) = old count(other) (the postcondition Result.count = a.count of
 * Listing 3).  The operands are never changed by a program, so the old count is the count
 * before or after the body alike.  Evaluated after the body; measure = count(n) - count(other). */
sg_status sg_program_count_eq(sg_program p, sg_clause kind, sg_node n, sg_node other, int32_t* id);
/* Mark `n` as a fusion split point of the execution plan (Section 5): it is materialized and
 * its consumers start a new pass. */
sg_status sg_program_split(sg_program p, sg_node n);
/* Run the program (the trigger update of Table 2; Section 5): plan, fuse, launch, then the
 * contract protocol of Section 4 (a failed require means the body's results are not
 * published).  Writes up to `cap` verdicts in clause order.  Returns SG_OK, SG_PRE_VIOLATED
 * (outputs unpublished) or SG_POST_VIOLATED, or an error code. */
sg_status sg_program_execute(sg_program p, sg_verdict* verdicts, int32_t cap, int32_t* nverdicts);
/* Asynchronous form of sg_program_execute, for loops that run a program repeatedly: launch
 * enqueues one execution on the context's stream and returns once it is enqueued; wait blocks
 * until the oldest pending execution has finished and returns exactly what sg_program_execute
 * would have returned for it (status, verdicts, published values).  Up to 4 executions of a
 * program may be pending (SG_E_STATE beyond that, or from wait with none pending).  While any
 * is pending the program is not changed: adding roots or clauses, split, set_plan, features,
 * time_plans, execute and a launch after a change of the context's mode return SG_E_STATE.
 * Outputs of a later launch overwrite those of an earlier one as the stream reaches it.
 * Releasing a program waits for its pending executions. */
sg_status sg_program_launch(sg_program p);
sg_status sg_program_wait(sg_program p, sg_verdict* verdicts, int32_t cap, int32_t* nverdicts);
sg_status sg_program_release(sg_program p);

/* update (Table 2) of roots without contracts (shorthand for a temporary program). */
sg_status sg_execute(sg_ctx ctx, const sg_node* roots, int32_t nroots);

/* ---- triggers and results (Section 5: scalar query, to_array) --------------------------- */

/* Scalar query (the trigger of Section 5 that returns a value, e.g. sum in Listing 4):
 * f = value as double (a float sum is rounded to binary32 first), i = integer value (counts,
 * int sums, int min/max).  Executes the node if needed.  SG_E_STATE when the value is
 * unpublished (a failed require). */
sg_status sg_scalar_get(sg_node s, double* f, int64_t* i);
/* float64 shadow of a float sum or avg node (accumulated in float64 in the same pass). */
sg_status sg_scalar_shadow(sg_node s, double* f64);
/* count (Table 2) of a computed collection. */
sg_status sg_count(sg_node c, int64_t* n);
/* item (Table 2): the item at 0-based index i (executes the collection if needed); f = its
 * value as double, iv = as integer (i32 collections).  Built-in precondition 0 <= i < count,
 * else SG_E_INVALID. */
sg_status sg_item(sg_node c, int64_t i, double* f, int64_t* iv);
/* Copy a collection to host memory in one copy (new_cursor of Table 2; Section 3.2), at most
 * cap elements; *n = its count. */
sg_status sg_to_host(sg_node c, void* dst, int64_t cap, int64_t* n);
/* Device address and count of a computed collection (valid until the node is released or
 * recomputed). */
sg_status sg_device_ptr(sg_node c, void** dev, int64_t* n);

/* ---- batched execution: many programs in one persistent launch -------------------------- */

/* Plan `n` programs (each a chain with its own contracts, Section 4) into one launch of the
 * streaming kernel; programs must contain no matrix product, sort or determinant
 * (SG_E_UNSUPPORTED).  The plan and its launch are captured into a HIP graph when
 * use_graph != 0 (the host-loop launch overhead of Section 6.1 paid once). */
sg_status sg_batch_create(sg_ctx ctx, const sg_program* progs, int32_t n, int use_graph, sg_batch* out);
/* Launch once (graph replay or direct launch); results are published to the programs' roots
 * and verdicts. status_out[n] receives each program's status, verdicts are written program
 * by program in clause order (up to cap). */
sg_status sg_batch_run(sg_batch b, int32_t* status_out, sg_verdict* verdicts, int32_t cap, int32_t* nverdicts);
/* Enqueue one launch without reading results back (for timing); sg_batch_run reads them. */
sg_status sg_batch_launch(sg_batch b);
sg_status sg_batch_release(sg_batch b);

/* ---- plans: autotuner and learned selector ------------------------------------------------ */

/* A launch plan of a program's streaming passes: block size (64..1024, multiple of 64),
 * 16-byte loads per lane and input (1, 2 or 4), sub-tiles per tile (1..64), and an optional
 * fusion split point (index into the program's split candidates -- its map/zip/filter nodes
 * in creation order -- or -1): the node is then materialized and its consumers start a new
 * pass. */
typedef struct sg_plan { int32_t block, unroll, substeps, split; } sg_plan;

typedef struct sg_mlp_s* sg_mlp;
typedef struct sg_tunedb_s* sg_tunedb;

sg_status sg_program_split_candidates(sg_program p, int32_t* n);
/* NULL restores the context defaults. */
sg_status sg_program_set_plan(sg_program p, const sg_plan* plan);
/* Cost-model features of (program, plan), 24 floats:
 *  0 affine/add_c/mul_c maps, 1 sqrt maps, 2 exp maps, 3 other unary maps, 4 zip add/sub,
 *  5 zip mul, 6 filters, 7 sums/averages, 8 min/max, 9 counts, 10 for_all/exists clauses,
 *  11 other clauses, 12 depth, 13 log2 length, 14 float32 data, 15 input collections,
 *  16 log2 block, 17 log2 unroll, 18 log2 sub-steps, 19 has split, 20 split position,
 *  21 passes, 22 bytes moved per element, 23 resident blocks per CU. */
sg_status sg_program_features(sg_program p, const sg_plan* plan, float* f24);
/* Autotuner of the optimizer's launch plans (Section 5's plan choice, measured): device time
 * in ms (median of reps runs after one warm-up) of every plan. */
sg_status sg_program_time_plans(sg_program p, const sg_plan* plans, int32_t n, int32_t reps, double* ms_out);
/* Time every plan, set the fastest on the program; *best its index, ms_out (n) the timings. */
sg_status sg_autotune(sg_program p, const sg_plan* plans, int32_t n, int32_t reps, int32_t* best, double* ms_out);

/* The cost model: a 24-64-64-1 float32 MLP with ReLU predicting log run time (us) from
 * standardized features.  Parameters (5825 floats): W1[24][64] b1[64] W2[64][64] b2[64]
 * W3[64] b3, initial values supplied by the caller. */
sg_status sg_mlp_create(sg_ctx ctx, const float* params, int64_t nparams, sg_mlp* out);
sg_status sg_mlp_release(sg_mlp m);
sg_status sg_mlp_get_params(sg_mlp m, float* params, int64_t nparams);
/* Loss (mean squared error) and gradient of one batch of B <= 128 samples (device X B x 24,
 * device targets T B) without updating: grad_host receives 5825 floats. */
sg_status sg_mlp_grad(sg_mlp m, const float* X_dev, const float* T_dev, int32_t B, float* grad_host, double* loss);
/* Adam training (beta 0.9/0.999, eps 1e-8) over n device samples in the given order, in
 * batches of `batch` <= 128, for `epochs` epochs; epoch_loss (host, epochs doubles) gets
 * each epoch's mean loss. */
sg_status sg_mlp_train(sg_mlp m, const float* X_dev, const float* T_dev, int64_t n, int32_t batch, int32_t epochs,
                       float lr, double* epoch_loss);
/* Predictions for n device samples (X n x 24) into device Y (n). */
sg_status sg_mlp_predict(sg_mlp m, const float* X_dev, int64_t n, float* Y_dev);
/* Standardization x' = (x - mean) / scale and the training range [lo, hi] of each feature. */
sg_status sg_mlp_set_norm(sg_mlp m, const float* mean24, const float* scale24, const float* lo24, const float* hi24);
/* The model's standardization (SG_E_STATE if none is set). */
sg_status sg_mlp_get_norm(sg_mlp m, float* mean24, float* scale24, float* lo24, float* hi24);
/* Learned selector: predict all candidates, set the argmin on the program unless a feature
 * is out of the training range or the best two predictions are closer than `margin` (log
 * units), in which case *fallback = 1 and the program's plan is unchanged (the caller runs
 * the autotuner).  pred_out (n, optional) receives the predictions. */
sg_status sg_select_plan(sg_mlp m, sg_program p, const sg_plan* plans, int32_t n, float margin, int32_t* best,
                         float* pred_out, int32_t* fallback);

/* Where a program's launch plan comes from (Section 5: the optimizer chooses how a merged plan
 * runs).  SG_PLAN_DEFAULT: the context's launch settings; SG_PLAN_AUTOTUNE: the autotuner;
 * SG_PLAN_LEARNED: the cost model, with the autotuner where it declines; SG_PLAN_SET: a plan
 * the caller set (sg_program_set_plan, sg_autotune, sg_select_plan). */
typedef enum sg_plan_source { SG_PLAN_DEFAULT = 0, SG_PLAN_AUTOTUNE = 1, SG_PLAN_LEARNED = 2, SG_PLAN_SET = 3 } sg_plan_source;
/* From now on, a program of ctx that has no plan of its own gets one before its first
 * execution or launch: with SG_PLAN_AUTOTUNE the candidates are timed (reps runs each, through
 * `db` when given: plans already recorded for the program's key are read, not timed) and the
 * fastest is kept; with SG_PLAN_LEARNED `model` (standardization set) chooses among them
 * (sg_select_plan with `margin`) and the autotuner decides where it falls back; SG_PLAN_DEFAULT
 * turns this off.  plans (n, copied; NULL/0 = the built-in candidates: ten launch shapes, plus
 * two with the first fusion split point when the program has one).  model and db are borrowed:
 * the caller keeps them alive until the source is set again or the context is destroyed.
 * Timing runs execute the program (their verdicts are not reported).  sg_program_set_plan(p,
 * NULL) lets the source choose again.  SG_E_INVALID for an unknown source, bad plans, reps < 1,
 * a negative margin, a missing model (learned) or a model or database of another context;
 * SG_E_STATE for a model without standardization. */
sg_status sg_ctx_set_plan_source(sg_ctx ctx, int32_t source, const sg_plan* plans, int32_t n, int32_t reps,
                                 sg_mlp model, sg_tunedb db, float margin);
/* The plan a program runs with (the context's settings where it has none) and how it was
 * chosen (an sg_plan_source value). */
sg_status sg_program_plan(sg_program p, sg_plan* plan, int32_t* source);

/* Training data of the cost model, prepared on the device: fits the model's standardization
 * (per feature: float64 mean and population standard deviation, scale = 1 where it is below
 * 1e-6, minimum and maximum) on the raw features X (n x 24, device), writes the standardized
 * features Xn = (X - mean) / scale (float32 operations; device, n x 24) and, when ms_dev (n
 * device doubles, measured milliseconds) is given, the targets T = RN32(log(1000 ms)) (device,
 * n floats).  SG_E_INVALID for n < 1 or buffers outside device allocations. */
sg_status sg_mlp_fit_data(sg_mlp m, const float* X_dev, const double* ms_dev, int64_t n, float* Xn_dev, float* T_dev);
/* Xn = (X - mean) / scale with the model's standardization (SG_E_STATE if none is set) and,
 * when ms_dev is given, the targets T as in sg_mlp_fit_data (held-out samples). */
sg_status sg_mlp_standardize(sg_mlp m, const float* X_dev, const double* ms_dev, int64_t n, float* Xn_dev, float* T_dev);
/* Save the cost model (parameters, Adam moments and step, standardization) to a file, and
 * create a model on `ctx` from one; training resumes where it stopped.  SG_E_STATE when the
 * model has no standardization yet; SG_E_INVALID for an unreadable or foreign file. */
sg_status sg_mlp_save(sg_mlp m, const char* path);
sg_status sg_mlp_load(sg_ctx ctx, const char* path, sg_mlp* out);

/* ---- the autotuner's timing database ------------------------------------------------------ */

/* Key of a program on its context's device: a 64-bit hash of its operations, constants,
 * element types, lengths (not the data), clauses, split points and the context's mode, with
 * the device's architecture and compute-unit count.  Equal programs on equal devices get
 * equal keys in every process. */
sg_status sg_program_key(sg_program p, uint64_t* key);
/* Open (creating if absent) an append-only text file of autotuner timings, one record per
 * line: "sgtune1 <key hex> <block> <unroll> <substeps> <split> <ms>"; the last record of a
 * (key, plan) pair wins.  SG_E_INVALID for a malformed record (its line is named) or a file
 * that cannot be appended to. */
sg_status sg_tunedb_open(sg_ctx ctx, const char* path, sg_tunedb* out);
sg_status sg_tunedb_close(sg_tunedb db);
/* Records read and appended so far, and distinct (key, plan) pairs. */
sg_status sg_tunedb_records(sg_tunedb db, int64_t* records, int64_t* distinct);
/* *ms = the recorded time of (key, plan), or -1 when there is none. */
sg_status sg_tunedb_lookup(sg_tunedb db, uint64_t key, const sg_plan* plan, double* ms);
/* Append one record (flushed before the call returns). */
sg_status sg_tunedb_record(sg_tunedb db, uint64_t key, const sg_plan* plan, double ms);
/* sg_autotune through the database: plans with a recorded time for this program's key are
 * not timed again; the others are timed (as sg_program_time_plans) and appended.  Sets the
 * fastest plan on the program; *best its index, ms_out (n, optional) every plan's time,
 * *measured (optional) how many plans were timed now. */
sg_status sg_autotune_db(sg_program p, sg_tunedb db, const sg_plan* plans, int32_t n, int32_t reps, int32_t* best,
                         double* ms_out, int32_t* measured);

/* ---- a call that allocates nothing ------------------------------------------------------ */

/* Bytes of static device work memory behind sg_product_check_noalloc (one copy per device,
 * held until the process ends). */
#define SG_NOALLOC_SCRATCH_BYTES (8u << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops
 * that must not call hipMalloc): the product check of sg_program_product as one call on
 * device pointers.  C (M x N), A (M x K), B (K x N) and R (nvec x N, 1 <= nvec <= 4) are
 * row-major float32 matrices in device memory, read only; the check and its tolerance are
 * those of sg_program_product.  The call enqueues its kernels on `hip_stream` (a hipStream_t of
 * the current device, NULL = the null stream) and returns without waiting; when the stream
 * reaches them, *verdict_dev (device memory the caller owns, 32 bytes) holds the verdict as
 * sg_program_execute would report it (contract_id 0, SG_ENSURE, SG_CHECK_PRODUCT).
 * Nothing is allocated: the work memory is the static array above, so the call fails with
 * SG_E_INVALID when 256 + the check's work (8 (N' + K' + M) + 8 S max(K, M) doubles, N' and K'
 * rounded up to multiples of 512, S the column slices of a pass) exceeds
 * SG_NOALLOC_SCRATCH_BYTES (every square size up to 32766 fits), and
 * calls on one device share that memory: calls that overlap on one device (several streams or
 * threads) race and must be ordered by the caller.  No device memory is touched before the
 * arguments are checked.  Errors: SG_E_INVALID (negative size, NULL pointer, too large),
 * SG_E_UNSUPPORTED (nvec outside 1..4), SG_E_DEVICE (HIP error); no context, so the message is
 * read with sg_last_error(NULL). */
sg_status sg_product_check_noalloc(const float* C_dev, const float* A_dev, const float* B_dev, const float* R_dev,
                                   int64_t M, int64_t N, int64_t K, int32_t nvec, void* hip_stream,
                                   sg_verdict* verdict_dev);

/* ---- host-side checks of device arithmetic (no GPU needed) ------------------------------ */

/* Evaluate the device code's correctly rounded binary32 exp on the host for n values;
 * *slow receives how many took the double-double path.  For tests. */
sg_status sg_host_exp_rn(const float* t, float* out, int64_t n, int64_t* slow);
/* Compile an expression agent (sg_fn_expr) into the register program a map gives it -- x and
 * the result in register 0, registers 1 .. registers-1 free -- and run that program on the
 * host in binary32 for n values; *nops = the program's length.  SG_E_UNSUPPORTED when the
 * expression needs more registers.  For tests of the expression compiler. */
sg_status sg_host_expr_run(const char* text, int32_t registers, const float* x, float* out, int64_t n, int32_t* nops);

#ifdef __cplusplus
}
#endif

#endif /* SAFEGPU_H */
