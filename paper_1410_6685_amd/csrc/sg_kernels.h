// Descriptors shared by the host planner and the streaming kernel.
//
// A fused pass ("instance") evaluates a small register program over one index space of n
// elements: element functions and zips (Section 3.2 project, Section 3.3 vector
// arithmetic), predicates and filters (Table 2), reductions (Section 3.3), and range
// contracts (Section 4) -- the merged kernel vertices of Figures 2 and 3.  Filters do not
// move data: they define nested index spaces as bit masks; a materialized filter output is
// written by stream compaction over one "scan space" per instance.
#pragma once
#ifndef __HIPCC_RTC__
#include <cstdint>
#else
// run-time compilation: fixed-width types without the C library headers
typedef __hip_internal::uint8_t uint8_t;
typedef __hip_internal::int32_t int32_t;
typedef __hip_internal::uint32_t uint32_t;
typedef __hip_internal::int64_t int64_t;
typedef __hip_internal::uint64_t uint64_t;
typedef unsigned long uintptr_t;
#define INT32_MAX 2147483647
#define INT32_MIN (-2147483647 - 1)
#endif

#ifndef SG_HD
#define SG_HD __host__ __device__ __forceinline__
#endif

namespace sg {

constexpr int NREG = 5;            // value registers per element
constexpr int MAX_IN = 4;          // loaded sources per instance
constexpr int MAX_OUT = 4;         // materialized outputs per instance
constexpr int MAX_SLOTS = 16;      // exact accumulators per instance
constexpr int MAX_SUMS = 4;        // float64 sums per instance (per-tile partials)
constexpr int MAX_SPACES = 8;      // index spaces; 0 = every in-bounds element
constexpr int MAX_DEFER = 2;       // contracts on the scan space (need compacted ranks)
constexpr int MAX_CEMIT = 2;       // compacted outputs per instance
constexpr int MAX_INLINE_OPS = 48; // program length of a single-instance launch
constexpr int MAX_WAVES = 16;      // 1024 threads per block
constexpr int TAG_WORDS = 1 + 2 * MAX_SUMS;  // per tile: done word, then each float64 sum as two halves
constexpr int MAX_SPREAD = 64;
constexpr int TILE_BUF = 32;       // tiles a block holds before publishing them

enum OpCode : uint8_t {
    OP_NOP = 0,
    MOV,  // register dst = register a
    // value ops work in place: register a = f(a), or a = a (op) b
    F_AFFINE, F_ADDC, F_MULC, F_SQUARE, F_NEG, F_ABS, F_SQRT, F_SQRT_ABS, F_EXP, F_EXP_NEG_SQ,
    F_ADD, F_SUB, F_MUL, F_DIV,
    // a = c0; a = a / c0; a = c0 / a (expression agents)
    F_CONST, F_DIVC, F_RDIVC,
    // i32 value ops (wrap modulo 2^32)
    I_AFFINE, I_ADDC, I_MULC, I_SQUARE, I_NEG, I_ABS, I_ADD, I_SUB, I_MUL, I_TO_F,
    // predicates push one bit per element onto a 4-deep stack
    P_TRUE, P_CMP_F, P_CMP_I, P_FINITE, P_RANGE_F, P_RANGE_I,
    // quotient check of a division: registers a = RN(n / d), b = n, dst = d
    P_QUOT,
    P_AND, P_OR, P_NOT,
    // FILTER pops: space[sp] = space[sp2] & top
    FILTER,
    // CHK_ALL / CHK_ANY pop: first element of space sp where top is false / true -> slot aux
    CHK_ALL, CHK_ANY,
    // first i with !(x[i] <= x[i+1]) over register a (loaded from input b) -> slot aux
    CHK_SORTED_F, CHK_SORTED_I,
    // reductions over space sp of register a
    RED_SUM_F,     // float64 sum -> sum index aux
    RED_ABSSUM_F,  // float64 sum of |x| -> sum index aux
    RED_SUM_I,     // int64 sum -> slot aux
    RED_MAX_F, RED_MIN_F, RED_MAX_I, RED_MIN_I,  // -> slot aux
    RED_COUNT,     // number of elements of space sp -> slot aux
    EMIT,          // write register a to output aux (space 0: dense; scan space: compacted)
    // a predicate and the CHK_ALL / CHK_ANY that pops it, as one operation (formed by the
    // run-time compiler for checks outside the compacted space): predicate opcode in pad,
    // its comparison in sp2, register a, constants c0 / c1; dst 0 = for_all, 1 = exists;
    // space sp, slot aux.  Same result as the pair.
    CHK_PRED,
    OP_COUNT_
};

enum CmpOp : uint8_t { CMP_LT = 0, CMP_LE, CMP_GT, CMP_GE, CMP_EQ, CMP_NE };

struct SgOp {
    uint8_t code, dst, a, b, sp, sp2, aux, pad;
    union { float f; int32_t i; } c0, c1;
};
static_assert(sizeof(SgOp) == 16, "op size");

// Every accumulator starts at 0 and is combined by add or by unsigned max, so no slot needs
// a type-specific initial value:
//   first index i   -> max of ~i (0 = none)          [SLOT_MAX64]
//   max of int key k -> max of k ^ 0x80000000         [SLOT_MAX32]
//   min of int key k -> max of ~(k ^ 0x80000000)      [SLOT_MAX32]
//   counts, int sums -> add                           [SLOT_ADD]
enum SlotKind : uint8_t { SLOT_NONE = 0, SLOT_ADD, SLOT_MAX64, SLOT_MAX32 };

struct InstDesc {
    const void* in[MAX_IN];
    void* out[MAX_OUT];
    int64_t n;              // element count when n_dev is null
    const int64_t* n_dev;   // device-resident element count (compacted upstream output)
    int64_t tile0;          // first global tile
    int64_t ntiles;
    int32_t prog_off, prog_len;
    int32_t nin;
    int32_t scan_space;     // 0: no compaction
    int32_t nsum;
    int32_t nslots;
    int32_t count_slot;     // slot holding the scan-space count (-1 if none)
    int32_t flags;          // bit 0: every input/output 16-byte aligned
    uint8_t slot_kind[MAX_SLOTS];
};

// Finalized per-instance results (device), read back once per execution.  slot[] holds the
// encoded accumulators (see SlotKind), sum[] the float64 sums.
struct InstResult {
    int64_t slot[MAX_SLOTS];
    double sum[MAX_SUMS];
    int64_t scan_count;
    uint32_t err;
    uint32_t pad0;
    int64_t pad[10];
};
static_assert(sizeof(InstResult) == 256, "result size");

enum ErrBits : uint32_t { ERR_LOOKBACK_TIMEOUT = 1u, ERR_FINALIZE_TIMEOUT = 2u };

// Spins of a bounded wait before it gives up and reports a device error (each spin sleeps
// about a microsecond).
constexpr uint32_t kDefaultWaitSpins = 1u << 22;

struct StreamArgs {
    const InstDesc* insts;      // batched launches: instance table (device)
    const SgOp* progs;          // batched launches: programs (device)
    const int32_t* tile_inst;   // batched launches: instance of every tile
    int64_t total_tiles;
    uint64_t* acc;              // ninst x MAX_SLOTS x spread accumulators (zero between launches)
    uint64_t* tags;             // total_tiles x TAG_WORDS epoch-tagged per-tile words
    uint64_t* lookback;         // total_tiles compaction descriptors (flag 2 | epoch 30 | count 32)
    InstResult* results;        // ninst
    const uint32_t* epoch_ptr;  // graph replays: device word advanced before every launch
    uint32_t epoch_val;         // direct launches: this launch's epoch
    int32_t ninst;
    int32_t substeps;           // sub-steps of blockDim.x * 4U elements per tile
    int32_t spread;             // accumulator copies per slot (spreads same-address atomics)
    int32_t lds_slots;          // per-lane exact accumulators kept in LDS (max over instances)
    int32_t lds_sums;           // per-lane float64 sums kept in LDS (max over instances)
    int32_t lds_cemit;          // compacted outputs staged in LDS (max over instances)
    uint32_t wait_limit;        // spin limit of bounded waits: 0 default, k > 0: k - 1 spins
    const uint32_t* limit_ptr;  // batched launches: the same limit in a device word (or null)
    InstDesc inst0;             // single-instance launches: the instance
    SgOp prog0[MAX_INLINE_OPS]; // single-instance launches: its program
};

}  // namespace sg
