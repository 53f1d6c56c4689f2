#pragma once
// Fused streaming pass: element functions, zips, filters with stream compaction,
// reductions and range contracts over one index space, in a single kernel.
//
// This is the merged kernel of the execution plan (Section 5, Figures 2 and 3).  The pass
// is a short register program.  The precompiled kernel interprets it (the opcode is
// uniform across the block), so one kernel serves every chain and many different chains
// can share one launch (batched mode); a specialized kernel, compiled at run time for one
// program, includes the same operation code with constant operands, so that the dispatch
// and every register index fold away (the paper generates and compiles one kernel per
// merged plan in the same way).
//
// Layout: a sub-tile is blockDim.x * 4U consecutive elements.  Wave w of the block owns the
// contiguous range [w*U*256, (w+1)*U*256) of the sub-tile; in chunk u, lane l holds
// elements u*256 + 4l .. u*256 + 4l + 3, loaded with one 16-byte load per input, so every
// load instruction of a wave reads 1 KiB contiguously.  Element values of one lane live in
// registers R[reg][4U]; index spaces (filters) and predicates are 4U-bit masks.
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#include "sg_exp.h"
#include "sg_kernels.h"

// The pass program: the interpreter by default; a specialized kernel supplies its own,
// with the facts below as constants (the interpreter takes them from the descriptor).
#ifndef SG_PROGRAM_INC
#define SG_PROGRAM_INC "sg_program_interp.inc"
#endif
#ifndef SG_GEN_HAS_SCAN
#define SG_GEN_HAS_SCAN 1  // the program may compact (has a scan space)
#endif
#ifndef SG_GEN_NSLOTS
#define SG_GEN_NSLOTS 1  // a specialized program's exact accumulators (kept in registers)
#endif
#ifndef SG_GEN_NSUMS
#define SG_GEN_NSUMS 1   // and its float64 sums
#endif
#ifndef SG_GEN_NIN
#define SG_GEN_NIN MAX_IN  // at most this many loaded sources
#endif
#ifndef SG_GEN_NBR_MASK
#define SG_GEN_NBR_MASK 0xF  // sources whose next element a sortedness check reads (bit per source)
#endif

namespace sg {

// ---- small helpers -------------------------------------------------------------------------

// a register-set index as a type (selects one of two copies of the sub-tile code)
template <int P>
struct SgPhase {
    static constexpr int value = P;
};

__device__ __forceinline__ float uf(uint32_t u) { return __builtin_bit_cast(float, u); }
__device__ __forceinline__ uint32_t fu(float f) { return __builtin_bit_cast(uint32_t, f); }
__device__ __forceinline__ int32_t ui(uint32_t u) { return (int32_t)u; }

// all ones when bit v of m is set, else zero
__device__ __forceinline__ uint32_t lane_mask_bit(uint32_t m, int v) {
    return (uint32_t)__builtin_amdgcn_sbfe((int)m, v, 1);  // one signed bit-field extract
}

__device__ __forceinline__ bool cmp_f(uint8_t op, float x, float c) {
    switch (op) {
        case CMP_LT: return x < c;
        case CMP_LE: return x <= c;
        case CMP_GT: return x > c;
        case CMP_GE: return x >= c;
        case CMP_EQ: return x == c;
        default: return x != c;
    }
}
__device__ __forceinline__ bool cmp_i(uint8_t op, int32_t x, int32_t c) {
    switch (op) {
        case CMP_LT: return x < c;
        case CMP_LE: return x <= c;
        case CMP_GT: return x > c;
        case CMP_GE: return x >= c;
        case CMP_EQ: return x == c;
        default: return x != c;
    }
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint64_t w = __shfl_xor(v, o);
        v = w < v ? w : v;
    }
    return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint64_t w = __shfl_xor(v, o);
        v = w > v ? w : v;
    }
    return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int32_t wave_max_i32(int32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

// Inclusive sum over the lanes of a wave (lane i gets lanes 0..i): shifts within rows of
// 16 lanes, then the row broadcasts of lane 15 and lane 31 (data-parallel primitives, no LDS).
__device__ __forceinline__ uint32_t wave_incl_add(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

// Block barrier that orders LDS only: global loads in flight (the next sub-tile's inputs)
// stay in flight across it, where __syncthreads() would first wait for every one of them.
// Used wherever the block exchanges only LDS data; global results other blocks read are
// ordered by their own atomics and waits.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int V>
__device__ __forceinline__ uint32_t all_bits() {
    return V >= 32 ? 0xFFFFFFFFu : ((1u << V) - 1u);
}

// Run BODY with `r` bound to the register chosen by a block-uniform index.  Written as a
// macro so that every case indexes the register file with constants (no private memory).
#define SG_ON_REG(idx, ...)                                  \
    switch (idx) {                                           \
        case 0: { uint32_t(&r)[V] = R[0]; __VA_ARGS__ } break; \
        case 1: { uint32_t(&r)[V] = R[1]; __VA_ARGS__ } break; \
        case 2: { uint32_t(&r)[V] = R[2]; __VA_ARGS__ } break; \
        case 3: { uint32_t(&r)[V] = R[3]; __VA_ARGS__ } break; \
        default: { uint32_t(&r)[V] = R[4]; __VA_ARGS__ } break; \
    }
// The current operation's register a (and, for MOV, its destination).  A specialized kernel
// indexes the register file with constants; the interpreter rebinds both to a copy of the
// operand, so that each operation's code exists once instead of once per register.
#define SG_ON_A(...) SG_ON_REG(op.a, __VA_ARGS__)
#define SG_ON_DST(...) SG_ON_REG(op.dst, __VA_ARGS__)

__device__ __forceinline__ uint32_t get_space(const uint32_t (&S)[MAX_SPACES], int s) {
    switch (s) {
        case 0: return S[0];
        case 1: return S[1];
        case 2: return S[2];
        case 3: return S[3];
        case 4: return S[4];
        case 5: return S[5];
        case 6: return S[6];
        default: return S[7];
    }
}
__device__ __forceinline__ void set_space(uint32_t (&S)[MAX_SPACES], int s, uint32_t v) {
    switch (s) {
        case 0: S[0] = v; break;
        case 1: S[1] = v; break;
        case 2: S[2] = v; break;
        case 3: S[3] = v; break;
        case 4: S[4] = v; break;
        case 5: S[5] = v; break;
        case 6: S[6] = v; break;
        default: S[7] = v; break;
    }
}

// Block-uniform reads of data that no kernel writes while this one runs (descriptor and
// program tables, tile map, a count written by an earlier launch): through the constant
// address space they are scalar loads, served by the scalar cache without a vector round trip.
#define SG_AS4 __attribute__((address_space(4)))
__device__ __forceinline__ uint32_t uload32(const void* p) {
    return *(const SG_AS4 uint32_t*)(const SG_AS4 char*)p;
}
__device__ __forceinline__ uint64_t uload64(const void* p) {
    const uint32_t lo = *(const SG_AS4 uint32_t*)(const SG_AS4 char*)p;
    const uint32_t hi = *((const SG_AS4 uint32_t*)(const SG_AS4 char*)p + 1);
    return ((uint64_t)hi << 32) | lo;
}
template <class T>
__device__ __forceinline__ T* uptr(const void* p) {
    return (T*)(uintptr_t)uload64(p);
}

// Input and output vectors are global memory, but their addresses come from the instance
// descriptor as integers.  Accessed through address-space-1 pointers they compile to global
// (not flat) instructions, whose completion is counted apart from LDS and scalar memory, so
// LDS traffic in a pass program never waits for the loads in flight.
typedef unsigned int sg_u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) uint32_t gu32;
typedef __attribute__((address_space(1))) sg_u32x4 gu4;
__device__ __forceinline__ const gu32* gin(uint64_t a) { return (const gu32*)(uintptr_t)a; }
__device__ __forceinline__ gu32* gout(uint64_t a) { return (gu32*)(uintptr_t)a; }

// Descriptor reads.  A single-instance launch keeps its descriptor and program in the kernel
// argument segment: they are read through the segment pointer (address space 4, scalar
// loads), never through the address of the by-value argument, which would make the
// compiler copy the whole argument block to private memory.  Batched launches read the
// descriptor and program tables in global memory, also with scalar loads.
typedef const __attribute__((address_space(4))) char* kptr;

template <bool INLINE>
__device__ __forceinline__ uint32_t d32(kptr kb, const char* gb, int off) {
    if constexpr (INLINE) return *(const __attribute__((address_space(4))) uint32_t*)(kb + off);
    else return uload32(gb + off);
}
template <bool INLINE>
__device__ __forceinline__ uint64_t d64(kptr kb, const char* gb, int off) {
    if constexpr (INLINE) {
        return *(const __attribute__((address_space(4))) uint64_t*)(kb + off);
    } else {
        return uload64(gb + off);
    }
}
template <bool INLINE>
__device__ __forceinline__ uint8_t d8_lane(kptr kb, const char* gb, int off) {  // per-lane index
    if constexpr (INLINE) return *(const __attribute__((address_space(4))) uint8_t*)(kb + off);
    else return *(const uint8_t*)(gb + off);
}

struct Lds {
    double exptab[1 << SG_EXPF_BITS];        // 2^(j/256) for the exp fast path
    uint64_t slot[MAX_WAVES][MAX_SLOTS];     // per-wave combines of the per-lane accumulators
    double sum[MAX_WAVES][MAX_SUMS];         // per-wave sums of the current tile
    double tsum[TILE_BUF][MAX_SUMS];         // sums of tiles not yet published
    int64_t tile[TILE_BUF];
    double fin[MAX_WAVES][MAX_SUMS];
    uint32_t rcnt[2][64];                    // kept values per LDS region, per staging buffer
    uint32_t roff[2][64];                    // their exclusive prefix within the tile
    uint32_t dfirst[2][MAX_DEFER][64];       // first failing compacted rank per region
    uint64_t ptotal[2];                      // kept values of the staged tile
    int64_t excl;                            // exclusive prefix of the tile being copied out
};

static_assert(sizeof(Lds) <= 10 * 1024, "static LDS bound assumed by the host's grid sizing");

__device__ __forceinline__ uint64_t tag_word(uint32_t epoch, uint32_t payload) {
    return ((uint64_t)epoch << 32) | payload;
}

// ---- the kernel ----------------------------------------------------------------------------
//
// A tile is `substeps` consecutive sub-tiles of blockDim.x * 4U elements of one instance.
// Tiles are assigned statically (block b takes tiles b, b + G, b + 2G, ... of a persistent
// grid that fits on the device at once), so nothing is handed out through a shared
// counter: same-address atomics serialize across the chip.  While a sub-tile's results are
// being combined, the loads of the block's next sub-tile are already in flight (they go
// into the value registers as soon as the program has finished with them).
//
// Accumulators are per lane, in LDS (dynamic part): exact slots (counts, int sums, min/max
// keys, first indices) are combined over the block once per instance and flushed to device
// accumulators spread over `spread` copies; float64 sums are combined once per tile in a
// fixed order (lanes, then waves).  A single-program pass keeps one running sum per block
// (its tiles in order) and publishes it once, in epoch-tagged 64-bit words indexed by block;
// a batched launch publishes per tile.  The block holding the instance's last tile waits
// until every word of the instance carries this launch's epoch (which also proves every
// contributing block has flushed), adds the sums in block (or tile) order and writes the
// result.  Sums are thus identical from run to run for a given launch configuration.
//
// Compaction: each wave packs the kept values of its part of a sub-tile into its own LDS
// region, and the block publishes the tile's count when the tile is done.  A single-program
// pass resolves the tile's exclusive prefix one tile later, while the block's next tile is
// staged in a second buffer: tiles are handed out in rounds of G (tile r*G + b to block b),
// the prefix of tile r*G + b is the base of round r plus the counts of tiles r*G .. r*G+b-1
// (all published a round ago, read in one step of 512 descriptors), and block G-1 publishes
// the next round's base when it resolves the last tile of a round.  No wait then sits on the
// path of the block's own loads; the copy-out of the staged regions is contiguous and
// coalesced.  A batched launch (many programs) resolves each tile at once by a decoupled
// look-back over the inclusive / aggregate counts of earlier tiles of its instance.  Waits
// only ever target lower-numbered tiles held by blocks that are all resident (the grid is
// sized by occupancy), so they end; every wait is bounded and reports a device error
// instead of hanging.
//
// Dynamic LDS layout (bytes): [lds_slots][blockDim] u64 | [lds_sums][blockDim] f64 |
// NBUF x [lds_cemit][substeps * waves][256U] u32 (NBUF = 2 for a single program, else 1).

constexpr int LB_WINDOW = 8;  // look-back descriptors per lane per step

// SPEC = 1 marks a kernel compiled at run time for one program (its own symbol in traces).
template <int U, bool INLINE, int LB, int SPEC = 0>
__global__ __launch_bounds__(LB, LB <= 256 ? 2 : 1) void stream_kernel(const StreamArgs A) {
    constexpr int V = 4 * U;
    constexpr int RW = 256 * U;  // elements of a wave's part of a sub-tile
    __shared__ Lds L;
    extern __shared__ uint64_t dyn[];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform over the wave, and visibly so
    const int B = blockDim.x;
    const int nwaves = B >> 6;
    const int C = A.substeps;
    const int64_t sub_elems = (int64_t)B * V;
    const uint32_t epoch = A.epoch_ptr
        ? __builtin_amdgcn_readfirstlane(__hip_atomic_load(A.epoch_ptr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        : A.epoch_val;
    // spin limit of every bounded wait: a device word (batches: settable between graph
    // replays) or the launch argument; raw 0 = the default, raw k = k - 1 spins (1: fail at once)
    const uint32_t wraw = A.limit_ptr
        ? __builtin_amdgcn_readfirstlane(__hip_atomic_load(A.limit_ptr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        : A.wait_limit;
    const uint32_t wlimit = wraw == 0 ? kDefaultWaitSpins : wraw - 1u;
    const int spread = A.spread;
    const int sp_idx = (int)(blockIdx.x % (unsigned)spread);
    const kptr kargs = (kptr)__builtin_amdgcn_kernarg_segment_ptr();
    const kptr kdesc = kargs + __builtin_offsetof(StreamArgs, inst0);
    const kptr kprog = kargs + __builtin_offsetof(StreamArgs, prog0);

    // Per-lane accumulators: a specialized kernel knows its slots and sums when it is compiled
    // and keeps them in registers (no LDS traffic in the sub-tile loop); the interpreter keeps
    // them in LDS, where a launch gives them lds_slots and lds_sums rows.
    constexpr bool RACC = SPEC == 1;
    constexpr int RNS = RACC && SG_GEN_NSLOTS > 0 ? SG_GEN_NSLOTS : 1;
    constexpr int RNU = RACC && SG_GEN_NSUMS > 0 ? SG_GEN_NSUMS : 1;
    uint64_t racc[RNS];
    double rsum[RNU];
#pragma unroll
    for (int i = 0; i < RNS; ++i) racc[i] = 0;
#pragma unroll
    for (int i = 0; i < RNU; ++i) rsum[i] = 0.0;
    uint64_t* lacc = dyn;                                        // [slot][B]
    double* lsum = (double*)(dyn + (int64_t)A.lds_slots * B);    // [sum][B]
    uint32_t* stage = (uint32_t*)(dyn + (int64_t)(A.lds_slots + A.lds_sums) * B);
    auto acc_add = [&](int k, uint64_t v) {
        if (RACC) {
#pragma unroll
            for (int i = 0; i < RNS; ++i) if (i == k) racc[i] += v;
        } else {
            lacc[k * B + tid] += v;
        }
    };
    auto acc_max = [&](int k, uint64_t v) {
        if (RACC) {
#pragma unroll
            for (int i = 0; i < RNS; ++i) if (i == k) racc[i] = v > racc[i] ? v : racc[i];
        } else {
            const uint64_t o = lacc[k * B + tid];
            lacc[k * B + tid] = v > o ? v : o;
        }
    };
    auto sum_add = [&](int k, double v) {
        if (RACC) {
#pragma unroll
            for (int i = 0; i < RNU; ++i) if (i == k) rsum[i] += v;
        } else {
            lsum[k * B + tid] += v;
        }
    };
    // read an accumulator and reset it
    auto acc_take = [&](int k) -> uint64_t {
        uint64_t v = 0;
        if (RACC) {
#pragma unroll
            for (int i = 0; i < RNS; ++i) if (i == k) { v = racc[i]; racc[i] = 0; }
        } else {
            v = lacc[k * B + tid];
            lacc[k * B + tid] = 0;
        }
        return v;
    };
    auto sum_take = [&](int k) -> double {
        double v = 0.0;
        if (RACC) {
#pragma unroll
            for (int i = 0; i < RNU; ++i) if (i == k) { v = rsum[i]; rsum[i] = 0.0; }
        } else {
            v = lsum[k * B + tid];
            lsum[k * B + tid] = 0.0;
        }
        return v;
    };

    // block-uniform state of the current instance
    int cur = -1, ntl = 0;
    const char* D = nullptr;     // batched: descriptor in global memory
    const char* prog = nullptr;  // batched: program in global memory
    int plen = 0, nin = 0, scan_space = 0, flags = 0, nsum = 0, ns = 0;
    int64_t n = 0, tile0 = 0, ntiles = 0;
    // program facts the tile end needs (block-uniform, the same for every sub-tile)
    int nce = 0, ce_reg0 = 0, ce_reg1 = 0, ce_out0 = 0, ce_out1 = 0;
    int nd = 0, d_slot0 = 0, d_slot1 = 0;

    for (int k = 0; k < A.lds_slots; ++k) lacc[k * B + tid] = 0;
    for (int k = 0; k < A.lds_sums; ++k) lsum[k * B + tid] = 0.0;
    for (int i = tid; i < (1 << SG_EXPF_BITS); i += blockDim.x) L.exptab[i] = SG_EXPF_TAB[i];
    lds_barrier();

    // Combine the block's exact accumulators of instance `cur`, publish its buffered tiles;
    // the block holding the instance's last tile finalizes.
    auto flush = [&]() {
        // single program: the block's sums, over lanes then waves in a fixed order
        if (INLINE) {
            for (int k = 0; k < nsum; ++k) {
                double s = sum_take(k);
                s = wave_sum_f64(s);
                if (lane == 0) L.sum[wave][k] = s;
            }
        }
        for (int k = 0; k < ns; ++k) {
            const uint8_t kind = d8_lane<INLINE>(kdesc, D, (int)__builtin_offsetof(InstDesc, slot_kind) + k);
            uint64_t v = acc_take(k);
            v = kind == SLOT_ADD ? (uint64_t)wave_sum_i64((int64_t)v) : wave_max_u64(v);
            if (lane == 0) L.slot[wave][k] = v;
        }
        __syncthreads();
        if (INLINE && tid < nsum) {
            double s = 0.0;
            for (int w = 0; w < nwaves; ++w) s += L.sum[w][tid];
            L.tsum[0][tid] = s;
        }
        if (tid < ns) {
            const uint8_t kind = d8_lane<INLINE>(kdesc, D, (int)__builtin_offsetof(InstDesc, slot_kind) + tid);
            uint64_t v = 0;
            for (int w = 0; w < nwaves; ++w) {
                const uint64_t x = L.slot[w][tid];
                v = kind == SLOT_ADD ? v + x : (x > v ? x : v);
            }
            uint64_t* g = A.acc + ((int64_t)cur * MAX_SLOTS + tid) * spread + sp_idx;
            if (v) {
                if (kind == SLOT_ADD) (void)__hip_atomic_fetch_add(g, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                else (void)__hip_atomic_fetch_max(g, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);  // accumulator updates complete before the tiles are published
        __syncthreads();
        // a single program publishes one running sum per block (its tiles in order), indexed
        // by block; a batched launch one word set per buffered tile
        bool has_last = false;
        if (INLINE) {
            has_last = (int64_t)blockIdx.x == (ntiles - 1) % (int64_t)gridDim.x;
        } else {
            for (int q = 0; q < ntl; ++q) has_last |= L.tile[q] == tile0 + ntiles - 1;
        }
        const int words = 1 + 2 * nsum;
        for (int idx = tid; idx < ntl * words; idx += B) {
            const int q = idx / words, w = idx % words;
            uint32_t payload = 0;
            if (w > 0) {
                const uint64_t bits = __builtin_bit_cast(uint64_t, L.tsum[q][(w - 1) >> 1]);
                payload = ((w - 1) & 1) ? (uint32_t)(bits >> 32) : (uint32_t)bits;  // low half first
            }
            const int64_t where = INLINE ? (int64_t)blockIdx.x : L.tile[q];
            __hip_atomic_store(&A.tags[where * TAG_WORDS + w], tag_word(epoch, payload), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        ntl = 0;
        if (!has_last) return;
        // ---- finalize the instance ----
        InstResult* res = A.results + cur;
        // word sets to wait for: one per block (single program; every block holds a tile) or
        // one per tile of the instance
        const int64_t nq = INLINE ? (int64_t)gridDim.x : ntiles;
        const int64_t q0 = INLINE ? 0 : tile0;
        for (uint32_t spins = 0;; ++spins) {
            if (spins >= wlimit) {  // bounded: report instead of hanging
                if (tid == 0) atomicOr(&res->err, (uint32_t)ERR_FINALIZE_TIMEOUT);
                break;
            }
            int ok = 1;
            for (int64_t q = tid; q < nq; q += B)
                for (int w = 0; w < words; ++w) {
                    const uint64_t x = __hip_atomic_load(&A.tags[(q0 + q) * TAG_WORDS + w], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                    ok &= (uint32_t)(x >> 32) == epoch;
                }
            if (__syncthreads_and(ok)) break;
            __builtin_amdgcn_s_sleep(2);
        }
        for (int k = 0; k < nsum; ++k) {
            double s = 0.0;
            for (int64_t q = tid; q < nq; q += B) {
                const uint64_t* tw = A.tags + (q0 + q) * TAG_WORDS + 1 + 2 * k;
                const uint64_t lo = __hip_atomic_load(tw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t hi = __hip_atomic_load(tw + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s += __builtin_bit_cast(double, ((hi & 0xFFFFFFFFull) << 32) | (lo & 0xFFFFFFFFull));
            }
            s = wave_sum_f64(s);
            if (lane == 0) L.fin[wave][k] = s;
        }
        __syncthreads();
        if (tid < nsum) {
            double s = 0.0;
            for (int w = 0; w < nwaves; ++w) s += L.fin[w][tid];
            res->sum[tid] = s;
        }
        const int count_slot = (int)d32<INLINE>(kdesc, D, (int)__builtin_offsetof(InstDesc, count_slot));
        if (tid < ns) {
            const uint8_t kind = d8_lane<INLINE>(kdesc, D, (int)__builtin_offsetof(InstDesc, slot_kind) + tid);
            uint64_t v = 0;
            uint64_t* g = A.acc + ((int64_t)cur * MAX_SLOTS + tid) * spread;
            for (int j = 0; j < spread; ++j) {
                const uint64_t x = __hip_atomic_load(g + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                v = kind == SLOT_ADD ? v + x : (x > v ? x : v);
                if (x) __hip_atomic_store(g + j, (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            res->slot[tid] = (int64_t)v;
            if (tid == count_slot) res->scan_count = (int64_t)v;
        }
        __syncthreads();
    };

    // ---- compaction state ----
    const int64_t stage_buf = (int64_t)A.lds_cemit * C * nwaves * RW;
    int sb = 0;          // staging buffer of the tile being computed
    int64_t pend = -1;   // single program: the tile staged in buffer sb ^ 1, awaiting its prefix
    int pnreg = 0;
    const uint64_t lb_epoch = (uint64_t)(epoch & 0x3FFFFFFFu) << 32;
    constexpr uint64_t LB_AGG = 1ull << 62, LB_INC = 2ull << 62;
    constexpr uint64_t LB_EPOCH_MASK = 0x3FFFFFFFull << 32;

    // every wave, single program: exclusive prefix of the staged tile `p` (buffer `buf`) from
    // its round's base and the counts of the round's earlier tiles (every wave reads the same
    // published values, so all get the same prefix, or -1 when none can be used); wave 0
    // publishes the next round's base when `p` closes a round
    auto resolve_round = [&](int64_t p, int buf) -> int64_t {
        const uint64_t total = L.ptotal[buf];
        const int64_t G = (int64_t)gridDim.x, local = p - tile0, r = local / G, b = local % G;
        uint64_t* rbase = A.lookback + A.total_tiles;  // base of round r at rbase[r]
        int64_t excl = 0;
        uint32_t spins = 0;
        // the round's base is loaded with the first window of counts (one round trip)
        for (int64_t j0 = 0; j0 == 0 || j0 < b; j0 += 64 * LB_WINDOW) {
            const bool want_base = j0 == 0 && r > 0;
            for (;;) {
                if (spins >= wlimit) { excl = -1; break; }
                const uint64_t bd = want_base ? ld_relaxed(&rbase[r]) : (LB_AGG | lb_epoch);
                uint64_t d[LB_WINDOW];
#pragma unroll
                for (int m = 0; m < LB_WINDOW; ++m) {
                    const int64_t k = j0 + 64 * m + lane;
                    d[m] = k < b ? ld_relaxed(&A.lookback[tile0 + r * G + k]) : (LB_AGG | lb_epoch);
                }
                bool valid = (bd & LB_EPOCH_MASK) == lb_epoch && (bd >> 62) != 0;
                int64_t part = 0;
#pragma unroll
                for (int m = 0; m < LB_WINDOW; ++m) {
                    valid &= (d[m] & LB_EPOCH_MASK) == lb_epoch && (d[m] >> 62) != 0;
                    part += (j0 + 64 * m + lane < b) ? (int64_t)(uint32_t)d[m] : 0;
                }
                if (__ballot(!valid) == 0) {
                    excl += (int64_t)(uint32_t)bd + wave_sum_i64(part);  // a base that was not loaded adds 0
                    break;
                }
                ++spins;
                __builtin_amdgcn_s_sleep(1);
            }
            if (excl < 0) break;
        }
        if (excl < 0 && lane == 0) atomicOr(&A.results[cur].err, (uint32_t)ERR_LOOKBACK_TIMEOUT);
        // the last tile of a full round opens the next one (its base is published even after
        // a timed-out wait, so that later rounds do not wait on it; the launch reports the error)
        if (b == G - 1 && (r + 1) * G < ntiles && wave == 0 && lane == 0)
            st_relaxed(&rbase[r + 1], LB_AGG | lb_epoch | (uint64_t)(uint32_t)((excl >= 0 ? (uint64_t)excl : 0) + total));
        if (excl >= 0 && (uint64_t)excl + total > (uint64_t)n) excl = -1;  // never past the capacity
        return excl;
    };

    // wave 0, batched launch: exclusive prefix of tile `pend` (buffer 0) by a decoupled
    // look-back; publishes its inclusive count and leaves the prefix (or -1) in L.excl
    auto resolve_chain = [&](int64_t pend) {
        const uint64_t total = L.ptotal[0];
        int64_t excl = 0;
        if (pend != tile0) {
            // descriptors at distance p + 1 = 1 + 64m + lane, nearest first
            int64_t j = pend - 1;
            for (uint32_t spins = 0;;) {
                if (spins >= wlimit) {
                    if (lane == 0) atomicOr(&A.results[cur].err, (uint32_t)ERR_LOOKBACK_TIMEOUT);
                    excl = -1;  // no prefix: nothing of this tile is written
                    break;
                }
                uint64_t d[LB_WINDOW];
#pragma unroll
                for (int m = 0; m < LB_WINDOW; ++m) {
                    const int64_t idx = j - 64 * m - lane;
                    d[m] = idx >= tile0 ? ld_relaxed(&A.lookback[idx]) : (LB_INC | lb_epoch);
                }
                int fi = 64 * LB_WINDOW;  // position of the nearest inclusive descriptor
                bool wait = false;
#pragma unroll
                for (int m = 0; m < LB_WINDOW; ++m) {
                    const bool valid = (d[m] & (0x3FFFFFFFull << 32)) == lb_epoch && (d[m] >> 62) != 0;
                    const uint64_t incm = __ballot(valid && (d[m] >> 62) == 2);
                    const uint64_t invm = __ballot(!valid);
                    if (fi == 64 * LB_WINDOW) {
                        const int f = incm ? __builtin_ctzll(incm) : 64;
                        const uint64_t need = f >= 63 ? ~0ull : ((2ull << f) - 1ull);
                        if (invm & need) wait = true;
                        if (incm) fi = 64 * m + f;
                    }
                }
                if (wait) {
                    ++spins;
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                int64_t part = 0;
#pragma unroll
                for (int m = 0; m < LB_WINDOW; ++m)
                    part += (64 * m + lane <= fi) ? (int64_t)(uint32_t)d[m] : 0;
                excl += wave_sum_i64(part);
                if (fi < 64 * LB_WINDOW) break;
                j -= 64 * LB_WINDOW;
            }
            // after a timed-out wait the prefix is unknown; publishing the tile's own count
            // keeps later tiles from waiting on it too (the launch reports the error)
            if (lane == 0)
                st_relaxed(&A.lookback[pend], LB_INC | lb_epoch | (uint64_t)(uint32_t)((excl >= 0 ? (uint64_t)excl : 0) + total));
        }
        if (excl >= 0 && (uint64_t)excl + total > (uint64_t)n) excl = -1;  // never past the capacity
        if (lane == 0) L.excl = excl;
    };
    // every wave: copy the regions this wave staged for the tile in `buf` out at `excl`;
    // deferred contract indices.  A wave reads only the regions it wrote, so it may stage
    // the next tile into the buffer as soon as its own copy is done.
    auto copy_out = [&](int buf, int nreg, int64_t excl) {
        const uint32_t* sbase = stage + buf * stage_buf;
        uint64_t dbest0 = 0, dbest1 = 0;
        for (int rg = wave; rg < nreg && excl >= 0; rg += nwaves) {
            const uint32_t cnt = L.rcnt[buf][rg];
            const int64_t ob = excl + L.roff[buf][rg];
            for (int ci = 0; ci < nce; ++ci) {
                gu32* q = gout(d64<INLINE>(kdesc, D, (int)__builtin_offsetof(InstDesc, out) + 8 * (ci == 0 ? ce_out0 : ce_out1)));
                const uint32_t* st = sbase + ((int64_t)ci * C * nwaves + rg) * RW;
                gu32* dst = q + ob;  // one base per region, 32-bit offsets per store
                // four reads in flight before their stores (i0 + 255 < RW: the unguarded
                // reads stay inside the region)
                for (uint32_t i0 = 0; i0 < cnt; i0 += 256) {
                    uint32_t w[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) w[k] = st[i0 + 64 * k + lane];
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (i0 + 64 * k + lane < cnt) dst[i0 + 64 * k + lane] = w[k];
                }
            }
            for (int ci = 0; ci < nd; ++ci) {
                const uint32_t f = L.dfirst[buf][ci][rg];
                if (f != 0xFFFFFFFFu) {
                    const uint64_t e = ~(uint64_t)(ob + f);
                    if (ci == 0) dbest0 = e > dbest0 ? e : dbest0;
                    else dbest1 = e > dbest1 ? e : dbest1;
                }
            }
        }
        if (lane == 0) {
            if (nd > 0 && dbest0) acc_max(d_slot0, dbest0);
            if (nd > 1 && dbest1) acc_max(d_slot1, dbest1);
        }
    };

    // Inputs of the block's next sub-tile.  The interpreter loads them into its registers R
    // once the program is done with R; a specialized kernel (few registers in use) loads them
    // before the program runs, so they are in flight for the whole sub-tile, into N: the other
    // of two register sets that alternate from sub-tile to sub-tile (a sub-tile whose inputs
    // were prefetched runs on the set that received them, so nothing is copied).
    constexpr bool EARLY = SPEC == 1;
    constexpr int NB = EARLY && SG_GEN_NIN > 1 ? (SG_GEN_NIN < MAX_IN ? SG_GEN_NIN : MAX_IN) : 1;
    uint32_t RB[EARLY ? 2 : 1][NREG][V];
    int ph = 0;  // specialized kernel: the register set of the sub-tile about to run
    // first element after each wave's part of a sub-tile (the sortedness check's neighbour
    // of the wave's last element), loaded with the part itself
    uint32_t NX[NB], nbr[NB];
    bool pf = false;  // the inputs of the sub-tile about to run are already loaded (R, or N if EARLY)
    const gu32* const safe = (const gu32*)(uintptr_t)A.tags;  // target of loads with no sub-tile to fetch

    for (int64_t t = blockIdx.x; t < A.total_tiles; t += gridDim.x) {
        const int64_t t_next = t + (int64_t)gridDim.x;
        const int inst = INLINE ? 0 : (int)uload32(A.tile_inst + t);
        if (inst != cur || ntl == TILE_BUF) {
            if (cur >= 0) flush();
            if (inst != cur) {
                cur = inst;
                pf = false;
                D = INLINE ? nullptr : (const char*)(A.insts + inst);
#define SG_D32(F) d32<INLINE>(kdesc, D, (int)__builtin_offsetof(InstDesc, F))
#define SG_D64(F) d64<INLINE>(kdesc, D, (int)__builtin_offsetof(InstDesc, F))
                prog = INLINE ? nullptr : (const char*)(A.progs + (int)SG_D32(prog_off));
                plen = (int)SG_D32(prog_len);
                const int64_t* n_dev = (const int64_t*)(uintptr_t)SG_D64(n_dev);
                n = n_dev ? (int64_t)uload64(n_dev) : (int64_t)SG_D64(n);
                tile0 = (int64_t)SG_D64(tile0);
                ntiles = (int64_t)SG_D64(ntiles);
                nin = (int)SG_D32(nin);
                scan_space = (int)SG_D32(scan_space);
                flags = (int)SG_D32(flags);
                nsum = (int)SG_D32(nsum);
                ns = (int)SG_D32(nslots);
#undef SG_D32
#undef SG_D64
            }
        }
        const int64_t local = t - tile0;
        // sub-tiles of this tile that hold elements (the first one always runs, so that an
        // empty instance still publishes and finalizes)
        int cend;
        {
            const int64_t rem = n - local * C * sub_elems;
            cend = rem <= 0 ? 1 : (int)((rem + sub_elems - 1) / sub_elems < C ? (rem + sub_elems - 1) / sub_elems : C);
        }

        auto subtile = [&](auto phase, const int c) {
            constexpr int P = decltype(phase)::value;
            uint32_t(&R)[NREG][V] = RB[P];
            uint32_t(&N)[NREG][V] = RB[EARLY ? 1 - P : 0];
            (void)N;
            const int64_t sub_base = (local * C + c) * sub_elems;
            const bool full = sub_base + sub_elems <= n;
            const bool vec = full && (flags & 1);
            const int64_t e0 = sub_base + (int64_t)wave * RW + lane * 4;

            uint32_t S[MAX_SPACES];
            uint32_t P0 = 0, P1 = 0, P2 = 0, P3 = 0;
            uint32_t D0 = 0, D1 = 0;

            auto elem = [&](int v) -> int64_t { return e0 + (v >> 2) * 256 + (v & 3); };
            auto first_of = [&](uint32_t m) -> uint64_t {
                if (!m) return ~0ull;
                return (uint64_t)elem(__builtin_ctz(m));
            };

            uint32_t inb = 0;
            if (full) {
                inb = all_bits<V>();
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) inb |= (elem(v) < n ? 1u : 0u) << v;
            }
            S[0] = inb;
#pragma unroll
            for (int s = 1; s < MAX_SPACES; ++s) S[s] = 0;
            if (EARLY) {
                // this sub-tile's inputs (a specialized kernel's instance has exactly
                // SG_GEN_NIN of them): prefetched into N by the previous sub-tile, else loaded
                // now; all of them have arrived before the next prefetch is issued
                if (pf) {
#pragma unroll
                    for (int k = 0; k < NB && k < SG_GEN_NIN; ++k) nbr[k] = NX[k];
                } else {
#pragma unroll
                    for (int k = 0; k < NB && k < SG_GEN_NIN; ++k) {
                        const gu32* q = gin(d64<INLINE>(kdesc, D, (int)__builtin_offsetof(InstDesc, in) + 8 * k));
                        if (vec) {
#pragma unroll
                            for (int u = 0; u < U; ++u) {
                                const sg_u32x4 w = *(const gu4*)(q + e0 + u * 256);
                                R[k][4 * u + 0] = w.x;
                                R[k][4 * u + 1] = w.y;
                                R[k][4 * u + 2] = w.z;
                                R[k][4 * u + 3] = w.w;
                            }
                        } else {
#pragma unroll
                            for (int v = 0; v < V; ++v) R[k][v] = (inb >> v) & 1u ? q[elem(v)] : 0u;
                        }
                        const int64_t ex = sub_base + (int64_t)(wave + 1) * RW;
                        nbr[k] = ((SG_GEN_NBR_MASK >> k) & 1) && ex < n ? q[ex] : 0u;
                    }
                }
#pragma unroll
                for (int k = 0; k < NB && k < SG_GEN_NIN; ++k) {
#pragma unroll
                    for (int v = 0; v < V; ++v) asm volatile("" ::"v"(R[k][v]));
                    asm volatile("" ::"v"(nbr[k]));
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int k = SG_GEN_NIN; k < NREG; ++k)
#pragma unroll
                    for (int v = 0; v < V; ++v) R[k][v] = 0u;
            } else {
#pragma unroll
                for (int k = 0; k < NREG; ++k) {
                    if (k < nin && k < SG_GEN_NIN) {
                        if (!pf) {
                            const gu32* q = gin(d64<INLINE>(kdesc, D, (int)__builtin_offsetof(InstDesc, in) + 8 * k));
                            if (vec) {
#pragma unroll
                                for (int u = 0; u < U; ++u) {
                                    const sg_u32x4 w = *(const gu4*)(q + e0 + u * 256);
                                    R[k][4 * u + 0] = w.x;
                                    R[k][4 * u + 1] = w.y;
                                    R[k][4 * u + 2] = w.z;
                                    R[k][4 * u + 3] = w.w;
                                }
                            } else {
#pragma unroll
                                for (int v = 0; v < V; ++v) R[k][v] = (inb >> v) & 1u ? q[elem(v)] : 0u;
                            }
                        }
                    } else {
#pragma unroll
                        for (int v = 0; v < V; ++v) R[k][v] = 0u;
                    }
                }
            }
            nce = 0;
            nd = 0;

            // the block's next sub-tile: this tile's next one, else the first of the next tile
            int64_t nb = -1;
            if (c + 1 < cend) nb = sub_base + sub_elems;
            else if (INLINE && t_next < A.total_tiles) nb = (t_next - tile0) * C * sub_elems;
            const bool nvec = nb >= 0 && nb + sub_elems <= n && (flags & 1);
            if (EARLY) {
                // issued without branches (a sub-tile with nothing to fetch loads from a
                // scratch word), so that nothing waits for these loads before the next sub-tile
                pf = nvec;
                const int64_t ne0 = nvec ? nb + (int64_t)wave * RW + lane * 4 : 0;
                const int64_t nex = nb + (int64_t)(wave + 1) * RW;
                const int ustep = nvec ? 256 : 0;
#pragma unroll
                for (int k = 0; k < NB && k < SG_GEN_NIN; ++k) {
                    const gu32* q = gin(d64<INLINE>(kdesc, D, (int)__builtin_offsetof(InstDesc, in) + 8 * k));
                    const gu32* qn = nvec ? q + ne0 : safe;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const sg_u32x4 w = *(const gu4*)(qn + u * ustep);
                        N[k][4 * u + 0] = w.x;
                        N[k][4 * u + 1] = w.y;
                        N[k][4 * u + 2] = w.z;
                        N[k][4 * u + 3] = w.w;
                    }
                    NX[k] = (SG_GEN_NBR_MASK >> k) & 1 ? *(nvec && nex < n ? q + nex : safe) : 0u;
                }
            }

#include SG_PROGRAM_INC

            // ---------------- compaction: pack kept values into this wave's LDS region ----------
            if (SG_GEN_HAS_SCAN && scan_space != 0) {
                const uint32_t keep = get_space(S, scan_space);
                // rank of value v within the region = (kept values of chunks before u)
                //   + (kept values of lanes below in chunk u) + (kept values j' < j of this lane).
                // Each lane counts its kept values per chunk (16-bit fields, two chunks per
                // word); one inclusive scan per word over the wave gives the lanes below, and
                // the last lane's sums are the chunk totals.
                constexpr int NCW = (U + 1) / 2;
                uint32_t cw[NCW], iw[NCW];
#pragma unroll
                for (int w = 0; w < NCW; ++w) {
                    const uint32_t lo = (uint32_t)__builtin_popcount((keep >> (8 * w)) & 0xFu);
                    const uint32_t hi = 2 * w + 1 < U ? (uint32_t)__builtin_popcount((keep >> (8 * w + 4)) & 0xFu) : 0u;
                    cw[w] = lo | (hi << 16);
                    iw[w] = wave_incl_add(cw[w]);
                }
                uint32_t lbase[U];
                uint32_t agg = 0;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int w = u >> 1, sh = 16 * (u & 1);
                    const uint32_t tot = ((uint32_t)__builtin_amdgcn_readlane((int)iw[w], 63) >> sh) & 0xFFFFu;
                    lbase[u] = agg + (((iw[w] - cw[w]) >> sh) & 0xFFFFu);  // fields never borrow
                    agg += tot;
                }
                auto rank_of = [&](int v) -> uint32_t {
                    const int u = v >> 2, jj = v & 3;
                    const uint32_t lowbits = (keep >> (4 * u)) & ((1u << jj) - 1u);
                    return lbase[u] + (uint32_t)__builtin_popcount(lowbits);
                };
                const int region = c * nwaves + wave;
                for (int ci = 0; ci < nce; ++ci) {
                    uint32_t* st = stage + sb * stage_buf + ((int64_t)ci * C * nwaves + region) * RW;
                    // kept values fill the region from the front in element order.  Within a
                    // chunk a lane's kept values are consecutive from lbase[u], so a pointer
                    // advanced by each element's keep bit addresses them, and a store runs
                    // only in the lanes whose element is kept (an execution mask, no branch):
                    // per element one bit extract, one compare and one add.
                    SG_ON_REG(ci == 0 ? ce_reg0 : ce_reg1, _Pragma("unroll") for (int u = 0; u < U; ++u) {
                        uint32_t* p = st + lbase[u];
                        _Pragma("unroll") for (int j = 0; j < 4; ++j) {
                            // the extracted bit is both the mask's source and the increment
                            // (through the empty asm the compiler does not test the bit apart)
                            uint32_t b = (keep >> (4 * u + j)) & 1u;
                            asm volatile("" : "+v"(b));
                            if (b) *p = r[4 * u + j];
                            if (j < 3) p += b;
                        }
                    })
                }
                for (int ci = 0; ci < nd; ++ci) {
                    const uint32_t hit = ci == 0 ? D0 : D1;
                    uint32_t f = hit ? rank_of(__builtin_ctz(hit)) : 0xFFFFFFFFu;
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) f = min(f, (uint32_t)__shfl_xor(f, o));
                    if (lane == 0) L.dfirst[sb][ci][region] = f;
                }
                if (lane == 0) L.rcnt[sb][region] = agg;
            }

            // ---------------- start the loads of the block's next sub-tile (interpreter) ----------
            if (!EARLY) {
                pf = nvec;
                if (pf) {
                    const int64_t ne0 = nb + (int64_t)wave * RW + lane * 4;
#pragma unroll
                    for (int k = 0; k < MAX_IN && k < NREG; ++k) {
                        if (k < nin && k < SG_GEN_NIN) {
                            const gu32* q = gin(d64<INLINE>(kdesc, D, (int)__builtin_offsetof(InstDesc, in) + 8 * k));
#pragma unroll
                            for (int u = 0; u < U; ++u) {
                                const sg_u32x4 w = *(const gu4*)(q + ne0 + u * 256);
                                R[k][4 * u + 0] = w.x;
                                R[k][4 * u + 1] = w.y;
                                R[k][4 * u + 2] = w.z;
                                R[k][4 * u + 3] = w.w;
                            }
                        }
                    }
                }
            }
        };
        for (int c = 0; c < cend; ++c) {
            if constexpr (EARLY) {
                if (ph) subtile(SgPhase<1>{}, c);
                else subtile(SgPhase<0>{}, c);
                if (pf) ph ^= 1;  // the next sub-tile's inputs are in the other set
            } else {
                subtile(SgPhase<0>{}, c);
            }
        }

        // ---------------- tile end: publish the tile's count; resolve and copy out a prefix ----
        if (SG_GEN_HAS_SCAN && scan_space != 0) {
            lds_barrier();
            const int nreg = cend * nwaves;  // regions written in this tile (at most 64)
            if (wave == 0) {
                const uint32_t cnt = lane < nreg ? L.rcnt[sb][lane] : 0u;
                uint32_t incl = cnt;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t y = __shfl_up(incl, o);
                    if (lane >= o) incl += y;
                }
                L.roff[sb][lane] = incl - cnt;
                const uint64_t total = (uint64_t)__shfl(incl, 63);
                if (lane == 0) {
                    L.ptotal[sb] = total;
                    st_relaxed(&A.lookback[t], (!INLINE && t == tile0 ? LB_INC : LB_AGG) | lb_epoch | total);
                }
                if (!INLINE) resolve_chain(t);
            }
            if (INLINE) {
                // the previous tile: its offsets and total were made visible by the barrier above
                if (pend >= 0) copy_out(sb ^ 1, pnreg, resolve_round(pend, sb ^ 1));
                pend = t;
                pnreg = nreg;
                sb ^= 1;
            } else {
                lds_barrier();
                copy_out(0, nreg, L.excl);
            }
        }
        // batched launch, tile end: its sums, added over the lanes and then the waves in a
        // fixed order, are buffered for publication (a single program keeps per-lane sums
        // until it flushes)
        if (!INLINE) {
            for (int k = 0; k < nsum; ++k) {
                double s = sum_take(k);
                s = wave_sum_f64(s);
                if (lane == 0) L.sum[wave][k] = s;
            }
            lds_barrier();
            if (tid < nsum) {
                double s = 0.0;
                for (int w = 0; w < nwaves; ++w) s += L.sum[w][tid];
                L.tsum[ntl][tid] = s;
            }
            if (tid == 0) L.tile[ntl] = t;
            lds_barrier();
        }
        ntl = INLINE ? 1 : ntl + 1;
    }
    // single program: the block's last staged tile (its offsets were written by wave 0 after
    // the last tile's first barrier)
    if (INLINE && SG_GEN_HAS_SCAN && pend >= 0) {
        lds_barrier();
        copy_out(sb ^ 1, pnreg, resolve_round(pend, sb ^ 1));
        lds_barrier();
    }
    if (cur >= 0) flush();
}

// zero a region of 64-bit words (accumulators, tags, look-back descriptors) without a
// memset node, so the call can sit inside a captured graph
__global__ void zero_kernel(uint64_t* p, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// set one 32-bit device word (one thread), so the call can sit in a stream a graph replays on
__global__ void set_word_kernel(uint32_t* p, uint32_t v) { *p = v; }

// advance the launch epoch of a captured graph (one thread)
__global__ void epoch_bump_kernel(uint32_t* e) {
    uint32_t v = (*e + 1u) & 0x3FFFFFFFu;
    *e = v ? v : 1u;
}

}  // namespace sg

