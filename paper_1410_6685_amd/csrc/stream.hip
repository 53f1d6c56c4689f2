// Fused streaming pass: element functions, zips, filters with stream compaction,
// reductions and range contracts over one index space, in a single kernel.
//
// This is the merged kernel of the execution plan (Section 5, Figures 2 and 3): where the
// paper instantiates one CUDA template per merged plan, this kernel interprets a short
// register program whose opcode is uniform across the block, so one precompiled kernel
// serves every chain, and many different chains can share one launch (batched mode).
//
// Layout: a tile is blockDim.x * 4U consecutive elements.  Wave w of the block owns the
// contiguous range [w*U*256, (w+1)*U*256) of the tile; in chunk u, lane l holds elements
// u*256 + 4l .. u*256 + 4l + 3, loaded with one 16-byte load per input, so every load
// instruction of a wave reads 1 KiB contiguously.  Element values of one lane live in
// registers R[reg][4U]; index spaces (filters) and predicates are 4U-bit masks.
//
// Exact accumulators (counts, int sums, min/max keys, first indices) are combined with
// device atomics once per block and instance; float64 sums are published per tile and added
// in tile order by the block that holds the instance's last tile, so sums are identical
// from run to run (for a given launch configuration).
#include <hip/hip_runtime.h>

#include "sg_exp.h"
#include "sg_kernels.h"

namespace sg {

// ---- small helpers -------------------------------------------------------------------------

__device__ __forceinline__ float uf(uint32_t u) { return __builtin_bit_cast(float, u); }
__device__ __forceinline__ uint32_t fu(float f) { return __builtin_bit_cast(uint32_t, f); }
__device__ __forceinline__ int32_t ui(uint32_t u) { return (int32_t)u; }

// order-preserving int32 key of a binary32 value (-0 < +0); NaN handled by the caller
__device__ __forceinline__ int32_t fkey(uint32_t b) {
    int32_t s = (int32_t)b;
    return s >= 0 ? s : (s ^ 0x7FFFFFFF);
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

// block-uniform loads from a descriptor in kernarg or global memory
__device__ __forceinline__ uint32_t uload32(const void* p) {
    return __builtin_amdgcn_readfirstlane(*(const uint32_t*)p);
}
__device__ __forceinline__ uint64_t uload64(const void* p) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(((const uint32_t*)p)[0]);
    const uint32_t hi = __builtin_amdgcn_readfirstlane(((const uint32_t*)p)[1]);
    return ((uint64_t)hi << 32) | lo;
}
template <class T>
__device__ __forceinline__ T* uptr(const void* p) {
    return (T*)(uintptr_t)uload64(p);
}

// Descriptor reads.  A single-instance launch keeps its descriptor and program in the kernel
// argument segment: they are read through the segment pointer (address space 4, scalar
// loads), never through the address of the by-value argument, which would make the
// compiler copy the whole argument block to private memory.  Batched launches read the
// descriptor table in global memory with block-uniform loads.
typedef const __attribute__((address_space(4))) char* kptr;

template <bool INLINE>
__device__ __forceinline__ uint32_t d32(kptr kb, const char* gb, int off) {
    if constexpr (INLINE) return *(const __attribute__((address_space(4))) uint32_t*)(kb + off);
    else return __builtin_amdgcn_readfirstlane(*(const uint32_t*)(gb + off));
}
template <bool INLINE>
__device__ __forceinline__ uint64_t d64(kptr kb, const char* gb, int off) {
    if constexpr (INLINE) {
        return *(const __attribute__((address_space(4))) uint64_t*)(kb + off);
    } else {
        const uint32_t lo = __builtin_amdgcn_readfirstlane(*(const uint32_t*)(gb + off));
        const uint32_t hi = __builtin_amdgcn_readfirstlane(*(const uint32_t*)(gb + off + 4));
        return ((uint64_t)hi << 32) | lo;
    }
}
template <bool INLINE>
__device__ __forceinline__ uint8_t d8_lane(kptr kb, const char* gb, int off) {  // per-lane index
    if constexpr (INLINE) return *(const __attribute__((address_space(4))) uint8_t*)(kb + off);
    else return *(const uint8_t*)(gb + off);
}

struct Lds {
    uint64_t slot[MAX_WAVES][MAX_SLOTS];   // per-wave accumulators of the current instance
    double sum[MAX_WAVES][MAX_SUMS];       // per-wave sums of the current tile
    double tsum[TILE_BUF][MAX_SUMS];       // sums of tiles not yet published
    int64_t tile[TILE_BUF];
    double fin[MAX_WAVES][MAX_SUMS];
    int32_t flag;
};

__device__ __forceinline__ uint64_t tag_word(uint32_t epoch, uint32_t payload) {
    return ((uint64_t)epoch << 32) | payload;
}

// ---- the kernel ----------------------------------------------------------------------------
//
// A tile is `substeps` sub-tiles of blockDim.x * 4U elements of one instance; tiles are
// assigned statically (block b takes tiles b, b + G, b + 2G, ... of a persistent grid that
// fits on the device at once) and a tile's sub-tiles are interleaved across the grid, so the
// waves running at the same time hold neighbouring elements.  Nothing is handed out through
// a shared counter: same-address atomics serialize across the chip.
//
// Per block and instance, exact accumulators live in LDS (one row per wave, no barriers) and
// are flushed to device accumulators once per instance, spread over `spread` copies.  Each
// tile's float64 sums, added over its waves in a fixed order, are then published in
// epoch-tagged 64-bit words; the block holding an instance's last tile waits until every
// tile word of the instance carries this launch's epoch (which also proves every
// contributing block has flushed), adds the sums in tile order and writes the result.
//
// Compaction uses a decoupled look-back per wave: each wave's chunk publishes its count,
// then walks back over earlier chunks' published counts (64 at a time) to its exclusive
// prefix, so the scan needs no block barrier.  Waits only ever target lower-numbered
// tiles, which blocks process in increasing order, so they end as long as the grid is
// resident; every wait is bounded and reports a device error instead of hanging.

template <int U, bool INLINE>
__global__ __launch_bounds__(1024) void stream_kernel(const StreamArgs A) {
    constexpr int V = 4 * U;
    __shared__ Lds L;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int nwaves = blockDim.x >> 6;
    const int C = A.substeps;
    const int64_t sub_elems = (int64_t)blockDim.x * V;
    const uint32_t epoch = A.epoch_ptr
        ? __builtin_amdgcn_readfirstlane(__hip_atomic_load(A.epoch_ptr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        : A.epoch_val;
    const int spread = A.spread;
    const int sp_idx = (int)(blockIdx.x % (unsigned)spread);
    const kptr kargs = (kptr)__builtin_amdgcn_kernarg_segment_ptr();
    const kptr kdesc = kargs + offsetof(StreamArgs, inst0);
    const kptr kprog = kargs + offsetof(StreamArgs, prog0);

    auto slot_add = [&](int k, uint64_t v) { L.slot[wave][k] += v; };
    auto slot_max = [&](int k, uint64_t v) { L.slot[wave][k] = v > L.slot[wave][k] ? v : L.slot[wave][k]; };

    // block-uniform state of the current instance
    int cur = -1, ntl = 0;
    const char* D = nullptr;     // batched: descriptor in global memory
    const char* prog = nullptr;  // batched: program in global memory
    int plen = 0, nin = 0, scan_space = 0, flags = 0, nsum = 0, ns = 0;
    int64_t n = 0, tile0 = 0, ntiles = 0;

    if (lane < MAX_SLOTS) L.slot[wave][lane] = 0;
    if (lane < MAX_SUMS) L.sum[wave][lane] = 0.0;

    // Publish the buffered tiles of instance `cur`; the block holding its last tile finalizes.
    auto flush = [&]() {
        __syncthreads();
        if (tid < ns) {
            const uint8_t kind = d8_lane<INLINE>(kdesc, D, (int)offsetof(InstDesc, slot_kind) + tid);
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
        bool has_last = false;
        for (int q = 0; q < ntl; ++q) has_last |= L.tile[q] == tile0 + ntiles - 1;
        const int words = 1 + 2 * nsum;
        for (int idx = tid; idx < ntl * words; idx += blockDim.x) {
            const int q = idx / words, w = idx % words;
            uint32_t payload = 0;
            if (w > 0) {
                const uint64_t bits = __builtin_bit_cast(uint64_t, L.tsum[q][(w - 1) >> 1]);
                payload = ((w - 1) & 1) ? (uint32_t)(bits >> 32) : (uint32_t)bits;  // low half first
            }
            __hip_atomic_store(&A.tags[L.tile[q] * TAG_WORDS + w], tag_word(epoch, payload), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        if (lane < MAX_SLOTS) L.slot[wave][lane] = 0;
        ntl = 0;
        if (!has_last) return;
        // ---- finalize the instance ----
        InstResult* res = A.results + cur;
        const int ok_words = words;
        for (uint32_t spins = 0;; ++spins) {
            int ok = 1;
            for (int64_t q = tid; q < ntiles; q += blockDim.x)
                for (int w = 0; w < ok_words; ++w) {
                    const uint64_t x = __hip_atomic_load(&A.tags[(tile0 + q) * TAG_WORDS + w], __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                    ok &= (uint32_t)(x >> 32) == epoch;
                }
            if (__syncthreads_and(ok)) break;
            if (spins > (1u << 22)) {
                if (tid == 0) atomicOr(&res->err, (uint32_t)ERR_FINALIZE_TIMEOUT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        for (int k = 0; k < nsum; ++k) {
            double s = 0.0;
            for (int64_t q = tid; q < ntiles; q += blockDim.x) {
                const uint64_t* tw = A.tags + (tile0 + q) * TAG_WORDS + 1 + 2 * k;
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
        const int count_slot = (int)d32<INLINE>(kdesc, D, (int)offsetof(InstDesc, count_slot));
        if (tid < ns) {
            const uint8_t kind = d8_lane<INLINE>(kdesc, D, (int)offsetof(InstDesc, slot_kind) + tid);
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

    for (int64_t t = blockIdx.x; t < A.total_tiles; t += gridDim.x) {
        const int inst = INLINE ? 0 : (int)uload32(A.tile_inst + t);
        if (inst != cur || ntl == TILE_BUF) {
            if (cur >= 0) flush();
            if (inst != cur) {
                cur = inst;
                D = INLINE ? nullptr : (const char*)(A.insts + inst);
#define SG_D32(F) d32<INLINE>(kdesc, D, (int)offsetof(InstDesc, F))
#define SG_D64(F) d64<INLINE>(kdesc, D, (int)offsetof(InstDesc, F))
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
        const int64_t lround = local / A.interleave, lcol = local % A.interleave;

        for (int c = 0; c < C; ++c) {
            // sub-tiles are interleaved across the grid so that the waves running at the
            // same time are neighbours in scan order
            const int64_t sub = (lround * C + c) * A.interleave + lcol;
            const int64_t sub_base = sub * sub_elems;
            if (sub_base >= n && !(local == 0 && c == 0)) break;
            const bool full = sub_base + sub_elems <= n;
            const bool vec = full && (flags & 1);
            const int64_t e0 = sub_base + (int64_t)wave * (U * 256) + lane * 4;

            uint32_t R[NREG][V];
            uint32_t S[MAX_SPACES];
            uint32_t P0 = 0, P1 = 0, P2 = 0, P3 = 0;
            int nce = 0, ce_reg0 = 0, ce_reg1 = 0, ce_out0 = 0, ce_out1 = 0;
            uint32_t D0 = 0, D1 = 0;
            int nd = 0, d_slot0 = 0, d_slot1 = 0;

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
#pragma unroll
            for (int k = 0; k < NREG; ++k) {
                if (k < nin && k < MAX_IN) {
                    const uint32_t* q = (const uint32_t*)(uintptr_t)d64<INLINE>(kdesc, D, (int)offsetof(InstDesc, in) + 8 * k);
                    if (vec) {
#pragma unroll
                        for (int u = 0; u < U; ++u) {
                            const uint4 w = *(const uint4*)(q + e0 + u * 256);
                            R[k][4 * u + 0] = w.x;
                            R[k][4 * u + 1] = w.y;
                            R[k][4 * u + 2] = w.z;
                            R[k][4 * u + 3] = w.w;
                        }
                    } else {
#pragma unroll
                        for (int v = 0; v < V; ++v) R[k][v] = (inb >> v) & 1u ? q[elem(v)] : 0u;
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) R[k][v] = 0u;
                }
            }

            for (int pc = 0; pc < plen; ++pc) {
                SgOp op;
                {
                    uint32_t* ow = (uint32_t*)&op;
#pragma unroll
                    for (int i = 0; i < 4; ++i) ow[i] = d32<INLINE>(kprog, prog, pc * (int)sizeof(SgOp) + 4 * i);
                }
                const uint8_t code = op.code;
                switch (code) {
                    case MOV: {
                        uint32_t y[V];
                        SG_ON_REG(op.a, _Pragma("unroll") for (int v = 0; v < V; ++v) y[v] = r[v];)
                        SG_ON_REG(op.dst, _Pragma("unroll") for (int v = 0; v < V; ++v) r[v] = y[v];)
                    } break;
    // in-place unary op on register op.a: r[v] = EXPR(a) with a the element's value
    #define SG_UNARY_F(CODE, EXPR) \
                    case CODE: { const float c0 = op.c0.f, c1 = op.c1.f; (void)c0; (void)c1; \
                        SG_ON_REG(op.a, _Pragma("unroll") for (int v = 0; v < V; ++v) { \
                            const float a = uf(r[v]); r[v] = fu(EXPR); }) } break;
    #define SG_UNARY_I(CODE, EXPR) \
                    case CODE: { const uint32_t c0 = (uint32_t)op.c0.i, c1 = (uint32_t)op.c1.i; (void)c0; (void)c1; \
                        SG_ON_REG(op.a, _Pragma("unroll") for (int v = 0; v < V; ++v) { \
                            const uint32_t a = r[v]; r[v] = (EXPR); }) } break;
    #define SG_BINARY(CODE, EXPR) \
                    case CODE: { uint32_t y[V]; \
                        SG_ON_REG(op.b, _Pragma("unroll") for (int v = 0; v < V; ++v) y[v] = r[v];) \
                        SG_ON_REG(op.a, _Pragma("unroll") for (int v = 0; v < V; ++v) { \
                            const uint32_t a = r[v], b = y[v]; r[v] = (EXPR); }) } break;
                    SG_UNARY_F(F_AFFINE, (a * c0) + c1)
                    SG_UNARY_F(F_ADDC, a + c0)
                    SG_UNARY_F(F_MULC, a * c0)
                    SG_UNARY_F(F_SQUARE, a * a)
                    SG_UNARY_F(F_NEG, -a)
                    SG_UNARY_F(F_ABS, __builtin_fabsf(a))
                    SG_UNARY_F(F_SQRT, __builtin_sqrtf(a))
                    SG_UNARY_F(F_SQRT_ABS, __builtin_sqrtf(__builtin_fabsf(a)))
                    case F_EXP: case F_EXP_NEG_SQ: {
                        // fast path for every element; the rare hard cases afterwards, one
                        // element per lane at a time
                        const bool nsq = code == F_EXP_NEG_SQ;
                        SG_ON_REG(op.a,
                            uint32_t hard = 0;
                            _Pragma("unroll") for (int v = 0; v < V; ++v) {
                                const float a = uf(r[v]);
                                bool h;
                                const float f = sgx::exp_rn_fast(nsq ? -(a * a) : a, h);
                                if (h) hard |= 1u << v; else r[v] = fu(f);
                                // one element's float64 temporaries live at a time
                                __builtin_amdgcn_sched_barrier(0);
                            }
                            while (hard) {
                                const int hv = __builtin_ctz(hard);
                                hard &= hard - 1u;
                                _Pragma("unroll") for (int v = 0; v < V; ++v) {
                                    if (v == hv) {
                                        const float a = uf(r[v]);
                                        r[v] = fu(sgx::exp_rn_slow(nsq ? -(a * a) : a));
                                    }
                                }
                            }
                        )
                    } break;
                    SG_UNARY_F(I_TO_F, (float)ui(r[v]))
                    SG_UNARY_I(I_AFFINE, a * c0 + c1)
                    SG_UNARY_I(I_ADDC, a + c0)
                    SG_UNARY_I(I_MULC, a * c0)
                    SG_UNARY_I(I_SQUARE, a * a)
                    SG_UNARY_I(I_NEG, 0u - a)
                    SG_UNARY_I(I_ABS, ui(a) < 0 ? 0u - a : a)
                    SG_BINARY(F_ADD, fu(uf(a) + uf(b)))
                    SG_BINARY(F_SUB, fu(uf(a) - uf(b)))
                    SG_BINARY(F_MUL, fu(uf(a) * uf(b)))
                    SG_BINARY(I_ADD, a + b)
                    SG_BINARY(I_SUB, a - b)
                    SG_BINARY(I_MUL, a * b)
    #undef SG_UNARY_F
    #undef SG_UNARY_I
    #undef SG_BINARY
                    // ---------------- predicates ----------------
    // push one bit per element: bit v = PRED(a) with a the element's bits
    #define SG_PRED(CODE, PRED) \
                    case CODE: { uint32_t bits = 0; \
                        SG_ON_REG(op.a, _Pragma("unroll") for (int v = 0; v < V; ++v) { \
                            const uint32_t a = r[v]; bits |= ((PRED) ? 1u : 0u) << v; }) \
                        P3 = P2; P2 = P1; P1 = P0; P0 = bits; } break;
                    case P_TRUE: { P3 = P2; P2 = P1; P1 = P0; P0 = all_bits<V>(); } break;
                    case P_CMP_F: {
                        const float c = op.c0.f;
                        uint32_t bits = 0;
                        switch (op.aux) {
    #define SG_CMPF(C, E) case C: SG_ON_REG(op.a, _Pragma("unroll") for (int v = 0; v < V; ++v) { \
                            const float a = uf(r[v]); bits |= ((E) ? 1u : 0u) << v; }) break;
                            SG_CMPF(CMP_LT, a < c)
                            SG_CMPF(CMP_LE, a <= c)
                            SG_CMPF(CMP_GT, a > c)
                            SG_CMPF(CMP_GE, a >= c)
                            SG_CMPF(CMP_EQ, a == c)
                            default: SG_ON_REG(op.a, _Pragma("unroll") for (int v = 0; v < V; ++v) {
                                const float a = uf(r[v]); bits |= ((a != c) ? 1u : 0u) << v; }) break;
    #undef SG_CMPF
                        }
                        P3 = P2; P2 = P1; P1 = P0; P0 = bits;
                    } break;
                    case P_CMP_I: {
                        const int32_t c = op.c0.i;
                        uint32_t bits = 0;
                        switch (op.aux) {
    #define SG_CMPI(C, E) case C: SG_ON_REG(op.a, _Pragma("unroll") for (int v = 0; v < V; ++v) { \
                            const int32_t a = ui(r[v]); bits |= ((E) ? 1u : 0u) << v; }) break;
                            SG_CMPI(CMP_LT, a < c)
                            SG_CMPI(CMP_LE, a <= c)
                            SG_CMPI(CMP_GT, a > c)
                            SG_CMPI(CMP_GE, a >= c)
                            SG_CMPI(CMP_EQ, a == c)
                            default: SG_ON_REG(op.a, _Pragma("unroll") for (int v = 0; v < V; ++v) {
                                const int32_t a = ui(r[v]); bits |= ((a != c) ? 1u : 0u) << v; }) break;
    #undef SG_CMPI
                        }
                        P3 = P2; P2 = P1; P1 = P0; P0 = bits;
                    } break;
                    SG_PRED(P_FINITE, (a & 0x7F800000u) != 0x7F800000u)
                    SG_PRED(P_RANGE_F, uf(a) >= op.c0.f && uf(a) <= op.c1.f)
                    SG_PRED(P_RANGE_I, ui(a) >= op.c0.i && ui(a) <= op.c1.i)
    #undef SG_PRED
                    case P_AND: { const uint32_t b = P0 & P1; P0 = b; P1 = P2; P2 = P3; } break;
                    case P_OR: { const uint32_t b = P0 | P1; P0 = b; P1 = P2; P2 = P3; } break;
                    case P_NOT: P0 = ~P0 & all_bits<V>(); break;
                    case FILTER: {
                        const uint32_t m = get_space(S, op.sp2) & P0;
                        set_space(S, op.sp, m);
                        P0 = P1; P1 = P2; P2 = P3;
                    } break;
                    // ---------------- contracts ----------------
                    case CHK_ALL: case CHK_ANY: {
                        const uint32_t m = get_space(S, op.sp);
                        const uint32_t hit = code == CHK_ALL ? (m & ~P0) : (m & P0);
                        P0 = P1; P1 = P2; P2 = P3;
                        if (op.sp != 0 && op.sp == scan_space) {
                            // index in the compacted space: resolved after the scan
                            if (nd == 0) { D0 = hit; d_slot0 = op.aux; }
                            else { D1 = hit; d_slot1 = op.aux; }
                            ++nd;
                        } else {
                            const uint64_t f = wave_max_u64(~first_of(hit));
                            if (lane == 0) slot_max(op.aux, f);
                        }
                    } break;
                    case CHK_SORTED_F: case CHK_SORTED_I: {
                        uint32_t bad = 0;
                        const uint32_t* q = (const uint32_t*)(uintptr_t)d64<INLINE>(kdesc, D, (int)offsetof(InstDesc, in) + 8 * op.b);
                        SG_ON_REG(op.a, 
    _Pragma("unroll")                         for (int u = 0; u < U; ++u) {
                                // all lanes take part in both shuffles; lane 63 then picks its neighbour
                                uint32_t nxt = __shfl_down(r[4 * u], 1);
                                const uint32_t nchunk = (u + 1 < U) ? __shfl(r[4 * ((u + 1) % U)], 0) : 0u;
                                if (lane == 63) {
                                    if (u + 1 < U) {
                                        nxt = nchunk;
                                    } else {
                                        const int64_t e = e0 + u * 256 + 4;
                                        nxt = e < n ? q[e] : 0u;
                                    }
                                }
    _Pragma("unroll")                             for (int j = 0; j < 4; ++j) {
                                    const int v = 4 * u + j;
                                    const uint32_t a = r[v];
                                    const uint32_t b = j < 3 ? r[v + (j < 3 ? 1 : 0)] : nxt;
                                    const bool ok = code == CHK_SORTED_F ? (uf(a) <= uf(b)) : (ui(a) <= ui(b));
                                    bad |= ((!ok && elem(v) + 1 < n) ? 1u : 0u) << v;
                                }
                            }
                        )
                        bad &= S[0];
                        const uint64_t f = wave_max_u64(~first_of(bad));
                        if (lane == 0) slot_max(op.aux, f);
                    } break;
                    // ---------------- reductions ----------------
                    case RED_SUM_F: case RED_ABSSUM_F: {
                        const uint32_t m = get_space(S, op.sp);
                        double acc = 0.0;
                        SG_ON_REG(op.a, 
    _Pragma("unroll")                         for (int v = 0; v < V; ++v) {
                                float f = uf(r[v]);
                                if (code == RED_ABSSUM_F) f = __builtin_fabsf(f);
                                acc += ((m >> v) & 1u) ? (double)f : 0.0;
                            }
                        )
                        acc = wave_sum_f64(acc);
                        if (lane == 0) L.sum[wave][op.aux] += acc;
                    } break;
                    case RED_SUM_I: {
                        const uint32_t m = get_space(S, op.sp);
                        int64_t acc = 0;
                        SG_ON_REG(op.a, 
    _Pragma("unroll")                         for (int v = 0; v < V; ++v) acc += ((m >> v) & 1u) ? (int64_t)ui(r[v]) : 0;
                        )
                        acc = wave_sum_i64(acc);
                        if (lane == 0) slot_add(op.aux, (uint64_t)acc);
                    } break;
                    case RED_MAX_F: case RED_MIN_F: case RED_MAX_I: case RED_MIN_I: {
                        // encoded so that the combine is an unsigned max with identity 0
                        const uint32_t m = get_space(S, op.sp);
                        const bool is_max = code == RED_MAX_F || code == RED_MAX_I;
                        const bool is_f = code == RED_MAX_F || code == RED_MIN_F;
                        uint32_t acc = 0;
                        SG_ON_REG(op.a, _Pragma("unroll") for (int v = 0; v < V; ++v) {
                            int32_t k;
                            if (is_f) {
                                const bool nan = (r[v] & 0x7FFFFFFFu) > 0x7F800000u;
                                k = nan ? (is_max ? INT32_MAX : INT32_MIN) : fkey(r[v]);
                            } else {
                                k = ui(r[v]);
                            }
                            uint32_t e = (uint32_t)k ^ 0x80000000u;
                            if (!is_max) e = ~e;
                            if ((m >> v) & 1u) acc = max(acc, e);
                        })
                        acc = wave_max_u32(acc);
                        if (lane == 0) slot_max(op.aux, (uint64_t)acc);
                    } break;
                    case RED_COUNT: {
                        const uint32_t m = get_space(S, op.sp);
                        const int64_t c = wave_sum_i64((int64_t)__builtin_popcount(m));
                        if (lane == 0) slot_add(op.aux, (uint64_t)c);
                    } break;
                    case EMIT: {
                        if (op.sp == 0) {
                            uint32_t* q = (uint32_t*)(uintptr_t)d64<INLINE>(kdesc, D, (int)offsetof(InstDesc, out) + 8 * op.aux);
                            SG_ON_REG(op.a, 
                                if (vec) {
    _Pragma("unroll")                                 for (int u = 0; u < U; ++u) {
                                        uint4 w;
                                        w.x = r[4 * u + 0]; w.y = r[4 * u + 1]; w.z = r[4 * u + 2]; w.w = r[4 * u + 3];
                                        *(uint4*)(q + e0 + u * 256) = w;
                                    }
                                } else {
    _Pragma("unroll")                                 for (int v = 0; v < V; ++v)
                                        if ((inb >> v) & 1u) q[elem(v)] = r[v];
                                }
                            )
                        } else if (nce == 0) {
                            ce_reg0 = op.a; ce_out0 = op.aux; ++nce;
                        } else {
                            ce_reg1 = op.a; ce_out1 = op.aux; ++nce;
                        }
                    } break;
                    default: break;
                }
            }


            // ---------------- compaction: ranks in the scan space, one look-back per wave --------
            if (scan_space != 0) {
                const uint32_t keep = get_space(S, scan_space);
                // rank of value v within the wave = (kept values of chunks before u)
                //   + (kept values of lanes below in chunk u) + (kept values j' < j of this lane)
                uint32_t lbase[U];
                uint32_t agg = 0;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    uint32_t below = 0, tot = 0;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const uint64_t b = __ballot((keep >> (4 * u + j)) & 1u);
                        below += __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
                        tot += (uint32_t)__builtin_popcountll(b);
                    }
                    lbase[u] = agg + below;
                    agg += tot;
                }
                const uint64_t ep = (uint64_t)(epoch & 0x3FFFFFFFu) << 32;
                const uint64_t AGG = 1ull << 62, INC = 2ull << 62;
                const int64_t g = (tile0 * C + sub) * nwaves + wave;  // this wave chunk
                const int64_t g0 = tile0 * C * nwaves;              // the instance's first chunk
                int64_t excl = 0;
                if (g == g0) {
                    if (lane == 0) st_relaxed(&A.lookback[g], INC | ep | agg);
                } else {
                    if (lane == 0) st_relaxed(&A.lookback[g], AGG | ep | agg);
                    int64_t j = g - 1;
                    for (uint32_t spins = 0;;) {
                        const int64_t idx = j - lane;
                        const uint64_t d = idx >= g0 ? ld_relaxed(&A.lookback[idx]) : (INC | ep);
                        const bool valid = (d & (0x3FFFFFFFull << 32)) == ep && (d >> 62) != 0;
                        const uint64_t incm = __ballot(valid && (d >> 62) == 2);
                        const uint64_t invm = __ballot(!valid);
                        const int fi = incm ? __builtin_ctzll(incm) : 64;
                        const uint64_t need = fi >= 63 ? ~0ull : ((2ull << fi) - 1ull);
                        if (invm & need) {
                            if (++spins > (1u << 22)) {
                                if (lane == 0) atomicOr(&A.results[cur].err, (uint32_t)ERR_LOOKBACK_TIMEOUT);
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                            continue;
                        }
                        excl += wave_sum_i64((lane <= fi) ? (int64_t)(uint32_t)d : 0);
                        if (fi < 64) break;
                        j -= 64;
                    }
                    if (lane == 0) st_relaxed(&A.lookback[g], INC | ep | (uint64_t)(uint32_t)(excl + agg));
                }
                auto rank_of = [&](int v) -> int64_t {
                    const int u = v >> 2, jj = v & 3;
                    const uint32_t lowbits = (keep >> (4 * u)) & ((1u << jj) - 1u);
                    return excl + lbase[u] + __builtin_popcount(lowbits);
                };
                for (int ci = 0; ci < nce; ++ci) {
                    uint32_t* q = (uint32_t*)(uintptr_t)d64<INLINE>(kdesc, D, (int)offsetof(InstDesc, out) + 8 * (ci == 0 ? ce_out0 : ce_out1));
                    SG_ON_REG(ci == 0 ? ce_reg0 : ce_reg1, _Pragma("unroll") for (int v = 0; v < V; ++v)
                        if ((keep >> v) & 1u) q[rank_of(v)] = r[v];)
                }
                for (int ci = 0; ci < nd; ++ci) {
                    const uint32_t hit = ci == 0 ? D0 : D1;
                    const uint64_t f = wave_max_u64(hit ? ~(uint64_t)rank_of(__builtin_ctz(hit)) : 0ull);
                    if (lane == 0) slot_max(ci == 0 ? d_slot0 : d_slot1, f);
                }
            }
        }
        // tile end: its sums, added over the waves in order, are buffered for publication
        __syncthreads();
        if (tid < nsum) {
            double s = 0.0;
            for (int w = 0; w < nwaves; ++w) s += L.sum[w][tid];
            L.tsum[ntl][tid] = s;
        }
        if (tid == 0) L.tile[ntl] = t;
        __syncthreads();
        if (lane < MAX_SUMS) L.sum[wave][lane] = 0.0;
        ++ntl;
    }
    if (cur >= 0) flush();
}

// zero a region of 64-bit words (accumulators, tags, look-back descriptors) without a
// memset node, so the call can sit inside a captured graph
__global__ void zero_kernel(uint64_t* p, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// advance the launch epoch of a captured graph (one thread)
__global__ void epoch_bump_kernel(uint32_t* e) {
    uint32_t v = (*e + 1u) & 0x3FFFFFFFu;
    *e = v ? v : 1u;
}

}  // namespace sg

// ---- launchers (host) ------------------------------------------------------------------------

extern "C++" hipError_t sg_launch_stream(const sg::StreamArgs& a, int unroll, bool inl, int grid, int block,
                                         hipStream_t s) {
    using namespace sg;
#define SG_LAUNCH(UU)                                                                        \
    if (inl) hipLaunchKernelGGL((stream_kernel<UU, true>), dim3(grid), dim3(block), 0, s, a); \
    else hipLaunchKernelGGL((stream_kernel<UU, false>), dim3(grid), dim3(block), 0, s, a);
    switch (unroll) {
        case 1: SG_LAUNCH(1); break;
        case 2: SG_LAUNCH(2); break;
        default: SG_LAUNCH(4); break;
    }
#undef SG_LAUNCH
    return hipGetLastError();
}

extern "C++" hipError_t sg_launch_zero(uint64_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int grid = (int)((n + 255) / 256);
    hipLaunchKernelGGL(sg::zero_kernel, dim3(grid), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

extern "C++" hipError_t sg_launch_epoch_bump(uint32_t* e, hipStream_t s) {
    hipLaunchKernelGGL(sg::epoch_bump_kernel, dim3(1), dim3(1), 0, s, e);
    return hipGetLastError();
}

extern "C++" int sg_stream_occupancy(int unroll, bool inl, int block) {
    using namespace sg;
    int nb = 0;
#define SG_OCC(UU)                                                                                      \
    if (inl) (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stream_kernel<UU, true>, block, 0);  \
    else (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, stream_kernel<UU, false>, block, 0);
    switch (unroll) {
        case 1: SG_OCC(1); break;
        case 2: SG_OCC(2); break;
        default: SG_OCC(4); break;
    }
#undef SG_OCC
    return nb > 0 ? nb : 1;
}
