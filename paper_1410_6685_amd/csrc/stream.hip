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
// Tiles are taken from an atomic ticket, so a tile waits only on tiles handed out earlier
// (decoupled look-back for compaction needs that forward-progress guarantee).  Exact
// accumulators (counts, int sums, min/max keys, first indices) are combined with device
// atomics; float64 sums are written per tile and added in tile order by the instance's
// last tile, so sums are identical from run to run.
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

struct Lds {
    uint64_t slot[MAX_WAVES][MAX_SLOTS];
    double sum[MAX_WAVES][MAX_SUMS];
    uint32_t wcount[MAX_WAVES];
    int64_t tile;
    int64_t prefix;
    int32_t last;
    int32_t pad;
    double fin[MAX_WAVES][MAX_SUMS];
};

// ---- the kernel ----------------------------------------------------------------------------

template <int U, bool INLINE>
__global__ __launch_bounds__(1024) void stream_kernel(const StreamArgs A) {
    constexpr int V = 4 * U;
    __shared__ Lds L;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int nwaves = blockDim.x >> 6;
    const int64_t tile_elems = (int64_t)blockDim.x * V;
    const uint32_t epoch = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(A.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) & 0x3FFFFFFFu;

    for (;;) {
        if (tid == 0) L.tile = (int64_t)atomicAdd(&A.counters[0], 1u);
        __syncthreads();
        const int64_t t = L.tile;
        if (t >= A.total_tiles) break;
        const int inst = INLINE ? 0 : (int)uload32(A.tile_inst + t);
        const InstDesc* D = INLINE ? &A.inst0 : (A.insts + inst);
        const SgOp* prog = INLINE ? A.prog0 : (A.progs + (int)uload32(&D->prog_off));
        const int plen = (int)uload32(&D->prog_len);
        const int64_t* n_dev = uptr<const int64_t>(&D->n_dev);
        const int64_t n = n_dev ? (int64_t)uload64(n_dev) : (int64_t)uload64(&D->n);
        const int64_t tile0 = (int64_t)uload64(&D->tile0);
        const int64_t ntiles = (int64_t)uload64(&D->ntiles);
        const int nin = (int)uload32(&D->nin);
        const int scan_space = (int)uload32(&D->scan_space);
        const int flags = (int)uload32(&D->flags);
        const int64_t local = t - tile0;
        const int64_t base = local * tile_elems;
        const bool full = base + tile_elems <= n;
        const bool vec = full && (flags & 1);
        const int64_t e0 = base + (int64_t)wave * (U * 256) + lane * 4;

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

        // in-bounds mask and loads of the sources into registers 0..nin-1
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
                const uint32_t* q = uptr<const uint32_t>(&D->in[k]);
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
                const uint32_t* pw = (const uint32_t*)(prog + pc);
                uint32_t* ow = (uint32_t*)&op;
#pragma unroll
                for (int i = 0; i < 4; ++i) ow[i] = __builtin_amdgcn_readfirstlane(pw[i]);
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
                        if (lane == 0) L.slot[wave][op.aux] = f;
                    }
                } break;
                case CHK_SORTED_F: case CHK_SORTED_I: {
                    uint32_t bad = 0;
                    const uint32_t* q = uptr<const uint32_t>(&D->in[op.b]);
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
                    if (lane == 0) L.slot[wave][op.aux] = f;
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
                    if (lane == 0) L.sum[wave][op.aux] = acc;
                } break;
                case RED_SUM_I: {
                    const uint32_t m = get_space(S, op.sp);
                    int64_t acc = 0;
                    SG_ON_REG(op.a, 
_Pragma("unroll")                         for (int v = 0; v < V; ++v) acc += ((m >> v) & 1u) ? (int64_t)ui(r[v]) : 0;
                    )
                    acc = wave_sum_i64(acc);
                    if (lane == 0) L.slot[wave][op.aux] = (uint64_t)acc;
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
                    if (lane == 0) L.slot[wave][op.aux] = (uint64_t)acc;
                } break;
                case RED_COUNT: {
                    const uint32_t m = get_space(S, op.sp);
                    const int64_t c = wave_sum_i64((int64_t)__builtin_popcount(m));
                    if (lane == 0) L.slot[wave][op.aux] = (uint64_t)c;
                } break;
                case EMIT: {
                    if (op.sp == 0) {
                        uint32_t* q = uptr<uint32_t>(&D->out[op.aux]);
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

        // ---------------- compaction: ranks in the scan space ----------------
        if (scan_space != 0) {
            const uint32_t keep = get_space(S, scan_space);
            // rank of value v within the wave = (kept values of chunks before u)
            //   + (kept values of lanes below in chunk u) + (kept values j' < j of this lane)
            uint32_t lbase[U];
            uint32_t running = 0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                uint32_t below = 0, tot = 0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const uint64_t b = __ballot((keep >> (4 * u + j)) & 1u);
                    below += __builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
                    tot += (uint32_t)__builtin_popcountll(b);
                }
                lbase[u] = running + below;
                running += tot;
            }
            if (lane == 0) L.wcount[wave] = running;
            __syncthreads();
            uint32_t woff = 0, agg = 0;
            for (int w = 0; w < nwaves; ++w) {
                const uint32_t c = L.wcount[w];
                woff += w < wave ? c : 0u;
                agg += c;
            }
            if (wave == 0) {
                // decoupled look-back over the tiles of this instance
                const uint64_t ep = (uint64_t)epoch << 32;
                const uint64_t AGG = 1ull << 62, INC = 2ull << 62;
                int64_t excl = 0;
                if (local == 0) {
                    if (lane == 0) st_relaxed(&A.lookback[t], INC | ep | agg);
                } else {
                    if (lane == 0) st_relaxed(&A.lookback[t], AGG | ep | agg);
                    int64_t j = t - 1;
                    uint32_t spins = 0;
                    for (;;) {
                        const int64_t idx = j - lane;
                        const uint64_t d = idx >= tile0 ? ld_relaxed(&A.lookback[idx]) : (INC | ep);
                        const bool valid = (d & (0x3FFFFFFFull << 32)) == ep && (d >> 62) != 0;
                        const uint64_t incm = __ballot(valid && (d >> 62) == 2);
                        const uint64_t invm = __ballot(!valid);
                        const int fi = incm ? __builtin_ctzll(incm) : 64;
                        const uint64_t need = fi >= 63 ? ~0ull : ((2ull << fi) - 1ull);
                        if (invm & need) {
                            if (++spins > (1u << 22)) {
                                if (lane == 0) atomicOr(&A.results[inst].err, (uint32_t)ERR_LOOKBACK_TIMEOUT);
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                            continue;
                        }
                        const int64_t vpart = (lane <= fi) ? (int64_t)(uint32_t)d : 0;
                        excl += wave_sum_i64(vpart);
                        if (fi < 64) break;
                        j -= 64;
                    }
                    if (lane == 0) st_relaxed(&A.lookback[t], INC | ep | (uint64_t)(uint32_t)(excl + agg));
                }
                if (lane == 0) L.prefix = excl;
            }
            __syncthreads();
            const int64_t tbase = L.prefix + woff;
            auto rank_of = [&](int v) -> int64_t {
                const int u = v >> 2, j = v & 3;
                const uint32_t lowbits = (keep >> (4 * u)) & ((1u << j) - 1u);
                return tbase + lbase[u] + __builtin_popcount(lowbits);
            };
            for (int c = 0; c < nce; ++c) {
                uint32_t* q = uptr<uint32_t>(&D->out[c == 0 ? ce_out0 : ce_out1]);
                SG_ON_REG(c == 0 ? ce_reg0 : ce_reg1, 
_Pragma("unroll")                     for (int v = 0; v < V; ++v)
                        if ((keep >> v) & 1u) q[rank_of(v)] = r[v];
                )
            }
            for (int c = 0; c < nd; ++c) {
                const uint32_t hit = c == 0 ? D0 : D1;
                const uint64_t f = wave_max_u64(hit ? ~(uint64_t)rank_of(__builtin_ctz(hit)) : 0ull);
                if (lane == 0) L.slot[wave][c == 0 ? d_slot0 : d_slot1] = f;
            }
        }
        __syncthreads();

        // ---------------- combine the tile over waves ----------------
        const int ns = (int)uload32(&D->nslots), nsum = (int)uload32(&D->nsum);
        if (tid < ns) {
            const uint8_t kind = D->slot_kind[tid];
            uint64_t* g = A.acc + (int64_t)inst * MAX_SLOTS + tid;
            if (kind == SLOT_ADD) {
                uint64_t s = 0;
                for (int w = 0; w < nwaves; ++w) s += L.slot[w][tid];
                if (s) atomicAdd((unsigned long long*)g, (unsigned long long)s);
            } else if (kind == SLOT_MAX64) {
                uint64_t m = 0;
                for (int w = 0; w < nwaves; ++w) m = L.slot[w][tid] > m ? L.slot[w][tid] : m;
                if (m) atomicMax((unsigned long long*)g, (unsigned long long)m);
            } else if (kind == SLOT_MAX32) {
                uint32_t m = 0;
                for (int w = 0; w < nwaves; ++w) m = max(m, (uint32_t)L.slot[w][tid]);
                if (m) atomicMax((unsigned int*)g, m);
            }
        } else if (tid >= MAX_SLOTS && tid < MAX_SLOTS + nsum) {
            const int k = tid - MAX_SLOTS;
            double s = 0.0;
            for (int w = 0; w < nwaves; ++w) s += L.sum[w][k];
            A.tile_sums[t * MAX_SUMS + k] = s;
        }
        // publish this tile; the instance's last tile finalizes it
        __syncthreads();
        if (tid == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const uint32_t done = atomicAdd(&A.counters[2 + inst], 1u);
            L.last = (int64_t)done + 1 == ntiles ? 1 : 0;
            if (L.last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (L.last) {
            InstResult* res = A.results + inst;
            // float64 sums: tile partials added in a fixed order over the block
            for (int k = 0; k < nsum; ++k) {
                double s = 0.0;
                for (int64_t q = tid; q < ntiles; q += blockDim.x) s += A.tile_sums[(tile0 + q) * MAX_SUMS + k];
                s = wave_sum_f64(s);
                if (lane == 0) L.fin[wave][k] = s;
            }
            __syncthreads();
            if (tid < nsum) {
                double s = 0.0;
                for (int w = 0; w < nwaves; ++w) s += L.fin[w][tid];
                res->sum[tid] = s;
            }
            const int count_slot = (int)uload32(&D->count_slot);
            if (tid < ns) {
                uint64_t* g = A.acc + (int64_t)inst * MAX_SLOTS + tid;
                const uint64_t v = __hip_atomic_load(g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                res->slot[tid] = (int64_t)v;
                __hip_atomic_store(g, (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (tid == count_slot) res->scan_count = (int64_t)v;
            }
            if (tid == 0) __hip_atomic_store(&A.counters[2 + inst], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
    // the last block to leave resets the ticket for the next launch
    if (tid == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const uint32_t d = atomicAdd(&A.counters[1], 1u);
        if (d + 1 == gridDim.x) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            atomicExch(&A.counters[0], 0u);
            atomicExch(&A.counters[1], 0u);
            atomicExch(A.epoch, (epoch + 1u) & 0x3FFFFFFFu);
        }
    }
}

// zero a region of 64-bit words (accumulators, counters, lookback descriptors) without a
// memset node, so the call can sit inside a captured graph
__global__ void zero_kernel(uint64_t* p, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
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
