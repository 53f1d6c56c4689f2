// Quicksort of the collection API (Section 4, Listing 3) run breadth-first on the GPU.
//
// The listing recurses: pivot = the item at index count // 2, three stable filters (less,
// equal, greater than the pivot), result = quicksort(less) ++ equal ++ quicksort(greater).
// Every collection of one recursion level is partitioned at once here.  A collection ("segment")
// keeps its place in the output: less occupies the front of its range, then equal, then
// greater, so every item's final position lies inside its segment's range.  The equal items
// are final at once and go straight to the output; the less and greater parts are the next
// level's segments.  Items no filter keeps (NaN against any pivot, or anything against a NaN
// pivot) are dropped, as the listing drops them: their slots at the end of the segment's range
// are filled with a NaN marker, and a final stable compaction removes the markers (a kept item
// is never NaN), so the result is the listing's concatenation and its count is what the
// postcondition count = old count compares.
//
// Large segments are partitioned by three kernels per level over 4096-item tiles: count the
// four classes per tile, scan the tile counts per segment, then scatter (LDS-staged, so that
// the writes of a tile are four contiguous runs).  Segments of at most 2048 items are finished
// by one workgroup each in LDS, all in one launch after the last level (a segment's items stay
// where its level wrote them): without NaN the recursion's result is the stable sort of the
// segment, which a bitonic network over (key, position) pairs computes; a segment holding a
// NaN runs the recursion itself, with the same pivot rule and stable three-way partition, all
// of the segment's sub-collections partitioned together in each round.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "sg_runtime.h"

namespace sgq {

constexpr int QB = 256;            // threads per block
constexpr int QPT = 16;            // items per thread
constexpr int QTE = QB * QPT;      // items per tile (4096)
constexpr uint32_t QHOLE = 0x7FC00000u;  // marker of a dropped item's slot (a quiet NaN)
constexpr int QPAD = QPT + 1;      // LDS row of one thread (bank-conflict padding)

struct Seg {
    int64_t start;   // first position of the segment (in the working buffers and the output)
    int64_t len;
    int64_t tile0;   // first tile of the segment
    int64_t pad;
};

__device__ __forceinline__ float uf(uint32_t u) { return __builtin_bit_cast(float, u); }

// class of item v against pivot p: 0 less, 1 equal, 2 greater, 3 dropped (IEEE: NaN compares false)
template <bool F>
__device__ __forceinline__ int qclass(uint32_t v, uint32_t p) {
    if (F) {
        const float a = uf(v), b = uf(p);
        return a < b ? 0 : a == b ? 1 : a > b ? 2 : 3;
    }
    const int32_t a = (int32_t)v, b = (int32_t)p;
    return a < b ? 0 : a == b ? 1 : 2;
}

// 4 x 16-bit class counters in one word (a tile or a leaf has at most 4096 items)
__device__ __forceinline__ uint64_t one_hot(int c) { return 1ull << (16 * c); }
__device__ __forceinline__ uint32_t field(uint64_t w, int c) { return (uint32_t)(w >> (16 * c)) & 0xFFFFu; }

__device__ __forceinline__ uint64_t wave_incl_sum(uint64_t v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(v, o);
        if (lane >= o) v += y;
    }
    return v;
}

// Block-wide exclusive scan of one 64-bit value per thread (QB threads); *total gets the sum.
__device__ __forceinline__ uint64_t block_excl_sum(uint64_t v, uint64_t* wsum, uint64_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t incl = wave_incl_sum(v, lane);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint64_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < QB / 64; ++w) {
        const uint64_t x = wsum[w];
        if (w < wave) base += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

// ---- level kernels: count, scan, scatter ---------------------------------------------------

template <bool F>
__global__ __launch_bounds__(QB) void q_count(const uint32_t* __restrict__ cur, const Seg* __restrict__ segs,
                                              const int32_t* __restrict__ tile_seg, uint4* __restrict__ tile_cnt) {
    __shared__ uint64_t wsum[QB / 64];
    const int64_t t = blockIdx.x;
    const Seg s = segs[tile_seg[t]];
    const uint32_t p = cur[s.start + s.len / 2];
    const int64_t lo = (t - s.tile0) * QTE, hi = std::min<int64_t>(lo + QTE, s.len);
    // the tile's QPT loads per thread are issued together (a fixed count, guarded), not one
    // round trip after another
    uint32_t x[QPT];
#pragma unroll
    for (int q = 0; q < QPT; ++q) {
        const int64_t i = lo + threadIdx.x + q * QB;
        x[q] = i < hi ? cur[s.start + i] : 0u;
    }
    uint64_t c = 0;
#pragma unroll
    for (int q = 0; q < QPT; ++q)
        if (lo + threadIdx.x + q * QB < hi) c += one_hot(qclass<F>(x[q], p));
    uint64_t tot;
    (void)block_excl_sum(c, wsum, &tot);
    if (threadIdx.x == 0) tile_cnt[t] = make_uint4(field(tot, 0), field(tot, 1), field(tot, 2), field(tot, 3));
}

// One block per segment: exclusive offsets of its tiles per class, and the segment's totals.
__global__ __launch_bounds__(QB) void q_scan(const Seg* __restrict__ segs, const uint4* __restrict__ tile_cnt,
                                             uint4* __restrict__ tile_off, ulonglong2* __restrict__ seg_tot) {
    __shared__ uint64_t wsum[QB / 64];
    const Seg s = segs[blockIdx.x];
    const int64_t nt = (s.len + QTE - 1) / QTE;
    // two 64-bit scans: classes 0,1 and classes 2,3 as 32-bit halves (a segment holds < 2^32 items)
    uint64_t carry01 = 0, carry23 = 0;
    for (int64_t c0 = 0; c0 < nt; c0 += QB) {
        const int64_t k = c0 + threadIdx.x;
        uint4 v = k < nt ? tile_cnt[s.tile0 + k] : make_uint4(0, 0, 0, 0);
        const uint64_t a = ((uint64_t)v.y << 32) | v.x, b = ((uint64_t)v.w << 32) | v.z;
        uint64_t ta, tb;
        const uint64_t ea = block_excl_sum(a, wsum, &ta) + carry01;
        const uint64_t eb = block_excl_sum(b, wsum, &tb) + carry23;
        if (k < nt) tile_off[s.tile0 + k] = make_uint4((uint32_t)ea, (uint32_t)(ea >> 32), (uint32_t)eb, (uint32_t)(eb >> 32));
        carry01 += ta;
        carry23 += tb;
    }
    if (threadIdx.x == 0) seg_tot[blockIdx.x] = make_ulonglong2(carry01, carry23);
}

// Scatter one tile: stable ranks per class in LDS, then four contiguous runs: less and greater
// to the next level's buffer (and to the output when that child holds one item), equal to the
// output, dropped slots as markers in the output.
template <bool F>
__global__ __launch_bounds__(QB) void q_scatter(const uint32_t* __restrict__ cur, uint32_t* __restrict__ nxt,
                                                uint32_t* __restrict__ out, const Seg* __restrict__ segs,
                                                const int32_t* __restrict__ tile_seg, const uint4* __restrict__ tile_off,
                                                const ulonglong2* __restrict__ seg_tot) {
    __shared__ uint32_t v[QB * QPAD];
    __shared__ uint32_t o[QTE];
    __shared__ uint64_t wsum[QB / 64];
    const int64_t t = blockIdx.x;
    const int si = tile_seg[t];
    const Seg s = segs[si];
    const uint32_t p = cur[s.start + s.len / 2];
    const int64_t lo = (t - s.tile0) * QTE;
    const int cnt = (int)std::min<int64_t>(QTE, s.len - lo);
    {
        uint32_t x[QPT];  // all loads in flight before the first is stored
#pragma unroll
        for (int q = 0; q < QPT; ++q) {
            const int i = threadIdx.x + q * QB;
            x[q] = i < cnt ? cur[s.start + lo + i] : 0u;
        }
#pragma unroll
        for (int q = 0; q < QPT; ++q) {
            const int i = threadIdx.x + q * QB;
            if (i < cnt) v[(i / QPT) * QPAD + i % QPT] = x[q];
        }
    }
    __syncthreads();
    // this thread's items: positions tid*16 .. tid*16+15 of the tile, in order
    const int first = threadIdx.x * QPT;
    uint64_t mine = 0;
    int cls[QPT];
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        cls[j] = first + j < cnt ? qclass<F>(v[threadIdx.x * QPAD + j], p) : -1;
        if (cls[j] >= 0) mine += one_hot(cls[j]);
    }
    uint64_t tot;
    const uint64_t ex = block_excl_sum(mine, wsum, &tot);
    const uint32_t base[4] = {0, field(tot, 0), field(tot, 0) + field(tot, 1), field(tot, 0) + field(tot, 1) + field(tot, 2)};
    uint32_t run[4] = {field(ex, 0), field(ex, 1), field(ex, 2), field(ex, 3)};
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        const int c = cls[j];
        if (c < 0) continue;
        uint32_t r = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k == c) r = base[k] + run[k]++;
        o[r] = v[threadIdx.x * QPAD + j];
    }
    __syncthreads();
    const ulonglong2 T = seg_tot[si];
    const uint64_t nL = (uint32_t)T.x, nE = (uint32_t)(T.x >> 32), nG = (uint32_t)T.y;
    const uint4 off = tile_off[t];
    for (int q = threadIdx.x; q < cnt; q += QB) {
        const uint32_t val = o[q];
        if ((uint32_t)q < base[1]) {
            const int64_t d = s.start + off.x + q;
            nxt[d] = val;
            if (nL == 1) out[d] = val;
        } else if ((uint32_t)q < base[2]) {
            out[s.start + nL + off.y + (q - base[1])] = val;
        } else if ((uint32_t)q < base[3]) {
            const int64_t d = s.start + nL + nE + off.z + (q - base[2]);
            nxt[d] = val;
            if (nG == 1) out[d] = val;
        } else {
            out[s.start + nL + nE + nG + off.w + (q - base[3])] = QHOLE;
        }
    }
}

// Order-preserving unsigned key: floats by value with -0 and +0 one key (they compare equal),
// int32 by value.  Not used for NaN.
template <bool F>
__device__ __forceinline__ uint32_t qkey(uint32_t u) {
    if (!F) return u ^ 0x80000000u;
    if ((u & 0x7FFFFFFFu) == 0) u = 0;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// ---- leaf kernel: one segment of at most 2048 items per block, finished in LDS ---------------
//
// Leaves holding a NaN (listed by q_leaf_net) run the recursion: each position
// carries the start and length of the sub-collection holding it; a round
// partitions every active sub-collection (length > 1) about its own pivot with one segmented
// scan of the four class counters, and the children become the next round's sub-collections.
// Equal items, one-item children and dropped slots are final.

struct Leaf {
    int64_t start, len;
    const uint32_t* src;  // the buffer holding the segment (the level that produced it wrote it there)
};

constexpr int LPT = 8;               // positions per thread in the leaf kernel
constexpr int QLEAF_N = QB * LPT;  // 2048: largest segment finished in LDS
constexpr uint16_t QFINAL = 0;       // length field of a final position

// The leaves without NaN: a bitonic network over (key, position) pairs in 24 KiB of LDS.  A leaf
// holding a NaN is left for q_leaf: its index goes to `nan_list`.
template <bool F>
__global__ __launch_bounds__(QB) void q_leaf_net(uint32_t* __restrict__ out, const Leaf* __restrict__ leaves,
                                                 uint32_t* __restrict__ nan_list, uint32_t* __restrict__ nan_count) {
    __shared__ uint32_t val[QLEAF_N];
    __shared__ uint64_t tot[QLEAF_N];
    const Leaf lf = leaves[blockIdx.x];
    const uint32_t* __restrict__ src = lf.src;
    const int n = (int)lf.len;
    // power of two >= n for the sorting network (n <= QLEAF_N)
    int P = 2;
    while (P < n) P <<= 1;
    bool nan = false;
    uint32_t xs[LPT];  // the segment's loads in flight together
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
        const int i = threadIdx.x + q * QB;
        xs[q] = i < n ? src[lf.start + i] : 0u;
    }
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
        const int i = threadIdx.x + q * QB;
        if (i >= P) continue;
        if (i < n) {
            val[i] = xs[q];
            nan |= F && (xs[q] & 0x7FFFFFFFu) > 0x7F800000u;
            tot[i] = ((uint64_t)qkey<F>(xs[q]) << 32) | (uint32_t)i;
        } else {
            tot[i] = ~0ull;  // above every key: padding sorts to the end
        }
    }
    if (__syncthreads_or(nan)) {
        if (threadIdx.x == 0) nan_list[atomicAdd(nan_count, 1u)] = blockIdx.x;
        return;
    }
    // No NaN: every filter keeps each item, and items that compare equal (including -0 and
    // +0) fall on the same side of every pivot, so the listing's recursion of stable
    // three-way partitions yields the items in ascending order with ties in input order,
    // i.e. the stable sort.  A bitonic network over (key, position) pairs computes it.
    // Each step compares the pairs (i, i + j) that differ in bit j of the position, ascending
    // where bit k of i is clear.  Pairs of one step are disjoint, so a thread loads all of its
    // pairs before it compares any (their LDS reads in flight together) and writes the
    // smaller and larger key of each without a branch (keys are distinct: the position is
    // part of the key).
    constexpr int PPT = QLEAF_N / 2 / QB;  // pairs per thread at the largest size
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            uint64_t ka[PPT], kc[PPT];
            int pi[PPT];
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                const int t = threadIdx.x + q * QB;
                pi[q] = ((t & ~(j - 1)) << 1) | (t & (j - 1));  // j is a power of two
                if (t < P / 2) {
                    ka[q] = tot[pi[q]];
                    kc[q] = tot[pi[q] + j];
                }
            }
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                if (threadIdx.x + q * QB < P / 2) {
                    const bool up = (pi[q] & k) == 0;
                    const uint64_t lo = ka[q] < kc[q] ? ka[q] : kc[q], hi = ka[q] < kc[q] ? kc[q] : ka[q];
                    tot[pi[q]] = up ? lo : hi;
                    tot[pi[q] + j] = up ? hi : lo;
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < n; i += QB) out[lf.start + i] = val[(uint32_t)tot[i] & 0xFFFFu];
}

template <bool F>
__global__ __launch_bounds__(QB) void q_leaf(uint32_t* __restrict__ out, const Leaf* __restrict__ leaves,
                                             const uint32_t* __restrict__ list, unsigned long long* __restrict__ dropped) {
    __shared__ uint32_t val[2][QLEAF_N];
    __shared__ uint16_t sst[2][QLEAF_N];  // start of the sub-collection holding the position
    __shared__ uint16_t sln[2][QLEAF_N];  // its length, QFINAL when the position is final
    __shared__ uint64_t tot[QLEAF_N];     // class totals of a sub-collection, at its start
    __shared__ uint64_t wsum[QB / 64];
    __shared__ uint32_t wflag[QB / 64];
    const Leaf lf = leaves[list[blockIdx.x]];
    const uint32_t* __restrict__ src = lf.src;
    const int n = (int)lf.len;
    uint32_t xs[LPT];  // the segment's loads in flight together
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
        const int i = threadIdx.x + q * QB;
        xs[q] = i < n ? src[lf.start + i] : 0u;
    }
#pragma unroll
    for (int q = 0; q < LPT; ++q) {
        const int i = threadIdx.x + q * QB;
        if (i < n) {
            val[0][i] = xs[q];
            sst[0][i] = 0;
            sln[0][i] = (uint16_t)(n > 1 ? n : QFINAL);
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int p0 = threadIdx.x * LPT;
    unsigned drops = 0;
    int b = 0;
    // every round finalizes at least the pivot of each active sub-collection, so at most n rounds
    for (int round = 0; round < QLEAF_N; ++round) {
        int cls[LPT];
        uint64_t incl[LPT];
        uint32_t flags = 0;
        uint64_t acc = 0;
        bool any = false;
#pragma unroll
        for (int j = 0; j < LPT; ++j) {
            const int pos = p0 + j;
            int c = -1;
            bool head = true;
            if (pos < n && sln[b][pos] != QFINAL) {
                const int s0 = sst[b][pos], L = sln[b][pos];
                c = qclass<F>(val[b][pos], val[b][s0 + L / 2]);
                head = pos == s0;
                any = true;
            }
            cls[j] = c;
            if (head) { flags |= 1u << j; acc = 0; }
            acc += c >= 0 ? one_hot(c) : 0;
            incl[j] = acc;  // inclusive counts since the last head inside this thread
        }
        // segmented inclusive scan of the thread aggregates over the wave: (has head, sum
        // since the last head); a later head resets the sum
        uint32_t hf = flags != 0;
        uint64_t sv = acc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t fy = __shfl_up(hf, o);
            const uint64_t sy = __shfl_up(sv, o);
            if (lane >= o) {
                if (!hf) sv += sy;
                hf |= fy;
            }
        }
        if (lane == 63) { wflag[wave] = hf; wsum[wave] = sv; }
        if (!__syncthreads_or(any)) break;
        // carry into this thread: the previous lane's aggregate, extended over earlier waves
        // while no head intervenes
        uint32_t pf = __shfl_up(hf, 1);
        uint64_t ps = __shfl_up(sv, 1);
        if (lane == 0) { pf = 0; ps = 0; }
        if (!pf) {
            for (int w = wave - 1; w >= 0; --w) {
                ps += wsum[w];
                if (wflag[w]) break;
            }
        }
        bool nohead = true;
#pragma unroll
        for (int j = 0; j < LPT; ++j) {
            nohead &= !((flags >> j) & 1u);
            if (nohead) incl[j] += ps;
        }
        // the last position of a sub-collection publishes the sub-collection's totals
#pragma unroll
        for (int j = 0; j < LPT; ++j) {
            const int pos = p0 + j;
            if (cls[j] < 0) continue;
            const int s0 = sst[b][pos], L = sln[b][pos];
            if (pos == s0 + L - 1) tot[s0] = incl[j];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < LPT; ++j) {
            const int pos = p0 + j;
            if (pos >= n) continue;
            const int c = cls[j];
            const uint32_t x = val[b][pos];
            if (c < 0) {  // final: stays where it is
                val[b ^ 1][pos] = x;
                sst[b ^ 1][pos] = (uint16_t)pos;
                sln[b ^ 1][pos] = QFINAL;
                continue;
            }
            const int s0 = sst[b][pos];
            const uint64_t T = tot[s0];
            const int nL = (int)field(T, 0), nE = (int)field(T, 1), nG = (int)field(T, 2);
            const int rank = (int)field(incl[j], c) - 1;
            int d, cs, cl;
            if (c == 0) { d = s0 + rank; cs = s0; cl = nL; }
            else if (c == 1) { d = s0 + nL + rank; cs = d; cl = 1; }
            else if (c == 2) { d = s0 + nL + nE + rank; cs = s0 + nL + nE; cl = nG; }
            else { d = s0 + nL + nE + nG + rank; cs = d; cl = 1; ++drops; }
            val[b ^ 1][d] = c == 3 ? QHOLE : x;
            sst[b ^ 1][d] = (uint16_t)cs;
            sln[b ^ 1][d] = (uint16_t)(cl > 1 ? cl : QFINAL);
        }
        __syncthreads();
        b ^= 1;
    }
    for (int i = threadIdx.x; i < n; i += QB) out[lf.start + i] = val[b][i];
    if (drops) atomicAdd(dropped, (unsigned long long)drops);
}

// ---- final compaction (only when items were dropped): keep every non-marker in order ------

__global__ __launch_bounds__(QB) void q_keep_count(const uint32_t* __restrict__ a, int64_t n, uint32_t* __restrict__ cnt) {
    __shared__ uint64_t wsum[QB / 64];
    const int64_t lo = (int64_t)blockIdx.x * QTE;
    uint64_t c = 0;
    for (int64_t i = lo + threadIdx.x; i < std::min<int64_t>(lo + QTE, n); i += QB) c += a[i] != QHOLE;
    uint64_t tot;
    (void)block_excl_sum(c, wsum, &tot);
    if (threadIdx.x == 0) cnt[blockIdx.x] = (uint32_t)tot;
}

__global__ __launch_bounds__(QB) void q_keep_scatter(const uint32_t* __restrict__ a, int64_t n,
                                                     const int64_t* __restrict__ off, uint32_t* __restrict__ out) {
    __shared__ uint64_t wsum[QB / 64];
    const int64_t lo = (int64_t)blockIdx.x * QTE;
    const int64_t first = lo + (int64_t)threadIdx.x * QPT;
    uint32_t x[QPT];
    uint64_t mine = 0;
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        x[j] = first + j < n ? a[first + j] : QHOLE;
        mine += x[j] != QHOLE;
    }
    uint64_t tot;
    int64_t d = off[blockIdx.x] + (int64_t)block_excl_sum(mine, wsum, &tot);
#pragma unroll
    for (int j = 0; j < QPT; ++j)
        if (x[j] != QHOLE) out[d++] = x[j];
}

__global__ void q_copy1(const uint32_t* __restrict__ a, uint32_t* __restrict__ b) { b[0] = a[0]; }

}  // namespace sgq

using namespace sgrt;

namespace sgrt {

// Sort the `m` items at `in` into `out` (capacity >= m); returns the count of the result (m
// minus the dropped items) in *count.  Work buffers come from the context's pool.
sg_status run_quicksort(sg_ctx_s* ctx, const void* in, void* out, int64_t m, bool is_f32, int64_t* count) {
    using namespace sgq;
    hipStream_t st = ctx->stream;
    const uint32_t* src = (const uint32_t*)in;
    uint32_t* dst = (uint32_t*)out;
    *count = m;
    if (m <= 0) return SG_OK;
    if (m == 1) {
        hipLaunchKernelGGL(q_copy1, dim3(1), dim3(1), 0, st, src, dst);
        SG_HIP(ctx, hipGetLastError());
        return SG_OK;
    }
    const int64_t max_tiles = (m + QTE - 1) / QTE + (m + QLEAF_N) / (QLEAF_N + 1) + 2;
    const int64_t max_segs = m / (QLEAF_N + 1) + 2;
    const int64_t max_leaves = m / 2 + 2;
    // device workspace: two item buffers, tables, counters
    const size_t b_items = (size_t)m * 4;
    const size_t b_segs = (size_t)max_segs * sizeof(Seg), b_tseg = (size_t)max_tiles * 4;
    const size_t b_cnt = (size_t)max_tiles * sizeof(uint4), b_tot = (size_t)max_segs * sizeof(ulonglong2);
    const size_t b_leaf = (size_t)std::min<int64_t>(max_leaves, m / 2 + 2) * sizeof(Leaf);
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_nanl = (size_t)std::min<int64_t>(max_leaves, m / 2 + 2) * 4;
    const size_t total = 2 * up(b_items) + up(b_segs) + up(b_tseg) + 2 * up(b_cnt) + up(b_tot) + up(b_leaf) +
                         up(b_nanl) + 256;
    char* w = (char*)dev_alloc(ctx, total);
    if (!w) return fail(ctx, SG_E_OOM, "quicksort: work memory");
    char* c = w;
    uint32_t* bufA = (uint32_t*)c; c += up(b_items);
    uint32_t* bufB = (uint32_t*)c; c += up(b_items);
    Seg* d_segs = (Seg*)c; c += up(b_segs);
    int32_t* d_tseg = (int32_t*)c; c += up(b_tseg);
    uint4* d_cnt = (uint4*)c; c += up(b_cnt);
    uint4* d_off = (uint4*)c; c += up(b_cnt);
    ulonglong2* d_tot = (ulonglong2*)c; c += up(b_tot);
    Leaf* d_leaf = (Leaf*)c; c += up(b_leaf);
    uint32_t* d_nanl = (uint32_t*)c; c += up(b_nanl);  // leaves holding a NaN
    unsigned long long* d_drop = (unsigned long long*)c;
    uint32_t* d_nanc = (uint32_t*)(d_drop + 1);          // their number
    auto done = [&](sg_status s) { dev_free(ctx, w); return s; };
#define SGQ_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t _e = (call);                                                        \
        if (_e != hipSuccess) return done(sgrt::hip_fail(ctx, _e, #call));            \
    } while (0)
    SGQ_HIP(hipMemsetAsync(d_drop, 0, 16, st));
    std::vector<Seg> segs;
    std::vector<int32_t> tseg;
    std::vector<Leaf> leaves;
    std::vector<ulonglong2> tots;
    int64_t dropped_host = 0;
    // level 0 reads the input in place; later levels alternate between the two buffers
    const uint32_t* cur = src;
    uint32_t* nxt = bufA;
    std::vector<Seg> active;
    if (m <= QLEAF_N) {
        leaves.push_back({0, m, src});
    } else {
        active.push_back({0, m, 0, 0});
    }
    while (!active.empty()) {
        segs.clear();
        tseg.clear();
        int64_t nt = 0;
        for (auto& s : active) {
            Seg q = s;
            q.tile0 = nt;
            const int64_t k = (s.len + QTE - 1) / QTE;
            for (int64_t i = 0; i < k; ++i) tseg.push_back((int32_t)segs.size());
            nt += k;
            segs.push_back(q);
        }
        SGQ_HIP(hipMemcpyAsync(d_segs, segs.data(), segs.size() * sizeof(Seg), hipMemcpyHostToDevice, st));
        SGQ_HIP(hipMemcpyAsync(d_tseg, tseg.data(), tseg.size() * 4, hipMemcpyHostToDevice, st));
        if (is_f32) hipLaunchKernelGGL(q_count<true>, dim3((unsigned)nt), dim3(QB), 0, st, cur, d_segs, d_tseg, d_cnt);
        else hipLaunchKernelGGL(q_count<false>, dim3((unsigned)nt), dim3(QB), 0, st, cur, d_segs, d_tseg, d_cnt);
        SGQ_HIP(hipGetLastError());
        hipLaunchKernelGGL(q_scan, dim3((unsigned)segs.size()), dim3(QB), 0, st, d_segs, d_cnt, d_off, d_tot);
        SGQ_HIP(hipGetLastError());
        if (is_f32)
            hipLaunchKernelGGL(q_scatter<true>, dim3((unsigned)nt), dim3(QB), 0, st, cur, nxt, dst, d_segs, d_tseg, d_off, d_tot);
        else
            hipLaunchKernelGGL(q_scatter<false>, dim3((unsigned)nt), dim3(QB), 0, st, cur, nxt, dst, d_segs, d_tseg, d_off, d_tot);
        SGQ_HIP(hipGetLastError());
        tots.resize(segs.size());
        SGQ_HIP(hipMemcpyAsync(tots.data(), d_tot, segs.size() * sizeof(ulonglong2), hipMemcpyDeviceToHost, st));
        SGQ_HIP(hipStreamSynchronize(st));
        std::vector<Seg> next;
        for (size_t i = 0; i < segs.size(); ++i) {
            const Seg& s = segs[i];
            const int64_t nL = (uint32_t)tots[i].x, nE = (uint32_t)(tots[i].x >> 32), nG = (uint32_t)tots[i].y;
            dropped_host += s.len - nL - nE - nG;
            const Seg kids[2] = {{s.start, nL, 0, 0}, {s.start + nL + nE, nG, 0, 0}};
            for (const Seg& k : kids) {
                if (k.len > QLEAF_N) next.push_back(k);
                else if (k.len >= 2) leaves.push_back({k.start, k.len, nxt});
            }
        }
        active.swap(next);
        cur = nxt;
        nxt = nxt == bufA ? bufB : bufA;
    }
    // Every leaf in one launch: a leaf's items stay where its level wrote them, since later
    // levels write only the ranges of the segments they partition, which are disjoint from it.
    if (!leaves.empty()) {
        SGQ_HIP(hipMemcpyAsync(d_leaf, leaves.data(), leaves.size() * sizeof(Leaf), hipMemcpyHostToDevice, st));
        const dim3 g((unsigned)leaves.size());
        if (is_f32) hipLaunchKernelGGL(q_leaf_net<true>, g, dim3(QB), 0, st, dst, d_leaf, d_nanl, d_nanc);
        else hipLaunchKernelGGL(q_leaf_net<false>, g, dim3(QB), 0, st, dst, d_leaf, d_nanl, d_nanc);
        SGQ_HIP(hipGetLastError());
        // the leaves holding a NaN run the listing's recursion (the order of the list is free:
        // each leaf writes only its own range)
        uint32_t nanc = 0;
        SGQ_HIP(hipMemcpyAsync(&nanc, d_nanc, 4, hipMemcpyDeviceToHost, st));
        SGQ_HIP(hipStreamSynchronize(st));
        if (nanc > 0) {
            if (is_f32) hipLaunchKernelGGL(q_leaf<true>, dim3(nanc), dim3(QB), 0, st, dst, d_leaf, d_nanl, d_drop);
            else hipLaunchKernelGGL(q_leaf<false>, dim3(nanc), dim3(QB), 0, st, dst, d_leaf, d_nanl, d_drop);
            SGQ_HIP(hipGetLastError());
        }
    }
    unsigned long long dleaf = 0;
    SGQ_HIP(hipMemcpyAsync(&dleaf, d_drop, 8, hipMemcpyDeviceToHost, st));
    SGQ_HIP(hipStreamSynchronize(st));
    const int64_t dropped = dropped_host + (int64_t)dleaf;
    if (dropped > 0) {
        // stable removal of the markers of dropped items: counts per tile, host prefix, scatter
        const int64_t tiles = (m + QTE - 1) / QTE;
        std::vector<uint32_t> cnt(tiles);
        std::vector<int64_t> off(tiles);
        SGQ_HIP(hipMemcpyAsync(bufA, dst, (size_t)m * 4, hipMemcpyDeviceToDevice, st));
        hipLaunchKernelGGL(q_keep_count, dim3((unsigned)tiles), dim3(QB), 0, st, bufA, m, (uint32_t*)d_cnt);
        SGQ_HIP(hipGetLastError());
        SGQ_HIP(hipMemcpyAsync(cnt.data(), d_cnt, tiles * 4, hipMemcpyDeviceToHost, st));
        SGQ_HIP(hipStreamSynchronize(st));
        int64_t run = 0;
        for (int64_t i = 0; i < tiles; ++i) { off[i] = run; run += cnt[i]; }
        SGQ_HIP(hipMemcpyAsync(d_cnt, off.data(), tiles * 8, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(q_keep_scatter, dim3((unsigned)tiles), dim3(QB), 0, st, bufA, m, (const int64_t*)d_cnt, dst);
        SGQ_HIP(hipGetLastError());
        SGQ_HIP(hipStreamSynchronize(st));
        if (run != m - dropped) return done(fail(ctx, SG_E_DEVICE, "quicksort: dropped-item accounting disagrees"));
    }
#undef SGQ_HIP
    *count = m - dropped;
    return done(SG_OK);
}

}  // namespace sgrt
