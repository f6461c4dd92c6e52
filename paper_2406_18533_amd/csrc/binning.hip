// Z-buffer construction (appendix A.2): per-tile depth-ordered instance lists.
//
// The order is lexicographic in (global tile, FP32 depth bits, Gaussian
// index). It is produced as a least-significant-digit-first radix sort whose
// low digits (depth) are sorted BEFORE the instances are duplicated per tile,
// and whose most significant digit, the view, is never sorted at all: every
// step keeps the views in their own contiguous segments.
//   1. compact the (view, Gaussian) pairs that touch at least one tile,
//      keeping (view-major, index) order;
//   2. stable radix sort of each view's pairs by FP32 depth bits (4 passes);
//   3. exclusive scan of their tile counts in that order -> instance offsets;
//   4. emit (tile, Gaussian index) per tile of each pair's rectangle
//      (grouped by view, since the pairs are);
//   5. stable radix sort of each view's instances by tile within the view
//      (13 bits, two passes, for a 1920x1080 view; 2-byte keys while a view
//      has at most 2^16 tiles, the last pass writing the global tile ids).
// Stability of step 5 keeps step 2's (depth, index) order inside each tile.
// Only step 5 runs over the duplicated instances, so the wide depth digits
// cost passes over the pairs, not over the (typically 5-10x larger)
// instance set, and its key is the tile within the view, not the global tile.
#include "common.hpp"

namespace gs {

constexpr int SB = 256;          // threads per block in the scan / sort kernels
constexpr int SITEMS = 16;       // items per thread
constexpr int STILE = SB * SITEMS;

__device__ __forceinline__ int64_t count_of(const int64_t *n_dev, int64_t n_max)
{
    if (!n_dev) return n_max;
    int64_t n = *n_dev;
    return n < n_max ? n : n_max;
}

template <typename U> __device__ __forceinline__ U wave_incl_scan(U x)
{
    int lane = threadIdx.x & 63;
    for (int off = 1; off < 64; off <<= 1) {
        U y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// Exclusive scan across the 256 threads of a block; `total` gets the sum.
template <typename U> __device__ __forceinline__ U block_excl_scan(U x, U &total)
{
    __shared__ U s_w[SB / 64];
    U inc = wave_incl_scan(x);
    int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    U off = 0;
    total = 0;
    for (int j = 0; j < SB / 64; j++) {
        U t = s_w[j];
        if (j < w) off += t;
        total += t;
    }
    __syncthreads();
    return off + inc - x;
}

// ---------------------------------------------------------------- generic scan
template <typename U, typename Load>
__global__ void __launch_bounds__(SB) scan_reduce_kernel(Load load, const int64_t *n_dev, int64_t n_max, U *partial)
{
    int64_t n = count_of(n_dev, n_max);
    int64_t base = (int64_t)blockIdx.x * STILE;
    U acc = 0;
    for (int j = 0; j < SITEMS; j++) {
        int64_t idx = base + (int64_t)j * SB + threadIdx.x;
        if (idx < n) acc += load(idx);
    }
    U total;
    block_excl_scan(acc, total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// LDS slot of item i of a 4096-item tile: one pad word per 32 items keeps
// the per-thread (blocked) accesses off a single bank.
__device__ __forceinline__ int pad_slot(int i) { return i + (i >> 5); }

// Second pass of the scan: each block adds up the sums of the blocks before
// it (its offset; block 0 also writes the grand total), scans its tile of
// 4096 items and stores the exclusive prefix of every item. Items are loaded
// and stored coalesced (item j*256 + thread of the tile) and transposed
// through LDS to the blocked order the scan needs.
template <typename U, typename Load, typename Store>
__global__ void __launch_bounds__(SB) scan_down_kernel(Load load, Store store, const int64_t *n_dev, int64_t n_max,
                                                       const U *partial, int64_t nb, int64_t *total_out)
{
    __shared__ U sm[STILE + STILE / 32];
    int64_t n = count_of(n_dev, n_max);
    int64_t base = (int64_t)blockIdx.x * STILE;
    if (blockIdx.x == 0 && total_out) {               // block-uniform
        U a = 0;
        for (int64_t j = threadIdx.x; j < nb; j += SB) a += partial[j];
        U all;
        block_excl_scan(a, all);
        if (threadIdx.x == 0) *total_out = (int64_t)all;
    }
    if (base >= n) return;
    U boff;                                           // sum of the blocks before this one
    {
        U a = 0;
        for (int64_t j = threadIdx.x; j < (int64_t)blockIdx.x; j += SB) a += partial[j];
        block_excl_scan(a, boff);
    }
    for (int j = 0; j < SITEMS; j++) {
        int i = j * SB + threadIdx.x;
        sm[pad_slot(i)] = base + i < n ? load(base + i) : U(0);
    }
    __syncthreads();
    U vals[SITEMS];
    U acc = 0;
    for (int j = 0; j < SITEMS; j++) {
        vals[j] = sm[pad_slot(threadIdx.x * SITEMS + j)];
        acc += vals[j];
    }
    U total;
    U run = block_excl_scan(acc, total) + boff;                  // (synchronises the block)
    for (int j = 0; j < SITEMS; j++) {
        sm[pad_slot(threadIdx.x * SITEMS + j)] = run;             // exclusive prefix, in place
        run += vals[j];
    }
    __syncthreads();
    U end = boff + total;
    for (int j = 0; j < SITEMS; j++) {
        int i = j * SB + threadIdx.x;
        if (base + i >= n) break;
        U pre = sm[pad_slot(i)];
        U nxt = i + 1 < STILE ? sm[pad_slot(i + 1)] : end;
        store(base + i, pre, (U)(nxt - pre));
    }
}

template <typename U, typename Load, typename Store>
static hipError_t device_scan(Load load, Store store, const int64_t *n_dev, int64_t n_max, U *partial,
                              int64_t *total_out, hipStream_t s)
{
    int64_t nb = (n_max + STILE - 1) / STILE;
    if (nb == 0) nb = 1;
    hipLaunchKernelGGL((scan_reduce_kernel<U, Load>), dim3((unsigned)nb), dim3(SB), 0, s, load, n_dev, n_max, partial);
    hipLaunchKernelGGL((scan_down_kernel<U, Load, Store>), dim3((unsigned)nb), dim3(SB), 0, s, load, store, n_dev,
                       n_max, (const U *)partial, nb, total_out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- functors
struct FlagLoad {
    const uint32_t *tiles;
    __device__ uint32_t operator()(int64_t f) const { return tiles[f] > 0u ? 1u : 0u; }
};

struct CompactStore {
    const uint32_t *depth;
    uint32_t *keys, *vals;
    __device__ void operator()(int64_t f, uint32_t pos, uint32_t flag) const
    {
        if (!flag) return;
        keys[pos] = depth[f];
        vals[pos] = (uint32_t)f;
    }
};

struct U32AsU64Load {
    const uint32_t *p;
    __device__ uint64_t operator()(int64_t j) const { return (uint64_t)p[j]; }
};

struct U64Store {
    uint64_t *out;
    __device__ void operator()(int64_t j, uint64_t pos, uint64_t) const { out[j] = pos; }
};

struct U32Load {
    const uint32_t *p;
    __device__ uint32_t operator()(int64_t j) const { return p[j]; }
};

struct U32Store {
    uint32_t *out;
    __device__ void operator()(int64_t j, uint32_t pos, uint32_t) const { out[j] = pos; }
};

// ---------------------------------------------------------------- radix sort
// View-segmented stable LSD radix sort of 32-bit (or, for tiles, 16-bit)
// keys with 32-bit values.
// The items of view v occupy [start[v], start[v + 1]) and a pass orders each
// view's items among themselves, by a digit of (key - base[v]): the views
// stay where they are. A block owns one 4096-item tile of one view (view v
// has tiles b0[v] .. b0[v + 1] - 1). A pass's histogram is laid out view
// first, then digit, then tile (entry RADIX b0[v] + d ntiles_v + t), so one
// exclusive scan over it gives every (view, digit, tile) its output offset.
struct SegPlan {
    int64_t start[MAXV + 1];
    int64_t b0[MAXV + 1];
    int64_t hist_n[10];   // histogram length RADIX b0[views] for RADIX = 2^bits
    uint32_t base[MAXV];
};

__device__ __forceinline__ void plan_finish(SegPlan *p, int views)
{
    int64_t b = 0;
    for (int v = 0; v < views; v++) {
        p->b0[v] = b;
        b += (p->start[v + 1] - p->start[v] + STILE - 1) / STILE;
    }
    p->b0[views] = b;
    for (int k = 0; k < 10; k++) p->hist_n[k] = b << k;
}

// Pair segments: the compacted pairs are in flat (view-major) order, so view
// v starts at the first flat index >= v n. One wavefront per view searches
// 64-ary: its lanes sample 64 evenly spaced entries of the current interval
// and a ballot narrows it 64-fold (four rounds for 16M pairs).
constexpr int PLAN_NT = 1024;

__global__ void __launch_bounds__(PLAN_NT) pair_plan_kernel(const uint32_t *__restrict__ flat, const int64_t *m_dev,
                                                            int64_t m_max, int64_t n, int views, SegPlan *plan)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t m = count_of(m_dev, m_max);
    for (int v = w; v < views; v += PLAN_NT / 64) {   // wave-uniform
        const uint64_t key = (uint64_t)v * (uint64_t)n;
        int64_t lo = 0, hi = m;                        // the answer lies in [lo, hi]
        while (lo < hi) {
            const int64_t step = (hi - lo + 63) / 64;
            const int64_t idx = lo + lane * step;
            const bool below = idx < hi && (uint64_t)flat[idx] < key;
            const int c = __popcll(__ballot(below));  // samples below the key: a prefix of the lanes
            if (c == 0) {
                hi = lo;
            } else {
                const int64_t nlo = lo + (int64_t)(c - 1) * step + 1;
                const int64_t nhi = lo + (int64_t)c * step < hi ? lo + (int64_t)c * step : hi;
                lo = nlo;
                hi = nhi;
            }
        }
        if (lane == 0) {
            plan->start[v] = lo;
            plan->base[v] = 0u;
        }
    }
    if (threadIdx.x == 0) plan->start[views] = m;
    __syncthreads();
    if (threadIdx.x == 0) plan_finish(plan, views);
}

// Instance segments: view v's instances start at the offset of its first
// pair (the emission keeps the pairs' view grouping); clipped to capacity.
__global__ void instance_plan_kernel(const SegPlan *__restrict__ pairs, const uint64_t *__restrict__ off,
                                     const int64_t *k_dev, int64_t cap, ViewTable vt, SegPlan *plan,
                                     int32_t *overflow)
{
    const int v = threadIdx.x, views = vt.nviews;
    int64_t K = *k_dev < cap ? *k_dev : cap;
    if (v == 0) *overflow = *k_dev > cap ? 1 : 0;
    const int64_t m = pairs->start[views];
    if (v < views) {
        int64_t j = pairs->start[v];
        int64_t st = j < m ? (int64_t)off[j] : K;
        plan->start[v] = st < K ? st : K;
        plan->base[v] = (uint32_t)vt.tile_base[v];
    }
    if (v == 0) plan->start[views] = K;
    __syncthreads();
    if (v == 0) plan_finish(plan, views);
}

// View and tile of block b (views are few: a uniform linear walk).
__device__ __forceinline__ int plan_view(const SegPlan *plan, int views, int64_t b)
{
    int v = 0;
    while (v + 1 < views && b >= plan->b0[v + 1]) v++;
    return v;
}

// Lanes with equal digits find each other with BITS ballots; their order
// inside the wave and the wave's running per-digit count give each element
// its rank among equal digits, in input order.
template <int BITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid)
{
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < BITS; b++) {
        bool bit = (d >> b) & 1u;
        uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
    }
    return peers;
}

// Keys are uint32 (FP32 depth bits, or global tile ids, whose digits are
// taken from key - base[v]) or, for the tile sort of views with at most 2^16
// tiles, uint16 tile ids within the view (LOCAL: base 0); the last pass of
// such a sort writes global ids (GLOBAL_OUT: key + base[v]).
template <int BITS, typename KI, bool LOCAL>
__global__ void __launch_bounds__(SB) seg_count_kernel(const KI *__restrict__ kin,
                                                       const SegPlan *__restrict__ plan, int views, int shift,
                                                       uint32_t *__restrict__ hist)
{
    constexpr int RADIX = 1 << BITS;
    __shared__ uint32_t s_cnt[SB / 64][RADIX];
    const int64_t b = blockIdx.x;
    if (b >= plan->b0[views]) return;
    const int v = plan_view(plan, views, b);
    const int64_t t = b - plan->b0[v], nt = plan->b0[v + 1] - plan->b0[v];
    const int64_t beg = plan->start[v] + t * STILE;
    const int64_t end = plan->start[v + 1] < beg + STILE ? plan->start[v + 1] : beg + STILE;
    const uint32_t kb = LOCAL ? 0u : plan->base[v];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int d = threadIdx.x; d < RADIX * (SB / 64); d += SB) (&s_cnt[0][0])[d] = 0;
    __syncthreads();
    const int64_t i0 = beg + (int64_t)w * (SITEMS * 64) + lane;
    uint32_t kk[SITEMS];
    for (int it = 0; it < SITEMS; it++) {          // all loads of the tile in flight at once
        int64_t idx = i0 + it * 64;
        kk[it] = idx < end ? (uint32_t)kin[idx] : 0u;
    }
    for (int it = 0; it < SITEMS; it++)             // counts only: LDS atomics, no ranks needed
        if (i0 + it * 64 < end) atomicAdd(&s_cnt[w][((kk[it] - kb) >> shift) & (RADIX - 1)], 1u);
    __syncthreads();
    for (int d = threadIdx.x; d < RADIX; d += SB) {
        uint32_t c = 0;
        for (int j = 0; j < SB / 64; j++) c += s_cnt[j][d];
        hist[RADIX * plan->b0[v] + d * nt + t] = c;
    }
}

template <int BITS, typename KI, typename KO, bool LOCAL, bool GLOBAL_OUT>
__global__ void __launch_bounds__(SB) seg_scatter_kernel(const KI *__restrict__ kin,
                                                         const uint32_t *__restrict__ vin,
                                                         KO *__restrict__ kout, uint32_t *__restrict__ vout,
                                                         const SegPlan *__restrict__ plan, int views, int shift,
                                                         const uint32_t *__restrict__ offs)
{
    constexpr int RADIX = 1 << BITS;
    constexpr int PER = (RADIX + SB - 1) / SB;
    __shared__ uint32_t s_key[STILE];
    __shared__ uint32_t s_val[STILE];
    __shared__ uint32_t s_cnt[SB / 64][RADIX];
    __shared__ uint32_t s_start[RADIX];
    __shared__ uint32_t s_goff[RADIX];
    const int64_t b = blockIdx.x;
    if (b >= plan->b0[views]) return;
    const int v = plan_view(plan, views, b);
    const int64_t t = b - plan->b0[v], nt = plan->b0[v + 1] - plan->b0[v];
    const int64_t beg = plan->start[v] + t * STILE;
    const int64_t end = plan->start[v + 1] < beg + STILE ? plan->start[v + 1] : beg + STILE;
    const uint32_t kb = LOCAL ? 0u : plan->base[v];
    const uint32_t kout_add = GLOBAL_OUT ? plan->base[v] : 0u;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int d = threadIdx.x; d < RADIX; d += SB) s_goff[d] = offs[RADIX * plan->b0[v] + d * nt + t];
    for (int d = threadIdx.x; d < RADIX * (SB / 64); d += SB) (&s_cnt[0][0])[d] = 0;
    const uint64_t lt = (1ull << lane) - 1ull;
    const int64_t i0 = beg + (int64_t)w * (SITEMS * 64) + lane;
    uint32_t key[SITEMS], val[SITEMS], rank[SITEMS];
    for (int it = 0; it < SITEMS; it++) {          // all loads of the tile in flight at once
        int64_t idx = i0 + it * 64;
        key[it] = idx < end ? (uint32_t)kin[idx] : 0u;
        val[it] = idx < end ? vin[idx] : 0u;
    }
    __syncthreads();
    for (int it = 0; it < SITEMS; it++) {
        bool valid = i0 + it * 64 < end;
        uint32_t d = ((key[it] - kb) >> shift) & (RADIX - 1);
        uint64_t peers = match_digit<BITS>(d, valid);
        uint32_t before = s_cnt[w][d];
        if (valid && (peers & lt) == 0) s_cnt[w][d] = before + (uint32_t)__popcll(peers);
        rank[it] = before + (uint32_t)__popcll(peers & lt);
    }
    __syncthreads();
    // wave prefixes per digit, then tile-local digit starts
    uint32_t tot[PER];
    uint32_t mysum = 0;
    for (int j = 0; j < PER; j++) {
        int d = threadIdx.x * PER + j;
        uint32_t tt = 0;
        if (d < RADIX) {
            uint32_t run = 0;
            for (int q = 0; q < SB / 64; q++) {
                uint32_t c = s_cnt[q][d];
                s_cnt[q][d] = run;
                run += c;
            }
            tt = run;
        }
        tot[j] = tt;
        mysum += tt;
    }
    uint32_t total;
    uint32_t run = block_excl_scan(mysum, total);
    for (int j = 0; j < PER; j++) {
        int d = threadIdx.x * PER + j;
        if (d < RADIX) s_start[d] = run;
        run += tot[j];
    }
    __syncthreads();
    for (int it = 0; it < SITEMS; it++) {
        if (i0 + it * 64 < end) {
            uint32_t d = ((key[it] - kb) >> shift) & (RADIX - 1);
            uint32_t pos = s_start[d] + s_cnt[w][d] + rank[it];
            s_key[pos] = key[it];
            s_val[pos] = val[it];
        }
    }
    __syncthreads();
    const int cnt = (int)(end - beg);
    for (int q = threadIdx.x; q < cnt; q += SB) {
        uint32_t k = s_key[q];
        uint32_t d = ((k - kb) >> shift) & (RADIX - 1);
        int64_t g = (int64_t)s_goff[d] + (q - (int64_t)s_start[d]);
        kout[g] = (KO)(k + kout_add);
        vout[g] = s_val[q];
    }
}

template <int BITS, typename KI, typename KO, bool LOCAL, bool GLOBAL_OUT>
static void seg_pass(const KI *kin, const uint32_t *vin, KO *ko, uint32_t *vo, const SegPlan *plan, int views,
                     int64_t nbmax, int shift, uint32_t *hist, uint32_t *partial, hipStream_t s)
{
    constexpr int RADIX = 1 << BITS;
    hipLaunchKernelGGL((seg_count_kernel<BITS, KI, LOCAL>), dim3((unsigned)nbmax), dim3(SB), 0, s, kin, plan, views,
                       shift, hist);
    (void)device_scan<uint32_t>(U32Load{hist}, U32Store{hist}, &plan->hist_n[BITS], (int64_t)RADIX * nbmax, partial,
                                nullptr, s);
    hipLaunchKernelGGL((seg_scatter_kernel<BITS, KI, KO, LOCAL, GLOBAL_OUT>), dim3((unsigned)nbmax), dim3(SB), 0, s, kin,
                       vin, ko, vo, plan, views, shift, (const uint32_t *)hist);
}

template <typename KI, typename KO, bool LOCAL, bool GLOBAL_OUT>
static void seg_pass_w(int width, const KI *kin, const uint32_t *vin, KO *ko, uint32_t *vo, const SegPlan *plan,
                       int views, int64_t nbmax, int shift, uint32_t *hist, uint32_t *partial, hipStream_t s)
{
    switch (width) {
    case 1: seg_pass<1, KI, KO, LOCAL, GLOBAL_OUT>(kin, vin, ko, vo, plan, views, nbmax, shift, hist, partial, s); break;
    case 2: seg_pass<2, KI, KO, LOCAL, GLOBAL_OUT>(kin, vin, ko, vo, plan, views, nbmax, shift, hist, partial, s); break;
    case 3: seg_pass<3, KI, KO, LOCAL, GLOBAL_OUT>(kin, vin, ko, vo, plan, views, nbmax, shift, hist, partial, s); break;
    case 4: seg_pass<4, KI, KO, LOCAL, GLOBAL_OUT>(kin, vin, ko, vo, plan, views, nbmax, shift, hist, partial, s); break;
    case 5: seg_pass<5, KI, KO, LOCAL, GLOBAL_OUT>(kin, vin, ko, vo, plan, views, nbmax, shift, hist, partial, s); break;
    case 6: seg_pass<6, KI, KO, LOCAL, GLOBAL_OUT>(kin, vin, ko, vo, plan, views, nbmax, shift, hist, partial, s); break;
    case 7: seg_pass<7, KI, KO, LOCAL, GLOBAL_OUT>(kin, vin, ko, vo, plan, views, nbmax, shift, hist, partial, s); break;
    default: seg_pass<8, KI, KO, LOCAL, GLOBAL_OUT>(kin, vin, ko, vo, plan, views, nbmax, shift, hist, partial, s); break;
    }
}

// Passes of a sort over the lowest `bits` key bits: digits of at most 8 bits,
// as even in width as possible.
static int seg_passes(int bits) { return bits < 1 ? 1 : (bits + 7) / 8; }

// Sorts (keys, vals) within each view segment over the lowest `bits` bits of
// key - base[v]. The result lands in keys/vals after an even number of
// passes and in kalt/valt after an odd one. n_max bounds the item count.
static hipError_t seg_radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *kalt, uint32_t *valt,
                                 const SegPlan *plan, int views, int64_t n_max, int bits, uint32_t *hist,
                                 uint32_t *partial, hipStream_t s)
{
    if (n_max == 0) return hipSuccess;
    const int64_t nbmax = (n_max + STILE - 1) / STILE + views;   // sum over views of ceil(count / STILE)
    if (bits < 1) bits = 1;
    const int passes = seg_passes(bits);
    const int digit = (bits + passes - 1) / passes;
    // A narrower digit goes first: the later passes read input already
    // ordered by the lower digits, where a block's items fall into long runs
    // per digit and a wide digit costs less (measured on tile sorts).
    const int first = bits - (passes - 1) * digit;
    uint32_t *kin = keys, *vin = vals, *ko = kalt, *vo = valt;
    for (int p = 0; p < passes; p++) {
        const int shift = p == 0 ? 0 : first + (p - 1) * digit;
        const int width = p == 0 ? first : digit;
        seg_pass_w<uint32_t, uint32_t, false, false>(width, kin, vin, ko, vo, plan, views, nbmax, shift, hist, partial,
                                                     s);
        uint32_t *tk = kin, *tv = vin;
        kin = ko; vin = vo; ko = tk; vo = tv;
    }
    return hipGetLastError();
}

// Tile sort with 16-bit keys (tiles within the view, at most 2^16 per view):
// the passes carry 2-byte keys between k16a and k16b and the values between
// their buffers; the last pass writes the global tile ids to tile_out and
// the values to val_out. The emission wrote (k16a, val_in); val_in is val_out
// for an even pass count and val_alt for an odd one, so the values end in
// val_out.
static hipError_t seg_tile_sort16(uint16_t *k16a, uint16_t *k16b, uint32_t *val_in, uint32_t *val_other,
                                  uint32_t *tile_out, uint32_t *val_out, const SegPlan *plan, int views, int64_t n_max,
                                  int bits, uint32_t *hist, uint32_t *partial, hipStream_t s)
{
    if (n_max == 0) return hipSuccess;
    const int64_t nbmax = (n_max + STILE - 1) / STILE + views;
    if (bits < 1) bits = 1;
    const int passes = seg_passes(bits);
    const int digit = (bits + passes - 1) / passes;
    const int first = bits - (passes - 1) * digit;   // narrower digit first, as above
    uint16_t *kin = k16a, *ko = k16b;
    uint32_t *vin = val_in, *vo = val_other;
    for (int p = 0; p < passes; p++) {
        const int shift = p == 0 ? 0 : first + (p - 1) * digit;
        const int width = p == 0 ? first : digit;
        if (p + 1 < passes) {
            seg_pass_w<uint16_t, uint16_t, true, false>(width, kin, vin, ko, vo, plan, views, nbmax, shift, hist,
                                                        partial, s);
            uint16_t *tk = kin; kin = ko; ko = tk;
            uint32_t *tv = vin; vin = vo; vo = tv;
        } else {
            seg_pass_w<uint16_t, uint32_t, true, true>(width, kin, vin, tile_out, val_out, plan, views, nbmax, shift,
                                                       hist, partial, s);
        }
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- emit and ranges
// One block emits the instances of 256 consecutive depth-sorted pairs. Their
// first-instance offsets (relative to the block's first instance) and tile
// rectangles go to LDS; each wavefront then writes a contiguous quarter of
// the block's instances, 64 at a time (coalesced). A wavefront finds the
// pair of its first instance by binary search once; inside a window of 64
// instances the pairs that start there are flagged in LDS, and each lane's
// pair is the window's first pair plus the flags at or below its lane
// (ballot + mbcnt). The tile follows from the position inside the pair's
// rectangle: row = floor((local + 1/2) / width) through a float reciprocal,
// exact because a view has at most 2^22 tiles, so local + 1/2 < 2^22 keeps
// the rounding error (below (local + 1/2) 2^-23 / width) under the
// 1/(2 width) distance of the quotient from an integer.
// K = uint32_t: global tile ids; K = uint16_t: tile ids within the view.
template <typename K>
__global__ void __launch_bounds__(256) emit_kernel(const uint64_t *__restrict__ rects, int64_t n, ViewTable vt,
                                                   const uint32_t *__restrict__ flat, const uint64_t *__restrict__ off,
                                                   const int64_t *m_dev, int64_t m_max, const int64_t *k_dev,
                                                   K *__restrict__ tile_out, uint32_t *__restrict__ id_out,
                                                   int64_t capacity)
{
    constexpr bool LOCAL = sizeof(K) == 2;
    __shared__ uint32_t s_off[256], s_xy[256], s_w[256], s_base[256], s_tx[256], s_id[256];
    __shared__ float s_rw[256];
    __shared__ uint32_t s_end;
    __shared__ uint8_t s_start[4][64];
    int64_t m = count_of(m_dev, m_max);
    int64_t j0 = (int64_t)blockIdx.x * 256;
    if (j0 >= m) return;
    int64_t j = j0 + threadIdx.x;
    int cnt = (int)(m - j0 < 256 ? m - j0 : 256);
    uint64_t e_beg = off[j0];
    if (j < m) {
        uint32_t f = flat[j];
        uint32_t v = f / (uint32_t)n;
        uint32_t i = f - v * (uint32_t)n;
        uint64_t r = rects[j];                       // x0, x1, y0, y1 in 16-bit fields
        uint32_t x0 = (uint32_t)(r & 0xffffu), x1 = (uint32_t)((r >> 16) & 0xffffu);
        uint32_t y0 = (uint32_t)((r >> 32) & 0xffffu);
        uint32_t w = x1 - x0 + 1;
        s_off[threadIdx.x] = (uint32_t)(off[j] - e_beg);
        s_xy[threadIdx.x] = x0 | (y0 << 16);
        s_w[threadIdx.x] = w;
        s_rw[threadIdx.x] = 1.0f / (float)w;
        s_base[threadIdx.x] = (uint32_t)vt.tile_base[v];
        s_tx[threadIdx.x] = (uint32_t)vt.tiles_x[v];
        s_id[threadIdx.x] = i;
    }
    if (threadIdx.x == 0) s_end = (uint32_t)(((j0 + 256 < m) ? off[j0 + 256] : (uint64_t)*k_dev) - e_beg);
    __syncthreads();
    uint64_t e_end = e_beg + s_end;
    if (e_end > (uint64_t)capacity) e_end = (uint64_t)capacity;
    if (e_end <= e_beg) return;
    uint32_t tot = (uint32_t)(e_end - e_beg);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t per = ((tot + 3) / 4 + 63) & ~63u;   // whole windows per wavefront
    uint32_t a = (uint32_t)w * per;
    uint32_t b = min(a + per, tot);
    if (a >= b) return;                            // wave-uniform
    int lo = 0, hi = cnt - 1;                      // last pair starting at or before a
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (s_off[mid] <= a) lo = mid;
        else hi = mid - 1;
    }
    int p = lo;   // every pair after p starts at or after the current window
    for (uint32_t e0 = a; e0 < b; e0 += 64) {
        int q = p + 1 + lane;
        uint32_t st = q < cnt ? s_off[q] : 0xffffffffu;
        s_start[w][lane] = 0;
        __builtin_amdgcn_wave_barrier();
        if (st - e0 < 64u) s_start[w][st - e0] = 1;   // pairs have distinct starts (each has >= 1 instance)
        __builtin_amdgcn_wave_barrier();
        uint32_t fl = s_start[w][lane];
        uint64_t mask = __ballot(fl != 0);
        uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        int pr = p + (int)(below + fl);            // pair of instance e0 + lane
        uint32_t e = e0 + (uint32_t)lane;
        if (e < b) {
            uint32_t local = e - s_off[pr];
            uint32_t wd = s_w[pr];
            uint32_t dy = (uint32_t)(((float)local + 0.5f) * s_rw[pr]);
            uint32_t dx = local - dy * wd;
            uint32_t xy = s_xy[pr];
            const uint32_t lt = ((xy >> 16) + dy) * s_tx[pr] + (xy & 0xffffu) + dx;   // tile within the view
            tile_out[e_beg + e] = (K)(LOCAL ? lt : s_base[pr] + lt);
            id_out[e_beg + e] = s_id[pr];
        }
        p = __shfl(pr, 63, 64);
        __builtin_amdgcn_wave_barrier();
    }
}

// Tile rectangles and tile counts of the visible pairs in depth order (one
// gather, so the offsets scan and the emission read them coalesced).
__global__ void gather_rects_kernel(const uint64_t *__restrict__ rects, const uint32_t *__restrict__ flat,
                                    const int64_t *m_dev, int64_t m_max, uint32_t *__restrict__ count_out,
                                    uint64_t *__restrict__ rect_out)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count_of(m_dev, m_max)) return;
    uint64_t r = rects[flat[j]];
    uint32_t x0 = (uint32_t)(r & 0xffffu), x1 = (uint32_t)((r >> 16) & 0xffffu);
    uint32_t y0 = (uint32_t)((r >> 32) & 0xffffu), y1 = (uint32_t)(r >> 48);
    count_out[j] = (x1 - x0 + 1) * (y1 - y0 + 1);
    rect_out[j] = r;
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t value)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) p[j] = value;
}

// Start and end of every tile's run in the sorted keys by binary search: a
// thread per tile finds the first key not below its tile; the run ends where
// the next tile's begins (the neighbouring lane's result; the last lane of a
// wavefront searches once more). An empty run is written as [0, 0).
__device__ __forceinline__ uint32_t first_not_below(const uint32_t *__restrict__ keys, uint32_t K, uint32_t x)
{
    uint32_t lo = 0, n = K;
    while (n > 0) {
        const uint32_t h = n >> 1;
        if (keys[lo + h] < x) {
            lo += h + 1;
            n -= h + 1;
        } else {
            n = h;
        }
    }
    return lo;
}

__global__ void __launch_bounds__(256) ranges_search_kernel(const uint32_t *__restrict__ tiles, const int64_t *k_dev,
                                                            int64_t cap, int64_t n_tiles, uint32_t *__restrict__ ranges)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const uint32_t K = (uint32_t)count_of(k_dev, cap);
    const uint32_t st = t < n_tiles ? first_not_below(tiles, K, (uint32_t)t) : K;
    uint32_t en = __shfl_down(st, 1, 64);
    if ((threadIdx.x & 63) == 63 && t < n_tiles) en = first_not_below(tiles, K, (uint32_t)(t + 1));
    if (t < n_tiles) {
        const bool any = en > st;
        ranges[2 * t] = any ? st : 0u;
        ranges[2 * t + 1] = any ? en : 0u;
    }
}

__global__ void overflow_kernel(const int64_t *k_dev, int64_t cap, int32_t *overflow)
{
    *overflow = *k_dev > cap ? 1 : 0;
}

template <typename T>
__global__ void keys64_kernel(const T *__restrict__ proj, int64_t n, ViewTable vt, const uint32_t *tiles,
                              const uint32_t *ids, const int64_t *k_dev, int64_t cap, uint64_t *out)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count_of(k_dev, cap)) return;
    uint32_t t = tiles[k];
    int v = view_of_tile(vt, (int32_t)t);
    const uint32_t *depth = side_depth<T>(proj, (int64_t)vt.nviews * n);
    out[k] = ((uint64_t)t << 32) | (uint64_t)depth[(int64_t)v * n + ids[k]];
}

// ---------------------------------------------------------------- workspace
struct BinWS {
    uint32_t *k1, *v1, *k1b, *v1b;   // [VN] depth keys / flat indices and alternates
    uint64_t *off;                   // [VN] instance offsets
    uint64_t *rect;                  // [VN] tile rectangles of the visible pairs in depth order
    uint32_t *talt, *ialt;           // [cap] alternate tile keys / ids
    uint32_t *hist;                  // [256 * nbmax] radix histograms
    uint64_t *partial;               // scan partials
    int64_t *m_dev;                  // visible pair count
    SegPlan *pplan, *iplan;          // view segments of the pairs and of the instances
};

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

size_t bin_ws_layout(int64_t vn, int64_t cap, char *base, BinWS *ws)
{
    int64_t big = vn > cap ? vn : cap;
    int64_t nbmax = (big + STILE - 1) / STILE + MAXV;
    int64_t hist_n = 256 * nbmax;
    int64_t part_n = (hist_n + STILE - 1) / STILE + (big + STILE - 1) / STILE + 8;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return base ? (void *)(base + at) : nullptr; };
    BinWS w;
    w.k1 = (uint32_t *)take(4 * vn);
    w.v1 = (uint32_t *)take(4 * vn);
    w.k1b = (uint32_t *)take(4 * vn);
    w.v1b = (uint32_t *)take(4 * vn);
    w.off = (uint64_t *)take(8 * vn);
    w.rect = (uint64_t *)take(8 * vn);
    w.talt = (uint32_t *)take(4 * cap);
    w.ialt = (uint32_t *)take(4 * cap);
    w.hist = (uint32_t *)take(4 * hist_n);
    w.partial = (uint64_t *)take(8 * part_n);
    w.m_dev = (int64_t *)take(64);
    w.pplan = (SegPlan *)take(sizeof(SegPlan));
    w.iplan = (SegPlan *)take(sizeof(SegPlan));
    if (ws) *ws = w;
    return o;
}

template <typename T>
hipError_t launch_bin_sort(const void *projv, int64_t n, const ViewTable &vt, gs_bins *b, bool check, int *capacity_err,
                           hipStream_t s)
{
    const T *proj = (const T *)projv;
    int64_t vn = (int64_t)vt.nviews * n;
    int64_t cap = b->capacity;
    BinWS ws;
    bin_ws_layout(vn, cap, (char *)b->workspace, &ws);
    hipError_t e;
    *capacity_err = 0;
    int64_t T_all = vt.total_tiles;
    // ranges start empty
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((2 * T_all + 255) / 256)), dim3(256), 0, s, b->ranges,
                       2 * T_all, 0u);
    const uint32_t *tiles = side_tiles<T>(proj, vn), *depth = side_depth<T>(proj, vn);
    // 1. compaction of pairs that touch a tile
    e = device_scan<uint32_t>(FlagLoad{tiles}, CompactStore{depth, ws.k1, ws.v1}, nullptr, vn,
                              (uint32_t *)ws.partial, ws.m_dev, s);
    if (e != hipSuccess) return e;
    if (vn > 0)
        hipLaunchKernelGGL(pair_plan_kernel, dim3(1), dim3(PLAN_NT), 0, s, (const uint32_t *)ws.v1,
                           (const int64_t *)ws.m_dev, vn, n, vt.nviews, ws.pplan);
    // 2. stable sort by FP32 depth bits within each view (4 passes: an even
    // count, so the result is back in k1 / v1)
    e = seg_radix_sort(ws.k1, ws.v1, ws.k1b, ws.v1b, ws.pplan, vt.nviews, vn, 32, ws.hist, (uint32_t *)ws.partial, s);
    if (e != hipSuccess) return e;
    // 3. instance offsets in depth order (the sorted depth keys are dead now:
    // their buffer holds the gathered tile counts)
    if (vn > 0)
        hipLaunchKernelGGL(gather_rects_kernel, dim3((unsigned)((vn + 255) / 256)), dim3(256), 0, s,
                           (const uint64_t *)side_rect<T>(proj, vn), (const uint32_t *)ws.v1,
                           (const int64_t *)ws.m_dev, vn, ws.k1, ws.rect);
    e = device_scan<uint64_t>(U32AsU64Load{ws.k1}, U64Store{ws.off}, ws.m_dev, vn, ws.partial, b->n_instances, s);
    if (e != hipSuccess) return e;
    if (vn == 0)   // (otherwise the instance plan writes the flag, or the capacity check below)
        hipLaunchKernelGGL(overflow_kernel, dim3(1), dim3(1), 0, s, (const int64_t *)b->n_instances, cap, b->overflow);
    if (check) {
        int64_t K = 0;
        e = hipMemcpyAsync(&K, b->n_instances, sizeof(int64_t), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (K > cap) {
            *capacity_err = 1;
            hipLaunchKernelGGL(overflow_kernel, dim3(1), dim3(1), 0, s, (const int64_t *)b->n_instances, cap,
                               b->overflow);
            return hipGetLastError();
        }
    }
    // 4. emission, grouped by view like the pairs; the tile passes are
    // arranged so the result lands in the caller's buffers
    int bits = 1;                                   // tile id within its view
    for (int v = 0; v < vt.nviews; v++)
        while ((int64_t(1) << bits) < (int64_t)(vt.tile_base[v + 1] - vt.tile_base[v])) bits++;
    const bool odd = seg_passes(bits) & 1;
    const dim3 eg((unsigned)((vn + 255) / 256)), eb(256);
    if (vn > 0 && bits <= 16) {
        // 2-byte tile keys within the view until the last pass, which writes
        // the global ids; both 2-byte key arrays fit in the alternate key buffer
        uint16_t *k16a = (uint16_t *)ws.talt, *k16b = k16a + cap;
        uint32_t *vin = odd ? ws.ialt : b->ids, *vother = odd ? b->ids : ws.ialt;
        hipLaunchKernelGGL(emit_kernel<uint16_t>, eg, eb, 0, s, (const uint64_t *)ws.rect, n, vt,
                           (const uint32_t *)ws.v1, (const uint64_t *)ws.off, (const int64_t *)ws.m_dev, vn,
                           (const int64_t *)b->n_instances, k16a, vin, cap);
        hipLaunchKernelGGL(instance_plan_kernel, dim3(1), dim3(MAXV), 0, s, (const SegPlan *)ws.pplan,
                           (const uint64_t *)ws.off, (const int64_t *)b->n_instances, cap, vt, ws.iplan, b->overflow);
        // 5. stable sort by tile within each view
        e = seg_tile_sort16(k16a, k16b, vin, vother, b->tile_keys, b->ids, ws.iplan, vt.nviews, cap, bits, ws.hist,
                            (uint32_t *)ws.partial, s);
        if (e != hipSuccess) return e;
    } else if (vn > 0) {
        uint32_t *ek = odd ? ws.talt : b->tile_keys, *ei = odd ? ws.ialt : b->ids;
        uint32_t *ak = odd ? b->tile_keys : ws.talt, *ai = odd ? b->ids : ws.ialt;
        hipLaunchKernelGGL(emit_kernel<uint32_t>, eg, eb, 0, s, (const uint64_t *)ws.rect, n, vt,
                           (const uint32_t *)ws.v1, (const uint64_t *)ws.off, (const int64_t *)ws.m_dev, vn,
                           (const int64_t *)b->n_instances, ek, ei, cap);
        hipLaunchKernelGGL(instance_plan_kernel, dim3(1), dim3(MAXV), 0, s, (const SegPlan *)ws.pplan,
                           (const uint64_t *)ws.off, (const int64_t *)b->n_instances, cap, vt, ws.iplan, b->overflow);
        // 5. stable sort by tile within each view
        e = seg_radix_sort(ek, ei, ak, ai, ws.iplan, vt.nviews, cap, bits, ws.hist, (uint32_t *)ws.partial, s);
        if (e != hipSuccess) return e;
    }
    if (cap > 0 && T_all > 0)
        hipLaunchKernelGGL(ranges_search_kernel, dim3((unsigned)((T_all + 255) / 256)), dim3(256), 0, s,
                           (const uint32_t *)b->tile_keys, (const int64_t *)b->n_instances, cap, T_all, b->ranges);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_keys64(const void *proj, int64_t n, const ViewTable &vt, const gs_bins *b, uint64_t *out,
                         hipStream_t s)
{
    int64_t cap = b->capacity;
    if (cap == 0) return hipSuccess;
    hipLaunchKernelGGL(keys64_kernel<T>, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, (const T *)proj, n, vt,
                       (const uint32_t *)b->tile_keys, (const uint32_t *)b->ids, (const int64_t *)b->n_instances, cap,
                       out);
    return hipGetLastError();
}

template hipError_t launch_bin_sort<float>(const void *, int64_t, const ViewTable &, gs_bins *, bool, int *, hipStream_t);
template hipError_t launch_bin_sort<double>(const void *, int64_t, const ViewTable &, gs_bins *, bool, int *,
                                            hipStream_t);
template hipError_t launch_keys64<float>(const void *, int64_t, const ViewTable &, const gs_bins *, uint64_t *,
                                         hipStream_t);
template hipError_t launch_keys64<double>(const void *, int64_t, const ViewTable &, const gs_bins *, uint64_t *,
                                          hipStream_t);

// ---------------------------------------------------------------- Algorithm 1
// Division points of the serialised tiles into Q cost-balanced chunks
// (Algorithm 1): CT = cumsum(ET) with ET_j = cost_j + 1 (a tile costs at
// least its fixed overhead), thresholds q * CT[last] / Q, DP[q] = first j
// with CT[j] >= threshold (left searchsorted), DP[Q] = T. Also resets the
// per-chunk cursors of the persistent render kernels.
struct CostLoad {
    const uint32_t *cost;
    __device__ uint64_t operator()(int64_t j) const { return (cost ? (uint64_t)cost[j] : 0ull) + 1ull; }
};

struct InclStore {
    uint64_t *ct;
    __device__ void operator()(int64_t j, uint64_t excl, uint64_t x) const { ct[j] = excl + x; }
};

__global__ void division_points_kernel(const uint64_t *__restrict__ ct, int32_t T_all, int32_t Q,
                                       int32_t *__restrict__ dp, int32_t *__restrict__ cursor,
                                       int32_t *__restrict__ dp_out)
{
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q > Q) return;
    int32_t r;
    if (q == Q) r = T_all;
    else {
        double th = (double)q * ((double)ct[T_all - 1] / (double)Q);
        int32_t lo = 0, hi = T_all;
        while (lo < hi) {
            int32_t mid = (lo + hi) >> 1;
            if ((double)ct[mid] < th) lo = mid + 1;
            else hi = mid;
        }
        r = lo;
    }
    dp[q] = r;
    if (q < Q) cursor[q] = r;
    if (dp_out) dp_out[q] = r;
}

hipError_t launch_plan(const uint32_t *cost, int32_t T_all, int32_t Q, uint64_t *ct, uint64_t *partial, int32_t *dp,
                       int32_t *cursor, int32_t *dp_out, hipStream_t s)
{
    if (T_all <= 0) return hipSuccess;
    hipError_t e = device_scan<uint64_t>(CostLoad{cost}, InclStore{ct}, nullptr, T_all, partial, nullptr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(division_points_kernel, dim3((unsigned)((Q + 256) / 256)), dim3(256), 0, s,
                       (const uint64_t *)ct, T_all, Q, dp, cursor, dp_out);
    return hipGetLastError();
}

// LPT order (longest processing time first): the tiles sorted by decreasing
// estimated cost, by a counting sort over LPT_BINS cost classes (4 per
// octave; an approximate order is all the greedy rule needs). With nseg > 1
// the tiles are first cut into nseg contiguous segments at the division
// points dp (Algorithm 1) and each segment is sorted in place, within its
// own range of the order. Within a class the order follows the arrival of
// the scatter's workgroups (roughly index order; the images do not depend
// on it).
__device__ __forceinline__ int lpt_bin(uint32_t c)
{
    int k = c == 0u ? 0 : 1 + (int)floorf(4.0f * __log2f((float)c));
    k = k < 0 ? 0 : (k > LPT_BINS - 1 ? LPT_BINS - 1 : k);
    return LPT_BINS - 1 - k;                       // class 0 = heaviest
}

__device__ __forceinline__ int lpt_seg(const int32_t *dp, int nseg, int32_t t)
{
    int sg = 0;
    for (int j = 1; j < nseg; j++) sg += t >= dp[j] ? 1 : 0;
    return sg;
}

__global__ void __launch_bounds__(256) lpt_hist_kernel(const uint32_t *__restrict__ cost, int32_t T_all,
                                                       const int32_t *__restrict__ dp, int nseg,
                                                       uint32_t *__restrict__ hist)
{
    __shared__ uint32_t h[LPT_SEGS * LPT_BINS];
    for (int j = threadIdx.x; j < nseg * LPT_BINS; j += 256) h[j] = 0u;
    __syncthreads();
    const int32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t < T_all) atomicAdd(&h[lpt_seg(dp, nseg, t) * LPT_BINS + lpt_bin(cost[t])], 1u);
    __syncthreads();
    for (int j = threadIdx.x; j < nseg * LPT_BINS; j += 256)
        if (h[j]) atomicAdd(&hist[j], h[j]);
}

// Exclusive prefix of each segment's class counts, heaviest class first,
// from the segment's first position (one block per segment). With head > 0
// only the heaviest classes that together hold at least `head` tiles keep
// their order; the classes after them form one bucket (cstar[segment] = the
// last ordered class), so the light tiles keep roughly their index order.
__global__ void __launch_bounds__(256) lpt_scan_kernel(const uint32_t *__restrict__ hist, const int32_t *__restrict__ dp,
                                                       uint32_t *__restrict__ cur, int32_t *__restrict__ cstar,
                                                       uint32_t head)
{
    __shared__ uint32_t v[256];
    __shared__ int cs;
    const int j = threadIdx.x, sg = blockIdx.x;
    const uint32_t hj = j < LPT_BINS ? hist[sg * LPT_BINS + j] : 0u;
    v[j] = hj;
    if (j == 0) cs = LPT_BINS - 1;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        uint32_t a = j >= o ? v[j - o] : 0u;
        __syncthreads();
        v[j] += a;
        __syncthreads();
    }
    if (head > 0u && j < LPT_BINS && v[j] >= head) atomicMin(&cs, j);
    __syncthreads();
    const uint32_t base = dp ? (uint32_t)dp[sg] : 0u;
    if (j < LPT_BINS && j <= cs) cur[sg * LPT_BINS + j] = base + v[j] - hj;
    if (j < LPT_BINS && j == cs + 1) cur[sg * LPT_BINS + j] = base + v[cs];   // the merged light bucket
    if (j == 0) cstar[sg] = cs;
}

__global__ void __launch_bounds__(256) lpt_scatter_kernel(const uint32_t *__restrict__ cost, int32_t T_all,
                                                          const int32_t *__restrict__ dp, int nseg,
                                                          uint32_t *__restrict__ cur, const int32_t *__restrict__ cstar,
                                                          int32_t *__restrict__ order)
{
    __shared__ uint32_t cnt[LPT_SEGS * LPT_BINS], base[LPT_SEGS * LPT_BINS];
    for (int j = threadIdx.x; j < nseg * LPT_BINS; j += 256) cnt[j] = 0u;
    __syncthreads();
    const int32_t t = blockIdx.x * 256 + threadIdx.x;
    int b = 0;
    uint32_t r = 0;
    if (t < T_all) {
        const int sg = lpt_seg(dp, nseg, t);
        b = sg * LPT_BINS + min(lpt_bin(cost[t]), cstar[sg] + 1);
        r = atomicAdd(&cnt[b], 1u);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < nseg * LPT_BINS; j += 256)
        if (cnt[j]) base[j] = atomicAdd(&cur[j], cnt[j]);
    __syncthreads();
    if (t < T_all) order[base[b] + r] = t;
}

hipError_t launch_lpt_plan(const uint32_t *cost, int32_t T_all, const int32_t *dp, int nseg, uint32_t head,
                           uint32_t *bins, int32_t *order, hipStream_t s)
{
    if (T_all <= 0) return hipSuccess;
    if (nseg < 1 || nseg > LPT_SEGS || (nseg > 1 && !dp)) return hipErrorInvalidValue;
    const unsigned g = (unsigned)((T_all + 255) / 256);
    const int64_t nb = (int64_t)nseg * LPT_BINS;
    int32_t *cstar = (int32_t *)(bins + 2 * (int64_t)LPT_SEGS * LPT_BINS);
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((2 * nb + 255) / 256)), dim3(256), 0, s, bins, 2 * nb, 0u);
    hipLaunchKernelGGL(lpt_hist_kernel, dim3(g), dim3(256), 0, s, cost, T_all, dp, nseg, bins);
    hipLaunchKernelGGL(lpt_scan_kernel, dim3((unsigned)nseg), dim3(256), 0, s, (const uint32_t *)bins,
                       nseg > 1 ? dp : nullptr, bins + nb, cstar, head);
    hipLaunchKernelGGL(lpt_scatter_kernel, dim3(g), dim3(256), 0, s, cost, T_all, dp, nseg, bins + nb,
                       (const int32_t *)cstar, order);
    return hipGetLastError();
}

// Exposed for the scheduler (cumulative tile cost).
hipError_t fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace gs
