// Device-side building blocks shared by the HIP kernels of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gs.h"

namespace gs {

constexpr int TILE = GS_TILE;
constexpr int MAXV = GS_MAX_VIEWS;
constexpr int LOSS_SUM_BLOCKS = 64;   // blocks of the fused loss's deterministic sum
constexpr int REC = GS_REC;

// Record slots of a projected (view, Gaussian) entry.
enum : int { R_U = 0, R_V = 1, R_A = 2, R_B = 3, R_C = 4, R_OPAC = 5, R_RGB = 6, R_RADIUS = 9, R_DEPTH = 10, R_TILES = 11 };
// Slots of a projected-gradient entry.
enum : int { D_U = 0, D_V = 1, D_A = 2, D_B = 3, D_C = 4, D_OPAC = 5, D_RGB = 6 };

// The projected buffer holds the [views][n][REC] records followed by three
// planar side arrays over the same (view, Gaussian) index: tiles touched
// (uint32), the FP32 bits of depth (uint32) and the touched tile rectangle
// (uint64: x0, x1, y0, y1 in 16-bit fields from the low end; 0 when no tile
// is touched). Binning and the backward read these fields contiguously
// instead of one field per record.
template <typename T> __host__ __device__ inline uint32_t *side_tiles(const void *proj, int64_t vn)
{
    return (uint32_t *)((char *)proj + vn * (int64_t)REC * (int64_t)sizeof(T));
}
template <typename T> __host__ __device__ inline uint32_t *side_depth(const void *proj, int64_t vn)
{
    return side_tiles<T>(proj, vn) + vn;
}
template <typename T> __host__ __device__ inline uint64_t *side_rect(const void *proj, int64_t vn)
{
    return (uint64_t *)(side_tiles<T>(proj, vn) + 2 * vn);   // 8-byte aligned: records and two uint32 arrays
}
__host__ __device__ inline uint64_t pack_rect(int x0, int x1, int y0, int y1)
{
    return (uint64_t)(uint16_t)x0 | ((uint64_t)(uint16_t)x1 << 16) | ((uint64_t)(uint16_t)y0 << 32) |
           ((uint64_t)(uint16_t)y1 << 48);
}

// Per-view image geometry, passed by value as a kernel argument.
struct ViewTable {
    int32_t nviews;
    int32_t total_tiles;
    int32_t tile_base[MAXV + 1];
    int32_t tiles_x[MAXV];
    int32_t width[MAXV];
    int32_t height[MAXV];
    int64_t pix_base[MAXV + 1];
};

ViewTable make_view_table(const gs_camera *cams, int32_t views);

// Deterministic sum of n per-tile loss shares into *loss: LOSS_SUM_BLOCKS
// block sums (written to bsum) in a fixed order, then one fixed tree.
hipError_t launch_tile_sum(const double *part, int64_t n, double *bsum, double *loss, hipStream_t s);

// Persistent-scheduler state inside the caller's workspace.
struct SchedState {
    int32_t *cursor;   // [queues] next tile of each queue
    int32_t *dp;       // [queues + 1] division points
    int32_t queues;    // multiple of 8
    int32_t *order;    // [total_tiles] tiles by decreasing estimated cost (LPT mode)
    uint32_t *bins;    // [2 * LPT_SEGS * LPT_BINS + LPT_SEGS] the LPT counting sort's histogram,
                       // cursors and last ordered class per segment
};

// Cost classes of the LPT order: 4 per octave of the estimated cost (a class
// spans a factor 2^(1/4) = 1.19), class 0 the heaviest; up to LPT_SEGS
// segments sorted separately (the XCD chunks of Algorithm 1).
constexpr int LPT_BINS = 136;
constexpr int LPT_SEGS = 8;
hipError_t launch_lpt_plan(const uint32_t *cost, int32_t T_all, const int32_t *dp, int nseg, uint32_t head,
                           uint32_t *bins, int32_t *order, hipStream_t s);

// Resolved launch shape of the render kernels.
struct LaunchShape {
    int mode, px, chunk, workers;
    SchedState S;
};

struct BinWS;

__device__ __forceinline__ int view_of_tile(const ViewTable &vt, int32_t g)
{
    int v = 0;
    while (v + 1 < vt.nviews && g >= vt.tile_base[v + 1]) v++;
    return v;
}

// Footprint rectangle in tiles, decided in FP32: pixels whose centre
// x + 1/2 lies in [u - r, u + r] (and likewise y), clipped to the image.
struct TileRect { int x0, x1, y0, y1; };

__device__ __forceinline__ bool tile_rect(float u, float v, float r, int W, int H, TileRect &t)
{
    if (!(r > 0.0f)) return false;
    float xlo = ceilf(__fsub_rn(__fsub_rn(u, r), 0.5f));
    float xhi = floorf(__fsub_rn(__fadd_rn(u, r), 0.5f));
    float ylo = ceilf(__fsub_rn(__fsub_rn(v, r), 0.5f));
    float yhi = floorf(__fsub_rn(__fadd_rn(v, r), 0.5f));
    xlo = fmaxf(xlo, 0.0f);
    ylo = fmaxf(ylo, 0.0f);
    xhi = fminf(xhi, (float)(W - 1));
    yhi = fminf(yhi, (float)(H - 1));
    if (!(xlo <= xhi) || !(ylo <= yhi)) return false;
    t.x0 = (int)xlo / TILE;
    t.x1 = (int)xhi / TILE;
    t.y0 = (int)ylo / TILE;
    t.y1 = (int)yhi / TILE;
    return true;
}

// Rasterizer constants (alpha clamp, skip threshold, transmittance stop).
template <typename T> struct K;
template <> struct K<float> {
    static constexpr float alpha_max = 0.99f;
    static constexpr float alpha_min = 1.0f / 255.0f;
    static constexpr float t_min = 1e-4f;
};
template <> struct K<double> {
    static constexpr double alpha_max = 0.99;
    static constexpr double alpha_min = 1.0 / 255.0;
    static constexpr double t_min = 1e-4;
};

__device__ __forceinline__ float exp2_t(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double exp2_t(double x) { return exp2(x); }

// Conic pre-scaled for the per-pixel exponent: with (na, nb, nc) =
// -(a/2, b, c/2) log2(e), the Gaussian falloff exp(-(a dx^2 + c dy^2)/2 -
// b dx dy) is exp2(na dx^2 + nb dx dy + nc dy^2).
template <typename T> __device__ __forceinline__ void scaled_conic(T a, T b, T c, T &na, T &nb, T &nc)
{
    const T l2e = T(1.4426950408889634);
    na = T(-0.5) * l2e * a;
    nb = -l2e * b;
    nc = T(-0.5) * l2e * c;
}

// Falloff terms that depend on the pixel column only. Every pixel a thread
// owns sits in the same column of the tile, so these are computed once per
// (thread, Gaussian) and shared by the thread's pixels.
template <typename T> struct ColTerms {
    T dx, dx2, qx, nbdx;   // offset, offset^2, na*offset^2, nb*offset
};

template <typename T> __device__ __forceinline__ ColTerms<T> col_terms(T pxc, T u, T na, T nb)
{
    ColTerms<T> c;
    c.dx = pxc - u;
    c.dx2 = c.dx * c.dx;
    c.qx = na * c.dx2;
    c.nbdx = nb * c.dx;
    return c;
}

// One (pixel, Gaussian) pair, evaluated without branches: row offset dy,
// falloff G, opacity times falloff og, alpha = min(0.99, og), and whether
// the pair counts (centre inside the radius circle, alpha >= 1/255). The
// exponent is qx + dy (nb dx + nc dy) in log2 units. Its sign test (skip a
// pair with a positive exponent) is left out: the conic is positive
// definite, so the exponent is positive only by rounding, within a few ulps
// of the sum of its terms' magnitudes, where G rounds to 1 as it does at
// the centre.
// Invalid lanes may hold inf or NaN in G/og/alpha; callers select on `ok`,
// never multiply by it. The forward and backward kernels both call this, so
// their decisions agree bit for bit.
template <typename T>
__device__ __forceinline__ bool eval_alpha(const ColTerms<T> &c, T pyc, T v, T r2, T nc, T o,
                                           T &dy, T &G, T &og, T &alpha)
{
    dy = pyc - v;
    T d2 = fma(dy, dy, c.dx2);
    T p2 = fma(dy, fma(nc, dy, c.nbdx), c.qx);
    G = exp2_t(p2);
    og = o * G;
    alpha = fmin(og, K<T>::alpha_max);
    return (d2 <= r2) & (alpha >= K<T>::alpha_min);
}

__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_t(double x) { return 1.0 / x; }
// 1 / sqrt(x): the hardware estimate in FP32 (about 1 ulp), exact rounding in FP64
__device__ __forceinline__ float rsq_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsq_t(double x) { return 1.0 / sqrt(x); }

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

// ------------------------------------------------------------------ addressing
// Element at a 32-bit byte offset from a wave-uniform base (the base MUST be
// the same in every active lane: it is taken from the first one): the base pointer
// (a row or a view's start) stays in scalar registers and the per-lane offset
// is one 32-bit register, so a load or store needs no per-lane 64-bit address
// arithmetic. The base goes through readfirstlane so that the compiler keeps
// it scalar instead of folding a row offset into the per-lane address, and
// the access is made in the global address space.
#define GS_GLOBAL __attribute__((address_space(1)))
template <typename U> __device__ __forceinline__ uint64_t uniform_addr(const U *p)
{
    uint64_t a = reinterpret_cast<uint64_t>(p);
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a), hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return ((uint64_t)hi << 32) | lo;
}
template <typename U> __device__ __forceinline__ U load_at(const U *base, uint32_t boff)
{
    return *(const GS_GLOBAL U *)((const GS_GLOBAL char *)uniform_addr(base) + boff);
}
template <typename U> __device__ __forceinline__ void store_at(U *base, uint32_t boff, U v)
{
    *(GS_GLOBAL U *)((GS_GLOBAL char *)uniform_addr(base) + boff) = v;
}
// four values in one aligned access (a builtin vector type: the HIP vector
// classes' operators take no address-space-qualified object)
template <typename T> using quad_t = T __attribute__((ext_vector_type(4)));
template <typename T> __device__ __forceinline__ void store4_at(T *base, uint32_t boff, T x, T y, T z, T w)
{
    store_at(reinterpret_cast<quad_t<T> *>(base), boff, quad_t<T>{x, y, z, w});
}
template <typename T> __device__ __forceinline__ quad_t<T> load4_at(const T *base, uint32_t boff)
{
    return load_at(reinterpret_cast<const quad_t<T> *>(base), boff);
}

template <int CTRL, int ROW_MASK> __device__ __forceinline__ float dpp_move(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, true));
}

// Sum over the 64 lanes of a wavefront; the result is valid in every lane.
__device__ __forceinline__ float wave_sum(float x)
{
    // Row-local inclusive scan (rows of 16 lanes), then carry rows into
    // later rows with the GFX9 row broadcasts; lane 63 ends with the total.
    x += dpp_move<0x111, 0xf>(x);  // row_shr:1
    x += dpp_move<0x112, 0xf>(x);  // row_shr:2
    x += dpp_move<0x114, 0xf>(x);  // row_shr:4
    x += dpp_move<0x118, 0xf>(x);  // row_shr:8
    x += dpp_move<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
    x += dpp_move<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

__device__ __forceinline__ double wave_sum(double x)
{
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t x)
{
    for (int off = 32; off > 0; off >>= 1) x = max(x, (uint32_t)__shfl_xor((int)x, off, 64));
    return x;
}

// One butterfly step of a transposed reduction: permlane32_swap exchanges
// the upper 32 lanes of `a` with the lower 32 lanes of `b`, so the sum holds
// a's pairwise half-sums in lanes 0-31 and b's in lanes 32-63.
__device__ __forceinline__ float fold32(float a, float b)
{
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// permlane16_swap exchanges the odd rows of `a` with the even rows of `b`:
// the sum holds a's row-pair sums in rows 0 and 2 and b's in rows 1 and 3.
__device__ __forceinline__ float fold16(float a, float b)
{
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Adds the wavefront sums of the per-lane values v[0..8] to dst[0..8], each
// times a factor, with two global atomic instructions: v[0..7] go through a
// transposed reduction (permlane32 and permlane16 swaps, a swap of row
// halves, a three-step row scan) that leaves component sum9_comp(lane) in
// every lane l with l % 8 == 7; v[8] goes through a plain DPP reduction and
// lane 6 adds it.
// sc is the factor for the component of the calling lane, sc8 the one of v[8].
__device__ __forceinline__ int sum9_comp(int lane)
{
    int row = (lane & 63) >> 4;
    int base = (row & 1) * 2 + (row >> 1);   // row 0 -> 0, 1 -> 2, 2 -> 1, 3 -> 3
    return base + ((lane & 8) ? 4 : 0);      // low half of a row: v[0..3], high half: v[4..7]
}

__device__ __forceinline__ void wave_sum9_atomic(const float (&v)[9], float *dst, float sc, float sc8)
{
    int lane = threadIdx.x & 63;
    // after fold32, rows 0-1 hold the first value of a pair, rows 2-3 the second
    float x01 = fold32(v[0], v[1]), x23 = fold32(v[2], v[3]);
    float x45 = fold32(v[4], v[5]), x67 = fold32(v[6], v[7]);
    // after fold16, rows 0..3 hold values (0, 2, 1, 3) and (4, 6, 5, 7)
    float z0 = fold16(x01, x23), z1 = fold16(x45, x67);
    // fold the row halves: lanes 0-7 of a row keep z0, lanes 8-15 z1
    bool hi = (lane & 8) != 0;
    float c = hi ? z1 : z0, d = hi ? z0 : z1;
    float r = c + dpp_move<0x128, 0xf>(d);          // row_ror:8: the other half of the row
    r += dpp_move<0x111, 0xf>(r);                   // row_shr:1
    r += dpp_move<0x112, 0xf>(r);                   // row_shr:2
    r += dpp_move<0x114, 0xf>(r);                   // row_shr:4: lane 8k+7 holds its 8 lanes' sum
    float s8 = wave_sum(v[8]);
    // one atomic instruction for all nine: lane 6 adds v[8] (a lane-dependent
    // address, so the compiler does not rewrite it as a wave-wide atomic)
    const bool l8 = lane == 6;
    const float val = l8 ? s8 * sc8 : r * sc;
    const uint32_t boff = 4u * (uint32_t)(l8 ? 8 : sum9_comp(lane));
    if ((lane & 7) == 7 || l8)
        __builtin_amdgcn_global_atomic_fadd_f32((GS_GLOBAL float *)((GS_GLOBAL char *)uniform_addr(dst) + boff), val);
}

// FP64: lane c (c < 9) adds component c, times sc (sc8 unused).
__device__ __forceinline__ void wave_sum9_atomic(const double (&v)[9], double *dst, double sc0, double)
{
    int lane = threadIdx.x & 63;
    double r = v[0];
    for (int c = 0; c < 9; c++) {
        double t = wave_sum(v[c]);
        r = lane == c ? t : r;
    }
    if (lane < 9) unsafeAtomicAdd(dst + lane, r * sc0);
}

__device__ __forceinline__ void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }

// ------------------------------------------------------------------ Adam
// Hyper-parameters of one Adam step after the batch scaling rules of paper
// section 4: lr already times sqrt(batch), betas already to the power batch.
struct AdamConst {
    double lr[6];      // per parameter group (row_group)
    double b1, b2;
    double eps;
    int32_t zero_grad;
};

// Parameter group of a row of the [59][n] parameter layout: position,
// log-scale, rotation, opacity logit, SH DC, SH rest.
__host__ __device__ __forceinline__ int row_group(int row)
{
    return row < 3 ? 0 : row < 6 ? 1 : row < 10 ? 2 : row < 11 ? 3 : row < 14 ? 4 : 5;
}

__device__ __forceinline__ float sqrt_t(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_t(double x) { return sqrt(x); }

// Step size lr / (1 - b1^t) and 1 / sqrt(1 - b2^t) of the current step, in
// the kernels' precision; every Adam kernel forms them this way so fused and
// separate updates agree bit for bit.
template <typename T> __device__ __forceinline__ T adam_step_size(double lr, double bc1) { return (T)lr * rcp_t((T)bc1); }
template <typename T> __device__ __forceinline__ T adam_inv_bc2s(double bc2s) { return rcp_t((T)bc2s); }

// One Adam update (torch.optim.Adam semantics: m and v, then
// p -= step m / (sqrt(v) / sqrt(1 - b2^t) + eps)); in FP32 the square root
// and the quotients use the hardware estimates (about 1 ulp each).
template <typename T>
__device__ __forceinline__ void adam_one(T &p, T g, T &m, T &v, T b1, T b2, T step, T inv_bc2s, T eps)
{
    m = b1 * m + (T(1) - b1) * g;
    v = b2 * v + (T(1) - b2) * g * g;
    T denom = sqrt_t(v) * inv_bc2s + eps;
    p = p - step * (m * rcp_t(denom));
}

// Moments, constants and the bias corrections of the current step (written
// by the prepare kernel: scratch[0] = 1 - b1^t, 0 for a skipped step;
// scratch[1] = sqrt(1 - b2^t)).
template <typename T> struct AdamRef {
    T *M, *V;
    AdamConst c;
    const double *scratch;
};

// Adam on CNT consecutive rows row0 .. row0 + CNT - 1 of Gaussian i with
// gradients g[r]: all loads are issued before any update, so the memory
// latency of the rows overlaps.
// ib = i * sizeof(T), the lane's byte offset in a row (n * sizeof(T) < 4 GiB).
template <typename T, int CNT>
__device__ __forceinline__ void adam_row_block(T *__restrict__ P, const AdamRef<T> &a, int row0, int64_t n, uint32_t ib,
                                               const T *g)
{
    double bc1 = a.scratch[0];
    if (bc1 == 0.0) return;                       // skipped step
    T *M = a.M;                                   // (no restrict: a later block's loads stay after this block's stores)
    T *V = a.V;
    T p[CNT], m[CNT], v[CNT];
#pragma unroll
    for (int r = 0; r < CNT; r++) {
        int64_t k = (int64_t)(row0 + r) * n;
        p[r] = load_at(P + k, ib);
        m[r] = load_at(M + k, ib);
        v[r] = load_at(V + k, ib);
    }
    T b1 = (T)a.c.b1, b2 = (T)a.c.b2, eps = (T)a.c.eps, ibc2s = adam_inv_bc2s<T>(a.scratch[1]);
#pragma unroll
    for (int r = 0; r < CNT; r++) {
        T step = adam_step_size<T>(a.c.lr[row_group(row0 + r)], bc1);
        adam_one(p[r], g[r], m[r], v[r], b1, b2, step, ibc2s, eps);
    }
#pragma unroll
    for (int r = 0; r < CNT; r++) {
        int64_t k = (int64_t)(row0 + r) * n;
        store_at(P + k, ib, p[r]);
        store_at(M + k, ib, m[r]);
        store_at(V + k, ib, v[r]);
    }
}

// The same update split in two, so that a caller can issue the next row
// block's loads before it updates and stores the current one: adam_load
// reads p, m, v of rows row0 .. row0 + CNT - 1, adam_store updates them with
// gradients g and writes them back (the arithmetic of adam_row_block). The
// caller tests adam_skipped once.
template <typename T, int CNT> struct AdamRows {
    T p[CNT], m[CNT], v[CNT];
};
template <typename T> __device__ __forceinline__ bool adam_skipped(const AdamRef<T> &a) { return a.scratch[0] == 0.0; }
template <typename T, int CNT>
__device__ __forceinline__ void adam_load(AdamRows<T, CNT> &b, const T *P, const AdamRef<T> &a, int row0, int64_t n,
                                          uint32_t ib)
{
#pragma unroll
    for (int r = 0; r < CNT; r++) {
        int64_t k = (int64_t)(row0 + r) * n;
        b.p[r] = load_at(P + k, ib);
        b.m[r] = load_at(a.M + k, ib);
        b.v[r] = load_at(a.V + k, ib);
    }
}
template <typename T, int CNT>
__device__ __forceinline__ void adam_store(AdamRows<T, CNT> &b, T *P, const AdamRef<T> &a, int row0, int64_t n,
                                           uint32_t ib, const T *g)
{
    double bc1 = a.scratch[0];
    T b1 = (T)a.c.b1, b2 = (T)a.c.b2, eps = (T)a.c.eps, ibc2s = adam_inv_bc2s<T>(a.scratch[1]);
#pragma unroll
    for (int r = 0; r < CNT; r++) {
        T step = adam_step_size<T>(a.c.lr[row_group(row0 + r)], bc1);
        adam_one(b.p[r], g[r], b.m[r], b.v[r], b1, b2, step, ibc2s, eps);
    }
#pragma unroll
    for (int r = 0; r < CNT; r++) {
        int64_t k = (int64_t)(row0 + r) * n;
        store_at(P + k, ib, b.p[r]);
        store_at(a.M + k, ib, b.m[r]);
        store_at(a.V + k, ib, b.v[r]);
    }
}

AdamConst make_adam_const(const gs_adam_hparams *h);
hipError_t launch_adam_prepare(int64_t *step, const AdamConst &c, double *scratch, const int32_t *skip, hipStream_t s);

}  // namespace gs
