// Adaptive densification (appendix A.1): the position-gradient statistic,
// the clone / split / prune classification with on-device compaction into
// new planar arrays, and the opacity reset.
//
// Plan: one thread per Gaussian classifies it (kept original, clone, split
// pair with surviving children) from the stored values only — log-scales and
// the opacity logit are compared with thresholds given in the same domain,
// the statistic's mean as sum >= threshold * count in double — and each
// 256-Gaussian block counts its classes with wavefront ballots; one
// workgroup scans the block counts into per-block output offsets. Apply:
// each block ranks its Gaussians within each class (ballot + prefix over
// the wavefronts), so every class keeps index order, and copies the 59 rows
// of parameters and moments to their new columns; split children get their
// offset means and shrunk log-scales. All of it is a streaming pass over the
// [59][n] arrays.
#include "common.hpp"

namespace gs {

constexpr int DBLK = 256;                 // Gaussians per block of the plan and apply passes
enum : uint8_t { DC_KEEP = 1, DC_CLONE = 2, DC_SPLIT = 4 };

struct DensifyThr {
    double grad, split_ls, prune_logit, prune_ls, prune_ls_child;
};

struct DensifyWS {
    uint8_t *cls;        // [n] class bits
    int64_t *bcount;     // [nb][3] per-block counts
    int64_t *boff;       // [nb][3] per-block exclusive offsets
    int64_t *totals;     // [3] K, C, S
};

static inline size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

static DensifyWS densify_ws(void *ws, int64_t n)
{
    const int64_t nb = (n + DBLK - 1) / DBLK;
    char *p = (char *)ws;
    DensifyWS w;
    w.cls = (uint8_t *)p;
    p += round256((size_t)n);
    w.bcount = (int64_t *)p;
    p += round256((size_t)nb * 3 * sizeof(int64_t));
    w.boff = (int64_t *)p;
    p += round256((size_t)nb * 3 * sizeof(int64_t));
    w.totals = (int64_t *)p;
    return w;
}

size_t densify_ws_bytes(int64_t n)
{
    const int64_t nb = (n + DBLK - 1) / DBLK;
    return round256((size_t)n) + 2 * round256((size_t)nb * 3 * sizeof(int64_t)) + 256;
}

template <typename T>
__global__ void __launch_bounds__(256) densify_stats_kernel(const T *__restrict__ proj, const T *__restrict__ dproj,
                                                            int64_t n, int32_t views, T scale,
                                                            float *__restrict__ accum, int32_t *__restrict__ count)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint32_t *tiles = side_tiles<T>(proj, (int64_t)views * n);
    T a = T(0);
    int32_t c = 0;
    for (int v = 0; v < views; v++) {
        const int64_t r = (int64_t)v * n + i;
        if (tiles[r] > 0) {
            const T du = dproj[r * REC + D_U], dv = dproj[r * REC + D_V];
            a += scale * sqrt(du * du + dv * dv);
            c++;
        }
    }
    if (c) {
        accum[i] += (float)a;
        count[i] += c;
    }
}

// Counts of the three class bits over the block (thread 0 holds them).
__device__ __forceinline__ void block_class_counts(uint8_t code, int (&out)[3])
{
    __shared__ int s[DBLK / 64][3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const uint64_t b = __ballot((code >> k) & 1);
        if (lane == 0) s[wave][k] = __popcll(b);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; k++) {
        int t = 0;
        for (int w = 0; w < DBLK / 64; w++) t += s[w][k];
        out[k] = t;
    }
}

template <typename T>
__global__ void __launch_bounds__(DBLK) densify_classify_kernel(const T *__restrict__ P, int64_t n,
                                                                const float *__restrict__ accum,
                                                                const int32_t *__restrict__ count, DensifyThr h,
                                                                DensifyWS w)
{
    const int64_t i = (int64_t)blockIdx.x * DBLK + threadIdx.x;
    uint8_t code = 0;
    if (i < n) {
        const T l0 = P[3 * n + i], l1 = P[4 * n + i], l2 = P[5 * n + i];
        const double ml = (double)fmax(l0, fmax(l1, l2)), lg = (double)P[10 * n + i];
        const int32_t c = count[i];
        const bool sel = c > 0 && (double)accum[i] >= h.grad * (double)c;
        const bool big = ml > h.split_ls;
        const bool pruned = lg < h.prune_logit || ml > h.prune_ls;
        const bool child_pruned = lg < h.prune_logit || ml > h.prune_ls_child;
        const bool split = sel && big;
        if (!split && !pruned) code |= DC_KEEP;
        if (sel && !big && !pruned) code |= DC_CLONE;
        if (split && !child_pruned) code |= DC_SPLIT;
        w.cls[i] = code;
    }
    int cnt[3];
    block_class_counts(code, cnt);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; k++) w.bcount[(int64_t)blockIdx.x * 3 + k] = cnt[k];
}

// Exclusive scan of the block counts of each class, one workgroup of 1024
// threads walking the blocks in order; totals into w.totals and counts_dev.
__global__ void __launch_bounds__(1024) densify_scan_kernel(DensifyWS w, int64_t nb, int64_t *counts_dev)
{
    __shared__ int64_t s_w[16];
    __shared__ int64_t s_carry;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < 3; k++) {
        if (threadIdx.x == 0) s_carry = 0;
        __syncthreads();
        for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
            const int64_t j = b0 + threadIdx.x;
            const int64_t val = j < nb ? w.bcount[j * 3 + k] : 0;
            int64_t x = val;
            for (int off = 1; off < 64; off <<= 1) {          // inclusive scan over the wavefront
                const int64_t y = __shfl_up(x, off, 64);
                if (lane >= off) x += y;
            }
            if (lane == 63) s_w[wave] = x;
            __syncthreads();
            int64_t before = s_carry;
            for (int q = 0; q < wave; q++) before += s_w[q];
            if (j < nb) w.boff[j * 3 + k] = before + x - val;
            __syncthreads();
            if (threadIdx.x == 1023) s_carry = before + x;     // the last thread's inclusive total
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            w.totals[k] = s_carry;
            counts_dev[k] = s_carry;
        }
        __syncthreads();
    }
}

template <typename T> __device__ __forceinline__ T exp_t(T x);
template <> __device__ __forceinline__ float exp_t<float>(float x) { return expf(x); }
template <> __device__ __forceinline__ double exp_t<double>(double x) { return exp(x); }

template <typename T>
__global__ void __launch_bounds__(DBLK) densify_apply_kernel(const T *__restrict__ P, const T *__restrict__ M,
                                                             const T *__restrict__ V, int64_t n,
                                                             const T *__restrict__ noise, DensifyWS w,
                                                             T *__restrict__ Po, T *__restrict__ Mo,
                                                             T *__restrict__ Vo, int64_t n_out, T shrink)
{
    __shared__ int s_rank[DBLK / 64][3];
    const int64_t i = (int64_t)blockIdx.x * DBLK + threadIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint8_t code = i < n ? w.cls[i] : 0;
    int rank[3];
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const uint64_t b = __ballot((code >> k) & 1);
        rank[k] = __popcll(b & below);
        if (lane == 0) s_rank[wave][k] = __popcll(b);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; k++)
        for (int q = 0; q < wave; q++) rank[k] += s_rank[q][k];
    if (i >= n || code == 0) return;
    const int64_t K = w.totals[0], C = w.totals[1], S = w.totals[2];
    const int64_t *bo = w.boff + (int64_t)blockIdx.x * 3;
    const int64_t dk = bo[0] + rank[0], dc = K + bo[1] + rank[1], d0 = K + C + bo[2] + rank[2], d1 = d0 + S;
    const bool keep = (code & DC_KEEP) && dk < n_out, clone = (code & DC_CLONE) && dc < n_out;
    const bool split = (code & DC_SPLIT) && d1 < n_out;
    T c0[3], c1[3];
    if (split) {
        T q[4], s[3];
        for (int r = 0; r < 4; r++) q[r] = P[(6 + r) * n + i];
        const T qn = T(1) / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const T qw = q[0] * qn, qx = q[1] * qn, qy = q[2] * qn, qz = q[3] * qn;
        const T R[3][3] = {{T(1) - T(2) * (qy * qy + qz * qz), T(2) * (qx * qy - qw * qz), T(2) * (qx * qz + qw * qy)},
                           {T(2) * (qx * qy + qw * qz), T(1) - T(2) * (qx * qx + qz * qz), T(2) * (qy * qz - qw * qx)},
                           {T(2) * (qx * qz - qw * qy), T(2) * (qy * qz + qw * qx), T(1) - T(2) * (qx * qx + qy * qy)}};
        for (int a = 0; a < 3; a++) s[a] = exp_t(P[(3 + a) * n + i]);
        for (int a = 0; a < 3; a++) {
            T o0 = T(0), o1 = T(0);
            for (int b = 0; b < 3; b++) {
                o0 += R[a][b] * (s[b] * noise[(0 * 3 + b) * n + i]);
                o1 += R[a][b] * (s[b] * noise[(1 * 3 + b) * n + i]);
            }
            const T mean = P[a * n + i];
            c0[a] = mean + o0;
            c1[a] = mean + o1;
        }
    }
    for (int r = 0; r < GS_PARAM_ROWS; r++) {
        const T p = P[(int64_t)r * n + i];
        const int64_t ro = (int64_t)r * n_out;
        if (keep) {
            Po[ro + dk] = p;
            Mo[ro + dk] = M[(int64_t)r * n + i];
            Vo[ro + dk] = V[(int64_t)r * n + i];
        }
        if (clone) {
            Po[ro + dc] = p;
            Mo[ro + dc] = T(0);
            Vo[ro + dc] = T(0);
        }
        if (split) {
            const T a = r < 3 ? c0[r] : (r < 6 ? p - shrink : p);
            const T b = r < 3 ? c1[r] : (r < 6 ? p - shrink : p);
            Po[ro + d0] = a;
            Po[ro + d1] = b;
            Mo[ro + d0] = T(0);
            Mo[ro + d1] = T(0);
            Vo[ro + d0] = T(0);
            Vo[ro + d1] = T(0);
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) reset_opacity_kernel(T *__restrict__ P, T *__restrict__ M, T *__restrict__ V,
                                                            int64_t n, T cap)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const T p = P[10 * n + i];
    P[10 * n + i] = p < cap ? p : cap;
    M[10 * n + i] = T(0);
    V[10 * n + i] = T(0);
}

template <typename T>
hipError_t launch_densify_stats(const void *proj, const void *dproj, int64_t n, int32_t views, double scale,
                                float *accum, int32_t *count, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(densify_stats_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       (const T *)proj, (const T *)dproj, n, views, (T)scale, accum, count);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_densify_plan(const void *params, int64_t n, const float *accum, const int32_t *count,
                               const gs_densify_hparams &h, void *workspace, int64_t *counts_dev, hipStream_t s)
{
    const DensifyWS w = densify_ws(workspace, n);
    const int64_t nb = (n + DBLK - 1) / DBLK;
    DensifyThr t;
    t.grad = h.grad_threshold;
    t.split_ls = h.split_log_scale;
    t.prune_logit = h.prune_logit;
    t.prune_ls = h.prune_log_scale;
    t.prune_ls_child = h.prune_log_scale + log(1.6);
    if (nb > 0)
        hipLaunchKernelGGL(densify_classify_kernel<T>, dim3((unsigned)nb), dim3(DBLK), 0, s, (const T *)params, n,
                           accum, count, t, w);
    hipLaunchKernelGGL(densify_scan_kernel, dim3(1), dim3(1024), 0, s, w, nb, counts_dev);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_densify_apply(const void *params, const void *m, const void *v, int64_t n, const void *noise,
                                const void *workspace, void *po, void *mo, void *vo, int64_t n_out, hipStream_t s)
{
    const DensifyWS w = densify_ws((void *)workspace, n);
    const int64_t nb = (n + DBLK - 1) / DBLK;
    if (nb == 0 || n_out == 0) return hipSuccess;
    hipLaunchKernelGGL(densify_apply_kernel<T>, dim3((unsigned)nb), dim3(DBLK), 0, s, (const T *)params,
                       (const T *)m, (const T *)v, n, (const T *)noise, w, (T *)po, (T *)mo, (T *)vo, n_out,
                       (T)log(1.6));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reset_opacity(void *params, void *m, void *v, int64_t n, double cap, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(reset_opacity_kernel<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (T *)params,
                       (T *)m, (T *)v, n, (T)cap);
    return hipGetLastError();
}

#define GS_DENSIFY_INST(T)                                                                                   \
    template hipError_t launch_densify_stats<T>(const void *, const void *, int64_t, int32_t, double, float *,  \
                                                int32_t *, hipStream_t);                                     \
    template hipError_t launch_densify_plan<T>(const void *, int64_t, const float *, const int32_t *,           \
                                               const gs_densify_hparams &, void *, int64_t *, hipStream_t);     \
    template hipError_t launch_densify_apply<T>(const void *, const void *, const void *, int64_t, const void *, \
                                                const void *, void *, void *, void *, int64_t, hipStream_t);    \
    template hipError_t launch_reset_opacity<T>(void *, void *, void *, int64_t, double, hipStream_t);
GS_DENSIFY_INST(float)
GS_DENSIFY_INST(double)
#undef GS_DENSIFY_INST

}  // namespace gs
