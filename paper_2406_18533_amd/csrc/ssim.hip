// L1 + D-SSIM loss and its gradient with respect to the rendered images (the
// loss step of section 2.1: L1 per pixel and SSIM over pixel windows). SSIM
// per colour channel with an 11x11 Gaussian window (standard deviation 1.5),
// zero padding, C1 = 0.01^2, C2 = 0.03^2; loss of a view = (1 - lam)
// mean|x - y| + lam (1 - mean SSIM) over its 3HW values, batch loss = mean
// over the views (times `scale`).
//
// SSIM needs four window-filtered fields: the means mx = G x and my = G y,
// s = G(x^2 + y^2) (so var_x + var_y = s - mx^2 - my^2) and f = G(x y) (so
// cov = f - mx my). The window is symmetric and zero-padded, so the gradient
// is G applied to three per-pixel coefficient maps:
//   dL/dx = G(a) + 2 x G(b) + y G(c) + the L1 term,
// with a = dL/dmx, b = dL/ds, c = dL/df at each pixel. Two passes, each an
// LDS-tiled separable stencil over 64x20 output tiles:
//  - forward: stage x, y with a 5-pixel halo, filter rows (four outputs per
//    item, 30 rows x 16 items over 256 threads) then columns (five outputs
//    per item, one item per thread), form SSIM and a, b, c (written out) and
//    the tile's loss share (FP32 over a thread's five pixels, then double in
//    a fixed order);
//  - backward: stage a, b, c with the halo, filter likewise, combine with x,
//    y and the L1 sign into dL/dx.
// The staged inputs and the row sums share one LDS buffer; the row sums are
// 64 floats wide, so the column pass reads them with two-row LDS reads at
// 64-float strides and no address arithmetic. Rows first beat columns first
// here: the column-first order needs fewer taps, but its reads of the
// 74-wide staged rows cost more than the taps it saves. Consecutive
// workgroup ids go to different XCDs; each XCD is given a contiguous run of
// tiles so that vertical neighbours (whose halos overlap) share its L2.
#include "common.hpp"

namespace gs {

constexpr int SR = 5;                     // window radius (11 taps)
constexpr int SWIN = 2 * SR + 1;
constexpr int OW = 64, OH = 20;           // output tile
constexpr int IW = OW + 2 * SR;           // 74 staged columns
constexpr int IH = OH + 2 * SR;           // 30 staged rows
constexpr int LW = 76;                    // LDS row stride of staged inputs: 16-byte rows, 2 zero columns
constexpr int SEG = 4;                    // outputs per horizontal item
constexpr int NSEG = OW / SEG;            // 16 items per row
constexpr int HITEMS = IH * NSEG;         // 480 horizontal items
constexpr int VSEG = 5;                   // outputs per vertical item: 64 columns x 4 items = 256 threads
constexpr int SSIM_THREADS = OW * (OH / VSEG);
static_assert(SSIM_THREADS == 256, "one vertical item per thread");
static_assert(HITEMS <= 2 * SSIM_THREADS, "at most two horizontal items per thread");
static_assert(SEG + 2 * SR <= 14 && (OW - SEG) + 14 <= LW, "a horizontal item reads 14 staged values");

struct SsimWindow {
    float f[SWIN];
    double d[SWIN];
};
__device__ __forceinline__ float win_at(const SsimWindow &w, int k, float) { return w.f[k]; }
__device__ __forceinline__ double win_at(const SsimWindow &w, int k, double) { return w.d[k]; }

// The 64x20 tiles of every view, row-major within a view, views in order.
struct SsimGrid {
    int32_t nt;
    int32_t base[MAXV + 1];
    int32_t tx[MAXV];
};

static SsimGrid ssim_grid(const ViewTable &vt)
{
    SsimGrid g;
    int32_t b = 0;
    for (int v = 0; v < vt.nviews; v++) {
        g.base[v] = b;
        g.tx[v] = (vt.width[v] + OW - 1) / OW;
        b += g.tx[v] * ((vt.height[v] + OH - 1) / OH);
    }
    g.base[vt.nviews] = b;
    g.nt = b;
    return g;
}

template <typename T> struct SsimArgs {
    const T *x, *y;          // rendered and target images, [3][H][W] per view, views concatenated
    T *dL;                   // like x
    T *ca, *cb, *cc;         // coefficient maps a, b, c (like x)
    double *part;            // [3 tiles] weighted loss shares
    double lam, scale;
};

struct SsimBlock {
    int W, H, x0, y0;
    int64_t base;            // first value of the channel plane
    double wv;               // scale / (3 H W views): weight of one value in the batch loss
    int32_t lin;             // (channel, tile) index, channel-major
};

// Workgroup b -> (channel, tile). Ids are dealt to the 8 XCDs in turn; the
// k-th XCD gets the k-th contiguous eighth of the (channel, tile) range.
// Returns false for the at most 7 spare workgroups of the rounded-up grid.
__device__ __forceinline__ bool ssim_block(const ViewTable &vt, const SsimGrid &sg, double scale, SsimBlock &B)
{
    const int32_t total = 3 * sg.nt, per = (total + 7) / 8;
    const int32_t lin = (int32_t)(blockIdx.x & 7) * per + (int32_t)(blockIdx.x >> 3);
    if (lin >= total) return false;
    const int ch = lin / sg.nt, t = lin - ch * sg.nt;
    int v = 0;
    while (v + 1 < vt.nviews && t >= sg.base[v + 1]) v++;
    const int local = t - sg.base[v], tx = sg.tx[v];
    B.W = vt.width[v];
    B.H = vt.height[v];
    B.x0 = (local % tx) * OW;
    B.y0 = (local / tx) * OH;
    const int64_t plane = (int64_t)B.W * B.H;
    B.base = 3 * vt.pix_base[v] + ch * plane;
    B.wv = scale / ((double)(3 * plane) * (double)vt.nviews);
    B.lin = lin;
    return true;
}

// Stages NI images of the tile plus halo into lds[NI][IH][LW], zero outside
// the image and in the two padding columns. Wave w takes rows w, w+4, ...;
// lane l columns l and 64 + l. Every load is issued before the first LDS
// write, so the workgroup waits for one memory latency, not one per row.
template <typename T, int NI>
__device__ __forceinline__ void stage(T *lds, const T *const (&src)[NI], const SsimBlock &B)
{
    constexpr int WAVES = SSIM_THREADS / 64, ROWS = (IH + WAVES - 1) / WAVES;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int xa = B.x0 - SR + lane, xb = xa + 64;
    const bool oka = xa >= 0 && xa < B.W;
    const bool okb = lane < IW - 64 && xb < B.W;
    T va[NI][ROWS], vb[NI][ROWS];
#pragma unroll
    for (int i = 0; i < ROWS; i++) {
        const int r = wave + WAVES * i, yy = B.y0 - SR + r;
        const bool rok = r < IH && yy >= 0 && yy < B.H;
        const int64_t row = B.base + (int64_t)yy * B.W;
#pragma unroll
        for (int k = 0; k < NI; k++) {
            va[k][i] = rok && oka ? src[k][row + xa] : T(0);
            vb[k][i] = rok && okb ? src[k][row + xb] : T(0);
        }
    }
#pragma unroll
    for (int i = 0; i < ROWS; i++) {
        const int r = wave + WAVES * i;
        if (r < IH) {
#pragma unroll
            for (int k = 0; k < NI; k++) {
                T *d = lds + (k * IH + r) * LW;
                d[lane] = va[k][i];
                if (lane < LW - 64) d[64 + lane] = vb[k][i];
            }
        }
    }
}

// 14 consecutive staged values from a 16-byte aligned position.
__device__ __forceinline__ void load14(const float *p, float (&v)[14])
{
    const float4 a = *(const float4 *)p, b = *(const float4 *)(p + 4), c = *(const float4 *)(p + 8);
    const float2 d = *(const float2 *)(p + 12);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    v[8] = c.x; v[9] = c.y; v[10] = c.z; v[11] = c.w;
    v[12] = d.x; v[13] = d.y;
}
__device__ __forceinline__ void load14(const double *p, double (&v)[14])
{
#pragma unroll
    for (int k = 0; k < 14; k += 2) {
        const double2 a = *(const double2 *)(p + k);
        v[k] = a.x;
        v[k + 1] = a.y;
    }
}

// Four outputs of a row filter: out[q] = sum_j w[j] in[q + j].
template <typename T>
__device__ __forceinline__ void row4(const SsimWindow &w, const T (&in)[14], T (&out)[SEG])
{
#pragma unroll
    for (int q = 0; q < SEG; q++) {
        T s = T(0);
#pragma unroll
        for (int j = 0; j < SWIN; j++) s = fma(win_at(w, j, T(0)), in[q + j], s);
        out[q] = s;
    }
}

template <typename T> __device__ __forceinline__ T rcp(T a);
template <> __device__ __forceinline__ float rcp<float>(float a) { return __builtin_amdgcn_rcpf(a); }
template <> __device__ __forceinline__ double rcp<double>(double a) { return 1.0 / a; }

// Horizontal items of this thread: write their row sums over the (now dead)
// staged inputs, NF fields [NF][IH][OW].
template <typename T, int NF>
__device__ __forceinline__ void store_rows(T *lds, const T (&h)[2][NF][SEG])
{
#pragma unroll
    for (int it = 0; it < 2; it++) {
        const int item = threadIdx.x + it * SSIM_THREADS;
        if (item < HITEMS) {
            const int r = item / NSEG, c0 = (item % NSEG) * SEG;
#pragma unroll
            for (int f = 0; f < NF; f++)
#pragma unroll
                for (int k = 0; k < SEG; k++) lds[(f * IH + r) * OW + c0 + k] = h[it][f][k];
        }
    }
}

// Column filter of NF row-sum fields: out[f][j] at output row VSEG q + j of column c.
template <typename T, int NF>
__device__ __forceinline__ void columns(const T *lds, const SsimWindow &win, int c, int q, T (&out)[NF][VSEG])
{
#pragma unroll
    for (int f = 0; f < NF; f++)
#pragma unroll
        for (int j = 0; j < VSEG; j++) out[f][j] = T(0);
#pragma unroll
    for (int i = 0; i < VSEG + 2 * SR; i++) {
#pragma unroll
        for (int f = 0; f < NF; f++) {
            const T val = lds[(f * IH + VSEG * q + i) * OW + c];
#pragma unroll
            for (int j = 0; j < VSEG; j++)
                if (i - j >= 0 && i - j < SWIN) out[f][j] = fma(win_at(win, i - j, T(0)), val, out[f][j]);
        }
    }
}

template <typename T, int NI, int NF> struct SsimLds {
    static constexpr int IN = NI * IH * LW, HF = NF * IH * OW;
    static constexpr int N = IN > HF ? IN : HF;
};

template <typename T>
__global__ void __launch_bounds__(SSIM_THREADS) ssim_fwd_kernel(ViewTable vt, SsimGrid sg, SsimWindow win,
                                                                SsimArgs<T> A)
{
    __shared__ __align__(16) T lds[SsimLds<T, 2, 4>::N];
    __shared__ double s_red[SSIM_THREADS / 64];
    SsimBlock B;
    if (!ssim_block(vt, sg, A.scale, B)) return;
    const T *const src[2] = {A.x, A.y};
    stage<T, 2>(lds, src, B);
    __syncthreads();

    // rows: the four fields at four outputs for each of (up to) two items
    T h[2][4][SEG];
#pragma unroll
    for (int it = 0; it < 2; it++) {
        const int item = threadIdx.x + it * SSIM_THREADS;
        if (item < HITEMS) {
            const int r = item / NSEG, c0 = (item % NSEG) * SEG;
            T xv[14], yv[14], pv[14], mv[14];
            load14(lds + r * LW + c0, xv);
            load14(lds + (IH + r) * LW + c0, yv);
#pragma unroll
            for (int k = 0; k < 14; k++) {
                pv[k] = fma(xv[k], xv[k], yv[k] * yv[k]);
                mv[k] = xv[k] * yv[k];
            }
            row4(win, xv, h[it][0]);
            row4(win, yv, h[it][1]);
            row4(win, pv, h[it][2]);
            row4(win, mv, h[it][3]);
        }
    }
    // this thread's vertical item: column c, output rows VSEG q .. VSEG q + VSEG - 1
    const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
    T xc[VSEG], yc[VSEG];
#pragma unroll
    for (int j = 0; j < VSEG; j++) {
        xc[j] = lds[(VSEG * q + j + SR) * LW + c + SR];
        yc[j] = lds[(IH + VSEG * q + j + SR) * LW + c + SR];
    }
    __syncthreads();
    store_rows<T, 4>(lds, h);
    __syncthreads();
    T m[4][VSEG];
    columns<T, 4>(lds, win, c, q, m);

    const T C1 = T(1e-4), C2 = T(9e-4);
    const T dS = (T)(-A.lam * B.wv);
    T l1sum = T(0), ssum = T(0);
    const int px = B.x0 + c;
#pragma unroll
    for (int j = 0; j < VSEG; j++) {
        const int py = B.y0 + VSEG * q + j;
        if (px < B.W && py < B.H) {
            const T mx = m[0][j], my = m[1][j];
            const T cm = fma(mx, mx, fma(my, my, C1));
            const T a1 = fma(T(2) * mx, my, C1);
            const T b1 = T(2) * (m[3][j] - mx * my) + C2;
            const T d = m[2][j] - mx * mx - my * my + C2;
            const T inv = rcp(cm * d);
            const T S = a1 * b1 * inv;
            const T dS_dd = -S * cm * inv;                 // d SSIM / d (var_x + var_y)
            const T dS_dcov = T(2) * a1 * inv;
            const T dS_dmx = T(2) * inv * (my * b1 - mx * S * d);
            const int64_t o = B.base + (int64_t)py * B.W + px;
            A.ca[o] = dS * (dS_dmx - T(2) * mx * dS_dd - my * dS_dcov);
            A.cb[o] = dS * dS_dd;
            A.cc[o] = dS * dS_dcov;
            l1sum += fabs(xc[j] - yc[j]);
            ssum += T(1) - S;
        }
    }
    double acc = (1.0 - A.lam) * (double)l1sum + A.lam * (double)ssum;
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);   // fixed order: deterministic
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) A.part[B.lin] = ((s_red[0] + s_red[1]) + (s_red[2] + s_red[3])) * B.wv;
}

template <typename T>
__global__ void __launch_bounds__(SSIM_THREADS) ssim_bwd_kernel(ViewTable vt, SsimGrid sg, SsimWindow win,
                                                                SsimArgs<T> A)
{
    __shared__ __align__(16) T lds[SsimLds<T, 3, 3>::N];
    SsimBlock B;
    if (!ssim_block(vt, sg, A.scale, B)) return;
    const T *const src[3] = {A.ca, A.cb, A.cc};
    stage<T, 3>(lds, src, B);
    __syncthreads();
    T h[2][3][SEG];
#pragma unroll
    for (int it = 0; it < 2; it++) {
        const int item = threadIdx.x + it * SSIM_THREADS;
        if (item < HITEMS) {
            const int r = item / NSEG, c0 = (item % NSEG) * SEG;
#pragma unroll
            for (int f = 0; f < 3; f++) {
                T v[14];
                load14(lds + (f * IH + r) * LW + c0, v);
                row4(win, v, h[it][f]);
            }
        }
    }
    __syncthreads();
    store_rows<T, 3>(lds, h);
    __syncthreads();
    const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
    T g[3][VSEG];
    columns<T, 3>(lds, win, c, q, g);
    const T l1 = (T)((1.0 - A.lam) * B.wv);
    const int px = B.x0 + c;
    T xv[VSEG], yv[VSEG];
#pragma unroll
    for (int j = 0; j < VSEG; j++) {   // all loads first
        const int py = B.y0 + VSEG * q + j;
        const bool ok = px < B.W && py < B.H;
        const int64_t o = B.base + (int64_t)py * B.W + px;
        xv[j] = ok ? A.x[o] : T(0);
        yv[j] = ok ? A.y[o] : T(0);
    }
#pragma unroll
    for (int j = 0; j < VSEG; j++) {
        const int py = B.y0 + VSEG * q + j;
        if (px < B.W && py < B.H) {
            const int64_t o = B.base + (int64_t)py * B.W + px;
            const T d = xv[j] - yv[j];
            A.dL[o] = g[0][j] + T(2) * xv[j] * g[1][j] + yv[j] * g[2][j] +
                      (d > T(0) ? l1 : (d < T(0) ? -l1 : T(0)));
        }
    }
}

static SsimWindow ssim_window()
{
    SsimWindow w;
    double s = 0.0, e[SWIN];
    for (int k = 0; k < SWIN; k++) {
        const double u = (double)(k - SR);
        e[k] = exp(-u * u / (2.0 * 1.5 * 1.5));
        s += e[k];
    }
    for (int k = 0; k < SWIN; k++) {
        w.d[k] = e[k] / s;
        w.f[k] = (float)w.d[k];
    }
    return w;
}

static size_t maps_bytes(const ViewTable &vt, size_t elem)
{
    return ((3 * (size_t)3 * (size_t)vt.pix_base[vt.nviews] * elem) + 255) & ~(size_t)255;
}

// Workspace: the three coefficient maps (like the images), then the loss
// shares of the (channel, tile) pairs and the block sums of their reduction.
size_t dssim_ws_bytes(const ViewTable &vt, size_t elem)
{
    return maps_bytes(vt, elem) + ((size_t)3 * ssim_grid(vt).nt + LOSS_SUM_BLOCKS) * sizeof(double);
}

template <typename T>
hipError_t launch_l1_dssim(const void *rgb, const void *target, const ViewTable &vt, double lam, double scale,
                           void *dL, double *loss, void *workspace, hipStream_t s)
{
    const int64_t vals = 3 * vt.pix_base[vt.nviews];
    const SsimGrid sg = ssim_grid(vt);
    T *maps = (T *)workspace;
    SsimArgs<T> A;
    A.x = (const T *)rgb;
    A.y = (const T *)target;
    A.dL = (T *)dL;
    A.ca = maps;
    A.cb = maps + vals;
    A.cc = maps + 2 * vals;
    A.part = (double *)((char *)workspace + maps_bytes(vt, sizeof(T)));
    A.lam = lam;
    A.scale = scale;
    if (sg.nt == 0) return hipSuccess;
    const SsimWindow w = ssim_window();
    const int64_t total = 3 * (int64_t)sg.nt;
    const unsigned grid = (unsigned)(8 * ((total + 7) / 8));
    hipLaunchKernelGGL(ssim_fwd_kernel<T>, dim3(grid), dim3(SSIM_THREADS), 0, s, vt, sg, w, A);
    hipLaunchKernelGGL(ssim_bwd_kernel<T>, dim3(grid), dim3(SSIM_THREADS), 0, s, vt, sg, w, A);
    return launch_tile_sum(A.part, total, A.part + total, loss, s);
}

template hipError_t launch_l1_dssim<float>(const void *, const void *, const ViewTable &, double, double, void *,
                                           double *, void *, hipStream_t);
template hipError_t launch_l1_dssim<double>(const void *, const void *, const ViewTable &, double, double, void *,
                                            double *, void *, hipStream_t);

}  // namespace gs
