// L1 + D-SSIM loss and its gradient with respect to the rendered images (the
// loss step of the paper's background section: L1 and SSIM over pixel
// windows). SSIM per colour channel with an 11x11 Gaussian window (standard
// deviation 1.5), zero padding, C1 = 0.01^2, C2 = 0.03^2; loss of a view =
// (1 - lam) mean|x - y| + lam (1 - mean SSIM) over its 3HW values, batch
// loss = mean over the views (times `scale`).
//
// SSIM depends on x through three window-filtered fields, the mean m = G x,
// the square e = G x^2 and the product f = G (x y); the window is symmetric
// and zero-padded, so the gradient is G applied to three per-pixel
// coefficient maps, dL/dx = G(a) + 2 x G(b) + y G(c). Two passes, one
// workgroup per 16x16 tile and channel (the render tiles), each staging the
// tile and a 5-pixel halo in LDS and filtering rows then columns:
//  - forward: the five moments of x and y, the SSIM map, the coefficients
//    a, b, c (written out) and the tile's loss share (double, no atomics);
//  - backward: G of the three coefficient maps, combined with x, y and the
//    L1 term into dL/dx.
// Both passes are HBM-bound streams.
#include "common.hpp"

namespace gs {

constexpr int SSIM_R = 5;                 // window radius (11 taps)
constexpr int SSIM_W = 2 * SSIM_R + 1;
constexpr int SSIM_T = TILE;              // 16x16 output pixels per workgroup
constexpr int SSIM_H = SSIM_T + 2 * SSIM_R;

struct SsimWindow {
    float f[SSIM_W];
    double d[SSIM_W];
};

__device__ __forceinline__ float win_at(const SsimWindow &w, int k, float) { return w.f[k]; }
__device__ __forceinline__ double win_at(const SsimWindow &w, int k, double) { return w.d[k]; }

template <typename T> struct SsimArgs {
    const T *x, *y;          // rendered and target images, [3][H][W] per view, views concatenated
    T *dL;                   // like x
    T *ca, *cb, *cc;         // gradient coefficients per pixel and channel (like x)
    double *part;            // [tiles][3] weighted loss shares
    double lam, scale;
};

// Pixel (py, px) of channel ch of tile g: the view, its size and the offset
// of the channel plane.
struct SsimTile {
    int W, H, x0, y0;
    int64_t plane, base;
    double wv;               // scale / (3 H W views): weight of one value in the batch loss
};

__device__ __forceinline__ SsimTile ssim_tile(const ViewTable &vt, int g, int ch, double scale)
{
    SsimTile t;
    const int v = view_of_tile(vt, g);
    const int local = g - vt.tile_base[v], TX = vt.tiles_x[v];
    t.W = vt.width[v];
    t.H = vt.height[v];
    t.x0 = (local % TX) * SSIM_T;
    t.y0 = (local / TX) * SSIM_T;
    t.plane = (int64_t)t.W * t.H;
    t.base = 3 * vt.pix_base[v] + ch * t.plane;
    t.wv = scale / ((double)(3 * t.plane) * (double)vt.nviews);
    return t;
}

template <typename T>
__global__ void __launch_bounds__(256) ssim_fwd_kernel(ViewTable vt, SsimWindow win, SsimArgs<T> A)
{
    __shared__ T sx[SSIM_H][SSIM_H], sy[SSIM_H][SSIM_H];
    __shared__ T hs[5][SSIM_H][SSIM_T];
    __shared__ double s_red[4];
    const int g = blockIdx.x, ch = blockIdx.y;
    const SsimTile t = ssim_tile(vt, g, ch, A.scale);
    for (int q = threadIdx.x; q < SSIM_H * SSIM_H; q += 256) {   // tile + halo, zero outside the image
        const int r = q / SSIM_H, c = q % SSIM_H;
        const int yy = t.y0 - SSIM_R + r, xx = t.x0 - SSIM_R + c;
        const bool in = yy >= 0 && yy < t.H && xx >= 0 && xx < t.W;
        const int64_t o = t.base + (int64_t)yy * t.W + xx;
        sx[r][c] = in ? A.x[o] : T(0);
        sy[r][c] = in ? A.y[o] : T(0);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < SSIM_H * SSIM_T; q += 256) {   // rows: window sums of x, y, x^2, y^2, xy
        const int r = q / SSIM_T, c = q % SSIM_T;
        T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0), s4 = T(0);
        for (int j = 0; j < SSIM_W; j++) {
            const T w = win_at(win, j, T(0)), a = sx[r][c + j], b = sy[r][c + j];
            s0 = fma(w, a, s0);
            s1 = fma(w, b, s1);
            s2 = fma(w, a * a, s2);
            s3 = fma(w, b * b, s3);
            s4 = fma(w, a * b, s4);
        }
        hs[0][r][c] = s0;
        hs[1][r][c] = s1;
        hs[2][r][c] = s2;
        hs[3][r][c] = s3;
        hs[4][r][c] = s4;
    }
    __syncthreads();
    const int ty = threadIdx.x / SSIM_T, tx = threadIdx.x % SSIM_T;
    T m[5] = {T(0), T(0), T(0), T(0), T(0)};
    for (int i = 0; i < SSIM_W; i++) {                            // columns: the five moments at this pixel
        const T w = win_at(win, i, T(0));
        for (int k = 0; k < 5; k++) m[k] = fma(w, hs[k][ty + i][tx], m[k]);
    }
    const int py = t.y0 + ty, px = t.x0 + tx;
    double acc = 0.0;
    if (py < t.H && px < t.W) {
        const T C1 = T(1e-4), C2 = T(9e-4);
        const T mx = m[0], my = m[1];
        const T vx = m[2] - mx * mx, vy = m[3] - my * my, cxy = m[4] - mx * my;
        const T a = T(2) * mx * my + C1, b = T(2) * cxy + C2;
        const T cm = mx * mx + my * my + C1, d = vx + vy + C2;
        const T S = a * b / (cm * d);
        const T dS = (T)(-A.lam * t.wv);                          // dL/dSSIM of this value
        const T dS_dmx = T(2) * my * b / (cm * d) - S * T(2) * mx / cm;
        const T dS_dvar = -S / d, dS_dcov = T(2) * a / (cm * d);
        const int64_t o = t.base + (int64_t)py * t.W + px;
        A.ca[o] = dS * (dS_dmx - T(2) * mx * dS_dvar - my * dS_dcov);
        A.cb[o] = dS * dS_dvar;
        A.cc[o] = dS * dS_dcov;
        const T diff = sx[ty + SSIM_R][tx + SSIM_R] - sy[ty + SSIM_R][tx + SSIM_R];
        acc = (1.0 - A.lam) * (double)fabs(diff) + A.lam * (1.0 - (double)S);
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);   // fixed order: deterministic
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) A.part[(int64_t)g * 3 + ch] = ((s_red[0] + s_red[1]) + (s_red[2] + s_red[3])) * t.wv;
}

template <typename T>
__global__ void __launch_bounds__(256) ssim_bwd_kernel(ViewTable vt, SsimWindow win, SsimArgs<T> A)
{
    __shared__ T sc[3][SSIM_H][SSIM_H];
    __shared__ T hs[3][SSIM_H][SSIM_T];
    const int g = blockIdx.x, ch = blockIdx.y;
    const SsimTile t = ssim_tile(vt, g, ch, A.scale);
    for (int q = threadIdx.x; q < SSIM_H * SSIM_H; q += 256) {   // coefficient maps, zero outside the image
        const int r = q / SSIM_H, c = q % SSIM_H;
        const int yy = t.y0 - SSIM_R + r, xx = t.x0 - SSIM_R + c;
        const bool in = yy >= 0 && yy < t.H && xx >= 0 && xx < t.W;
        const int64_t o = t.base + (int64_t)yy * t.W + xx;
        sc[0][r][c] = in ? A.ca[o] : T(0);
        sc[1][r][c] = in ? A.cb[o] : T(0);
        sc[2][r][c] = in ? A.cc[o] : T(0);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < SSIM_H * SSIM_T; q += 256) {
        const int r = q / SSIM_T, c = q % SSIM_T;
        T s0 = T(0), s1 = T(0), s2 = T(0);
        for (int j = 0; j < SSIM_W; j++) {
            const T w = win_at(win, j, T(0));
            s0 = fma(w, sc[0][r][c + j], s0);
            s1 = fma(w, sc[1][r][c + j], s1);
            s2 = fma(w, sc[2][r][c + j], s2);
        }
        hs[0][r][c] = s0;
        hs[1][r][c] = s1;
        hs[2][r][c] = s2;
    }
    __syncthreads();
    const int ty = threadIdx.x / SSIM_T, tx = threadIdx.x % SSIM_T;
    const int py = t.y0 + ty, px = t.x0 + tx;
    if (py >= t.H || px >= t.W) return;
    T G[3] = {T(0), T(0), T(0)};
    for (int i = 0; i < SSIM_W; i++) {
        const T w = win_at(win, i, T(0));
        for (int k = 0; k < 3; k++) G[k] = fma(w, hs[k][ty + i][tx], G[k]);
    }
    const int64_t o = t.base + (int64_t)py * t.W + px;
    const T x = A.x[o], y = A.y[o], d = x - y;
    const T l1 = (T)((1.0 - A.lam) * t.wv);
    A.dL[o] = G[0] + T(2) * x * G[1] + y * G[2] + (d > T(0) ? l1 : (d < T(0) ? -l1 : T(0)));
}

static SsimWindow ssim_window()
{
    SsimWindow w;
    double s = 0.0, e[SSIM_W];
    for (int k = 0; k < SSIM_W; k++) {
        const double u = (double)(k - SSIM_R);
        e[k] = exp(-u * u / (2.0 * 1.5 * 1.5));
        s += e[k];
    }
    for (int k = 0; k < SSIM_W; k++) {
        w.d[k] = e[k] / s;
        w.f[k] = (float)w.d[k];
    }
    return w;
}

// Workspace: the three coefficient maps (like the images), then the tiles'
// loss shares and the block sums of their reduction.
size_t dssim_ws_bytes(const ViewTable &vt, size_t elem)
{
    const size_t maps = 3 * (size_t)3 * (size_t)vt.pix_base[vt.nviews] * elem;
    return ((maps + 255) & ~(size_t)255) + ((size_t)vt.total_tiles * 3 + LOSS_SUM_BLOCKS) * sizeof(double);
}

template <typename T>
hipError_t launch_l1_dssim(const void *rgb, const void *target, const ViewTable &vt, double lam, double scale,
                           void *dL, double *loss, void *workspace, hipStream_t s)
{
    const int64_t vals = 3 * vt.pix_base[vt.nviews];
    T *maps = (T *)workspace;
    const size_t mb = ((3 * (size_t)vals * sizeof(T)) + 255) & ~(size_t)255;
    SsimArgs<T> A;
    A.x = (const T *)rgb;
    A.y = (const T *)target;
    A.dL = (T *)dL;
    A.ca = maps;
    A.cb = maps + vals;
    A.cc = maps + 2 * vals;
    A.part = (double *)((char *)workspace + mb);
    A.lam = lam;
    A.scale = scale;
    if (vt.total_tiles == 0) return hipSuccess;
    const SsimWindow w = ssim_window();
    const dim3 grid((unsigned)vt.total_tiles, 3);
    hipLaunchKernelGGL(ssim_fwd_kernel<T>, grid, dim3(256), 0, s, vt, w, A);
    hipLaunchKernelGGL(ssim_bwd_kernel<T>, grid, dim3(256), 0, s, vt, w, A);
    return launch_tile_sum(A.part, (int64_t)vt.total_tiles * 3, A.part + (int64_t)vt.total_tiles * 3, loss, s);
}

template hipError_t launch_l1_dssim<float>(const void *, const void *, const ViewTable &, double, double, void *,
                                           double *, void *, hipStream_t);
template hipError_t launch_l1_dssim<double>(const void *, const void *, const ViewTable &, double, double, void *,
                                            double *, void *, hipStream_t);

}  // namespace gs
