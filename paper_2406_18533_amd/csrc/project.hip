// Gaussian transformation forward and backward (paper section 2.1 step 1;
// appendix A.3: both are Gaussian-wise).
//  - forward: one lane per (view, Gaussian); a wavefront takes 64
//    consecutive Gaussians of one view at a time (planar rows, so every
//    parameter load and record store is coalesced), and the views of one
//    64-Gaussian chunk run back to back on one XCD, so the chunk's parameters
//    come from HBM once and from that XCD's L2 for the other views;
//  - backward: one thread per Gaussian, summing over the views in registers.
#include "common.hpp"

namespace gs {

template <typename T> struct Camera {
    T R[9], t[3], cen[3];
    T fx, fy, cx, cy, znear, limx, limy;
    int W, H;
};

template <typename T> __device__ __forceinline__ Camera<T> load_camera(const gs_camera *c)
{
    Camera<T> k;
    for (int j = 0; j < 9; j++) k.R[j] = (T)c->R[j];
    for (int j = 0; j < 3; j++) k.t[j] = (T)c->t[j];
    for (int j = 0; j < 3; j++)
        k.cen[j] = (T)(-(c->R[j] * c->t[0] + c->R[3 + j] * c->t[1] + c->R[6 + j] * c->t[2]));
    k.fx = (T)c->fx; k.fy = (T)c->fy; k.cx = (T)c->cx; k.cy = (T)c->cy;
    k.znear = (T)c->znear;
    // Guard band of the Jacobian: 1.3x the tangent of the half field of view.
    k.limx = (T)(1.3 * (0.5 * c->width / c->fx));
    k.limy = (T)(1.3 * (0.5 * c->height / c->fy));
    k.W = c->width;
    k.H = c->height;
    return k;
}

// The cameras of the launch in the kernels' precision, formed once per
// workgroup into LDS (the conversions from the double-precision camera
// structs and the camera centres are wave-uniform work that every thread
// would otherwise repeat for every view). Must be reached by all threads.
template <typename T> __device__ __forceinline__ void stage_cameras(Camera<T> *cs, const gs_camera *cams, int views)
{
    if ((int)threadIdx.x < views) cs[threadIdx.x] = load_camera<T>(cams + threadIdx.x);
    __syncthreads();
}

// View-independent part: scale, rotation, opacity and the factor
// M = R(q) diag(s) of the 3D covariance Sigma = M M^T.
template <typename T> struct Shape {
    T s[3], q[4], qn, Rq[9], M[9];
    T opac;
    bool ok;
};

template <typename T> __device__ __forceinline__ void quat_matrix(const T q[4], T R[9])
{
    T w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = T(1) - T(2) * (y * y + z * z); R[1] = T(2) * (x * y - w * z); R[2] = T(2) * (x * z + w * y);
    R[3] = T(2) * (x * y + w * z); R[4] = T(1) - T(2) * (x * x + z * z); R[5] = T(2) * (y * z - w * x);
    R[6] = T(2) * (x * z - w * y); R[7] = T(2) * (y * z + w * x); R[8] = T(1) - T(2) * (x * x + y * y);
}

template <typename T> __device__ __forceinline__ bool finite(T x) { return isfinite(x); }

template <typename T>
__device__ __forceinline__ void shape_from(const T ls[3], const T qr[4], T logit, Shape<T> &S)
{
    S.ok = finite(ls[0]) && finite(ls[1]) && finite(ls[2]) && finite(qr[0]) && finite(qr[1]) && finite(qr[2]) &&
           finite(qr[3]) && finite(logit);
    for (int j = 0; j < 3; j++) S.s[j] = exp(ls[j]);
    // reciprocals and the normalisation by the hardware estimates (about
    // 1 ulp in FP32; the quotients are not correctly rounded anywhere in the
    // method's tolerances)
    T q2 = qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3];
    S.ok = S.ok && q2 > T(0);
    T iq = rsq_t(q2);
    S.qn = q2 * iq;
    for (int j = 0; j < 4; j++) S.q[j] = qr[j] * iq;
    quat_matrix(S.q, S.Rq);
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) S.M[3 * r + c] = S.Rq[3 * r + c] * S.s[c];
    S.opac = rcp_t(T(1) + exp(-logit));
}

template <typename T>
__device__ __forceinline__ void make_shape(const T *P, int64_t n, int64_t i, Shape<T> &S)
{
    const uint32_t ib = (uint32_t)i * (uint32_t)sizeof(T);
    T ls[3], qr[4];
    for (int j = 0; j < 3; j++) ls[j] = load_at(P + (3 + j) * n, ib);
    for (int j = 0; j < 4; j++) qr[j] = load_at(P + (6 + j) * n, ib);
    shape_from(ls, qr, load_at(P + 10 * n, ib), S);
}

// Per-view geometry of one Gaussian.
template <typename T> struct Geo {
    T y[3], iz, xi, eta;
    bool xi_cl, eta_cl;
    T J00, J02, J11, J12;
    T Tm[6];
    T N[6];           // Tm M: the screen covariance is N N^T + 0.3 I
    T A, B, C, det;
    T u, v, conic[3], radius;
    bool visible;   // in front of znear, finite
    int tiles;
    TileRect rect;
};

template <typename T>
__device__ __forceinline__ void make_geo(const T x[3], const Shape<T> &S, const Camera<T> &k, Geo<T> &g)
{
    g.visible = false;
    g.tiles = 0;
    // (explicit fused multiply-adds: every kernel that calls this gets the
    // same roundings, whatever the compiler would contract)
    for (int r = 0; r < 3; r++)
        g.y[r] = fma(k.R[3 * r], x[0], fma(k.R[3 * r + 1], x[1], fma(k.R[3 * r + 2], x[2], k.t[r])));
    T z = g.y[2];
    if (!S.ok || !(z > k.znear)) return;
    g.iz = rcp_t(z);
    T xr = g.y[0] * g.iz, yr = g.y[1] * g.iz;
    g.u = fma(k.fx, xr, k.cx);
    g.v = fma(k.fy, yr, k.cy);
    g.xi_cl = xr < -k.limx || xr > k.limx;
    g.eta_cl = yr < -k.limy || yr > k.limy;
    g.xi = fmin(fmax(xr, -k.limx), k.limx);
    g.eta = fmin(fmax(yr, -k.limy), k.limy);
    g.J00 = k.fx * g.iz;
    g.J02 = -k.fx * g.xi * g.iz;
    g.J11 = k.fy * g.iz;
    g.J12 = -k.fy * g.eta * g.iz;
    for (int c = 0; c < 3; c++) {
        g.Tm[c] = fma(g.J00, k.R[c], g.J02 * k.R[6 + c]);
        g.Tm[3 + c] = fma(g.J11, k.R[3 + c], g.J12 * k.R[6 + c]);
    }
    // Screen covariance N N^T + 0.3 I with N = Tm M (2x3). Its entries and
    // determinant are formed as sums of squares (Lagrange identity
    // |n0|^2 |n1|^2 - (n0.n1)^2 = |n0 x n1|^2), so thin footprints keep
    // their FP32 accuracy.
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++)
            g.N[3 * r + c] = fma(g.Tm[3 * r], S.M[c], fma(g.Tm[3 * r + 1], S.M[3 + c], g.Tm[3 * r + 2] * S.M[6 + c]));
    const T *n0 = g.N, *n1 = g.N + 3;
    T a0 = fma(n0[0], n0[0], fma(n0[1], n0[1], n0[2] * n0[2]));
    T c0 = fma(n1[0], n1[0], fma(n1[1], n1[1], n1[2] * n1[2]));
    T b0 = fma(n0[0], n1[0], fma(n0[1], n1[1], n0[2] * n1[2]));
    T x0 = fma(n0[1], n1[2], -(n0[2] * n1[1])), x1 = fma(n0[2], n1[0], -(n0[0] * n1[2]));
    T x2 = fma(n0[0], n1[1], -(n0[1] * n1[0]));
    g.A = a0 + T(0.3);
    g.B = b0;
    g.C = c0 + T(0.3);
    g.det = fma(x0, x0, fma(x1, x1, x2 * x2)) + fma(T(0.3), a0 + c0, T(0.09));
    if (!(g.det > T(0)) || !finite(g.det)) return;
    T id = rcp_t(g.det);
    g.conic[0] = g.C * id;
    g.conic[1] = -g.B * id;
    g.conic[2] = g.A * id;
    T mid = T(0.5) * (g.A + g.C);
    T hd = T(0.5) * (g.A - g.C);
    T lmax = mid + sqrt(fma(hd, hd, g.B * g.B));
    g.radius = ceil(T(3) * sqrt(lmax));
    if (!finite(g.radius) || !finite(g.u) || !finite(g.v)) return;
    g.visible = true;
    if (tile_rect((float)g.u, (float)g.v, (float)g.radius, k.W, k.H, g.rect))
        g.tiles = (g.rect.x1 - g.rect.x0 + 1) * (g.rect.y1 - g.rect.y0 + 1);
}

// Real orthonormal spherical harmonics of degree <= 3 (Condon-Shortley phase)
// as polynomials in the unit direction; coefficients from
// K_lm = sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) and the Legendre derivatives.
#define GS_SQRT(v) ((T)__builtin_sqrt(v))

template <typename T> __device__ __forceinline__ void sh_basis(T x, T y, T z, T Y[16])
{
    constexpr double PI = 3.14159265358979323846;
    const T c0 = GS_SQRT(1.0 / (4.0 * PI)), c1 = GS_SQRT(3.0 / (4.0 * PI));
    const T c2a = GS_SQRT(15.0 / (4.0 * PI)), c2b = GS_SQRT(5.0 / (16.0 * PI)), c2c = GS_SQRT(15.0 / (16.0 * PI));
    const T c3a = GS_SQRT(35.0 / (32.0 * PI)), c3b = GS_SQRT(105.0 / (4.0 * PI)), c3c = GS_SQRT(21.0 / (32.0 * PI));
    const T c3d = GS_SQRT(7.0 / (16.0 * PI)), c3e = GS_SQRT(105.0 / (16.0 * PI));
    T xx = x * x, yy = y * y, zz = z * z;
    Y[0] = c0;
    Y[1] = -c1 * y; Y[2] = c1 * z; Y[3] = -c1 * x;
    Y[4] = c2a * x * y; Y[5] = -c2a * y * z; Y[6] = c2b * (T(3) * zz - T(1)); Y[7] = -c2a * x * z;
    Y[8] = c2c * (xx - yy);
    Y[9] = -c3a * y * (T(3) * xx - yy); Y[10] = c3b * x * y * z; Y[11] = -c3c * y * (T(5) * zz - T(1));
    Y[12] = c3d * z * (T(5) * zz - T(3)); Y[13] = -c3c * x * (T(5) * zz - T(1)); Y[14] = c3e * z * (xx - yy);
    Y[15] = -c3a * x * (xx - T(3) * yy);
}

// sum_k w_k grad Y_k of the polynomial forms above (before projection onto
// the sphere's tangent plane); w(k) gives the weight of basis function k.
template <typename T, typename W> __device__ __forceinline__ void sh_grad(T x, T y, T z, W w, T g[3])
{
    constexpr double PI = 3.14159265358979323846;
    const T c1 = GS_SQRT(3.0 / (4.0 * PI));
    const T c2a = GS_SQRT(15.0 / (4.0 * PI)), c2b = GS_SQRT(5.0 / (16.0 * PI)), c2c = GS_SQRT(15.0 / (16.0 * PI));
    const T c3a = GS_SQRT(35.0 / (32.0 * PI)), c3b = GS_SQRT(105.0 / (4.0 * PI)), c3c = GS_SQRT(21.0 / (32.0 * PI));
    const T c3d = GS_SQRT(7.0 / (16.0 * PI)), c3e = GS_SQRT(105.0 / (16.0 * PI));
    T xx = x * x, yy = y * y, zz = z * z;
    T gx = T(0), gy = T(0), gz = T(0);
    gy += -c1 * w(1);
    gz += c1 * w(2);
    gx += -c1 * w(3);
    gx += c2a * y * w(4); gy += c2a * x * w(4);
    gy += -c2a * z * w(5); gz += -c2a * y * w(5);
    gz += c2b * T(6) * z * w(6);
    gx += -c2a * z * w(7); gz += -c2a * x * w(7);
    gx += c2c * T(2) * x * w(8); gy += -c2c * T(2) * y * w(8);
    gx += -c3a * T(6) * x * y * w(9); gy += -c3a * (T(3) * xx - T(3) * yy) * w(9);
    gx += c3b * y * z * w(10); gy += c3b * x * z * w(10); gz += c3b * x * y * w(10);
    gy += -c3c * (T(5) * zz - T(1)) * w(11); gz += -c3c * T(10) * y * z * w(11);
    gz += c3d * (T(15) * zz - T(3)) * w(12);
    gx += -c3c * (T(5) * zz - T(1)) * w(13); gz += -c3c * T(10) * x * z * w(13);
    gx += c3e * T(2) * x * z * w(14); gy += -c3e * T(2) * y * z * w(14); gz += c3e * (xx - yy) * w(14);
    gx += -c3a * (T(3) * xx - T(3) * yy) * w(15); gy += c3a * T(6) * x * y * w(15);
    g[0] = gx; g[1] = gy; g[2] = gz;
}
#undef GS_SQRT

template <typename T> using V4 = typename Vec4<T>::type;

// Forward work items: (view v, 64-Gaussian chunk c), one per wavefront. The
// items of XCD x (workgroups b with b mod 8 = x) are the chunks
// c = 8 k + x, k = 0, 1, ..., each with all its views in turn (item s of the
// XCD is k = s div views, v = s mod views), so the views of one chunk run
// back to back on one XCD and its parameters come from that XCD's L2 after
// the first view. Workgroups of four wavefronts take four consecutive items
// (one-wavefront workgroups made workgroup dispatch, not the work, the
// limit). Only pairs that touch a tile write a record and the depth /
// rectangle side arrays; every pair writes its tiles touched (0 when culled
// or off-screen).
// One (view, Gaussian) pair. ib = i * sizeof(T) is the lane's byte offset in
// a parameter row (n * sizeof(T) < 4 GiB); view_out and the side arrays of
// the view are wave-uniform bases, indexed by the Gaussian (n * 48 B < 4 GiB).
template <typename T>
__device__ __forceinline__ void project_item(const T *__restrict__ P, int64_t n, const Camera<T> &k, int64_t vn,
                                             int64_t vbase, uint32_t i, T *__restrict__ out)
{
    const uint32_t ib = i * (uint32_t)sizeof(T);
    auto row = [&](int r) { return load_at(P + r * n, ib); };
    // the position and the shape rows in one round of loads (nearly every
    // pair is in front of the camera; the colour rows wait for the footprint)
    T x[3] = {row(0), row(1), row(2)};
    T ls[3] = {row(3), row(4), row(5)};
    T qr[4] = {row(6), row(7), row(8), row(9)};
    T logit = row(10);
    bool xok = finite(x[0]) && finite(x[1]) && finite(x[2]);
    T z = k.R[6] * x[0] + k.R[7] * x[1] + k.R[8] * x[2] + k.t[2];
    uint32_t tiles = 0;
    if (xok && z > k.znear) {
        Shape<T> S;
        shape_from(ls, qr, logit, S);
        Geo<T> g;
        make_geo(x, S, k, g);
        if (g.visible && g.tiles > 0) {
            tiles = (uint32_t)g.tiles;
            T d[3] = {x[0] - k.cen[0], x[1] - k.cen[1], x[2] - k.cen[2]};
            T idn = rsq_t(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            T Y[16];
            sh_basis(d[0] * idn, d[1] * idn, d[2] * idn, Y);
            T acc[3] = {T(0), T(0), T(0)};
            for (int k2 = 0; k2 < 16; k2++)
                for (int ch = 0; ch < 3; ch++) acc[ch] = fma(row(11 + 3 * k2 + ch), Y[k2], acc[ch]);
            T rgb[3];
            for (int ch = 0; ch < 3; ch++) {
                T a = acc[ch] + T(0.5);
                rgb[ch] = a > T(0) ? a : T(0);
            }
            T *rec = out + vbase * REC;
            const uint32_t rb = i * (uint32_t)(REC * sizeof(T));
            store4_at(rec, rb, g.u, g.v, g.conic[0], g.conic[1]);
            store4_at(rec + 4, rb, g.conic[2], S.opac, rgb[0], rgb[1]);
            store4_at(rec + 8, rb, rgb[2], g.radius, g.y[2], (T)g.tiles);
            store_at(side_depth<T>(out, vn) + vbase, 4 * i, __float_as_uint((float)g.y[2]));
            store_at(side_rect<T>(out, vn) + vbase, 8 * i, pack_rect(g.rect.x0, g.rect.x1, g.rect.y0, g.rect.y1));
        }
    }
    store_at(side_tiles<T>(out, vn) + vbase, 4 * i, tiles);
}

template <typename T>
__global__ void __launch_bounds__(256) project_fwd_kernel(const T *__restrict__ P, int64_t n,
                                                          const gs_camera *__restrict__ cams, int32_t views,
                                                          T *__restrict__ out)
{
    const int x = blockIdx.x & 7;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t s = (int64_t)(blockIdx.x >> 3) * 4 + wave;               // item of XCD x
    const int64_t kk = s / views;
    const int v = (int)(s - kk * views);
    const int64_t i = (kk * 8 + x) * 64 + (threadIdx.x & 63);
    __shared__ Camera<T> cs[MAXV];
    stage_cameras(cs, cams, views);                // once per workgroup, not per item
    if (i >= n) return;
    project_item(P, n, cs[v], (int64_t)views * n, (int64_t)v * n, (uint32_t)i, out);
}

// Transformation backward: chain rule from the per-view record gradients
// d(u, v, a, b, c, opacity, rgb) to the 59 parameters, summed over views in
// registers; each parameter gradient is added once (no atomics). One thread
// per Gaussian, in two phases that keep register pressure apart:
//  - geometry: position (through u, v and the perspective Jacobian), scale,
//    rotation and opacity;
//  - colour, all three channels: per seen view the direction and the SH
//    basis are formed once, each channel's clamp is tested (the raw colour
//    summed in the forward's order, so the mask agrees), the SH gradients of
//    the unclamped channels are accumulated (rows 11 + 3 k + c) and so is
//    the position gradient through the viewing direction, which is linear
//    in the weights: one sh_grad of the clamp-masked channel sum of
//    dL/drgb_c sh_c.
// The records are read once and, with `clear`, zeroed after use.
//
// With ADAM the Adam step is applied to the parameters instead of adding
// into grad: the gradient is the same expression, summed in the same order
// ((0 + geometry part) + colour part for the position), so the result equals
// the two separate calls bit for bit, and grad is left untouched. Rows 3-10
// are updated after the geometry phase (nothing reads them later); position
// and SH rows, read before, are updated at the end. Gaussians seen by no view
// get the Adam step with a zero gradient on all 59 rows.

// Geometry part for Gaussian i, seen by the views in vis: the position
// gradient gpos and the gradients g8 of rows 3-10 (log-scales, rotation,
// opacity logit).
template <typename T>
__device__ __forceinline__ void geom_grads(const T *__restrict__ P, int64_t n, int64_t i, const T x[3],
                                           const Camera<T> *cs, int32_t views, uint64_t vis,
                                           const T *__restrict__ dproj, T gpos[3], T g8[8])
{
    Shape<T> S;
    make_shape(P, n, i, S);
    T gmean[3] = {0, 0, 0}, gM[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, gop = T(0);
    // each lane's next seen view's record gradient is loaded before the
    // current view's chain rule, so the loads overlap the arithmetic
    uint64_t rem = vis;
    quad_t<T> n0 = {}, n1 = {};
    // (the view differs between lanes, so these addresses are per lane)
    auto rec_of = [&](uint64_t r) {
        return reinterpret_cast<const quad_t<T> *>(dproj + ((int64_t)__builtin_ctzll(r) * n + i) * REC);
    };
    if (rem) {
        n0 = rec_of(rem)[0];
        n1 = rec_of(rem)[1];
    }
    for (int v = 0; v < views; v++) {
        if (!((vis >> v) & 1ull)) continue;
        const quad_t<T> d0 = n0, d1 = n1;
        rem &= rem - 1ull;
        if (rem) {
            n0 = rec_of(rem)[0];
            n1 = rec_of(rem)[1];
        }
        T du = d0.x, dv = d0.y, da = d0.z, db = d0.w, dc = d1.x, dop = d1.y;
        const Camera<T> &k = cs[v];
        Geo<T> g;
        make_geo(x, S, k, g);
        T iz = g.iz, iz2 = iz * iz;
        T dy[3];
        dy[0] = du * k.fx * iz;
        dy[1] = dv * k.fy * iz;
        dy[2] = -(du * k.fx * g.y[0] + dv * k.fy * g.y[1]) * iz2;
        // conic Q = Sigma'^-1 = (C, -B, A) / det. With Gc = [[da, db/2],
        // [db/2, dc]] the gradient w.r.t. Sigma' is H = -Q Gc Q, and with
        // Sigma' = N N^T + 0.3 I, dL/dN = 2 H N. H is formed in the
        // eigenbasis (e1, e2) of Sigma': for a thin footprint its entries in
        // image coordinates are large terms that cancel, and FP32 loses the
        // part along the long axis; in the eigenbasis H is diagonal-scaled,
        // -(e_i^T Gc e_j) / (l_i l_j), with l2 = det / l1 (no cancellation),
        // and N is projected onto e1, e2 before the product.
        T hd = T(0.5) * (g.A - g.C), mid = T(0.5) * (g.A + g.C);
        T rr = sqrt(hd * hd + g.B * g.B);
        T l1 = mid + rr, l2 = g.det / l1;
        T ex = T(1), ey = T(0);
        if (rr > T(0)) {
            T px = hd >= T(0) ? hd + rr : g.B, py = hd >= T(0) ? g.B : rr - hd;
            T inv = rsq_t(px * px + py * py);
            ex = px * inv;
            ey = py * inv;
        }
        T hdb = T(0.5) * db;
        T g11 = ex * (da * ex + hdb * ey) + ey * (hdb * ex + dc * ey);
        T g22 = ey * (da * ey - hdb * ex) - ex * (hdb * ey - dc * ex);
        T g12 = ex * (hdb * ex - da * ey) + ey * (dc * ex - hdb * ey);
        T il1 = rcp_t(l1), il2 = rcp_t(l2);
        T h11 = -g11 * il1 * il1, h22 = -g22 * il2 * il2, h12 = -g12 * il1 * il2;
        T dN[6];
        for (int c = 0; c < 3; c++) {
            T p1 = ex * g.N[c] + ey * g.N[3 + c];        // e1^T N
            T p2 = ex * g.N[3 + c] - ey * g.N[c];        // e2^T N, e2 = (-ey, ex)
            T r1 = h11 * p1 + h12 * p2, r2 = h12 * p1 + h22 * p2;
            dN[c] = T(2) * (ex * r1 - ey * r2);
            dN[3 + c] = T(2) * (ey * r1 + ex * r2);
        }
        T dT0[3], dT1[3];
        for (int c = 0; c < 3; c++) {
            dT0[c] = dN[0] * S.M[3 * c] + dN[1] * S.M[3 * c + 1] + dN[2] * S.M[3 * c + 2];
            dT1[c] = dN[3] * S.M[3 * c] + dN[4] * S.M[3 * c + 1] + dN[5] * S.M[3 * c + 2];
        }
        for (int c = 0; c < 3; c++)
            for (int k2 = 0; k2 < 3; k2++) gM[3 * c + k2] += g.Tm[c] * dN[k2] + g.Tm[3 + c] * dN[3 + k2];
        // Tm = J R
        T dJ00 = dT0[0] * k.R[0] + dT0[1] * k.R[1] + dT0[2] * k.R[2];
        T dJ02 = dT0[0] * k.R[6] + dT0[1] * k.R[7] + dT0[2] * k.R[8];
        T dJ11 = dT1[0] * k.R[3] + dT1[1] * k.R[4] + dT1[2] * k.R[5];
        T dJ12 = dT1[0] * k.R[6] + dT1[1] * k.R[7] + dT1[2] * k.R[8];
        dy[2] += -(dJ00 * k.fx + dJ11 * k.fy) * iz2 + (dJ02 * k.fx * g.xi + dJ12 * k.fy * g.eta) * iz2;
        T dxi = -dJ02 * k.fx * iz, deta = -dJ12 * k.fy * iz;
        if (!g.xi_cl) { dy[0] += dxi * iz; dy[2] -= dxi * g.y[0] * iz2; }
        if (!g.eta_cl) { dy[1] += deta * iz; dy[2] -= deta * g.y[1] * iz2; }
        for (int c = 0; c < 3; c++) gmean[c] += k.R[c] * dy[0] + k.R[3 + c] * dy[1] + k.R[6 + c] * dy[2];
        gop += dop;
    }
    // M = Rq diag(s) -> scale and rotation
    T gls[3], dRq[9];
    for (int c = 0; c < 3; c++) {
        T acc = T(0);
        for (int r = 0; r < 3; r++) {
            dRq[3 * r + c] = gM[3 * r + c] * S.s[c];
            acc += gM[3 * r + c] * S.Rq[3 * r + c];
        }
        gls[c] = acc * S.s[c];
    }
    T w = S.q[0], qx = S.q[1], qy = S.q[2], qz = S.q[3];
    T dq[4];
    dq[0] = T(2) * (-qz * dRq[1] + qy * dRq[2] + qz * dRq[3] - qx * dRq[5] - qy * dRq[6] + qx * dRq[7]);
    dq[1] = T(2) * (qy * dRq[1] + qz * dRq[2] + qy * dRq[3] - T(2) * qx * dRq[4] - w * dRq[5] + qz * dRq[6] +
                    w * dRq[7] - T(2) * qx * dRq[8]);
    dq[2] = T(2) * (-T(2) * qy * dRq[0] + qx * dRq[1] + w * dRq[2] + qx * dRq[3] + qz * dRq[5] - w * dRq[6] +
                    qz * dRq[7] - T(2) * qy * dRq[8]);
    dq[3] = T(2) * (-T(2) * qz * dRq[0] - w * dRq[1] + qx * dRq[2] + w * dRq[3] - T(2) * qz * dRq[4] +
                    qy * dRq[5] + qx * dRq[6] + qy * dRq[7]);
    T dot = dq[0] * S.q[0] + dq[1] * S.q[1] + dq[2] * S.q[2] + dq[3] * S.q[3];
    T iqn = rcp_t(S.qn);
    for (int c = 0; c < 3; c++) {
        gpos[c] = gmean[c];
        g8[c] = gls[c];
    }
    for (int j = 0; j < 4; j++) g8[3 + j] = (dq[j] - S.q[j] * dot) * iqn;
    g8[7] = gop * S.opac * (T(1) - S.opac);
}

template <typename T, bool ADAM>
__global__ void __launch_bounds__(256) project_bwd_kernel(T *__restrict__ P, int64_t n,
                                                          const gs_camera *__restrict__ cams, int32_t views,
                                                          const T *__restrict__ proj, T *__restrict__ dproj, int clear,
                                                          T *__restrict__ grad, AdamRef<T> ad)
{
    __shared__ Camera<T> cs[MAXV];
    stage_cameras(cs, cams, views);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t ib = (uint32_t)i * (uint32_t)sizeof(T);          // lane offset in a parameter row
    uint64_t vis = 0;
    const uint32_t *tiles = side_tiles<T>(proj, (int64_t)views * n);
    for (int v = 0; v < views; v++)
        if (load_at(tiles + (int64_t)v * n, 4u * (uint32_t)i) > 0u) vis |= 1ull << v;
    // Gaussians seen by no view have nothing to add and, with ADAM, take the
    // step with a zero gradient. Seen and unseen Gaussians share wavefronts
    // (visibility is scattered over the index range), so the gradients are
    // formed under `seen` and every Adam block below runs once for all lanes.
    const bool seen = vis != 0;
    if (!ADAM && !seen) return;
    T x[3] = {T(0), T(0), T(0)};
    if (seen) {
        x[0] = load_at(P, ib);
        x[1] = load_at(P + n, ib);
        x[2] = load_at(P + 2 * n, ib);
    }
    T gpos[3] = {T(0), T(0), T(0)};
    {
        T g8[8] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
        if (seen) geom_grads(P, n, i, x, cs, views, vis, dproj, gpos, g8);
        if (!ADAM) {
            for (int r = 0; r < 8; r++) store_at(grad + (3 + r) * n, ib, load_at(grad + (3 + r) * n, ib) + g8[r]);
        } else {
            for (int r = 0; r < 8; r++) g8[r] = T(0) + g8[r];   // as += into a zero gradient
            adam_row_block<T, 8>(P, ad, 3, n, ib, g8);          // rows 3-10
        }
    }
    asm volatile("" ::: "memory");
    T gsh[3][16];
    for (int k2 = 0; k2 < 16; k2++)
        for (int c = 0; c < 3; c++) gsh[c][k2] = T(0);
    T gmean[3] = {0, 0, 0};
    if (seen) {
        T sh[3][16];
        for (int k2 = 0; k2 < 16; k2++)
            for (int c = 0; c < 3; c++) sh[c][k2] = load_at(P + (11 + 3 * k2 + c) * n, ib);
        uint64_t rem = vis;                  // the next seen view's colour gradient is loaded ahead
        T nrgb[3] = {T(0), T(0), T(0)};
        // (per-lane addresses: the next seen view differs between lanes)
        auto rgb_of = [&](uint64_t r) { return dproj + ((int64_t)__builtin_ctzll(r) * n + i) * REC + D_RGB; };
        if (rem) {
            const T *dr = rgb_of(rem);
            for (int c = 0; c < 3; c++) nrgb[c] = dr[c];
        }
        for (int v = 0; v < views; v++) {
            if (!((vis >> v) & 1ull)) continue;
            T drgb[3] = {nrgb[0], nrgb[1], nrgb[2]};
            rem &= rem - 1ull;
            if (rem) {
                const T *dr = rgb_of(rem);
                for (int c = 0; c < 3; c++) nrgb[c] = dr[c];
            }
            const T *cen = cs[v].cen;
            T d[3] = {x[0] - cen[0], x[1] - cen[1], x[2] - cen[2]};
            T idn = rsq_t(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);   // as the forward, so the clamp agrees
            T dir[3] = {d[0] * idn, d[1] * idn, d[2] * idn};
            T Y[16];
            sh_basis(dir[0], dir[1], dir[2], Y);
            T raw[3] = {T(0), T(0), T(0)};   // each summed in the forward's order, so the clamp mask agrees
            for (int k2 = 0; k2 < 16; k2++)
                for (int c = 0; c < 3; c++) raw[c] = fma(sh[c][k2], Y[k2], raw[c]);
            T a[3];                          // dL/drgb of the unclamped channels, 0 for clamped ones
            for (int c = 0; c < 3; c++) a[c] = raw[c] + T(0.5) > T(0) ? drgb[c] : T(0);
            if (!(raw[0] + T(0.5) > T(0)) && !(raw[1] + T(0.5) > T(0)) && !(raw[2] + T(0.5) > T(0))) continue;
            for (int k2 = 0; k2 < 16; k2++)
                for (int c = 0; c < 3; c++) gsh[c][k2] = fma(a[c], Y[k2], gsh[c][k2]);
            T gd[3];
            sh_grad(dir[0], dir[1], dir[2], [&](int k2) { return fma(a[2], sh[2][k2], fma(a[1], sh[1][k2], a[0] * sh[0][k2])); },
                    gd);
            T dd = gd[0] * dir[0] + gd[1] * dir[1] + gd[2] * dir[2];
            for (int j = 0; j < 3; j++) gmean[j] += (gd[j] - dir[j] * dd) * idn;
        }
    }
    if (!ADAM) {
        for (int k2 = 0; k2 < 16; k2++)
            for (int c = 0; c < 3; c++) {
                T *row = grad + (11 + 3 * k2 + c) * n;
                store_at(row, ib, load_at(row, ib) + gsh[c][k2]);
            }
        for (int j = 0; j < 3; j++) store_at(grad + j * n, ib, (load_at(grad + j * n, ib) + gpos[j]) + gmean[j]);
    } else if (!adam_skipped(ad)) {
        // position rows, then the SH rows 11 .. 58 eight at a time (row - 11
        // = 3 k + c), each block's loads issued before the previous block is
        // updated and stored: two blocks in flight
        T g3[3];
        for (int j = 0; j < 3; j++) g3[j] = (T(0) + gpos[j]) + gmean[j];
        AdamRows<T, 3> b3;
        AdamRows<T, 8> cur, nxt;
        adam_load(b3, P, ad, 0, n, ib);
        adam_load(cur, P, ad, 11, n, ib);
        adam_store(b3, P, ad, 0, n, ib, g3);
#pragma unroll
        for (int b = 0; b < 6; b++) {
            if (b < 5) adam_load(nxt, P, ad, 11 + 8 * (b + 1), n, ib);
            T gb[8];
#pragma unroll
            for (int r = 0; r < 8; r++) {
                const int t = 8 * b + r;
                gb[r] = T(0) + gsh[t % 3][t / 3];
            }
            adam_store(cur, P, ad, 11 + 8 * b, n, ib, gb);
            if (b < 5) cur = nxt;
        }
    }
    if (clear) {
        const uint32_t rb = (uint32_t)i * (uint32_t)(REC * sizeof(T));
        for (int v = 0; v < views; v++)
            if ((vis >> v) & 1ull) {
                T *rec = dproj + (int64_t)v * n * REC;
                store4_at(rec, rb, T(0), T(0), T(0), T(0));
                store4_at(rec + 4, rb, T(0), T(0), T(0), T(0));
                store4_at(rec + 8, rb, T(0), T(0), T(0), T(0));
            }
    }
}

template <typename T>
hipError_t launch_project_fwd(const void *P, int64_t n, const gs_camera *cams, int32_t views, void *out,
                              hipStream_t s)
{
    if (n == 0) return hipSuccess;
    // each XCD takes ceil(chunks / 8) chunks x views items, four per workgroup
    int64_t items_per_xcd = ((n + 63) / 64 + 7) / 8 * views;
    int64_t grid = 8 * ((items_per_xcd + 3) / 4);
    hipLaunchKernelGGL(project_fwd_kernel<T>, dim3((unsigned)grid), dim3(256), 0, s, (const T *)P, n, cams, views,
                       (T *)out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_project_bwd(const void *P, int64_t n, const gs_camera *cams, int32_t views, const void *proj,
                              void *dproj, int clear, void *grad, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    AdamRef<T> none{};
    hipLaunchKernelGGL((project_bwd_kernel<T, false>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       const_cast<T *>((const T *)P), n, cams, views, (const T *)proj, (T *)dproj, clear, (T *)grad,
                       none);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_project_bwd_adam(void *P, int64_t n, const gs_camera *cams, int32_t views, const void *proj,
                                   void *dproj, void *grad, void *m, void *v, const gs_adam_hparams *h,
                                   int64_t *step, double *scratch, const int32_t *skip, hipStream_t s)
{
    AdamRef<T> ad{(T *)m, (T *)v, make_adam_const(h), scratch};
    hipError_t e = launch_adam_prepare(step, ad.c, scratch, skip, s);
    if (n == 0 || e != hipSuccess) return e;
    hipLaunchKernelGGL((project_bwd_kernel<T, true>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (T *)P, n,
                       cams, views, (const T *)proj, (T *)dproj, 1, (T *)grad, ad);
    return hipGetLastError();
}

template hipError_t launch_project_fwd<float>(const void *, int64_t, const gs_camera *, int32_t, void *, hipStream_t);
template hipError_t launch_project_fwd<double>(const void *, int64_t, const gs_camera *, int32_t, void *, hipStream_t);
template hipError_t launch_project_bwd<float>(const void *, int64_t, const gs_camera *, int32_t, const void *, void *,
                                              int, void *, hipStream_t);
template hipError_t launch_project_bwd<double>(const void *, int64_t, const gs_camera *, int32_t, const void *, void *,
                                               int, void *, hipStream_t);
template hipError_t launch_project_bwd_adam<float>(void *, int64_t, const gs_camera *, int32_t, const void *, void *,
                                                   void *, void *, void *, const gs_adam_hparams *, int64_t *,
                                                   double *, const int32_t *, hipStream_t);
template hipError_t launch_project_bwd_adam<double>(void *, int64_t, const gs_camera *, int32_t, const void *, void *,
                                                    void *, void *, void *, const gs_adam_hparams *, int64_t *,
                                                    double *, const int32_t *, hipStream_t);

}  // namespace gs
