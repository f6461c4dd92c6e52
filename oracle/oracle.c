/*
 * FP64 CPU oracle of the batched 3D Gaussian Splatting training step.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link or call
 * this file: it is loaded by the tests, by the smoke check and by the CPU
 * baseline leg of the benchmark. It shares no code, header, table or
 * constant with the HIP path.
 *
 * What it computes (section "Background on 3D Gaussian Training" of the
 * paper, steps 1-3, plus back-propagation and the optimizer of the section
 * "Scaling Hyperparameters for Batched Training"):
 *
 *   1. Gaussian transformation: per (view, Gaussian) the on-screen position,
 *      depth, footprint radius and view-dependent colour from the Gaussian's
 *      position, scale + rotation (covariance), opacity and 48 SH values.
 *   2. Rendering: for each pixel the Gaussians whose footprint contains it,
 *      composed front to back by increasing depth until an opacity threshold.
 *   3. Loss: per-pixel L1 (kept in the Python shim, it is one line).
 *   4. Back-propagation of 1-3 to every parameter.
 *   5. Adam with the learning rate scaled by sqrt(batch) (eq. "lambda") and
 *      both moment decay rates raised to the power batch (eq. "beta").
 *
 * The paper does not print the rasterizer's formulas or constants; the
 * readings taken here (EWA projection with a 0.3 px low-pass, radius =
 * ceil(3 sqrt(lambda_max)), alpha clamped at 0.99, skipped below 1/255, stop
 * before a blend that would bring T below 1e-4, degree-3 real orthonormal SH
 * with +0.5 offset and clamp at 0, 16x16 tiles, pixel centres at +0.5) are the
 * ones listed in the design notes of the repository and are the same readings
 * the HIP path implements independently.
 *
 * Everything is double precision except where a floating-point value decides
 * an integer for binning (the tile rectangle of a Gaussian, the depth key):
 * those decisions take FP32 inputs and FP32 arithmetic, the precision the
 * GPU kernels compute in.
 *
 * Parity pins of every function live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ONF 12 /* projected fields per (view, Gaussian), see oracle_project */
#define TILE 16

/* ------------------------------------------------------------------ cameras
 * A camera is 19 doubles: width, height, fx, fy, cx, cy, R[9] (world to
 * camera, row-major), t[3], znear. Camera frame: +x right, +y down, +z
 * forward. */
typedef struct {
    int W, H;
    double fx, fy, cx, cy, R[9], t[3], znear;
} cam_t;

static cam_t cam_load(const double *c)
{
    cam_t k;
    k.W = (int)c[0];
    k.H = (int)c[1];
    k.fx = c[2]; k.fy = c[3]; k.cx = c[4]; k.cy = c[5];
    for (int j = 0; j < 9; j++) k.R[j] = c[6 + j];
    for (int j = 0; j < 3; j++) k.t[j] = c[15 + j];
    k.znear = c[18];
    return k;
}

/* ------------------------------------------------------------------ spherical harmonics
 * Real orthonormal spherical harmonics Y_lm, l <= 3, index k = l*l + l + m.
 * Written from the definition: with the Condon-Shortley phase inside the
 * associated Legendre function P_l^m(z) = (-1)^m (1-z^2)^(m/2) d^m P_l/dz^m,
 * and sin^m(theta) e^{i m phi} = (x + i y)^m on the unit sphere,
 *   m = 0 : Y = K_l0 P_l(z)
 *   m > 0 : Y = sqrt(2) K_lm (-1)^m P_l^(m)(z) Re (x+iy)^m
 *   m < 0 : Y = sqrt(2) K_l|m| (-1)^|m| P_l^(|m|)(z) Im (x+iy)^|m|
 * with K_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!). These are polynomials in
 * (x, y, z); their gradient is taken on that polynomial extension and the
 * caller projects it onto the sphere's tangent plane. */
static double fact(int n) { double f = 1.0; for (int i = 2; i <= n; i++) f *= i; return f; }

static void legendre_coeffs(double leg[4][4])
{
    memset(leg, 0, sizeof(double) * 16);
    leg[0][0] = 1.0;           /* P0 = 1 */
    leg[1][1] = 1.0;           /* P1 = z */
    for (int n = 1; n < 3; n++) /* (n+1) P_{n+1} = (2n+1) z P_n - n P_{n-1} */
        for (int j = 0; j < 4; j++) {
            double zpn = j > 0 ? leg[n][j - 1] : 0.0;
            leg[n + 1][j] = ((2 * n + 1) * zpn - n * leg[n - 1][j]) / (n + 1);
        }
}

static double poly(const double *c, double z) { return c[0] + z * (c[1] + z * (c[2] + z * c[3])); }

static void sh_basis(const double d[3], double Y[16], double dY[16][3])
{
    double leg[4][4];
    legendre_coeffs(leg);
    double x = d[0], y = d[1], z = d[2];
    /* re[m] + i im[m] = (x + i y)^m */
    double re[4], im[4];
    re[0] = 1.0; im[0] = 0.0;
    for (int m = 1; m < 4; m++) {
        re[m] = re[m - 1] * x - im[m - 1] * y;
        im[m] = re[m - 1] * y + im[m - 1] * x;
    }
    for (int l = 0; l <= 3; l++)
        for (int m = -l; m <= l; m++) {
            int am = m < 0 ? -m : m;
            int k = l * l + l + m;
            /* A = (-1)^am d^am P_l / dz^am, and its derivative */
            double A[4] = {0, 0, 0, 0}, dA[4] = {0, 0, 0, 0};
            for (int j = 0; j < 4; j++) A[j] = leg[l][j];
            for (int r = 0; r < am; r++) {
                for (int j = 0; j < 3; j++) A[j] = (j + 1) * A[j + 1];
                A[3] = 0.0;
            }
            if (am & 1) for (int j = 0; j < 4; j++) A[j] = -A[j];
            for (int j = 0; j < 3; j++) dA[j] = (j + 1) * A[j + 1];
            double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * fact(l - am) / fact(l + am));
            double Az = poly(A, z), dAz = poly(dA, z);
            if (m == 0) {
                Y[k] = K * Az;
                dY[k][0] = 0.0; dY[k][1] = 0.0; dY[k][2] = K * dAz;
            } else {
                double c = sqrt(2.0) * K;
                if (m > 0) {
                    Y[k] = c * Az * re[am];
                    dY[k][0] = c * Az * am * re[am - 1];
                    dY[k][1] = -c * Az * am * im[am - 1];
                    dY[k][2] = c * dAz * re[am];
                } else {
                    Y[k] = c * Az * im[am];
                    dY[k][0] = c * Az * am * im[am - 1];
                    dY[k][1] = c * Az * am * re[am - 1];
                    dY[k][2] = c * dAz * im[am];
                }
            }
        }
}

/* Exported for the basis pins (comparison with scipy's complex harmonics). */
void oracle_sh_basis(const double *dirs, int64_t n, double *Y /*[n][16]*/, double *dY /*[n][16][3]*/)
{
    for (int64_t i = 0; i < n; i++) {
        double yy[16], dd[16][3];
        sh_basis(dirs + 3 * i, yy, dd);
        memcpy(Y + 16 * i, yy, sizeof yy);
        if (dY) memcpy(dY + 48 * i, dd, sizeof dd);
    }
}

/* ------------------------------------------------------------------ geometry helpers */
static void quat_rot(const double q[4], double R[9]) /* unit q = (w, x, y, z) */
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* d R_e / d q_j for the 9 entries e and the 4 components j = (w, x, y, z). */
static void quat_rot_jac(const double q[4], double J[9][4])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double t[9][4] = {
        {0, 0, -4 * y, -4 * z},
        {-2 * z, 2 * y, 2 * x, -2 * w},
        {2 * y, 2 * z, 2 * w, 2 * x},
        {2 * z, 2 * y, 2 * x, 2 * w},
        {0, -4 * x, 0, -4 * z},
        {-2 * x, -2 * w, 2 * z, 2 * y},
        {-2 * y, 2 * z, -2 * w, 2 * x},
        {2 * x, 2 * w, 2 * z, 2 * y},
        {0, -4 * x, -4 * y, 0},
    };
    memcpy(J, t, sizeof t);
}

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* Everything the transformation of one (view, Gaussian) produces, including
 * the intermediates its derivative needs. */
typedef struct {
    int culled;
    double s[3], qn, qh[4], Rq[9], M[9], Sig[9];
    double y[3], xi, eta, xi_clamped, eta_clamped, J[6], Tm[6];
    double A, B, C, det, a, b, c, lmax, r_exact, radius;
    double u, v, depth, opac;
    double dir[3], dnorm, Y[16], dY[16][3], raw[3], rgb[3];
} proj_t;

static int finite_all(const double *p, int n)
{
    for (int j = 0; j < n; j++) if (!isfinite(p[j])) return 0;
    return 1;
}

/* Gaussian transformation of Gaussian i (parameter rows of P with stride N)
 * for camera k: section "Background on 3D Gaussian Training", step 1. */
static void project_one(const double *P, int64_t N, int64_t i, const cam_t *k, proj_t *o)
{
    memset(o, 0, sizeof *o);
    double x[3], ls[3], q[4], logit, sh[48];
    for (int j = 0; j < 3; j++) x[j] = P[(0 + j) * N + i];
    for (int j = 0; j < 3; j++) ls[j] = P[(3 + j) * N + i];
    for (int j = 0; j < 4; j++) q[j] = P[(6 + j) * N + i];
    logit = P[10 * N + i];
    for (int j = 0; j < 48; j++) sh[j] = P[(11 + j) * N + i];
    o->culled = 1;
    if (!finite_all(x, 3) || !finite_all(ls, 3) || !finite_all(q, 4) || !isfinite(logit) || !finite_all(sh, 48))
        return;
    /* activation: s = exp(l), q normalised, Sigma = R diag(s^2) R^T, opacity = sigmoid */
    for (int j = 0; j < 3; j++) o->s[j] = exp(ls[j]);
    o->qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(o->qn > 0.0)) return;
    for (int j = 0; j < 4; j++) o->qh[j] = q[j] / o->qn;
    quat_rot(o->qh, o->Rq);
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) o->M[3 * r + c] = o->Rq[3 * r + c] * o->s[c];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            double acc = 0.0;
            for (int j = 0; j < 3; j++) acc += o->M[3 * r + j] * o->M[3 * c + j];
            o->Sig[3 * r + c] = acc;
        }
    o->opac = 1.0 / (1.0 + exp(-logit));
    /* camera transform and near-plane cull */
    for (int r = 0; r < 3; r++)
        o->y[r] = k->R[3 * r] * x[0] + k->R[3 * r + 1] * x[1] + k->R[3 * r + 2] * x[2] + k->t[r];
    double z = o->y[2];
    if (!(z > k->znear)) return;
    o->u = k->fx * o->y[0] / z + k->cx;
    o->v = k->fy * o->y[1] / z + k->cy;
    o->depth = z;
    /* EWA: Jacobian of the perspective map at the (guard-banded) centre */
    double limx = 1.3 * (0.5 * k->W / k->fx), limy = 1.3 * (0.5 * k->H / k->fy);
    double xr = o->y[0] / z, yr = o->y[1] / z;
    o->xi = clampd(xr, -limx, limx);
    o->eta = clampd(yr, -limy, limy);
    o->xi_clamped = (xr < -limx || xr > limx);
    o->eta_clamped = (yr < -limy || yr > limy);
    o->J[0] = k->fx / z; o->J[1] = 0.0;        o->J[2] = -k->fx * o->xi / z;
    o->J[3] = 0.0;       o->J[4] = k->fy / z;  o->J[5] = -k->fy * o->eta / z;
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++) {
            double acc = 0.0;
            for (int j = 0; j < 3; j++) acc += o->J[3 * r + j] * k->R[3 * j + c];
            o->Tm[3 * r + c] = acc;
        }
    double S2[4];
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 2; c++) {
            double acc = 0.0;
            for (int m = 0; m < 3; m++)
                for (int n = 0; n < 3; n++) acc += o->Tm[3 * r + m] * o->Sig[3 * m + n] * o->Tm[3 * c + n];
            S2[2 * r + c] = acc;
        }
    o->A = S2[0] + 0.3;
    o->B = S2[1];
    o->C = S2[3] + 0.3;
    o->det = o->A * o->C - o->B * o->B;
    if (!(o->det > 0.0) || !isfinite(o->det)) return;
    o->a = o->C / o->det;
    o->b = -o->B / o->det;
    o->c = o->A / o->det;
    double mid = 0.5 * (o->A + o->C);
    double disc = mid * mid - o->det;
    o->lmax = mid + sqrt(disc > 0.0 ? disc : 0.0);
    o->r_exact = 3.0 * sqrt(o->lmax);
    o->radius = ceil(o->r_exact);
    if (!isfinite(o->radius) || !isfinite(o->u) || !isfinite(o->v)) return;
    /* colour from the SH by the world-space viewing direction */
    double cen[3];
    for (int c = 0; c < 3; c++)
        cen[c] = -(k->R[c] * k->t[0] + k->R[3 + c] * k->t[1] + k->R[6 + c] * k->t[2]);
    double dd[3] = {x[0] - cen[0], x[1] - cen[1], x[2] - cen[2]};
    o->dnorm = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
    for (int j = 0; j < 3; j++) o->dir[j] = dd[j] / o->dnorm;
    sh_basis(o->dir, o->Y, o->dY);
    for (int ch = 0; ch < 3; ch++) {
        double acc = 0.0;
        for (int kk = 0; kk < 16; kk++) acc += sh[3 * kk + ch] * o->Y[kk];
        o->raw[ch] = acc + 0.5;
        o->rgb[ch] = o->raw[ch] > 0.0 ? o->raw[ch] : 0.0;
    }
    o->culled = 0;
}

/* Projected fields per (view, Gaussian), planar [ONF][N]:
 * 0 u, 1 v, 2 depth, 3-5 conic (a, b, c), 6 opacity, 7-9 rgb, 10 radius
 * (integer valued, 0 = culled), 11 unrounded 3*sqrt(lambda_max). */
int oracle_project(const double *P, int64_t N, const double *cam, double *out)
{
    cam_t k = cam_load(cam);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        proj_t o;
        project_one(P, N, i, &k, &o);
        double f[ONF] = {0};
        if (!o.culled) {
            f[0] = o.u; f[1] = o.v; f[2] = o.depth;
            f[3] = o.a; f[4] = o.b; f[5] = o.c; f[6] = o.opac;
            f[7] = o.rgb[0]; f[8] = o.rgb[1]; f[9] = o.rgb[2];
            f[10] = o.radius; f[11] = o.r_exact;
        }
        for (int j = 0; j < ONF; j++) out[j * N + i] = f[j];
    }
    return 0;
}

/* ------------------------------------------------------------------ binning
 * 16x16 tiles (section "Pixel-wise Distribution" and appendix "Scheduling
 * Granularity"). The pixel rectangle of a Gaussian is the bounding box of its
 * footprint circle over pixel centres (p + 1/2), clipped to the image; its
 * tiles are those that rectangle meets. Computed in FP32 from FP32 inputs. */
static int tile_rect(float u, float v, float r, int W, int H, int *tx0, int *tx1, int *ty0, int *ty1)
{
    if (!(r > 0.0f)) return 0;
    float xlo = ceilf(u - r - 0.5f), xhi = floorf(u + r - 0.5f);
    float ylo = ceilf(v - r - 0.5f), yhi = floorf(v + r - 0.5f);
    xlo = fmaxf(xlo, 0.0f); ylo = fmaxf(ylo, 0.0f);
    xhi = fminf(xhi, (float)(W - 1)); yhi = fminf(yhi, (float)(H - 1));
    if (!(xlo <= xhi) || !(ylo <= yhi)) return 0;
    *tx0 = (int)xlo / TILE; *tx1 = (int)xhi / TILE;
    *ty0 = (int)ylo / TILE; *ty1 = (int)yhi / TILE;
    return 1;
}

static int64_t tiles_of(int W) { return (W + TILE - 1) / TILE; }

/* Number of tiles touched per (view, Gaussian); inputs concatenated per view [V][N]. */
int64_t oracle_tiles_touched(const float *u, const float *v, const float *r, int64_t N, int32_t V,
                             const int32_t *Ws, const int32_t *Hs, int32_t *out)
{
    int64_t K = 0;
    for (int32_t vi = 0; vi < V; vi++)
        for (int64_t i = 0; i < N; i++) {
            int64_t j = (int64_t)vi * N + i;
            int a, b, c, d;
            int32_t n = 0;
            if (tile_rect(u[j], v[j], r[j], Ws[vi], Hs[vi], &a, &b, &c, &d)) n = (b - a + 1) * (d - c + 1);
            out[j] = n;
            K += n;
        }
    return K;
}

typedef struct { uint64_t key; uint32_t id; } inst_t;

static int inst_cmp(const void *pa, const void *pb)
{
    const inst_t *a = pa, *b = pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->id < b->id ? -1 : (a->id > b->id ? 1 : 0);
}

/* Instances (global tile, depth) -> Gaussian, sorted lexicographically by
 * (global tile id, FP32 bits of depth, Gaussian index), plus [start, end) per
 * global tile (0, 0 when empty). Global tile id = tiles of earlier views +
 * ty * tiles_x + tx. Requires capacity >= K (see oracle_tiles_touched). */
int64_t oracle_bin(const float *u, const float *v, const float *r, const float *depth, int64_t N, int32_t V,
                   const int32_t *Ws, const int32_t *Hs, int64_t capacity,
                   uint64_t *keys, uint32_t *ids, uint32_t *ranges)
{
    int64_t ntiles = 0;
    for (int32_t vi = 0; vi < V; vi++) ntiles += tiles_of(Ws[vi]) * tiles_of(Hs[vi]);
    inst_t *buf = NULL;
    int64_t K = 0, cap = 1024;
    buf = malloc(sizeof(inst_t) * cap);
    int64_t base = 0;
    for (int32_t vi = 0; vi < V; vi++) {
        int64_t TX = tiles_of(Ws[vi]);
        for (int64_t i = 0; i < N; i++) {
            int64_t j = (int64_t)vi * N + i;
            int a, b, c, d;
            if (!tile_rect(u[j], v[j], r[j], Ws[vi], Hs[vi], &a, &b, &c, &d)) continue;
            float df = depth[j];
            uint32_t dbits;
            memcpy(&dbits, &df, 4);
            for (int ty = c; ty <= d; ty++)
                for (int tx = a; tx <= b; tx++) {
                    if (K == cap) { cap *= 2; buf = realloc(buf, sizeof(inst_t) * cap); }
                    uint64_t tile = (uint64_t)(base + (int64_t)ty * TX + tx);
                    buf[K].key = (tile << 32) | dbits;
                    buf[K].id = (uint32_t)i;
                    K++;
                }
        }
        base += TX * tiles_of(Hs[vi]);
    }
    if (K > capacity) { free(buf); return -K; }
    qsort(buf, (size_t)K, sizeof(inst_t), inst_cmp);
    for (int64_t t = 0; t < 2 * ntiles; t++) ranges[t] = 0;
    for (int64_t k2 = 0; k2 < K; k2++) {
        keys[k2] = buf[k2].key;
        ids[k2] = buf[k2].id;
        uint64_t tile = buf[k2].key >> 32;
        if (k2 == 0 || (buf[k2 - 1].key >> 32) != tile) ranges[2 * tile] = (uint32_t)k2;
        if (k2 == K - 1 || (buf[k2 + 1].key >> 32) != tile) ranges[2 * tile + 1] = (uint32_t)(k2 + 1);
    }
    free(buf);
    return K;
}

/* ------------------------------------------------------------------ rendering
 * Section "Background on 3D Gaussian Training", step 2: for a pixel p, the
 * Gaussians whose footprint radius contains p, in increasing depth, alpha
 * composed front to back until the transmittance threshold. */
#define ALPHA_MAX 0.99
#define ALPHA_MIN (1.0 / 255.0)
#define T_MIN 1e-4

typedef struct {
    int inside;    /* passes the circle test and power <= 0 */
    double dx, dy, G, og, alpha;
    double alpha_rel;   /* bound on the relative error of alpha in FP32 */
    double alpha_mrel;  /* the decision margin's relative width (alpha_rel with a 4x safety) */
} pair_t;

/* Ambiguity margins. A decision is ambiguous when the quantity it compares
 * is within rounding of its threshold: pos_tol (pixels) bounds how far the
 * compared implementation's projected centre may sit from this one's (0
 * when both render the same projected records). */
typedef struct { double pos_tol, t_tol; } tol_t;

/* The binary decisions of one pixel's walk (circle, exponent sign, alpha
 * threshold, transmittance stop) that fall within rounding of their
 * thresholds. An implementation in lower precision may take either branch
 * of such a decision and still be right, so the walk can be re-run with the
 * flip_at-th ambiguous decision taken the other way; count is the number of
 * ambiguous decisions met, unresolved is set by an ambiguity that a single
 * flip does not describe (two contributors whose depth order may differ). */
typedef struct { int count, flip_at, unresolved; } amb_t;

static int decide(amb_t *am, int outcome, int ambiguous)
{
    if (!am || !ambiguous) return outcome;
    int k = am->count++;
    return k == am->flip_at ? !outcome : outcome;
}

/* One (pixel, Gaussian) pair. proj is planar [ONF][N]. fragile (nullable):
 * the Gaussian's radius may round to the next integer in the compared
 * implementation, which moves its circle test on the annulus
 * r - 1 <= d <= r + 1. */
static void eval_pair(const double *proj, int64_t N, uint32_t id, int px, int py, const tol_t *tol, int fragile,
                      amb_t *am, pair_t *e)
{
    double u = proj[0 * N + id], v = proj[1 * N + id], r = proj[10 * N + id];
    double a = proj[3 * N + id], b = proj[4 * N + id], c = proj[5 * N + id], o = proj[6 * N + id];
    double pt = tol ? tol->pos_tol : 0.0;
    e->inside = 0;
    e->dx = px + 0.5 - u;
    e->dy = py + 0.5 - v;
    double d2 = e->dx * e->dx + e->dy * e->dy, r2 = r * r;
    int amb = fabs(d2 - r2) <= 1e-6 * (r2 > 1.0 ? r2 : 1.0) + 2.0 * r * pt + pt * pt;
    if (fragile) {
        /* the unrounded radius sits near the integer m, so the other side
         * may hold m or m + 1: the circle test differs on m <= d <= m + 1 */
        double m = nearbyint(proj[11 * N + id]);
        if (d2 >= m * m && d2 <= (m + 1.0) * (m + 1.0)) amb = 1;
    }
    if (!decide(am, d2 <= r2, amb)) return;
    double qa = 0.5 * a * e->dx * e->dx, qc = 0.5 * c * e->dy * e->dy, qb = b * e->dx * e->dy;
    double power = -qa - qc - qb;
    amb = fabs(power) <= 1e-6 * (fabs(qa) + fabs(qb) + fabs(qc)) && (qa + qc) > 0.0;
    if (!decide(am, power <= 0.0, amb)) return;
    e->G = exp(power);
    e->og = o * e->G;
    e->alpha = e->og < ALPHA_MAX ? e->og : ALPHA_MAX;
    /* Rounding of the exponent in FP32: its three terms are formed and summed
     * with a few roundings each, so the error is bounded by a small multiple
     * of the unit roundoff times S = |qa| + |qb| + |qc| (not |power|: for a
     * thin footprint the terms are large and cancel), plus the exp and the
     * opacity product: about 9 u S + 4 u with u = 2^-24 (alpha_rel); four
     * times that is the decision margin. Against another implementation's
     * own projection the exponent also carries its conic's error (1e-5
     * relative to the terms) and the change when the centre moves by
     * pos_tol. */
    double S = fabs(qa) + fabs(qb) + fabs(qc);
    double ulp = 5.9604644775390625e-8;                 /* 2^-24 */
    double cr = (pt > 0.0 ? 1e-5 * S : 0.0);
    double mrel = 1e-6 + 2e-6 * S + cr;
    e->alpha_rel = e->og < ALPHA_MAX ? 9.0 * ulp * S + 4.0 * ulp + cr : 1e-7;
    e->alpha_mrel = e->og < ALPHA_MAX ? mrel : 1e-7;
    double lmargin = mrel + 2.0 * sqrt(fabs(power) * (a + c)) * pt;
    amb = fabs(log(e->alpha / ALPHA_MIN)) <= lmargin;
    if (!decide(am, e->alpha >= ALPHA_MIN, amb)) return;
    e->inside = 1;
}

static int depth_near(const double *proj, int64_t N, uint32_t i0, uint32_t i1)
{
    float d0 = (float)proj[2 * N + i0], d1 = (float)proj[2 * N + i1];
    uint32_t b0, b1;
    memcpy(&b0, &d0, 4);
    memcpy(&b1, &d1, 4);
    uint32_t gap = b0 > b1 ? b0 - b1 : b1 - b0;
    return gap <= 2;
}

/* Forward composition of one pixel over list[0..n). Writes colour, T, the
 * position after the last blended entry, the number blended and the number
 * of entries evaluated; am (nullable) tracks and flips ambiguous decisions. */
static void composite_pixel(const double *proj, int64_t N, const uint32_t *list, int64_t n, int px, int py,
                            const double *bg, const uint8_t *fragile, int depth_check, const tol_t *tol,
                            amb_t *am, double out[3], double *Tout, uint32_t *last, uint32_t *ncontrib,
                            int64_t *evaluated, double *bound)
{
    double T = 1.0, C[3] = {0, 0, 0};
    uint32_t lastp = 0, nc = 0;
    int64_t prev = -1;
    int64_t ev = 0;
    /* bound on the relative error of T in FP32: per blend the update's own
     * roundings, plus 1 - alpha's, which grows as alpha / (1 - alpha) times
     * alpha's relative error (t_rel); the stop decision's margin grows the
     * same way from alpha's margin (t_mrel) */
    double t_rel = 0.0, t_mrel = 0.0;
    /* first-order colour error from alpha's relative error: moving alpha_i
     * by a fraction e changes the colour by at most e alpha_i T_i times the
     * largest colour of the pixel (its own, or what lies behind it) */
    double cmax = 0.0, werr = 0.0;
    for (int ch = 0; ch < 3; ch++) cmax = fmax(cmax, fabs(bg[ch]));
    for (int64_t k = 0; k < n; k++) {
        /* two adjacent entries of the list that both reach this pixel and
         * whose FP32 depths nearly tie: the compared implementation (which
         * rounds its own depths) may hold them in the other order */
        int swap = 0;
        if (am && depth_check && k + 1 < n && depth_near(proj, N, list[k], list[k + 1])) {
            pair_t t0, t1;
            eval_pair(proj, N, list[k], px, py, tol, fragile ? fragile[list[k]] : 0, NULL, &t0);
            eval_pair(proj, N, list[k + 1], px, py, tol, fragile ? fragile[list[k + 1]] : 0, NULL, &t1);
            if (t0.inside && t1.inside) swap = decide(am, 0, 1);
        }
        int stop = 0;
        for (int s = 0; s <= swap && !stop; s++) {
            int64_t pos = k + s;
            uint32_t id = list[swap ? k + 1 - s : k];
            pair_t e;
            eval_pair(proj, N, id, px, py, tol, fragile ? fragile[id] : 0, am, &e);
            ev++;
            if (!e.inside) continue;
            double Tn = T * (1.0 - e.alpha);
            double tr = t_rel + 1.2e-7 + e.alpha / (1.0 - e.alpha) * e.alpha_rel;
            double tm = t_mrel + 2.4e-7 + e.alpha / (1.0 - e.alpha) * e.alpha_mrel;
            int amb = fabs(Tn - T_MIN) <= ((tol ? tol->t_tol : 1e-5) + tm) * T_MIN;
            if (decide(am, Tn < T_MIN, amb)) { stop = 1; break; }
            /* a near tie with a contributor that is not the adjacent entry */
            if (am && depth_check && prev >= 0 && (int64_t)lastp != pos && depth_near(proj, N, (uint32_t)prev, id))
                am->unresolved = 1;
            for (int ch = 0; ch < 3; ch++) {
                C[ch] += proj[(7 + ch) * N + id] * e.alpha * T;
                cmax = fmax(cmax, fabs(proj[(7 + ch) * N + id]));
            }
            werr += e.alpha * T * e.alpha_rel;
            T = Tn;
            t_rel = tr;
            t_mrel = tm;
            lastp = (uint32_t)(pos + 1);
            nc++;
            prev = id;
        }
        if (stop) break;
        k += swap;
    }
    for (int ch = 0; ch < 3; ch++) out[ch] = C[ch] + T * bg[ch];
    *Tout = T;
    *last = lastp;
    *ncontrib = nc;
    *evaluated = ev;
    if (bound) *bound = fmax(cmax * (werr + T * t_rel), T * t_rel);
}

/* Tiled render of one view. proj: [ONF][N] of this view; ids/ranges: the
 * sorted instances and the view's slice of per-tile [start, end) ranges
 * (T_view entries, positions index ids). Outputs are planar [3][H][W] colour,
 * [H][W] transmittance, last position, contributor count and ambiguity class:
 * 0 no decision within rounding of its threshold; 1 exactly one, and the
 * nullable alternative outputs (rgb_alt, T_alt, last_alt) hold the walk with
 * that decision taken the other way; 2 more than one, or a depth-order tie.
 * counts[0] = list entries evaluated, counts[1] = blended pairs (nominal walk).
 * bound (nullable): per pixel, a first-order bound of how far an FP32
 * evaluation of the same walk may put its colour and T, from the relative
 * error bound of each blended alpha (the larger of the two branches). */
int oracle_render(const double *proj, int64_t N, int32_t W, int32_t H, const uint32_t *ids,
                  const uint32_t *ranges, const double *bg, const uint8_t *fragile, int32_t depth_check,
                  double pos_tol, double t_tol,
                  double *rgb, double *Tout, uint32_t *last, uint32_t *ncontrib, uint8_t *amb, int64_t *counts,
                  double *rgb_alt, double *T_alt, uint32_t *last_alt, double *bound)
{
    tol_t tol = {pos_tol, t_tol};
    int64_t TX = tiles_of(W), TY = tiles_of(H);
    int64_t ev_total = 0, nc_total = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : ev_total, nc_total)
    for (int64_t t = 0; t < TX * TY; t++) {
        int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
        int tx = (int)(t % TX), ty = (int)(t / TX);
        for (int py = ty * TILE; py < ty * TILE + TILE && py < H; py++)
            for (int px = tx * TILE; px < tx * TILE + TILE && px < W; px++) {
                double c[3], T;
                uint32_t l, nc;
                int64_t ev;
                amb_t am = {0, -1, 0};
                double bd, bda = 0.0;
                composite_pixel(proj, N, ids + s, e - s, px, py, bg, fragile, depth_check, &tol, &am, c, &T, &l,
                                &nc, &ev, &bd);
                int64_t p = (int64_t)py * W + px;
                for (int ch = 0; ch < 3; ch++) rgb[(int64_t)ch * W * H + p] = c[ch];
                Tout[p] = T;
                last[p] = l;
                if (ncontrib) ncontrib[p] = nc;
                ev_total += ev;
                nc_total += nc;
                uint8_t cls = am.unresolved || am.count > 1 ? 2 : (uint8_t)am.count;
                double ca[3] = {c[0], c[1], c[2]}, Ta = T;
                uint32_t la = l;
                if (cls == 1) {
                    /* the other branch of the one ambiguous decision; it is
                     * a single alternative only if that walk meets no other */
                    amb_t alt = {0, 0, 0};
                    uint32_t nca;
                    int64_t eva;
                    composite_pixel(proj, N, ids + s, e - s, px, py, bg, fragile, depth_check, &tol, &alt, ca, &Ta,
                                    &la, &nca, &eva, &bda);
                    if (alt.unresolved || alt.count > 1) cls = 2;
                }
                if (amb) amb[p] = cls;
                if (rgb_alt)
                    for (int ch = 0; ch < 3; ch++) rgb_alt[(int64_t)ch * W * H + p] = ca[ch];
                if (T_alt) T_alt[p] = Ta;
                if (last_alt) last_alt[p] = la;
                if (bound) bound[p] = fmax(bd, bda);
            }
    }
    if (counts) { counts[0] = ev_total; counts[1] = nc_total; }
    return 0;
}

static int64_t *g_sort_keys; /* qsort context for the brute-force order */
static int brute_cmp(const void *pa, const void *pb)
{
    uint32_t a = *(const uint32_t *)pa, b = *(const uint32_t *)pb;
    uint64_t ka = (uint64_t)g_sort_keys[a], kb = (uint64_t)g_sort_keys[b];
    if (ka != kb) return ka < kb ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* The plain definition without tiling: every pixel against every Gaussian
 * with a positive radius, in increasing (FP32 depth bits, index). */
int oracle_render_brute(const double *proj, int64_t N, int32_t W, int32_t H, const double *bg,
                        double *rgb, double *Tout, uint32_t *ncontrib)
{
    uint32_t *order = malloc(sizeof(uint32_t) * (N > 0 ? N : 1));
    int64_t *keys = malloc(sizeof(int64_t) * (N > 0 ? N : 1));
    int64_t n = 0;
    for (int64_t i = 0; i < N; i++) {
        float df = (float)proj[2 * N + i];
        uint32_t bits;
        memcpy(&bits, &df, 4);
        keys[i] = bits;
        if (proj[10 * N + i] > 0.0) order[n++] = (uint32_t)i;
    }
    g_sort_keys = keys;
    qsort(order, (size_t)n, sizeof(uint32_t), brute_cmp);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < (int64_t)W * H; p++) {
        int px = (int)(p % W), py = (int)(p / W);
        double c[3], T;
        uint32_t l, nc;
        int64_t ev;
        composite_pixel(proj, N, order, n, px, py, bg, NULL, 0, NULL, NULL, c, &T, &l, &nc, &ev, NULL);
        for (int ch = 0; ch < 3; ch++) rgb[(int64_t)ch * W * H + p] = c[ch];
        Tout[p] = T;
        if (ncontrib) ncontrib[p] = nc;
    }
    free(order);
    free(keys);
    return 0;
}

/* ------------------------------------------------------------------ render backward
 * Chain rule of the composition, per pixel, with the forward list stored
 * (no division): with B the colour composed behind entry k (starting at the
 * background and updated after use as B <- alpha_k c_k + (1 - alpha_k) B),
 *   dL/dc_k     = alpha_k T_k g
 *   dL/dalpha_k = T_k <g, c_k - B>
 * then alpha = min(0.99, o exp(power)) with
 * power = -(a dx^2 + c dy^2)/2 - b dx dy and (dx, dy) = pixel centre - (u, v).
 * Writes, per Gaussian of this view, d/d(u, v, a, b, c, opacity, r, g, b)
 * planar [9][N], accumulated (+=). */
typedef struct { uint32_t k; double alpha, T, G, og, dx, dy; } rec_t;

int oracle_render_bwd(const double *proj, int64_t N, int32_t W, int32_t H, const uint32_t *ids,
                      const uint32_t *ranges, const double *bg, const double *dL_drgb, double *dproj)
{
    int64_t TX = tiles_of(W), TY = tiles_of(H);
    int64_t kbeg = -1, kend = 0;
    for (int64_t t = 0; t < TX * TY; t++)
        if (ranges[2 * t + 1] > ranges[2 * t]) {
            if (kbeg < 0) kbeg = ranges[2 * t];
            kend = ranges[2 * t + 1];
        }
    if (kbeg < 0) return 0;
    /* per sorted instance partial sums (each instance belongs to one tile) */
    double *part = calloc((size_t)(kend - kbeg) * 9, sizeof(double));
    if (!part) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < TX * TY; t++) {
        int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
        if (e <= s) continue;
        rec_t *recs = malloc(sizeof(rec_t) * (size_t)(e - s));
        int tx = (int)(t % TX), ty = (int)(t / TX);
        for (int py = ty * TILE; py < ty * TILE + TILE && py < H; py++)
            for (int px = tx * TILE; px < tx * TILE + TILE && px < W; px++) {
                int64_t p = (int64_t)py * W + px;
                /* forward, storing the blended entries */
                double T = 1.0;
                int64_t nr = 0;
                for (int64_t k = s; k < e; k++) {
                    pair_t pe;
                    eval_pair(proj, N, ids[k], px, py, NULL, 0, NULL, &pe);
                    if (!pe.inside) continue;
                    double Tn = T * (1.0 - pe.alpha);
                    if (Tn < T_MIN) break;
                    rec_t rr = {(uint32_t)k, pe.alpha, T, pe.G, pe.og, pe.dx, pe.dy};
                    recs[nr++] = rr;
                    T = Tn;
                }
                double g[3];
                for (int ch = 0; ch < 3; ch++) g[ch] = dL_drgb[(int64_t)ch * W * H + p];
                double Bc[3] = {bg[0], bg[1], bg[2]};
                for (int64_t j = nr - 1; j >= 0; j--) {
                    rec_t *rr = &recs[j];
                    uint32_t id = ids[rr->k];
                    double *out = part + (size_t)(rr->k - kbeg) * 9;
                    double col[3] = {proj[7 * N + id], proj[8 * N + id], proj[9 * N + id]};
                    double dalpha = 0.0;
                    for (int ch = 0; ch < 3; ch++) {
                        out[6 + ch] += rr->alpha * rr->T * g[ch];
                        dalpha += rr->T * g[ch] * (col[ch] - Bc[ch]);
                        Bc[ch] = rr->alpha * col[ch] + (1.0 - rr->alpha) * Bc[ch];
                    }
                    if (rr->og > ALPHA_MAX) continue; /* clamped: alpha constant */
                    double o = proj[6 * N + id];
                    double a = proj[3 * N + id], b = proj[4 * N + id], c = proj[5 * N + id];
                    double dpower = dalpha * o * rr->G;
                    out[5] += dalpha * rr->G;
                    out[0] += dpower * (a * rr->dx + b * rr->dy);
                    out[1] += dpower * (b * rr->dx + c * rr->dy);
                    out[2] += -0.5 * dpower * rr->dx * rr->dx;
                    out[3] += -dpower * rr->dx * rr->dy;
                    out[4] += -0.5 * dpower * rr->dy * rr->dy;
                }
            }
        free(recs);
    }
    for (int64_t k = kbeg; k < kend; k++) {
        uint32_t id = ids[k];
        for (int j = 0; j < 9; j++) dproj[(int64_t)j * N + id] += part[(size_t)(k - kbeg) * 9 + j];
    }
    free(part);
    return 0;
}

/* ------------------------------------------------------------------ transformation backward
 * From d/d(u, v, a, b, c, opacity, rgb) of one view back to the 59 parameters
 * of each Gaussian, accumulated (+=) into grad [59][N]. Depth and radius are
 * piecewise constant and carry no gradient. Every intermediate of
 * project_one is treated as its own variable and differentiated by explicit
 * index sums. */
int oracle_project_bwd(const double *P, int64_t N, const double *cam, const double *dproj, double *grad)
{
    cam_t k = cam_load(cam);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        proj_t o;
        project_one(P, N, i, &k, &o);
        if (o.culled) continue;
        double du = dproj[0 * N + i], dv = dproj[1 * N + i];
        double da = dproj[2 * N + i], db = dproj[3 * N + i], dc = dproj[4 * N + i];
        double dop = dproj[5 * N + i];
        double drgb[3] = {dproj[6 * N + i], dproj[7 * N + i], dproj[8 * N + i]};
        double g[59];
        memset(g, 0, sizeof g);
        double z = o.y[2];
        double dy[3] = {0, 0, 0};
        /* u = fx y0/z + cx, v = fy y1/z + cy */
        dy[0] += du * k.fx / z;
        dy[1] += dv * k.fy / z;
        dy[2] += -du * k.fx * o.y[0] / (z * z) - dv * k.fy * o.y[1] / (z * z);
        /* conic (a, b, c) = (C, -B, A)/det, det = A C - B^2 */
        double d2 = o.det * o.det;
        double dA = da * (-o.C * o.C / d2) + db * (o.B * o.C / d2) + dc * (-o.B * o.B / d2);
        double dB = da * (2.0 * o.B * o.C / d2) + db * (-1.0 / o.det - 2.0 * o.B * o.B / d2) + dc * (2.0 * o.A * o.B / d2);
        double dC = da * (-o.B * o.B / d2) + db * (o.A * o.B / d2) + dc * (-o.A * o.A / d2);
        /* A = S'00 + 0.3, B = S'01, C = S'11 with S' = Tm Sig Tm^T */
        double dSig[9] = {0}, dTm[6] = {0};
        const int jk[3][2] = {{0, 0}, {0, 1}, {1, 1}};
        const double w3[3] = {dA, dB, dC};
        for (int e = 0; e < 3; e++) {
            int j = jk[e][0], kk = jk[e][1];
            double w = w3[e];
            for (int m = 0; m < 3; m++)
                for (int n = 0; n < 3; n++) {
                    dSig[3 * m + n] += w * o.Tm[3 * j + m] * o.Tm[3 * kk + n];
                    dTm[3 * j + m] += w * o.Sig[3 * m + n] * o.Tm[3 * kk + n];
                    dTm[3 * kk + n] += w * o.Tm[3 * j + m] * o.Sig[3 * m + n];
                }
        }
        /* Tm = J Rcam */
        double dJ[6] = {0};
        for (int r = 0; r < 2; r++)
            for (int p = 0; p < 3; p++)
                for (int m = 0; m < 3; m++) dJ[3 * r + p] += dTm[3 * r + m] * k.R[3 * p + m];
        /* J00 = fx/z, J02 = -fx xi/z, J11 = fy/z, J12 = -fy eta/z */
        dy[2] += dJ[0] * (-k.fx / (z * z)) + dJ[4] * (-k.fy / (z * z));
        dy[2] += dJ[2] * (k.fx * o.xi / (z * z)) + dJ[5] * (k.fy * o.eta / (z * z));
        double dxi = dJ[2] * (-k.fx / z), deta = dJ[5] * (-k.fy / z);
        if (!o.xi_clamped) { dy[0] += dxi / z; dy[2] += -dxi * o.y[0] / (z * z); }
        if (!o.eta_clamped) { dy[1] += deta / z; dy[2] += -deta * o.y[1] / (z * z); }
        /* y = Rcam x + t */
        for (int c = 0; c < 3; c++) g[c] += k.R[c] * dy[0] + k.R[3 + c] * dy[1] + k.R[6 + c] * dy[2];
        /* Sig = M M^T */
        double dM[9] = {0};
        for (int p = 0; p < 3; p++)
            for (int kk = 0; kk < 3; kk++) {
                double acc = 0.0;
                for (int n = 0; n < 3; n++) acc += dSig[3 * p + n] * o.M[3 * n + kk] + dSig[3 * n + p] * o.M[3 * n + kk];
                dM[3 * p + kk] = acc;
            }
        /* M = Rq diag(s) */
        double dRq[9], ds[3] = {0, 0, 0};
        for (int r = 0; r < 3; r++)
            for (int c = 0; c < 3; c++) {
                dRq[3 * r + c] = dM[3 * r + c] * o.s[c];
                ds[c] += dM[3 * r + c] * o.Rq[3 * r + c];
            }
        for (int c = 0; c < 3; c++) g[3 + c] += ds[c] * o.s[c];
        /* Rq = R(qhat), qhat = q/|q| */
        double Jq[9][4], dqh[4] = {0, 0, 0, 0};
        quat_rot_jac(o.qh, Jq);
        for (int e = 0; e < 9; e++)
            for (int j = 0; j < 4; j++) dqh[j] += dRq[e] * Jq[e][j];
        double dot = dqh[0] * o.qh[0] + dqh[1] * o.qh[1] + dqh[2] * o.qh[2] + dqh[3] * o.qh[3];
        for (int j = 0; j < 4; j++) g[6 + j] += (dqh[j] - o.qh[j] * dot) / o.qn;
        /* opacity = sigmoid(logit) */
        g[10] += dop * o.opac * (1.0 - o.opac);
        /* colour = max(0, sum_k sh_k Y_k(dir) + 1/2) */
        double ddir[3] = {0, 0, 0};
        for (int ch = 0; ch < 3; ch++) {
            if (!(o.raw[ch] > 0.0)) continue;
            for (int kk = 0; kk < 16; kk++) {
                g[11 + 3 * kk + ch] += drgb[ch] * o.Y[kk];
                double coef = P[(11 + 3 * kk + ch) * N + i];
                for (int j = 0; j < 3; j++) ddir[j] += drgb[ch] * coef * o.dY[kk][j];
            }
        }
        double dd = ddir[0] * o.dir[0] + ddir[1] * o.dir[1] + ddir[2] * o.dir[2];
        for (int j = 0; j < 3; j++) g[j] += (ddir[j] - o.dir[j] * dd) / o.dnorm;
        for (int j = 0; j < 59; j++) grad[(int64_t)j * N + i] += g[j];
    }
    return 0;
}

/* ------------------------------------------------------------------ optimizer
 * Adam (no weight decay, bias correction from step 1) with the batch scaling
 * rules: learning rate lr * sqrt(batch) (eq. "lambda") and decay rates
 * beta^batch for both moments (eq. "beta"). lr6 holds one base rate per
 * group: rows 0-2 (mean), 3-5 (log-scale), 6-9 (quaternion), 10 (opacity),
 * 11-13 (SH degree 0), 14-58 (SH degree >= 1). Arrays are [59][N]; t is the
 * step number after this update (1 on the first call). */
static int row_group(int row)
{
    if (row < 3) return 0;
    if (row < 6) return 1;
    if (row < 10) return 2;
    if (row < 11) return 3;
    if (row < 14) return 4;
    return 5;
}

int oracle_adam(double *p, const double *g, double *m, double *v, int64_t N, const double *lr6,
                double beta1, double beta2, double eps, int32_t batch, int64_t t)
{
    double b1 = pow(beta1, batch), b2 = pow(beta2, batch);
    double bc1 = 1.0 - pow(b1, (double)t), bc2 = 1.0 - pow(b2, (double)t);
    for (int row = 0; row < 59; row++) {
        double lr = lr6[row_group(row)] * sqrt((double)batch);
        double step = lr / bc1;
        for (int64_t i = 0; i < N; i++) {
            int64_t j = (int64_t)row * N + i;
            m[j] = b1 * m[j] + (1.0 - b1) * g[j];
            v[j] = b2 * v[j] + (1.0 - b2) * g[j] * g[j];
            double denom = sqrt(v[j]) / sqrt(bc2) + eps;
            p[j] -= step * m[j] / denom;
        }
    }
    return 0;
}
