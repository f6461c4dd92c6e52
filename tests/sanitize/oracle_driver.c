/* Runs every entry of the FP64 oracle on a small seeded scene, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure:
 * tests/test_oracle_sanitized.py compiles this file together with
 * oracle/oracle.c and runs it). Two views of ragged sizes (partial edge
 * tiles), Gaussians in front of, beside and behind the cameras, one with a
 * zero quaternion and one with a non-finite parameter (both culled). Exits 0
 * when every call returned and the tiled render agrees with the brute-force
 * render of the same view; a sanitizer report ends the process with an
 * error first. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ONF 12
#define F_U 0
#define F_V 1
#define F_DEPTH 2
#define F_RADIUS 10

int oracle_project(const double *P, int64_t N, const double *cam, double *out);
int64_t oracle_tiles_touched(const float *u, const float *v, const float *r, int64_t N, int32_t V,
                             const int32_t *Ws, const int32_t *Hs, int32_t *out);
int64_t oracle_bin(const float *u, const float *v, const float *r, const float *depth, int64_t N, int32_t V,
                   const int32_t *Ws, const int32_t *Hs, int64_t capacity, uint64_t *keys, uint32_t *ids,
                   uint32_t *ranges);
int oracle_render(const double *proj, int64_t N, int32_t W, int32_t H, const uint32_t *ids,
                  const uint32_t *ranges, const double *bg, const uint8_t *fragile, int32_t depth_check,
                  double pos_tol, double t_tol, double *rgb, double *Tout, uint32_t *last, uint32_t *ncontrib,
                  uint8_t *amb, int64_t *counts, double *rgb_alt, double *T_alt, uint32_t *last_alt,
                  double *bound);
int oracle_render_brute(const double *proj, int64_t N, int32_t W, int32_t H, const double *bg, double *rgb,
                        double *Tout, uint32_t *ncontrib);
int oracle_render_bwd(const double *proj, int64_t N, int32_t W, int32_t H, const uint32_t *ids,
                      const uint32_t *ranges, const double *bg, const double *dL_drgb, double *dproj);
int oracle_project_bwd(const double *P, int64_t N, const double *cam, const double *dproj, double *grad);
int oracle_adam(double *p, const double *g, double *m, double *v, int64_t N, const double *lr6, double beta1,
                double beta2, double eps, int32_t batch, int64_t t);
void oracle_sh_basis(const double *dirs, int64_t n, double *Y, double *dY);

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double urand(void) /* splitmix64, mapped to [0, 1) */
{
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static void *xcalloc(size_t n, size_t s)
{
    void *p = calloc(n ? n : 1, s);
    if (!p) { fprintf(stderr, "out of memory\n"); exit(3); }
    return p;
}

int main(void)
{
    const int64_t N = 320;
    const int32_t V = 2;
    const int32_t Ws[2] = {45, 30}, Hs[2] = {37, 21};
    double cams[2][19];
    for (int c = 0; c < V; c++) {
        double *k = cams[c];
        memset(k, 0, sizeof cams[c]);
        k[0] = Ws[c]; k[1] = Hs[c];
        k[2] = k[3] = 0.5 * Ws[c] / tan(M_PI / 6.0); /* 60 degree horizontal field of view */
        k[4] = 0.5 * Ws[c]; k[5] = 0.5 * Hs[c];
        double a = c ? 0.3 : 0.0;                    /* second camera turned about y */
        k[6] = cos(a); k[8] = sin(a); k[10] = 1.0; k[12] = -sin(a); k[14] = cos(a);
        k[15] = 0.0; k[16] = 0.0; k[17] = 4.0; k[18] = 0.2;
    }
    double *P = xcalloc(59 * N, sizeof(double));
    for (int64_t i = 0; i < N; i++) {
        for (int j = 0; j < 3; j++) P[j * N + i] = (urand() - 0.5) * (j == 2 ? 9.0 : 5.0);
        for (int j = 3; j < 6; j++) P[j * N + i] = -2.5 + 1.5 * urand();
        for (int j = 6; j < 10; j++) P[j * N + i] = urand() - 0.5;
        P[10 * N + i] = 4.0 * urand() - 2.0;
        for (int j = 11; j < 59; j++) P[j * N + i] = (urand() - 0.5) * (j < 14 ? 2.0 : 0.4);
    }
    for (int j = 6; j < 10; j++) P[j * N + 5] = 0.0; /* zero quaternion: culled */
    P[7 * N + 9] = NAN;                              /* non-finite parameter: culled */

    double *proj[2];
    float *u = xcalloc(V * N, sizeof(float)), *v = xcalloc(V * N, sizeof(float));
    float *r = xcalloc(V * N, sizeof(float)), *d = xcalloc(V * N, sizeof(float));
    for (int c = 0; c < V; c++) {
        proj[c] = xcalloc(ONF * N, sizeof(double));
        oracle_project(P, N, cams[c], proj[c]);
        for (int64_t i = 0; i < N; i++) {
            u[c * N + i] = (float)proj[c][F_U * N + i];
            v[c * N + i] = (float)proj[c][F_V * N + i];
            r[c * N + i] = (float)proj[c][F_RADIUS * N + i];
            d[c * N + i] = (float)proj[c][F_DEPTH * N + i];
        }
    }
    int32_t *touched = xcalloc(V * N, sizeof(int32_t));
    int64_t K = oracle_tiles_touched(u, v, r, N, V, Ws, Hs, touched);
    int64_t tb[3] = {0, 0, 0};
    for (int c = 0; c < V; c++) tb[c + 1] = tb[c] + (int64_t)((Ws[c] + 15) / 16) * ((Hs[c] + 15) / 16);
    uint64_t *keys = xcalloc(K, sizeof(uint64_t));
    uint32_t *ids = xcalloc(K, sizeof(uint32_t));
    uint32_t *ranges = xcalloc(2 * tb[V], sizeof(uint32_t));
    int64_t got = oracle_bin(u, v, r, d, N, V, Ws, Hs, K, keys, ids, ranges);
    if (got != K) { fprintf(stderr, "bin: %lld instances, expected %lld\n", (long long)got, (long long)K); return 1; }

    const double bg[3] = {0.1, 0.2, 0.3};
    double *grad = xcalloc(59 * N, sizeof(double)), *gsum = xcalloc(59 * N, sizeof(double));
    double worst = 0.0;
    int64_t evaluated = 0;
    for (int c = 0; c < V; c++) {
        const int64_t HW = (int64_t)Ws[c] * Hs[c];
        double *rgb = xcalloc(3 * HW, sizeof(double)), *T = xcalloc(HW, sizeof(double));
        double *rgb_alt = xcalloc(3 * HW, sizeof(double)), *T_alt = xcalloc(HW, sizeof(double));
        double *bound = xcalloc(HW, sizeof(double));
        uint32_t *last = xcalloc(HW, sizeof(uint32_t)), *nc = xcalloc(HW, sizeof(uint32_t));
        uint32_t *last_alt = xcalloc(HW, sizeof(uint32_t));
        uint8_t *amb = xcalloc(HW, 1), *fragile = xcalloc(N, 1);
        int64_t counts[2] = {0, 0};
        fragile[3] = 1;
        oracle_render(proj[c], N, Ws[c], Hs[c], K ? ids : NULL, ranges + 2 * tb[c], bg, fragile, 1, 1e-6, 1e-5,
                      rgb, T, last, nc, amb, counts, rgb_alt, T_alt, last_alt, bound);
        evaluated += counts[0];
        double *rgb_b = xcalloc(3 * HW, sizeof(double)), *T_b = xcalloc(HW, sizeof(double));
        uint32_t *nc_b = xcalloc(HW, sizeof(uint32_t));
        oracle_render_brute(proj[c], N, Ws[c], Hs[c], bg, rgb_b, T_b, nc_b);
        for (int64_t p = 0; p < 3 * HW; p++) {
            double e = fabs(rgb[p] - rgb_b[p]);
            if (isnan(e)) worst = INFINITY;
            else if (e > worst) worst = e;
        }
        double *dL = xcalloc(3 * HW, sizeof(double)), *dproj = xcalloc(9 * N, sizeof(double));
        for (int64_t p = 0; p < 3 * HW; p++) dL[p] = urand() - 0.5;
        if (oracle_render_bwd(proj[c], N, Ws[c], Hs[c], K ? ids : NULL, ranges + 2 * tb[c], bg, dL, dproj) != 0) {
            fprintf(stderr, "render backward failed\n");
            return 1;
        }
        oracle_project_bwd(P, N, cams[c], dproj, grad);
        for (int64_t q = 0; q < 59 * N; q++) gsum[q] += grad[q];
        free(rgb); free(T); free(rgb_alt); free(T_alt); free(bound); free(last); free(nc); free(last_alt);
        free(amb); free(fragile); free(rgb_b); free(T_b); free(nc_b); free(dL); free(dproj);
    }
    double *m = xcalloc(59 * N, sizeof(double)), *vv = xcalloc(59 * N, sizeof(double));
    const double lr6[6] = {1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3, 1.25e-4};
    for (int64_t t = 1; t <= 3; t++) oracle_adam(P, gsum, m, vv, N, lr6, 0.9, 0.999, 1e-15, V, t);
    int bad = 0;
    for (int64_t q = 0; q < 59 * N; q++)
        if (q / N != 7 || q % N != 9) bad += !isfinite(P[q]);
    double dirs[3 * 4] = {0, 0, 1, 1, 0, 0, 0.6, 0.8, 0, -0.36, 0.48, 0.8}, Y[4 * 16], dY[4 * 16 * 3];
    oracle_sh_basis(dirs, 4, Y, dY);
    printf("instances %lld, pairs evaluated %lld, tiled vs brute max diff %.3g, non-finite parameters %d\n",
           (long long)K, (long long)evaluated, worst, bad);
    free(P); free(u); free(v); free(r); free(d); free(touched); free(keys); free(ids); free(ranges);
    free(grad); free(gsum); free(m); free(vv);
    for (int c = 0; c < V; c++) free(proj[c]);
    return (worst <= 1e-12 && bad == 0 && K > 0) ? 0 : 2;
}
