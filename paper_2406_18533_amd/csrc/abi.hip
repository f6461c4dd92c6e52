// C ABI entry points: argument checks, view tables, dtype dispatch.
// Every entry point returns a gs_status; no exception leaves this file.
#include <math.h>
#include <string.h>

#include <mutex>
#include <string>

#include "common.hpp"

namespace gs {

template <typename T> hipError_t launch_project_fwd(const void *, int64_t, const gs_camera *, int32_t, void *, hipStream_t);
template <typename T>
hipError_t launch_project_bwd(const void *, int64_t, const gs_camera *, int32_t, const void *, void *, int, void *,
                              hipStream_t);
template <typename T>
hipError_t launch_project_bwd_adam(void *, int64_t, const gs_camera *, int32_t, const void *, void *, void *, void *,
                                   void *, const gs_adam_hparams *, int64_t *, double *, const int32_t *, hipStream_t);
template <typename T>
hipError_t launch_bin_sort(const void *, int64_t, const ViewTable &, gs_bins *, bool, int *, hipStream_t);
template <typename T>
hipError_t launch_keys64(const void *, int64_t, const ViewTable &, const gs_bins *, uint64_t *, hipStream_t);
size_t bin_ws_layout(int64_t vn, int64_t cap, char *base, BinWS *ws);
template <typename T>
hipError_t launch_render_fwd(const ViewTable &, const void *, int64_t, const gs_bins *, const float *,
                             const LaunchShape &, void *, void *, uint32_t *, uint32_t *, uint32_t *, uint64_t *,
                             const void *, double, void *, double *, double *, hipStream_t);
template <typename T>
hipError_t launch_render_bwd(const ViewTable &, const void *, int64_t, const gs_bins *, const float *,
                             const LaunchShape &, const void *, const uint32_t *, const void *, void *, hipStream_t);
hipError_t launch_plan(const uint32_t *, int32_t, int32_t, uint64_t *, uint64_t *, int32_t *, int32_t *, int32_t *,
                       hipStream_t);
template <typename T>
hipError_t launch_adam(void *, void *, void *, void *, int64_t, const gs_adam_hparams *, int64_t *, double *,
                       const int32_t *, hipStream_t);
template <typename T>
hipError_t launch_l1(const void *, const void *, const ViewTable &, double, void *, double *, void *, hipStream_t);
size_t loss_ws_bytes(int32_t views);
template <typename T>
hipError_t launch_l1_dssim(const void *, const void *, const ViewTable &, double, double, void *, double *, void *,
                           hipStream_t);
size_t dssim_ws_bytes(const ViewTable &vt, size_t elem);
template <typename T>
hipError_t launch_densify_stats(const void *, const void *, int64_t, int32_t, double, float *, int32_t *, hipStream_t);
template <typename T>
hipError_t launch_densify_plan(const void *, int64_t, const float *, const int32_t *, const gs_densify_hparams &,
                               void *, int64_t *, hipStream_t);
template <typename T>
hipError_t launch_densify_apply(const void *, const void *, const void *, int64_t, const void *, const void *, void *,
                                void *, void *, int64_t, hipStream_t);
template <typename T> hipError_t launch_reset_opacity(void *, void *, void *, int64_t, double, hipStream_t);
size_t densify_ws_bytes(int64_t n);

ViewTable make_view_table(const gs_camera *cams, int32_t views)
{
    ViewTable vt;
    memset(&vt, 0, sizeof vt);
    vt.nviews = views;
    int32_t tb = 0;
    int64_t pb = 0;
    for (int v = 0; v < views; v++) {
        int tx = (cams[v].width + TILE - 1) / TILE, ty = (cams[v].height + TILE - 1) / TILE;
        vt.tile_base[v] = tb;
        vt.tiles_x[v] = tx;
        vt.width[v] = cams[v].width;
        vt.height[v] = cams[v].height;
        vt.pix_base[v] = pb;
        tb += tx * ty;
        pb += (int64_t)cams[v].width * cams[v].height;
    }
    vt.tile_base[views] = tb;
    vt.pix_base[views] = pb;
    vt.total_tiles = tb;
    return vt;
}

}  // namespace gs

using namespace gs;

static thread_local std::string g_err;

static gs_status fail(gs_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

static gs_status hip_status(hipError_t e, const char *where)
{
    if (e == hipSuccess) return GS_OK;
    return fail(GS_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

static bool cams_ok(const gs_camera *cams, int32_t views, std::string &why)
{
    if (!cams) { why = "null host cameras"; return false; }
    if (views < 1 || views > GS_MAX_VIEWS) { why = "views must be in [1, 64]"; return false; }
    int64_t tiles = 0;
    for (int v = 0; v < views; v++) {
        const gs_camera &c = cams[v];
        if (c.width < 1 || c.height < 1 || c.width > 65536 || c.height > 65536) { why = "bad image size"; return false; }
        if (!(c.fx > 0) || !(c.fy > 0) || !isfinite(c.cx) || !isfinite(c.cy) || !(c.znear > 0)) {
            why = "bad intrinsics";
            return false;
        }
        int64_t vt = (int64_t)((c.width + 15) / 16) * ((c.height + 15) / 16);
        if (vt > (int64_t(1) << 22)) { why = "image too large (at most 2^22 tiles per view)"; return false; }
        tiles += vt;
    }
    if (tiles >= (int64_t(1) << 31)) { why = "too many tiles"; return false; }
    return true;
}

static bool dtype_ok(gs_dtype d) { return d == GS_F32 || d == GS_F64; }

#define CHECK_ARG(cond, msg) \
    do { if (!(cond)) return fail(GS_ERR_ARG, msg); } while (0)

static int g_cus = 0;

static int cu_count()
{
    if (g_cus > 0) return g_cus;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) g_cus = p.multiProcessorCount;
    if (g_cus <= 0) g_cus = 256;
    return g_cus;
}

// Fixed scratch of the no-allocation forward (gs_render_fwd_l1_noalloc): the
// per-tile loss shares and the 64 block sums of their deterministic sum, for
// up to GS_NOALLOC_MAX_TILES tiles. Each device holds its own copy for the
// life of the process. In host code `scratch` only names the symbol: kernels
// get the device address that hipGetSymbolAddress returns for the current
// device, kept in g_scratch_dev.
static __device__ __align__(256) double scratch[GS_NOALLOC_MAX_TILES + LOSS_SUM_BLOCKS];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_dev[MAX_DEVICES];

// Device address of `scratch` on the current device, resolved once per
// device (gs_init does it; a first call on a device that skipped gs_init
// does it then).
static gs_status scratch_address(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e, "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) return fail(GS_ERR_ARG, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e, "hipGetSymbolAddress(scratch)");
        g_scratch_dev[dev] = (double *)p;
    }
    *out = g_scratch_dev[dev];
    return GS_OK;
}

extern "C" {

const char *gs_version(void) { return GS_VERSION_STRING; }

const char *gs_last_error(void) { return g_err.c_str(); }

gs_status gs_init(int32_t device)
{
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return hip_status(e, "hipSetDevice");
    hipDeviceProp_t p;
    e = hipGetDeviceProperties(&p, device);
    if (e != hipSuccess) return hip_status(e, "hipGetDeviceProperties");
    if (strncmp(p.gcnArchName, "gfx950", 6) != 0)
        return fail(GS_ERR_UNSUPPORTED, std::string("device is ") + p.gcnArchName + ", this library is built for gfx950");
    g_cus = p.multiProcessorCount;
    double *sp = nullptr;
    return scratch_address(&sp);
}

size_t gs_projected_bytes(gs_dtype dtype, int64_t n, int32_t views)
{
    if (n < 0 || views < 0 || !dtype_ok(dtype)) return 0;
    return (size_t)n * (size_t)views * (GS_REC * (dtype == GS_F64 ? 8 : 4) + 16);
}

int64_t gs_total_tiles(const gs_camera *cams, int32_t views)
{
    std::string why;
    if (!cams_ok(cams, views, why)) { fail(GS_ERR_ARG, why); return -1; }
    return make_view_table(cams, views).total_tiles;
}

int64_t gs_total_pixels(const gs_camera *cams, int32_t views)
{
    std::string why;
    if (!cams_ok(cams, views, why)) { fail(GS_ERR_ARG, why); return -1; }
    return make_view_table(cams, views).pix_base[views];
}

size_t gs_bin_workspace_bytes(int64_t n, int32_t views, int64_t capacity, int64_t total_tiles)
{
    (void)total_tiles;
    if (n < 0 || views < 1 || capacity < 0) return 0;
    return bin_ws_layout(n * views, capacity, nullptr, nullptr);
}

// Scheduler workspace: cursor[Q] | dp[Q + 1] | ct[T] (uint64) | scan partials, each 256-byte aligned.
struct SchedWS {
    size_t cursor, dp, ct, partial, order, bins, total;
};

static SchedWS sched_ws(int64_t total_tiles, int32_t q)
{
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    SchedWS w;
    size_t t = (size_t)(total_tiles > 0 ? total_tiles : 1);
    w.cursor = 0;
    w.dp = al(4 * (size_t)q);
    w.ct = w.dp + al(4 * ((size_t)q + 1));
    w.partial = w.ct + al(8 * t);
    w.order = w.partial + al(8 * (t / 4096 + 8));
    w.bins = w.order + al(4 * t);
    w.total = w.bins + al(4 * (2 * (size_t)LPT_SEGS * (size_t)LPT_BINS + (size_t)LPT_SEGS));
    return w;
}

size_t gs_sched_workspace_bytes(int64_t total_tiles, int32_t queues)
{
    if (queues <= 0) queues = 64;
    return sched_ws(total_tiles, queues).total;
}

size_t gs_loss_workspace_bytes(const gs_camera *cams, int32_t views)
{
    std::string why;
    if (!cams_ok(cams, views, why)) return 0;
    size_t tiles = ((size_t)make_view_table(cams, views).total_tiles + LOSS_SUM_BLOCKS) * sizeof(double);   // gs_render_fwd_l1
    size_t ws = loss_ws_bytes(views);
    return ws > tiles ? ws : tiles;
}

size_t gs_loss_dssim_workspace_bytes(gs_dtype dtype, const gs_camera *cams, int32_t views)
{
    std::string why;
    if (!dtype_ok(dtype)) {
        fail(GS_ERR_ARG, "bad dtype");
        return 0;
    }
    if (!cams_ok(cams, views, why)) {
        fail(GS_ERR_ARG, why);
        return 0;
    }
    return dssim_ws_bytes(make_view_table(cams, views), dtype == GS_F32 ? sizeof(float) : sizeof(double));
}

gs_status gs_project(gs_dtype dtype, const void *params, int64_t n, const gs_camera *cams_dev,
                     const gs_camera *cams_host, int32_t views, void *projected, void *stream)
{
    std::string why;
    CHECK_ARG(dtype_ok(dtype), "bad dtype");
    CHECK_ARG(cams_ok(cams_host, views, why), why);
    CHECK_ARG(n >= 0 && (uint64_t)n * (uint64_t)views < (uint64_t(1) << 32), "n * views must be < 2^32");
    CHECK_ARG((uint64_t)n * GS_REC * (dtype == GS_F32 ? 4u : 8u) < (uint64_t(1) << 32),
              "one view's records must be < 4 GiB (n < 89M in FP32, 44M in FP64)");
    CHECK_ARG(n == 0 || (params && cams_dev && projected), "null pointer");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = dtype == GS_F32 ? launch_project_fwd<float>(params, n, cams_dev, views, projected, s)
                                   : launch_project_fwd<double>(params, n, cams_dev, views, projected, s);
    return hip_status(e, "gs_project");
}

static bool bins_ok(const gs_bins *b, int64_t n, int32_t views, std::string &why)
{
    if (!b) { why = "null bins"; return false; }
    if (b->capacity < 0 || b->capacity >= (int64_t(1) << 32) - 1) { why = "capacity must be < 2^32 - 1"; return false; }
    if (!b->tile_keys || !b->ids || !b->ranges || !b->n_instances || !b->overflow) { why = "null bins buffer"; return false; }
    if (!b->workspace || b->workspace_bytes < bin_ws_layout(n * views, b->capacity, nullptr, nullptr)) {
        why = "bins workspace too small";
        return false;
    }
    return true;
}

gs_status gs_bin_sort(gs_dtype dtype, const void *projected, int64_t n, const gs_camera *cams_host, int32_t views,
                      gs_bins *bins, int32_t check, void *stream)
{
    std::string why;
    CHECK_ARG(dtype_ok(dtype), "bad dtype");
    CHECK_ARG(cams_ok(cams_host, views, why), why);
    CHECK_ARG(n >= 0 && (uint64_t)n * (uint64_t)views < (uint64_t(1) << 32), "n * views must be < 2^32");
    CHECK_ARG(bins_ok(bins, n, views, why), why);
    CHECK_ARG(n == 0 || projected, "null projected");
    ViewTable vt = make_view_table(cams_host, views);
    int cap_err = 0;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = dtype == GS_F32 ? launch_bin_sort<float>(projected, n, vt, bins, check != 0, &cap_err, s)
                                   : launch_bin_sort<double>(projected, n, vt, bins, check != 0, &cap_err, s);
    if (e != hipSuccess) return hip_status(e, "gs_bin_sort");
    if (cap_err) return fail(GS_ERR_CAPACITY, "more instances than bins->capacity");
    return GS_OK;
}

gs_status gs_bins_keys64(gs_dtype dtype, const void *projected, int64_t n, const gs_camera *cams_host, int32_t views,
                         const gs_bins *bins, uint64_t *keys_out, void *stream)
{
    std::string why;
    CHECK_ARG(dtype_ok(dtype), "bad dtype");
    CHECK_ARG(cams_ok(cams_host, views, why), why);
    CHECK_ARG(bins_ok(bins, n, views, why), why);
    CHECK_ARG(keys_out && projected, "null pointer");
    ViewTable vt = make_view_table(cams_host, views);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = dtype == GS_F32 ? launch_keys64<float>(projected, n, vt, bins, keys_out, s)
                                   : launch_keys64<double>(projected, n, vt, bins, keys_out, s);
    return hip_status(e, "gs_bins_keys64");
}

static bool sched_shape(const gs_sched *sc, int64_t total_tiles, LaunchShape &sh, std::string &why)
{
    sh.mode = GS_SCHED_PER_TILE;
    sh.px = 1;
    sh.chunk = 64;
    sh.workers = 0;
    sh.S.cursor = nullptr;
    sh.S.dp = nullptr;
    sh.S.queues = 0;
    sh.S.order = nullptr;
    sh.S.bins = nullptr;
    if (!sc) return true;
    if (sc->mode != GS_SCHED_PER_TILE && sc->mode != GS_SCHED_PERSISTENT && sc->mode != GS_SCHED_XCD_SPLIT &&
        sc->mode != GS_SCHED_LPT && sc->mode != GS_SCHED_XCD_LPT && sc->mode != GS_SCHED_LPT_HEAD) {
        why = "bad sched mode";
        return false;
    }
    if (sc->px_per_thread != 1 && sc->px_per_thread != 2 && sc->px_per_thread != 4) { why = "px_per_thread"; return false; }
    if (sc->chunk != 32 && sc->chunk != 64 && sc->chunk != 128 && sc->chunk != 256) { why = "chunk"; return false; }
    sh.mode = sc->mode;
    sh.px = sc->px_per_thread;
    sh.chunk = sc->chunk;
    const bool lpt = sh.mode == GS_SCHED_LPT || sh.mode == GS_SCHED_XCD_LPT || sh.mode == GS_SCHED_LPT_HEAD;
    if (lpt && !sc->tile_cost) sh.mode = GS_SCHED_PER_TILE;   // no costs: index order
    if (lpt && sc->tile_cost) {
        if (!sc->workspace || sc->workspace_bytes < gs_sched_workspace_bytes(total_tiles, 8)) {
            why = "sched workspace too small";
            return false;
        }
        SchedWS L = sched_ws(total_tiles, 8);
        char *w = (char *)sc->workspace;
        sh.S.order = (int32_t *)(w + L.order);
        sh.S.bins = (uint32_t *)(w + L.bins);
    }
    if (sh.mode == GS_SCHED_PERSISTENT || sh.mode == GS_SCHED_XCD_SPLIT || sh.mode == GS_SCHED_XCD_LPT) {
        int q = sh.mode == GS_SCHED_PERSISTENT ? (sc->queues > 0 ? sc->queues : 64) : 8;
        if (q % 8 != 0 || q > (1 << 16)) { why = "queues must be a positive multiple of 8"; return false; }
        if (!sc->workspace || sc->workspace_bytes < gs_sched_workspace_bytes(total_tiles, q)) {
            why = "sched workspace too small";
            return false;
        }
        if (sc->workers < 0 || sc->workers % 8 != 0) { why = "workers must be a multiple of 8"; return false; }
        char *w = (char *)sc->workspace;
        SchedWS L = sched_ws(total_tiles, q);
        sh.S.queues = q;
        sh.S.cursor = (int32_t *)(w + L.cursor);
        sh.S.dp = (int32_t *)(w + L.dp);
        int wk = sc->workers;
        if (wk == 0) wk = cu_count() * 8 * sh.px;  // about 32 wavefronts per CU
        sh.workers = wk;
    }
    return true;
}

static hipError_t run_plan(const gs_sched *sc, const LaunchShape &sh, int32_t total_tiles, int32_t *dp_out,
                           hipStream_t s)
{
    if (sh.mode == GS_SCHED_LPT)
        return launch_lpt_plan(sc->tile_cost, total_tiles, nullptr, 1, 0u, sh.S.bins, sh.S.order, s);
    if (sh.mode == GS_SCHED_LPT_HEAD)   // the heaviest eighth of the tiles first, the rest in index order
        return launch_lpt_plan(sc->tile_cost, total_tiles, nullptr, 1, (uint32_t)((total_tiles + 7) / 8), sh.S.bins,
                               sh.S.order, s);
    SchedWS L = sched_ws(total_tiles, sh.S.queues);
    char *w = (char *)sc->workspace;
    hipError_t e = launch_plan(sc->tile_cost, total_tiles, sh.S.queues, (uint64_t *)(w + L.ct),
                               (uint64_t *)(w + L.partial), sh.S.dp, sh.S.cursor, dp_out, s);
    if (e != hipSuccess || sh.mode != GS_SCHED_XCD_LPT) return e;
    return launch_lpt_plan(sc->tile_cost, total_tiles, sh.S.dp, 8, 0u, sh.S.bins, sh.S.order, s);
}

gs_status gs_sched_plan(const gs_sched *sched, const gs_camera *cams_host, int32_t views, int32_t *dp_out, void *stream)
{
    std::string why;
    CHECK_ARG(cams_ok(cams_host, views, why), why);
    CHECK_ARG(sched && sched->mode == GS_SCHED_PERSISTENT, "gs_sched_plan needs a persistent sched");
    ViewTable vt = make_view_table(cams_host, views);
    LaunchShape sh;
    CHECK_ARG(sched_shape(sched, vt.total_tiles, sh, why), why);
    return hip_status(run_plan(sched, sh, vt.total_tiles, dp_out, (hipStream_t)stream), "gs_sched_plan");
}

gs_status gs_render_fwd(gs_dtype dtype, const void *projected, int64_t n, const gs_bins *bins,
                        const gs_camera *cams_host, int32_t views, const float *bg, const gs_sched *sched, void *rgb,
                        void *final_T, uint32_t *last, uint32_t *tile_work_fwd, uint32_t *tile_work_bwd,
                        uint64_t *pair_stats, void *stream)
{
    std::string why;
    CHECK_ARG(dtype_ok(dtype), "bad dtype");
    CHECK_ARG(cams_ok(cams_host, views, why), why);
    CHECK_ARG(bins_ok(bins, n, views, why), why);
    CHECK_ARG(bg && rgb && final_T && last && projected, "null pointer");
    ViewTable vt = make_view_table(cams_host, views);
    LaunchShape sh;
    CHECK_ARG(sched_shape(sched, vt.total_tiles, sh, why), why);
    hipStream_t s = (hipStream_t)stream;
    if (sh.mode != GS_SCHED_PER_TILE) {
        hipError_t e = run_plan(sched, sh, vt.total_tiles, nullptr, s);
        if (e != hipSuccess) return hip_status(e, "gs_render_fwd plan");
    }
    hipError_t e = dtype == GS_F32
                       ? launch_render_fwd<float>(vt, projected, n, bins, bg, sh, rgb, final_T, last, tile_work_fwd,
                                                  tile_work_bwd, pair_stats, nullptr, 0.0, nullptr, nullptr, nullptr,
                                                  s)
                       : launch_render_fwd<double>(vt, projected, n, bins, bg, sh, rgb, final_T, last, tile_work_fwd,
                                                   tile_work_bwd, pair_stats, nullptr, 0.0, nullptr, nullptr, nullptr,
                                                   s);
    return hip_status(e, "gs_render_fwd");
}

gs_status gs_render_fwd_l1(gs_dtype dtype, const void *projected, int64_t n, const gs_bins *bins,
                           const gs_camera *cams_host, int32_t views, const float *bg, const gs_sched *sched,
                           void *rgb, void *final_T, uint32_t *last, uint32_t *tile_work_fwd, uint32_t *tile_work_bwd,
                           const void *target, double scale, void *dL_drgb, double *loss_dev, void *workspace,
                           size_t workspace_bytes, void *stream)
{
    std::string why;
    CHECK_ARG(dtype_ok(dtype), "bad dtype");
    CHECK_ARG(cams_ok(cams_host, views, why), why);
    CHECK_ARG(bins_ok(bins, n, views, why), why);
    CHECK_ARG(bg && rgb && final_T && last && projected, "null pointer");
    CHECK_ARG(target && dL_drgb && loss_dev && workspace, "null pointer");
    CHECK_ARG(isfinite(scale), "bad scale");
    ViewTable vt = make_view_table(cams_host, views);
    CHECK_ARG(workspace_bytes >= ((size_t)vt.total_tiles + LOSS_SUM_BLOCKS) * sizeof(double), "loss workspace too small");
    LaunchShape sh;
    CHECK_ARG(sched_shape(sched, vt.total_tiles, sh, why), why);
    hipStream_t s = (hipStream_t)stream;
    if (sh.mode != GS_SCHED_PER_TILE) {
        hipError_t e = run_plan(sched, sh, vt.total_tiles, nullptr, s);
        if (e != hipSuccess) return hip_status(e, "gs_render_fwd_l1 plan");
    }
    hipError_t e = dtype == GS_F32
                       ? launch_render_fwd<float>(vt, projected, n, bins, bg, sh, rgb, final_T, last, tile_work_fwd,
                                                  tile_work_bwd, nullptr, target, scale, dL_drgb, loss_dev,
                                                  (double *)workspace, s)
                       : launch_render_fwd<double>(vt, projected, n, bins, bg, sh, rgb, final_T, last, tile_work_fwd,
                                                   tile_work_bwd, nullptr, target, scale, dL_drgb, loss_dev,
                                                   (double *)workspace, s);
    return hip_status(e, "gs_render_fwd_l1");
}

gs_status gs_render_fwd_l1_noalloc(gs_dtype dtype, const void *projected, int64_t n, const gs_bins *bins,
                                   const gs_camera *cams_host, int32_t views, const float *bg, const gs_sched *sched,
                                   void *rgb, void *final_T, uint32_t *last, uint32_t *tile_work_fwd,
                                   uint32_t *tile_work_bwd, const void *target, double scale, void *dL_drgb,
                                   double *loss_dev, void *stream)
{
    std::string why;
    CHECK_ARG(cams_ok(cams_host, views, why), why);
    int64_t tiles = make_view_table(cams_host, views).total_tiles;
    if (tiles > GS_NOALLOC_MAX_TILES)
        return fail(GS_ERR_ARG, "gs_render_fwd_l1_noalloc: " + std::to_string(tiles) + " tiles exceed its fixed scratch of " +
                                    std::to_string(GS_NOALLOC_MAX_TILES) + " tiles; use gs_render_fwd_l1");
    double *ws = nullptr;
    gs_status st = scratch_address(&ws);
    if (st != GS_OK) return st;
    // every tile share is written before the sum reads it: nothing to clear
    return gs_render_fwd_l1(dtype, projected, n, bins, cams_host, views, bg, sched, rgb, final_T, last, tile_work_fwd,
                            tile_work_bwd, target, scale, dL_drgb, loss_dev, ws,
                            sizeof(double) * ((size_t)GS_NOALLOC_MAX_TILES + LOSS_SUM_BLOCKS), stream);
}

gs_status gs_render_bwd_pixels(gs_dtype dtype, const void *projected, int64_t n, const gs_bins *bins,
                               const gs_camera *cams_host, int32_t views, const float *bg, const gs_sched *sched,
                               const void *final_T, const uint32_t *last, const void *dL_drgb, void *dprojected,
                               void *stream)
{
    std::string why;
    CHECK_ARG(dtype_ok(dtype), "bad dtype");
    CHECK_ARG(cams_ok(cams_host, views, why), why);
    CHECK_ARG(bins_ok(bins, n, views, why), why);
    CHECK_ARG(bg && final_T && last && dL_drgb && dprojected && projected, "null pointer");
    ViewTable vt = make_view_table(cams_host, views);
    LaunchShape sh;
    CHECK_ARG(sched_shape(sched, vt.total_tiles, sh, why), why);
    hipStream_t s = (hipStream_t)stream;
    if (sh.mode != GS_SCHED_PER_TILE) {
        hipError_t e = run_plan(sched, sh, vt.total_tiles, nullptr, s);
        if (e != hipSuccess) return hip_status(e, "gs_render_bwd_pixels plan");
    }
    hipError_t e = dtype == GS_F32
                       ? launch_render_bwd<float>(vt, projected, n, bins, bg, sh, final_T, last, dL_drgb, dprojected, s)
                       : launch_render_bwd<double>(vt, projected, n, bins, bg, sh, final_T, last, dL_drgb, dprojected,
                                                   s);
    return hip_status(e, "gs_render_bwd_pixels");
}

gs_status gs_project_bwd(gs_dtype dtype, const void *params, int64_t n, const gs_camera *cams_dev,
                         const gs_camera *cams_host, int32_t views, const void *projected, void *dprojected,
                         int32_t clear, void *grad, void *stream)
{
    std::string why;
    CHECK_ARG(dtype_ok(dtype), "bad dtype");
    CHECK_ARG(cams_ok(cams_host, views, why), why);
    CHECK_ARG(n >= 0 && (uint64_t)n * (uint64_t)views < (uint64_t(1) << 32), "n * views must be < 2^32");
    CHECK_ARG(n == 0 || (params && cams_dev && projected && dprojected && grad), "null pointer");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = dtype == GS_F32
                       ? launch_project_bwd<float>(params, n, cams_dev, views, projected, dprojected, clear, grad, s)
                       : launch_project_bwd<double>(params, n, cams_dev, views, projected, dprojected, clear, grad, s);
    return hip_status(e, "gs_project_bwd");
}

gs_status gs_render_bwd(gs_dtype dtype, const void *params, int64_t n, const void *projected, const gs_bins *bins,
                        const gs_camera *cams_dev, const gs_camera *cams_host, int32_t views, const float *bg,
                        const gs_sched *sched, const void *final_T, const uint32_t *last, const void *dL_drgb,
                        void *dprojected, void *grad, void *stream)
{
    CHECK_ARG(params && grad && cams_dev, "null pointer");
    gs_status st = gs_render_bwd_pixels(dtype, projected, n, bins, cams_host, views, bg, sched, final_T, last,
                                        dL_drgb, dprojected, stream);
    if (st != GS_OK) return st;
    return gs_project_bwd(dtype, params, n, cams_dev, cams_host, views, projected, dprojected, 1, grad, stream);
}

gs_status gs_loss_l1(gs_dtype dtype, const void *rgb, const void *target, const gs_camera *cams_host, int32_t views,
                     double scale, void *dL_drgb, double *loss_dev, void *workspace, size_t workspace_bytes,
                     void *stream)
{
    std::string why;
    CHECK_ARG(dtype_ok(dtype), "bad dtype");
    CHECK_ARG(cams_ok(cams_host, views, why), why);
    CHECK_ARG(rgb && target && dL_drgb && loss_dev && workspace, "null pointer");
    CHECK_ARG(workspace_bytes >= loss_ws_bytes(views), "loss workspace too small");
    ViewTable vt = make_view_table(cams_host, views);
    hipStream_t s = (hipStream_t)stream;
    CHECK_ARG(isfinite(scale), "bad scale");
    hipError_t e = dtype == GS_F32 ? launch_l1<float>(rgb, target, vt, scale, dL_drgb, loss_dev, workspace, s)
                                   : launch_l1<double>(rgb, target, vt, scale, dL_drgb, loss_dev, workspace, s);
    return hip_status(e, "gs_loss_l1");
}

gs_status gs_loss_l1_dssim(gs_dtype dtype, const void *rgb, const void *target, const gs_camera *cams_host,
                           int32_t views, double lam, double scale, void *dL_drgb, double *loss_dev, void *workspace,
                           size_t workspace_bytes, void *stream)
{
    std::string why;
    CHECK_ARG(dtype_ok(dtype), "bad dtype");
    CHECK_ARG(cams_ok(cams_host, views, why), why);
    CHECK_ARG(rgb && target && dL_drgb && loss_dev && workspace, "null pointer");
    CHECK_ARG(dL_drgb != rgb && dL_drgb != target, "dL_drgb aliases an input");
    CHECK_ARG(isfinite(scale), "bad scale");
    CHECK_ARG(lam >= 0.0 && lam <= 1.0, "lam outside [0, 1]");
    ViewTable vt = make_view_table(cams_host, views);
    const size_t elem = dtype == GS_F32 ? sizeof(float) : sizeof(double);
    CHECK_ARG(workspace_bytes >= dssim_ws_bytes(vt, elem), "loss workspace too small");
    CHECK_ARG(((uintptr_t)workspace & 7) == 0, "workspace not 8-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = dtype == GS_F32
                       ? launch_l1_dssim<float>(rgb, target, vt, lam, scale, dL_drgb, loss_dev, workspace, s)
                       : launch_l1_dssim<double>(rgb, target, vt, lam, scale, dL_drgb, loss_dev, workspace, s);
    return hip_status(e, "gs_loss_l1_dssim");
}

gs_status gs_densify_stats(gs_dtype dtype, const void *projected, const void *dprojected, int64_t n, int32_t views,
                           double scale, float *accum, int32_t *count, void *stream)
{
    CHECK_ARG(dtype_ok(dtype), "bad dtype");
    CHECK_ARG(n >= 0 && views >= 1 && views <= GS_MAX_VIEWS, "bad n or views");
    CHECK_ARG(n == 0 || (projected && dprojected && accum && count), "null pointer");
    CHECK_ARG(isfinite(scale), "bad scale");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = dtype == GS_F32
                       ? launch_densify_stats<float>(projected, dprojected, n, views, scale, accum, count, s)
                       : launch_densify_stats<double>(projected, dprojected, n, views, scale, accum, count, s);
    return hip_status(e, "gs_densify_stats");
}

size_t gs_densify_workspace_bytes(int64_t n) { return n < 0 ? 0 : densify_ws_bytes(n); }

gs_status gs_densify_plan(gs_dtype dtype, const void *params, int64_t n, const float *accum, const int32_t *count,
                          const gs_densify_hparams *h, void *workspace, size_t workspace_bytes, int64_t *counts_dev,
                          void *stream)
{
    CHECK_ARG(dtype_ok(dtype), "bad dtype");
    CHECK_ARG(n >= 0, "n < 0");
    CHECK_ARG(h && workspace && counts_dev, "null pointer");
    CHECK_ARG(n == 0 || (params && accum && count), "null pointer");
    CHECK_ARG(isfinite(h->grad_threshold) && h->grad_threshold >= 0.0, "bad gradient threshold");
    CHECK_ARG(!isnan(h->split_log_scale) && !isnan(h->prune_logit) && !isnan(h->prune_log_scale), "NaN threshold");
    CHECK_ARG(workspace_bytes >= densify_ws_bytes(n), "densify workspace too small");
    CHECK_ARG(((uintptr_t)workspace & 255) == 0, "workspace not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = dtype == GS_F32 ? launch_densify_plan<float>(params, n, accum, count, *h, workspace, counts_dev, s)
                                   : launch_densify_plan<double>(params, n, accum, count, *h, workspace, counts_dev, s);
    return hip_status(e, "gs_densify_plan");
}

gs_status gs_densify_apply(gs_dtype dtype, const void *params, const void *m, const void *v, int64_t n,
                           const void *noise, const void *workspace, size_t workspace_bytes, void *params_out,
                           void *m_out, void *v_out, int64_t n_out, void *stream)
{
    CHECK_ARG(dtype_ok(dtype), "bad dtype");
    CHECK_ARG(n >= 0 && n_out >= 0, "n < 0");
    CHECK_ARG(workspace, "null pointer");
    CHECK_ARG(n == 0 || (params && m && v && noise), "null pointer");
    CHECK_ARG(n_out == 0 || (params_out && m_out && v_out), "null pointer");
    CHECK_ARG(n_out <= 2 * n, "n_out larger than any plan allows");
    CHECK_ARG(n_out == 0 || (params_out != params && params_out != m && params_out != v && m_out != params &&
                             m_out != m && m_out != v && v_out != params && v_out != m && v_out != v),
              "outputs alias inputs");
    CHECK_ARG(workspace_bytes >= densify_ws_bytes(n), "densify workspace too small");
    CHECK_ARG(((uintptr_t)workspace & 255) == 0, "workspace not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = dtype == GS_F32
                       ? launch_densify_apply<float>(params, m, v, n, noise, workspace, params_out, m_out, v_out,
                                                     n_out, s)
                       : launch_densify_apply<double>(params, m, v, n, noise, workspace, params_out, m_out, v_out,
                                                      n_out, s);
    return hip_status(e, "gs_densify_apply");
}

gs_status gs_reset_opacity(gs_dtype dtype, void *params, void *m, void *v, int64_t n, double max_logit, void *stream)
{
    CHECK_ARG(dtype_ok(dtype), "bad dtype");
    CHECK_ARG(n >= 0, "n < 0");
    CHECK_ARG(n == 0 || (params && m && v), "null pointer");
    CHECK_ARG(!isnan(max_logit), "NaN max_logit");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = dtype == GS_F32 ? launch_reset_opacity<float>(params, m, v, n, max_logit, s)
                                   : launch_reset_opacity<double>(params, m, v, n, max_logit, s);
    return hip_status(e, "gs_reset_opacity");
}

gs_status gs_adam_step(gs_dtype dtype, void *params, void *grad, void *m, void *v, int64_t n,
                       const gs_adam_hparams *h, int64_t *step_dev, double *scratch, const int32_t *skip_flag,
                       void *stream)
{
    CHECK_ARG(dtype_ok(dtype), "bad dtype");
    CHECK_ARG(h && step_dev && scratch, "null pointer");
    CHECK_ARG(n >= 0, "n < 0");
    CHECK_ARG(n == 0 || (params && grad && m && v), "null pointer");
    CHECK_ARG(h->batch_size >= 1, "batch_size must be >= 1");
    CHECK_ARG(h->beta1 >= 0 && h->beta1 < 1 && h->beta2 >= 0 && h->beta2 < 1 && h->eps >= 0, "bad betas / eps");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = dtype == GS_F32 ? launch_adam<float>(params, grad, m, v, n, h, step_dev, scratch, skip_flag, s)
                                   : launch_adam<double>(params, grad, m, v, n, h, step_dev, scratch, skip_flag, s);
    return hip_status(e, "gs_adam_step");
}

gs_status gs_project_bwd_adam(gs_dtype dtype, void *params, int64_t n, const gs_camera *cams_dev,
                              const gs_camera *cams_host, int32_t views, const void *projected, void *dprojected,
                              void *grad, void *m, void *v, const gs_adam_hparams *h, int64_t *step_dev,
                              double *scratch, const int32_t *skip_flag, void *stream)
{
    std::string why;
    CHECK_ARG(dtype_ok(dtype), "bad dtype");
    CHECK_ARG(cams_ok(cams_host, views, why), why);
    CHECK_ARG(n >= 0 && (uint64_t)n * (uint64_t)views < (uint64_t(1) << 32), "n * views must be < 2^32");
    CHECK_ARG(h && step_dev && scratch, "null pointer");
    CHECK_ARG(n == 0 || (params && cams_dev && projected && dprojected && grad && m && v), "null pointer");
    CHECK_ARG(h->batch_size >= 1, "batch_size must be >= 1");
    CHECK_ARG(h->beta1 >= 0 && h->beta1 < 1 && h->beta2 >= 0 && h->beta2 < 1 && h->eps >= 0, "bad betas / eps");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = dtype == GS_F32
                       ? launch_project_bwd_adam<float>(params, n, cams_dev, views, projected, dprojected, grad, m, v,
                                                        h, step_dev, scratch, skip_flag, s)
                       : launch_project_bwd_adam<double>(params, n, cams_dev, views, projected, dprojected, grad, m,
                                                         v, h, step_dev, scratch, skip_flag, s);
    return hip_status(e, "gs_project_bwd_adam");
}

}  // extern "C"
