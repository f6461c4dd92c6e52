// Render forward and backward over 16x16 pixel tiles (paper section 2.1 step
// 2; appendix A.3: render and its backward are pixel-wise), and the
// scheduler that spreads the tiles of a whole batch over the GPU.
//
// A tile is worked by one workgroup of 256/PX threads, each owning PX pixels.
// The tile's depth-ordered list is staged CHUNK records at a time into LDS
// (one gathered 48-byte record per entry), and every thread walks the staged
// records for its pixels. In the backward pass the list is walked in reverse
// from the tile's largest `last`, the blend is undone with T_k = T_{k+1} /
// (1 - alpha_k), and the nine per-Gaussian gradient sums of a wavefront are
// reduced together (a transposed permlane/DPP reduction) before three global
// atomics.
//
// Work distribution:
//  - per-tile mode: one workgroup per tile; workgroup b runs tile
//    (b mod 8) * ceil(T/8) + b div 8, so each XCD (workgroups are dealt
//    round-robin to the 8 XCDs) sees a contiguous eighth of the serialised
//    tiles and neighbouring tiles share that XCD's L2;
//  - XCD-split mode: as per-tile, but the eighth of the tiles each XCD takes
//    is a cost-balanced contiguous chunk (Algorithm 1 with G = 8);
//  - persistent mode: a fixed grid of workgroups takes tiles from Q queues.
//    The queues are the contiguous, cost-balanced chunks of Algorithm 1
//    (division points) computed from per-tile costs; queue q belongs to XCD
//    q div (Q/8). A workgroup drains its home queue, then steals from the
//    other queues of its XCD, then from the other XCDs.
#include "common.hpp"

namespace gs {

template <typename T> using V4 = typename Vec4<T>::type;

template <typename T> struct FwdArgs {
    const T *proj;
    int64_t n;
    const uint32_t *ids;
    const uint32_t *ranges;
    T bg[3];
    T *rgb;
    T *finalT;
    uint32_t *last;
    uint32_t *work_fwd;
    uint32_t *work_bwd;
    unsigned long long *stats;   // [2]: pairs evaluated, pairs blended (STATS variants only)
    // L1 loss fused into the output stage (target null: no loss)
    const T *target;             // like rgb
    T *dL;                       // like rgb: scale sign(rgb - target) / (3 H W views)
    double *loss_tile;           // [total tiles]: the tile's share of the loss
    double loss_scale;
};

template <typename T> struct BwdArgs {
    const T *proj;
    int64_t n;
    const uint32_t *ids;
    const uint32_t *ranges;
    T bg[3];
    const T *finalT;
    const uint32_t *last;
    const T *dL;
    T *dproj;
};

// BWD: the backward also needs the raw conic and the Gaussian index; the
// forward leaves them out, which keeps its LDS per workgroup small enough
// for eight workgroups of one wavefront per SIMD.
// The fourth slot of b, c and d carries an integer's bits, so one 16-byte
// load per vector brings every per-record value.
template <typename T, int CHUNK, bool BWD> struct Stage {
    V4<T> a[CHUNK];               // u, v, r^2, opacity
    V4<T> b[BWD ? CHUNK : 1];     // conic a, b, c, Gaussian index
    V4<T> c[CHUNK];               // r, g, b, 1 + position of the record in the tile's list
    V4<T> d[CHUNK];               // scaled conic na, nb, nc (see scaled_conic), bands
                                  // (bit k: the record may touch pixel rows 4k..4k+3 of the tile)
    uint32_t wcnt[4];
};

__device__ __forceinline__ float u32_bits(uint32_t x, float) { return __uint_as_float(x); }
__device__ __forceinline__ double u32_bits(uint32_t x, double) { return __longlong_as_double((long long)x); }
__device__ __forceinline__ uint32_t bits_u32(float v) { return __float_as_uint(v); }
__device__ __forceinline__ uint32_t bits_u32(double v) { return (uint32_t)__double_as_longlong(v); }
// the integer carried in a staged vector's fourth slot, read as a wave-uniform value
template <typename T> __device__ __forceinline__ uint32_t staged_u32(T v)
{
    return __builtin_amdgcn_readfirstlane(bits_u32(v));
}

// Per-record constants of the culling tests below.
template <typename T> struct CullRec {
    T u, v, a, b, c;
    T ia, ic;      // 1/a, 1/c
    T r2c;         // radius^2 with a relative and an absolute slack
    T lim;         // log(255 opacity) + 0.01: the exponent bound where alpha reaches 1/255
};

__device__ __forceinline__ float log_t(float x) { return __logf(x); }
__device__ __forceinline__ double log_t(double x) { return log(x); }

template <typename T> __device__ __forceinline__ CullRec<T> cull_rec(T u, T v, T r2, T a, T b, T c, T o)
{
    CullRec<T> k;
    k.u = u; k.v = v; k.a = a; k.b = b; k.c = c;
    k.ia = rcp_t(a);
    k.ic = rcp_t(c);
    k.r2c = r2 * T(1.001) + T(0.01);
    k.lim = log_t(o * T(255)) + T(0.01);
    return k;
}

// Minimum over the box [lx, hx] x [ly, hy] of the quadratic form
// a dx^2 + 2 b dx dy + c dy^2 (positive definite), with (dx, dy) measured from
// the centre (u, v); 0 if the centre is inside the box. On each edge the
// minimiser along the free coordinate is clamped into the edge; an inexact
// minimiser only raises the value by a second-order amount.
template <typename T>
__device__ __forceinline__ T box_min_quadratic(T lx, T hx, T ly, T hy, const CullRec<T> &k)
{
    if (lx <= T(0) && hx >= T(0) && ly <= T(0) && hy >= T(0)) return T(0);
    auto edge_x = [&](T dx) {        // dx fixed, dy free in [ly, hy]
        T dy = fmin(fmax(-k.b * dx * k.ic, ly), hy);
        return fma(k.a * dx, dx, fma(T(2) * k.b * dx, dy, k.c * dy * dy));
    };
    auto edge_y = [&](T dy) {        // dy fixed, dx free in [lx, hx]
        T dx = fmin(fmax(-k.b * dy * k.ia, lx), hx);
        return fma(k.a * dx, dx, fma(T(2) * k.b * dx, dy, k.c * dy * dy));
    };
    return fmin(fmin(edge_x(lx), edge_x(hx)), fmin(edge_y(ly), edge_y(hy)));
}

// Conservative test that a record cannot reach alpha >= 1/255 inside its
// footprint circle at any pixel centre in [bx0, bx1] x [by0, by1]. A pixel
// keeps a Gaussian only if its centre is within the radius and
// o exp(-q/2) >= 1/255 with q the conic's quadratic form; the test culls when
// the circle misses the whole box, or when the box minimum of q already gives
// alpha below 1/255 by a margin that bounds the rounding of the per-pixel
// evaluation (16 FP32 ulps of the largest term a dx^2 + c dy^2 over the box,
// plus 0.01). A culled record is thus skipped at every pixel anyway and the
// image is unchanged.
template <typename T>
__device__ __forceinline__ bool box_culls(const CullRec<T> &k, T bx0, T bx1, T by0, T by1)
{
    T lx = bx0 - k.u, hx = bx1 - k.u, ly = by0 - k.v, hy = by1 - k.v;
    T ex = fmax(fmax(lx, -hx), T(0)), ey = fmax(fmax(ly, -hy), T(0));
    if (ex * ex + ey * ey > k.r2c) return true;                   // circle misses every centre
    T qmin = box_min_quadratic(lx, hx, ly, hy, k);
    T dmax2 = fmax(lx * lx, hx * hx) + fmax(ly * ly, hy * hy);
    T margin = T(1e-6) * (k.a + k.c) * dmax2;
    return T(0.5) * qmin > k.lim + margin;
}

// Records of one chunk held in registers between the gather and the LDS
// commit, so the next chunk's gathers are in flight while the current chunk
// is composited.
template <typename T, int CHUNK, int NT> struct Fetched {
    static constexpr int R = (CHUNK + NT - 1) / NT;
    V4<T> r0[R], r1[R], r2[R];
    uint32_t id[R];
    int cnt;
    uint32_t pos0;
};

template <typename T, int CHUNK, int NT>
__device__ __forceinline__ void fetch_records(Fetched<T, CHUNK, NT> &f, const T *__restrict__ proj, int64_t vbase,
                                              const uint32_t *__restrict__ ids, int64_t first, int cnt, uint32_t pos0)
{
    f.cnt = cnt;
    f.pos0 = pos0;
    for (int rr = 0; rr < Fetched<T, CHUNK, NT>::R; rr++) {
        int q = rr * NT + threadIdx.x;
        if (q < cnt) {
            uint32_t id = ids[first + q];
            const V4<T> *rec = reinterpret_cast<const V4<T> *>(proj + (vbase + id) * REC);
            f.id[rr] = id;
            f.r0[rr] = rec[0];
            f.r1[rr] = rec[1];
            f.r2[rr] = rec[2];
        }
    }
}

// Commits fetched records that can touch the tile to LDS, compacted in list
// order, with a mask of the four 16x4 pixel bands of the tile each can touch;
// returns how many were kept. A band is exactly one wavefront's pixels in
// every launch shape, so the render loops skip a band with a wave-uniform
// branch.
// Bands a commit may keep: bit k of `allow`, and only for records whose
// 1 + position is at most last[k] (the backward's largest last of band k).
struct BandLimit {
    uint32_t allow;
    uint32_t last[4];
};

template <typename T, int CHUNK, int NT, bool BWD>
__device__ __forceinline__ int commit_records(Stage<T, CHUNK, BWD> &st, const Fetched<T, CHUNK, NT> &f, T bx0, T by0,
                                              const BandLimit &lim)
{
    constexpr int NW = NT / 64;
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t lt = (1ull << lane) - 1ull;
    int kept = 0;
    for (int rr = 0; rr < Fetched<T, CHUNK, NT>::R; rr++) {
        int q = rr * NT + threadIdx.x;
        if (rr * NT >= f.cnt) break;
        uint32_t bands = 0;
        V4<T> sa, sb, sc;
        if (q < f.cnt) {
            V4<T> r0v = f.r0[rr], r1 = f.r1[rr], r2 = f.r2[rr];
            T rad = r2.y;
            sa = V4<T>{r0v.x, r0v.y, rad * rad, r1.y};
            sb = V4<T>{r0v.z, r0v.w, r1.x, T(0)};
            sc = V4<T>{r1.z, r1.w, r2.x, T(0)};
            if (sa.w >= K<T>::alpha_min) {   // alpha <= opacity everywhere
                CullRec<T> k = cull_rec(sa.x, sa.y, sa.z, sb.x, sb.y, sb.z, sa.w);
                const uint32_t k1 = f.pos0 + (uint32_t)q + 1u;
                for (int band = 0; band < 4; band++)
                    if (((lim.allow >> band) & 1u) && k1 <= lim.last[band] &&
                        !box_culls(k, bx0, bx0 + T(15), by0 + T(4 * band), by0 + T(4 * band + 3)))
                        bands |= 1u << band;
            }
        }
        bool keep = bands != 0;
        uint64_t m = __ballot(keep);
        int off = kept;
        if (NW > 1) {
            if (lane == 0) st.wcnt[w] = (uint32_t)__popcll(m);
            __syncthreads();
            int tot = 0;
            for (int j = 0; j < NW; j++) {
                int c = (int)st.wcnt[j];
                if (j < w) off += c;
                tot += c;
            }
            __syncthreads();
            kept += tot;
        } else {
            kept += __popcll(m);
        }
        if (keep) {
            int slot = off + __popcll(m & lt);
            T na, nb, nc;
            scaled_conic(sb.x, sb.y, sb.z, na, nb, nc);
            st.a[slot] = sa;
            if constexpr (BWD) st.b[slot] = V4<T>{sb.x, sb.y, sb.z, u32_bits(f.id[rr], T(0))};
            st.c[slot] = V4<T>{sc.x, sc.y, sc.z, u32_bits(f.pos0 + (uint32_t)q + 1u, T(0))};
            st.d[slot] = V4<T>{na, nb, nc, u32_bits(bands, T(0))};
        }
    }
    return kept;
}

// ------------------------------------------------------------------ forward tile
template <typename T, int PX, int CHUNK, bool STATS>
__device__ void fwd_tile(int32_t g, const ViewTable &vt, const FwdArgs<T> &A, Stage<T, CHUNK, false> &st,
                         uint32_t *s_red)
{
    uint32_t n_eval = 0, n_blend = 0;
    constexpr int NT = 256 / PX;
    const int wave_id = NT == 64 ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int v = view_of_tile(vt, g);
    int local = g - vt.tile_base[v];
    int TX = vt.tiles_x[v];
    int tx = local % TX, ty = local / TX;
    int W = vt.width[v], H = vt.height[v];
    // a thread's pixels share one column: NT is a multiple of the tile width
    const T pxc = (T)(tx * TILE + (threadIdx.x & 15)) + T(0.5);
    // Tr: transmittance, stored negated once the pixel is finished (it
    // saturated, or it lies outside the image), which saves a flag per pixel
    T pyc[PX], Tr[PX], C[PX][3];
    uint32_t lastp[PX];
    bool inside[PX];
    for (int j = 0; j < PX; j++) {
        int p = threadIdx.x + j * NT;
        int px = tx * TILE + (p & 15), py = ty * TILE + (p >> 4);
        inside[j] = px < W && py < H;
        pyc[j] = (T)py + T(0.5);
        Tr[j] = inside[j] ? T(1) : T(-1);
        C[j][0] = C[j][1] = C[j][2] = T(0);
        lastp[j] = 0;
    }
    uint32_t s = A.ranges[2 * (int64_t)g], e = A.ranges[2 * (int64_t)g + 1];
    int64_t vbase = (int64_t)v * A.n;
    uint32_t walked = 0;
    if (threadIdx.x == 0) *s_red = 0;
    T bx0 = (T)(tx * TILE) + T(0.5), by0 = (T)(ty * TILE) + T(0.5);
    Fetched<T, CHUNK, NT> fr;
    if (s < e) fetch_records<T, CHUNK, NT>(fr, A.proj, vbase, A.ids, s, (int)min((uint32_t)CHUNK, e - s), 0u);
    for (uint32_t base = s; base < e; base += CHUNK) {
        __syncthreads();
        // bit j (NT/64): slot j of this wavefront still has an unfinished pixel
        uint32_t live_bands = 0;
        for (int j = 0; j < PX; j++)
            live_bands |= (__ballot(Tr[j] > T(0)) != 0 ? 1u : 0u) << (j * (NT / 64));
        // one wavefront per tile: its finished bands need no staged records
        const BandLimit lim{NT == 64 ? live_bands : 0xfu, {~0u, ~0u, ~0u, ~0u}};
        int kept = commit_records<T, CHUNK, NT>(st, fr, bx0, by0, lim);
        int cnt = fr.cnt;
        __syncthreads();
        uint32_t nb = base + CHUNK;
        if (nb < e) fetch_records<T, CHUNK, NT>(fr, A.proj, vbase, A.ids, nb, (int)min((uint32_t)CHUNK, e - nb), nb - s);
        if (live_bands == 0) kept = 0;            // this wavefront's pixels are all finished
        // records in groups of eight; between groups, drop finished bands and
        // leave once every pixel of the wavefront is finished
        for (int q0 = 0; q0 < kept; q0 += 8) {
            const int q1 = min(q0 + 8, kept);
            for (int q = q0; q < q1; q++) {
                V4<T> ra = st.a[q], rd = st.d[q], rc = st.c[q];
                uint32_t bm = (staged_u32(rd.w) >> wave_id) & live_bands;   // wave-uniform
                uint32_t pos1 = bits_u32(rc.w);
                ColTerms<T> col = col_terms(pxc, ra.x, rd.x, rd.y);
                for (int j = 0; j < PX; j++) {
                    if ((bm >> (j * (NT / 64))) & 1u) {   // wave-uniform: the record can touch this band
                        T dy, G, og, alpha;
                        bool ok = eval_alpha(col, pyc[j], ra.y, ra.z, rd.z, ra.w, dy, G, og, alpha);
                        // A finished pixel holds -T: then Tn < 0 fails the blend
                        // test below and -|T| leaves it unchanged, so `ok` needs
                        // no separate live test.
                        T Tj = Tr[j];
                        T Tn = fma(-alpha, Tj, Tj);                 // T (1 - alpha)
                        bool bl = ok && (Tn >= K<T>::t_min);   // (Tn is finite wherever ok holds)
                        T w = bl ? alpha * Tj : T(0);
                        C[j][0] = fma(rc.x, w, C[j][0]);
                        C[j][1] = fma(rc.y, w, C[j][1]);
                        C[j][2] = fma(rc.z, w, C[j][2]);
                        Tr[j] = bl ? Tn : (ok ? -fabs(Tj) : Tj);   // stop: mark finished
                        lastp[j] = bl ? pos1 : lastp[j];
                        if (STATS) {
                            n_eval += Tj > T(0) ? 1u : 0u;
                            n_blend += bl ? 1u : 0u;
                        }
                    }
                }
            }
            live_bands = 0;
            for (int j = 0; j < PX; j++)
                live_bands |= (__ballot(Tr[j] > T(0)) != 0 ? 1u : 0u) << (j * (NT / 64));
            if (live_bands == 0) break;
        }
        bool alldone = true;
        for (int j = 0; j < PX; j++) alldone &= Tr[j] < T(0);
        walked += cnt;
        if (!__syncthreads_or(!alldone)) break;
    }
    uint32_t mylast = 0;
    const int64_t plane = (int64_t)W * H;
    // per-element L1 weight, computed exactly as the standalone loss does
    const double wd = A.target ? A.loss_scale / ((double)(3 * plane) * (double)vt.nviews) : 0.0;
    double labs = 0.0;
    for (int j = 0; j < PX; j++) {
        if (!inside[j]) continue;
        int p = threadIdx.x + j * NT;
        int px = tx * TILE + (p & 15), py = ty * TILE + (p >> 4);
        int64_t pix = vt.pix_base[v] + (int64_t)py * W + px;
        int64_t o = 3 * vt.pix_base[v] + (int64_t)py * W + px;
        T Tf = fabs(Tr[j]);
        T out[3];
        for (int ch = 0; ch < 3; ch++) {
            out[ch] = C[j][ch] + Tf * A.bg[ch];
            A.rgb[o + ch * plane] = out[ch];
        }
        if (A.target) {                     // L1: gradient now, loss summed per tile
            T w = (T)wd;
            for (int ch = 0; ch < 3; ch++) {
                T d = out[ch] - A.target[o + ch * plane];
                A.dL[o + ch * plane] = d > T(0) ? w : (d < T(0) ? -w : T(0));
                labs += (double)(d < T(0) ? -d : d);
            }
        }
        A.finalT[pix] = Tf;
        A.last[pix] = lastp[j];
        mylast = max(mylast, lastp[j]);
    }
    if (A.target) {                         // the tile's share of the loss (no atomics: deterministic)
        for (int off = 32; off > 0; off >>= 1) labs += __shfl_xor(labs, off, 64);
        if (NT == 64) {
            if (threadIdx.x == 0) A.loss_tile[g] = labs * wd;
        } else {
            __shared__ double s_l[NT / 64];
            if ((threadIdx.x & 63) == 0) s_l[threadIdx.x >> 6] = labs;
            __syncthreads();
            if (threadIdx.x == 0) {
                double t = 0.0;
                for (int k = 0; k < NT / 64; k++) t += s_l[k];
                A.loss_tile[g] = t * wd;
            }
        }
    }
    if (A.work_bwd) atomicMax(s_red, mylast);
    if (STATS) {
        atomicAdd(A.stats, (unsigned long long)n_eval);
        atomicAdd(A.stats + 1, (unsigned long long)n_blend);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (A.work_fwd) A.work_fwd[g] = walked;
        if (A.work_bwd) A.work_bwd[g] = *s_red;
    }
}

// ------------------------------------------------------------------ backward tile
template <typename T, int PX, int CHUNK>
__device__ void bwd_tile(int32_t g, const ViewTable &vt, const BwdArgs<T> &A, Stage<T, CHUNK, true> &st,
                         uint32_t *s_red)
{
    constexpr int NT = 256 / PX;
    int v = view_of_tile(vt, g);
    int local = g - vt.tile_base[v];
    int TX = vt.tiles_x[v];
    int tx = local % TX, ty = local / TX;
    int W = vt.width[v], H = vt.height[v];
    const int wave_id = NT == 64 ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const T pxc = (T)(tx * TILE + (threadIdx.x & 15)) + T(0.5);   // one column per thread
    // Sg: the colour composited behind the current Gaussian, dotted with the
    // pixel's colour gradient (only that product enters the gradients)
    T pyc[PX], Tr[PX], gr[PX][3], Sg[PX];
    uint32_t L[PX];
    uint32_t mymax = 0;
    int64_t plane = (int64_t)W * H;
    for (int j = 0; j < PX; j++) {
        int p = threadIdx.x + j * NT;
        int px = tx * TILE + (p & 15), py = ty * TILE + (p >> 4);
        bool in = px < W && py < H;
        pyc[j] = (T)py + T(0.5);
        int64_t pix = vt.pix_base[v] + (int64_t)py * W + px;
        const T *dl = A.dL + 3 * vt.pix_base[v] + (int64_t)py * W + px;
        Tr[j] = in ? A.finalT[pix] : T(1);
        L[j] = in ? A.last[pix] : 0u;
        for (int ch = 0; ch < 3; ch++) gr[j][ch] = in ? dl[ch * plane] : T(0);
        Sg[j] = fma(gr[j][0], A.bg[0], fma(gr[j][1], A.bg[1], gr[j][2] * A.bg[2]));
        mymax = max(mymax, L[j]);
    }
    // factors of the summed components: d/d(a, b, c) of the exponent
    // -(a dx^2 + c dy^2)/2 - b dx dy are -1/2, -1, -1/2 times the sums kept
    const int comp = sizeof(T) == 4 ? sum9_comp(threadIdx.x) : (int)(threadIdx.x & 63);   // component this lane adds
    const T sc = (comp == 2 || comp == 4) ? T(-0.5) : comp == 3 ? T(-1) : T(1);
    // per band (one wavefront's pixels) the largest last, held by lane
    // j (NT/64) of the wavefront: one compare and ballot per record then give
    // the bands that still have a contributor behind the record
    uint32_t Lv = 0;
    for (int j = 0; j < PX; j++) {
        uint32_t lb = __builtin_amdgcn_readfirstlane(wave_max(L[j]));
        Lv = (int)(threadIdx.x & 63) == j * (NT / 64) ? lb : Lv;
    }
    if (threadIdx.x == 0) *s_red = 0;
    __syncthreads();
    atomicMax(s_red, mymax);
    __syncthreads();
    uint32_t Lmax = *s_red;
    uint32_t s = A.ranges[2 * (int64_t)g];
    int64_t vbase = (int64_t)v * A.n;
    T bx0 = (T)(tx * TILE) + T(0.5), by0 = (T)(ty * TILE) + T(0.5);
    Fetched<T, CHUNK, NT> fr;
    if (Lmax > 0) {
        int64_t lo0 = (int64_t)Lmax - CHUNK > 0 ? (int64_t)Lmax - CHUNK : 0;
        fetch_records<T, CHUNK, NT>(fr, A.proj, vbase, A.ids, (int64_t)s + lo0, (int)(Lmax - lo0), (uint32_t)lo0);
    }
    // one wavefront per tile: a band takes no record past its largest last
    BandLimit lim{0xfu, {~0u, ~0u, ~0u, ~0u}};
    if (NT == 64)
        for (int j = 0; j < PX && j < 4; j++) lim.last[j] = __builtin_amdgcn_readlane(Lv, j);
    for (int64_t hi = Lmax; hi > 0; hi -= CHUNK) {
        __syncthreads();
        int kept = commit_records<T, CHUNK, NT>(st, fr, bx0, by0, lim);
        __syncthreads();
        int64_t lo = hi - CHUNK > 0 ? hi - CHUNK : 0;
        if (lo > 0) {
            int64_t lo2 = lo - CHUNK > 0 ? lo - CHUNK : 0;
            fetch_records<T, CHUNK, NT>(fr, A.proj, vbase, A.ids, (int64_t)s + lo2, (int)(lo - lo2), (uint32_t)lo2);
        }
        for (int q = kept - 1; q >= 0; q--) {
            V4<T> ra = st.a[q], rb = st.b[q], rc = st.c[q], rd = st.d[q];
            const uint32_t k1 = bits_u32(rc.w);                   // 1 + the record's position
            uint32_t bm = staged_u32(rd.w) >> wave_id;
            if constexpr (NT != 64)   // (one wavefront per tile: the commit already dropped such bands)
                bm &= (uint32_t)__ballot(k1 <= Lv);               // the position is below the largest last of band j
            // dL/d(exponent) moments over this thread's pixels: they share the column
            // (one dx), so the position and conic sums factor through
            // D0 = sum d, D1 = sum d dy, D2 = sum d dy^2 (d = dL/d exponent)
            T D0 = T(0), D1 = T(0), D2 = T(0), acc[9];
            for (int c = 5; c < 9; c++) acc[c] = T(0);
            bool any = false;
            ColTerms<T> col = col_terms(pxc, ra.x, rd.x, rd.y);
            const T dx = col.dx;
            // The pairs of this record over the thread's pixels. The 0.99 clamp
            // of alpha has no gradient; it is tested in every pair (one loop
            // for every record: a second copy for records that cannot reach
            // the clamp made the compiler copy the loop-carried T and S at
            // every record).
            for (int j = 0; j < PX; j++) {
                if (!((bm >> (j * (NT / 64))) & 1u)) continue;     // wave-uniform band skip
                T dy, G, og, alpha;
                bool ok = eval_alpha(col, pyc[j], ra.y, ra.z, rd.z, ra.w, dy, G, og, alpha);
                if (ok && k1 <= L[j]) {   // lanes whose pixel blended this Gaussian
                    any = true;
                    T Tk = Tr[j] * rcp_t(T(1) - alpha);   // transmittance in front of this Gaussian
                    T w = alpha * Tk;
                    T gx = gr[j][0], gy = gr[j][1], gz = gr[j][2];
                    acc[6] = fma(w, gx, acc[6]);
                    acc[7] = fma(w, gy, acc[7]);
                    acc[8] = fma(w, gz, acc[8]);
                    T cg = fma(rc.x, gx, fma(rc.y, gy, rc.z * gz));
                    T diff = cg - Sg[j];
                    T dalpha = diff * Tk;
                    Sg[j] = fma(alpha, diff, Sg[j]);      // alpha c + (1 - alpha) S
                    Tr[j] = Tk;
                    T live = og <= K<T>::alpha_max ? dalpha : T(0);   // the clamped pair passes no gradient
                    T dpow = live * og;
                    T hy = dpow * dy;
                    acc[5] = fma(live, G, acc[5]);
                    D0 += dpow;
                    D1 += hy;
                    D2 = fma(hy, dy, D2);
                }
            }
            // d/du, d/dv through (dx, dy) and d/d(a, b, c) (times -1/2, -1, -1/2 after the reduction)
            T hx = dx * D0;
            acc[0] = fma(rb.x, hx, rb.y * D1);
            acc[1] = fma(rb.y, hx, rb.z * D1);
            acc[2] = dx * hx;
            acc[3] = dx * D1;
            acc[4] = D2;
            if (__ballot(any) == 0) continue;
            wave_sum9_atomic(acc, A.dproj + (vbase + staged_u32(rb.w)) * REC, sc, T(1));
        }
    }
}

// ------------------------------------------------------------------ kernels
__device__ __forceinline__ int32_t per_tile_index(int32_t b, int32_t T_all)
{
    int32_t per = (T_all + 7) / 8;
    return (b & 7) * per + (b >> 3);
}

// Claims the next tile for this workgroup in persistent mode; -1 when every
// queue is drained. Home queue first, then the rest of the XCD, then others.
__device__ __forceinline__ int32_t claim(const SchedState &S, int &qi, int32_t *s_item)
{
    if (threadIdx.x == 0) {
        int Q = S.queues, per = Q / 8;
        int x = blockIdx.x & 7;
        int home = x * per + (int)((blockIdx.x >> 3) % per);
        int32_t item = -1;
        while (qi < Q) {
            int q;
            if (qi < per) q = x * per + (home - x * per + qi) % per;
            else {
                int o = qi - per;                 // other XCDs, nearest first
                int xo = (x + 1 + o / per) & 7;
                q = xo * per + o % per;
            }
            int32_t end = S.dp[q + 1];
            if (__hip_atomic_load(S.cursor + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < end) {
                int32_t got = atomicAdd(S.cursor + q, 1);
                if (got < end) { item = got; break; }
            }
            qi++;
        }
        *s_item = item;
    }
    __syncthreads();
    int32_t item = *s_item;
    __syncthreads();
    return item;
}

template <typename T, int PX, int CHUNK, bool STATS>
__global__ void __launch_bounds__(256 / PX) __attribute__((amdgpu_waves_per_eu(7))) render_fwd_kernel(ViewTable vt, FwdArgs<T> A)
{
    __shared__ Stage<T, CHUNK, false> st;
    __shared__ uint32_t s_red;
    int32_t g = per_tile_index(blockIdx.x, vt.total_tiles);
    if (g >= vt.total_tiles) return;
    fwd_tile<T, PX, CHUNK, STATS>(g, vt, A, st, &s_red);
}

template <typename T, int PX, int CHUNK, bool STATS>
__global__ void __launch_bounds__(256 / PX) __attribute__((amdgpu_waves_per_eu(7)))
render_fwd_persistent(ViewTable vt, FwdArgs<T> A, SchedState S)
{
    __shared__ Stage<T, CHUNK, false> st;
    __shared__ uint32_t s_red;
    __shared__ int32_t s_item;
    int qi = 0;
    for (;;) {
        int32_t g = claim(S, qi, &s_item);
        if (g < 0) break;
        fwd_tile<T, PX, CHUNK, STATS>(g, vt, A, st, &s_red);
    }
}

template <typename T, int PX, int CHUNK>
__global__ void __launch_bounds__(256 / PX) __attribute__((amdgpu_waves_per_eu(6)))
render_bwd_kernel(ViewTable vt, BwdArgs<T> A)
{
    __shared__ Stage<T, CHUNK, true> st;
    __shared__ uint32_t s_red;
    int32_t g = per_tile_index(blockIdx.x, vt.total_tiles);
    if (g >= vt.total_tiles) return;
    bwd_tile<T, PX, CHUNK>(g, vt, A, st, &s_red);
}

template <typename T, int PX, int CHUNK>
__global__ void __launch_bounds__(256 / PX) __attribute__((amdgpu_waves_per_eu(6)))
render_bwd_persistent(ViewTable vt, BwdArgs<T> A, SchedState S)
{
    __shared__ Stage<T, CHUNK, true> st;
    __shared__ uint32_t s_red;
    __shared__ int32_t s_item;
    int qi = 0;
    for (;;) {
        int32_t g = claim(S, qi, &s_item);
        if (g < 0) break;
        bwd_tile<T, PX, CHUNK>(g, vt, A, st, &s_red);
    }
}

// Cost-balanced XCD split: the serialised tiles are cut into 8 contiguous
// chunks of equal estimated cost by Algorithm 1 with G = 8 (dp[0..8], from
// the previous iteration's per-tile work), and XCD x (the workgroups b with
// b mod 8 = x) takes chunk x in order, workgroup b its tiles
// dp[x] + b div 8 + k per, k = 0, 1, ... (per = grid / 8). Adjacent tiles
// stay on one XCD's L2 as in the per-tile launch, but the XCDs finish
// together when the views' costs differ.
template <typename T, int PX, int CHUNK, bool STATS>
__global__ void __launch_bounds__(256 / PX) __attribute__((amdgpu_waves_per_eu(7)))
render_fwd_xcd(ViewTable vt, FwdArgs<T> A, const int32_t *__restrict__ dp)
{
    __shared__ Stage<T, CHUNK, false> st;
    __shared__ uint32_t s_red;
    const int x = blockIdx.x & 7;
    const int32_t per = (int32_t)(gridDim.x >> 3), hi = dp[x + 1];
    for (int32_t g = dp[x] + (int32_t)(blockIdx.x >> 3); g < hi; g += per) {
        fwd_tile<T, PX, CHUNK, STATS>(g, vt, A, st, &s_red);
        __syncthreads();
    }
}

template <typename T, int PX, int CHUNK>
__global__ void __launch_bounds__(256 / PX) __attribute__((amdgpu_waves_per_eu(6)))
render_bwd_xcd(ViewTable vt, BwdArgs<T> A, const int32_t *__restrict__ dp)
{
    __shared__ Stage<T, CHUNK, true> st;
    __shared__ uint32_t s_red;
    const int x = blockIdx.x & 7;
    const int32_t per = (int32_t)(gridDim.x >> 3), hi = dp[x + 1];
    for (int32_t g = dp[x] + (int32_t)(blockIdx.x >> 3); g < hi; g += per) {
        bwd_tile<T, PX, CHUNK>(g, vt, A, st, &s_red);
        __syncthreads();
    }
}

// LPT order: workgroup b takes the b-th heaviest tile of the previous
// iteration's per-tile work (order from launch_lpt_plan), so the long tiles
// start first and the launch ends on short ones; workgroups are dealt to
// the XCDs round-robin, which spreads the heavy tiles over all of them.
template <typename T, int PX, int CHUNK, bool STATS>
__global__ void __launch_bounds__(256 / PX) __attribute__((amdgpu_waves_per_eu(7)))
render_fwd_lpt(ViewTable vt, FwdArgs<T> A, const int32_t *__restrict__ order)
{
    __shared__ Stage<T, CHUNK, false> st;
    __shared__ uint32_t s_red;
    if ((int32_t)blockIdx.x >= vt.total_tiles) return;
    fwd_tile<T, PX, CHUNK, STATS>(order[blockIdx.x], vt, A, st, &s_red);
}

template <typename T, int PX, int CHUNK>
__global__ void __launch_bounds__(256 / PX) __attribute__((amdgpu_waves_per_eu(6)))
render_bwd_lpt(ViewTable vt, BwdArgs<T> A, const int32_t *__restrict__ order)
{
    __shared__ Stage<T, CHUNK, true> st;
    __shared__ uint32_t s_red;
    if ((int32_t)blockIdx.x >= vt.total_tiles) return;
    bwd_tile<T, PX, CHUNK>(order[blockIdx.x], vt, A, st, &s_red);
}

// XCD split with the LPT order inside each chunk: XCD x takes chunk x of
// Algorithm 1 (G = 8) as in the XCD split, its tiles heaviest first (order
// holds each chunk's tiles in decreasing cost, at the chunk's positions).
template <typename T, int PX, int CHUNK, bool STATS>
__global__ void __launch_bounds__(256 / PX) __attribute__((amdgpu_waves_per_eu(7)))
render_fwd_xcd_lpt(ViewTable vt, FwdArgs<T> A, const int32_t *__restrict__ dp, const int32_t *__restrict__ order)
{
    __shared__ Stage<T, CHUNK, false> st;
    __shared__ uint32_t s_red;
    const int x = blockIdx.x & 7;
    const int32_t per = (int32_t)(gridDim.x >> 3), hi = dp[x + 1];
    for (int32_t j = dp[x] + (int32_t)(blockIdx.x >> 3); j < hi; j += per) {
        fwd_tile<T, PX, CHUNK, STATS>(order[j], vt, A, st, &s_red);
        __syncthreads();
    }
}

template <typename T, int PX, int CHUNK>
__global__ void __launch_bounds__(256 / PX) __attribute__((amdgpu_waves_per_eu(6)))
render_bwd_xcd_lpt(ViewTable vt, BwdArgs<T> A, const int32_t *__restrict__ dp, const int32_t *__restrict__ order)
{
    __shared__ Stage<T, CHUNK, true> st;
    __shared__ uint32_t s_red;
    const int x = blockIdx.x & 7;
    const int32_t per = (int32_t)(gridDim.x >> 3), hi = dp[x + 1];
    for (int32_t j = dp[x] + (int32_t)(blockIdx.x >> 3); j < hi; j += per) {
        bwd_tile<T, PX, CHUNK>(order[j], vt, A, st, &s_red);
        __syncthreads();
    }
}

// ------------------------------------------------------------------ launchers
#define GS_DISPATCH_SHAPE(T, PX, CH, CALL)                                                                   \
    do {                                                                                                     \
        if (PX == 1 && CH == 32) { CALL(T, 1, 32); }                                                         \
        else if (PX == 1 && CH == 64) { CALL(T, 1, 64); }                                                    \
        else if (PX == 1 && CH == 128) { CALL(T, 1, 128); }                                                  \
        else if (PX == 1 && CH == 256) { CALL(T, 1, 256); }                                                  \
        else if (PX == 2 && CH == 32) { CALL(T, 2, 32); }                                                    \
        else if (PX == 2 && CH == 64) { CALL(T, 2, 64); }                                                    \
        else if (PX == 2 && CH == 128) { CALL(T, 2, 128); }                                                  \
        else if (PX == 2 && CH == 256) { CALL(T, 2, 256); }                                                  \
        else if (PX == 4 && CH == 32) { CALL(T, 4, 32); }                                                    \
        else if (PX == 4 && CH == 64) { CALL(T, 4, 64); }                                                    \
        else if (PX == 4 && CH == 128) { CALL(T, 4, 128); }                                                  \
        else { CALL(T, 4, 256); }                                                                            \
    } while (0)

// Sum of the per-tile loss shares in a fixed order (deterministic): block b
// adds slice b of the tiles (a fixed strided split over its threads, then a
// fixed tree), and one wavefront adds the block sums with a fixed tree.
__global__ void __launch_bounds__(256) loss_tiles_part_kernel(const double *__restrict__ part, int64_t n,
                                                             double *__restrict__ bsum)
{
    __shared__ double s[256];
    const int64_t per = (n + LOSS_SUM_BLOCKS - 1) / LOSS_SUM_BLOCKS;
    const int64_t b0 = (int64_t)blockIdx.x * per, b1 = b0 + per < n ? b0 + per : n;
    double a = 0.0;
    for (int64_t j = b0 + threadIdx.x; j < b1; j += 256) a += part[j];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = s[0];
}

__global__ void __launch_bounds__(64) loss_tiles_final_kernel(const double *__restrict__ bsum, double *__restrict__ loss)
{
    double a = bsum[threadIdx.x];   // LOSS_SUM_BLOCKS == 64: one per lane
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    if (threadIdx.x == 0) *loss = a;
}

hipError_t launch_tile_sum(const double *part, int64_t n, double *bsum, double *loss, hipStream_t s)
{
    hipLaunchKernelGGL(loss_tiles_part_kernel, dim3(LOSS_SUM_BLOCKS), dim3(256), 0, s, part, n, bsum);
    hipLaunchKernelGGL(loss_tiles_final_kernel, dim3(1), dim3(64), 0, s, (const double *)bsum, loss);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_render_fwd(const ViewTable &vt, const void *proj, int64_t n, const gs_bins *b, const float *bg,
                             const LaunchShape &sh, void *rgb, void *finalT, uint32_t *last, uint32_t *wf,
                             uint32_t *wb, uint64_t *stats, const void *target, double loss_scale, void *dL,
                             double *loss, double *loss_tiles, hipStream_t s)
{
    FwdArgs<T> A;
    A.target = (const T *)target;
    A.dL = (T *)dL;
    A.loss_tile = loss_tiles;
    A.loss_scale = loss_scale;
    A.proj = (const T *)proj;
    A.n = n;
    A.ids = b->ids;
    A.ranges = b->ranges;
    for (int c = 0; c < 3; c++) A.bg[c] = (T)bg[c];
    A.rgb = (T *)rgb;
    A.finalT = (T *)finalT;
    A.last = last;
    A.work_fwd = wf;
    A.work_bwd = wb;
    A.stats = (unsigned long long *)stats;
    if (vt.total_tiles == 0) return hipSuccess;
    unsigned grid_tiles = (unsigned)(8 * ((vt.total_tiles + 7) / 8));
#define GS_FWD_S(TT, P, C, ST)                                                                               \
    if (sh.mode == GS_SCHED_PERSISTENT)                                                                      \
        hipLaunchKernelGGL((render_fwd_persistent<TT, P, C, ST>), dim3(sh.workers), dim3(256 / P), 0, s, vt, A, \
                           sh.S);                                                                            \
    else if (sh.mode == GS_SCHED_XCD_SPLIT)                                                                  \
        hipLaunchKernelGGL((render_fwd_xcd<TT, P, C, ST>), dim3(grid_tiles), dim3(256 / P), 0, s, vt, A,      \
                           (const int32_t *)sh.S.dp);                                                        \
    else if (sh.mode == GS_SCHED_LPT || sh.mode == GS_SCHED_LPT_HEAD)                                        \
        hipLaunchKernelGGL((render_fwd_lpt<TT, P, C, ST>), dim3(grid_tiles), dim3(256 / P), 0, s, vt, A,      \
                           (const int32_t *)sh.S.order);                                                     \
    else if (sh.mode == GS_SCHED_XCD_LPT)                                                                    \
        hipLaunchKernelGGL((render_fwd_xcd_lpt<TT, P, C, ST>), dim3(grid_tiles), dim3(256 / P), 0, s, vt, A,  \
                           (const int32_t *)sh.S.dp, (const int32_t *)sh.S.order);                           \
    else                                                                                                     \
        hipLaunchKernelGGL((render_fwd_kernel<TT, P, C, ST>), dim3(grid_tiles), dim3(256 / P), 0, s, vt, A);
#define GS_FWD(TT, P, C)                                                                                     \
    if (stats) { GS_FWD_S(TT, P, C, true) } else { GS_FWD_S(TT, P, C, false) }
    if (sizeof(T) == 8) {
        GS_FWD(T, 1, 64);
    } else {
        GS_DISPATCH_SHAPE(T, sh.px, sh.chunk, GS_FWD);
    }
#undef GS_FWD
#undef GS_FWD_S
    if (target) return launch_tile_sum(loss_tiles, (int64_t)vt.total_tiles, loss_tiles + vt.total_tiles, loss, s);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_render_bwd(const ViewTable &vt, const void *proj, int64_t n, const gs_bins *b, const float *bg,
                             const LaunchShape &sh, const void *finalT, const uint32_t *last, const void *dL,
                             void *dproj, hipStream_t s)
{
    BwdArgs<T> A;
    A.proj = (const T *)proj;
    A.n = n;
    A.ids = b->ids;
    A.ranges = b->ranges;
    for (int c = 0; c < 3; c++) A.bg[c] = (T)bg[c];
    A.finalT = (const T *)finalT;
    A.last = last;
    A.dL = (const T *)dL;
    A.dproj = (T *)dproj;
    if (vt.total_tiles == 0) return hipSuccess;
    unsigned grid_tiles = (unsigned)(8 * ((vt.total_tiles + 7) / 8));
#define GS_BWD(TT, P, C)                                                                                     \
    if (sh.mode == GS_SCHED_PERSISTENT)                                                                      \
        hipLaunchKernelGGL((render_bwd_persistent<TT, P, C>), dim3(sh.workers), dim3(256 / P), 0, s, vt, A, sh.S); \
    else if (sh.mode == GS_SCHED_XCD_SPLIT)                                                                  \
        hipLaunchKernelGGL((render_bwd_xcd<TT, P, C>), dim3(grid_tiles), dim3(256 / P), 0, s, vt, A,          \
                           (const int32_t *)sh.S.dp);                                                        \
    else if (sh.mode == GS_SCHED_LPT || sh.mode == GS_SCHED_LPT_HEAD)                                        \
        hipLaunchKernelGGL((render_bwd_lpt<TT, P, C>), dim3(grid_tiles), dim3(256 / P), 0, s, vt, A,          \
                           (const int32_t *)sh.S.order);                                                     \
    else if (sh.mode == GS_SCHED_XCD_LPT)                                                                    \
        hipLaunchKernelGGL((render_bwd_xcd_lpt<TT, P, C>), dim3(grid_tiles), dim3(256 / P), 0, s, vt, A,      \
                           (const int32_t *)sh.S.dp, (const int32_t *)sh.S.order);                           \
    else                                                                                                     \
        hipLaunchKernelGGL((render_bwd_kernel<TT, P, C>), dim3(grid_tiles), dim3(256 / P), 0, s, vt, A);
    if (sizeof(T) == 8) {
        GS_BWD(T, 1, 64);
    } else {
        GS_DISPATCH_SHAPE(T, sh.px, sh.chunk, GS_BWD);
    }
#undef GS_BWD
    return hipGetLastError();
}

template hipError_t launch_render_fwd<float>(const ViewTable &, const void *, int64_t, const gs_bins *, const float *,
                                             const LaunchShape &, void *, void *, uint32_t *, uint32_t *, uint32_t *,
                                             uint64_t *, const void *, double, void *, double *, double *,
                                             hipStream_t);
template hipError_t launch_render_fwd<double>(const ViewTable &, const void *, int64_t, const gs_bins *, const float *,
                                              const LaunchShape &, void *, void *, uint32_t *, uint32_t *, uint32_t *,
                                              uint64_t *, const void *, double, void *, double *, double *,
                                              hipStream_t);
template hipError_t launch_render_bwd<float>(const ViewTable &, const void *, int64_t, const gs_bins *, const float *,
                                             const LaunchShape &, const void *, const uint32_t *, const void *, void *,
                                             hipStream_t);
template hipError_t launch_render_bwd<double>(const ViewTable &, const void *, int64_t, const gs_bins *, const float *,
                                              const LaunchShape &, const void *, const uint32_t *, const void *, void *,
                                              hipStream_t);

}  // namespace gs
