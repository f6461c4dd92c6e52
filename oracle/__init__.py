"""FP64 CPU oracle of the batched 3DGS training step: TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. The product path never does.

It follows the paper's pipeline (section "Background on 3D Gaussian
Training": Gaussian transformation, rendering, loss, back-propagation) and
the Adam scaling rules of section "Scaling Hyperparameters for Batched
Training" (eqs. "lambda" and "beta"). The arithmetic lives in ``oracle.c``;
this module marshals numpy arrays and writes the L1 loss, which is one line.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

ONF = 12          # projected fields per (view, Gaussian)
TILE = 16
F_U, F_V, F_DEPTH, F_A, F_B, F_C, F_OPAC, F_R, F_G, F_BL, F_RADIUS, F_REXACT = range(ONF)

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        d, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        L.oracle_project.argtypes = [d, i64, d, d]
        L.oracle_tiles_touched.argtypes = [d, d, d, i64, i32, d, d, d]
        L.oracle_tiles_touched.restype = i64
        L.oracle_bin.argtypes = [d, d, d, d, i64, i32, d, d, i64, d, d, d]
        L.oracle_bin.restype = i64
        L.oracle_render.argtypes = [d, i64, i32, i32, d, d, d, d, i32, C.c_double, C.c_double, d, d, d, d, d, d,
                                    d, d, d, d]
        L.oracle_render_brute.argtypes = [d, i64, i32, i32, d, d, d, d]
        L.oracle_render_bwd.argtypes = [d, i64, i32, i32, d, d, d, d, d]
        L.oracle_render_bwd.restype = C.c_int
        L.oracle_project_bwd.argtypes = [d, i64, d, d, d]
        L.oracle_adam.argtypes = [d, d, d, d, i64, d, C.c_double, C.c_double, C.c_double, i32, i64]
        L.oracle_sh_basis.argtypes = [d, i64, d, d]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=np.float64)


def pack_camera(cam: dict) -> np.ndarray:
    return np.concatenate([
        [cam["width"], cam["height"], cam["fx"], cam["fy"], cam["cx"], cam["cy"]],
        np.asarray(cam["R"], dtype=np.float64).reshape(9),
        np.asarray(cam["t"], dtype=np.float64).reshape(3),
        [cam["znear"]],
    ]).astype(np.float64)


def tiles_xy(cam: dict):
    return (cam["width"] + TILE - 1) // TILE, (cam["height"] + TILE - 1) // TILE


def tile_base(cams: list) -> list:
    base, out = 0, []
    for c in cams:
        out.append(base)
        tx, ty = tiles_xy(c)
        base += tx * ty
    out.append(base)
    return out


# ----------------------------------------------------------------------------- steps
def sh_basis(dirs: np.ndarray, with_grad: bool = False):
    dirs = _f64(dirs).reshape(-1, 3)
    n = dirs.shape[0]
    Y = np.zeros((n, 16))
    dY = np.zeros((n, 16, 3)) if with_grad else None
    lib().oracle_sh_basis(_p(dirs), n, _p(Y), _p(dY) if with_grad else None)
    return (Y, dY) if with_grad else Y


def project(P, cam: dict) -> np.ndarray:
    """Gaussian transformation of every Gaussian for one view: [ONF][N]."""
    P = _f64(P)
    N = P.shape[1]
    out = np.zeros((ONF, N))
    lib().oracle_project(_p(P), N, _p(pack_camera(cam)), _p(out))
    return out


def _f32(a) -> np.ndarray:
    if hasattr(a, "detach"):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=np.float32)


def tiles_touched(u, v, r, cams: list) -> np.ndarray:
    """Tiles touched per (view, Gaussian) from FP32 u, v, radius ([V][N])."""
    u, v, r = _f32(u), _f32(v), _f32(r)
    V, N = u.shape
    Ws = np.array([c["width"] for c in cams], dtype=np.int32)
    Hs = np.array([c["height"] for c in cams], dtype=np.int32)
    out = np.zeros((V, N), dtype=np.int32)
    lib().oracle_tiles_touched(_p(u), _p(v), _p(r), N, V, _p(Ws), _p(Hs), _p(out))
    return out


def bin_sort(u, v, r, depth, cams: list):
    """Sorted instances: keys (u64: global tile << 32 | FP32 depth bits), ids
    (Gaussian index) and per-global-tile [start, end) ranges."""
    u, v, r, depth = _f32(u), _f32(v), _f32(r), _f32(depth)
    V, N = u.shape
    K = int(tiles_touched(u, v, r, cams).astype(np.int64).sum())
    Ws = np.array([c["width"] for c in cams], dtype=np.int32)
    Hs = np.array([c["height"] for c in cams], dtype=np.int32)
    T = tile_base(cams)[-1]
    keys = np.zeros(max(K, 1), dtype=np.uint64)
    ids = np.zeros(max(K, 1), dtype=np.uint32)
    ranges = np.zeros((T, 2), dtype=np.uint32)
    got = lib().oracle_bin(_p(u), _p(v), _p(r), _p(depth), N, V, _p(Ws), _p(Hs), K, _p(keys), _p(ids), _p(ranges))
    assert got == K, (got, K)
    return keys[:K], ids[:K], ranges


def render(proj, cam: dict, ids, ranges_view, bg=(0.0, 0.0, 0.0), fragile=None, depth_check=False,
           pos_tol: float = 0.0, t_tol: float = 1e-5) -> dict:
    """Tiled render of one view from projected fields [ONF][N] (FP64).

    "amb" classifies each pixel by the decisions of its walk (circle test,
    exponent sign, alpha >= 1/255, transmittance stop) that lie within
    rounding of their thresholds, where a lower-precision implementation may
    rightly take either branch: 0 none; 1 exactly one, and "rgb_alt",
    "T_alt", "last_alt" hold the result with that decision taken the other
    way; 2 more than one, or two contributors whose depth order is a near
    tie. fragile/depth_check/pos_tol/t_tol only widen those margins.
    "bound" is a first-order bound, per pixel, of how far an FP32 walk may
    put colour and T from these values, from each blended alpha's relative
    error bound (large only where a thin footprint's exponent terms cancel)."""
    proj = _f64(proj)
    N = proj.shape[1]
    W, H = cam["width"], cam["height"]
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    ranges_view = np.ascontiguousarray(ranges_view, dtype=np.uint32)
    bgv = np.asarray(bg, dtype=np.float64)
    rgb = np.zeros((3, H, W))
    T = np.zeros((H, W))
    last = np.zeros((H, W), dtype=np.uint32)
    rgb_alt = np.zeros((3, H, W))
    T_alt = np.zeros((H, W))
    last_alt = np.zeros((H, W), dtype=np.uint32)
    nc = np.zeros((H, W), dtype=np.uint32)
    amb = np.zeros((H, W), dtype=np.uint8)
    counts = np.zeros(2, dtype=np.int64)
    bound = np.zeros((H, W))
    fr = None if fragile is None else np.ascontiguousarray(fragile, dtype=np.uint8)
    lib().oracle_render(_p(proj), N, W, H, _p(ids) if ids.size else None, _p(ranges_view), _p(bgv),
                        _p(fr) if fr is not None else None, int(depth_check), float(pos_tol), float(t_tol),
                        _p(rgb), _p(T), _p(last), _p(nc), _p(amb), _p(counts), _p(rgb_alt), _p(T_alt), _p(last_alt),
                        _p(bound))
    return {"rgb": rgb, "T": T, "last": last, "ncontrib": nc, "amb": amb,
            "rgb_alt": rgb_alt, "T_alt": T_alt, "last_alt": last_alt, "bound": bound,
            "evaluated": int(counts[0]), "blended": int(counts[1])}


def image_mismatch(o: dict, rgb, T=None, last=None, tol: float = 1e-5):
    """Compares another implementation's image of one view with an oracle
    render ``o``. A pixel with no ambiguous decision must match the oracle's
    result; one with exactly one must match either branch (its colour, and T
    and last when given, all from the same branch); pixels of class 2 are
    left out. A pixel whose FP32 error bound ("bound") exceeds tol may
    differ by that bound instead: the error reported for it is what exceeds
    bound - tol. Returns (max error over the compared pixels, mask of those
    pixels, number of class-1 pixels that matched the alternative)."""
    rgb = np.asarray(rgb, dtype=np.float64)

    def err(ref_rgb, ref_T, ref_last):
        e = np.max(np.abs(rgb - ref_rgb), axis=0)
        if T is not None:
            e = np.maximum(e, np.abs(np.asarray(T, dtype=np.float64) - ref_T))
        if last is not None:
            e = np.where(np.asarray(last).view(np.uint32) == ref_last, e, np.inf)
        return e

    e0 = err(o["rgb"], o["T"], o["last"])
    e1 = err(o["rgb_alt"], o["T_alt"], o["last_alt"])
    cls = o["amb"]
    e = np.where(cls == 0, e0, np.minimum(e0, e1))
    if "bound" in o:
        e = e - np.maximum(o["bound"] - tol, 0.0)
    compared = cls <= 1
    took_alt = int(((cls == 1) & (e1 < e0) & (e1 <= tol)).sum())
    return float(np.max(e[compared], initial=0.0)), compared, took_alt


def render_brute(proj, cam: dict, bg=(0.0, 0.0, 0.0)) -> dict:
    proj = _f64(proj)
    N = proj.shape[1]
    W, H = cam["width"], cam["height"]
    rgb = np.zeros((3, H, W))
    T = np.zeros((H, W))
    nc = np.zeros((H, W), dtype=np.uint32)
    bgv = np.asarray(bg, dtype=np.float64)
    lib().oracle_render_brute(_p(proj), N, W, H, _p(bgv), _p(rgb), _p(T), _p(nc))
    return {"rgb": rgb, "T": T, "ncontrib": nc}


def render_bwd(proj, cam: dict, ids, ranges_view, dL_drgb, bg=(0.0, 0.0, 0.0)) -> np.ndarray:
    """d/d(u, v, conic a, b, c, opacity, r, g, b) per Gaussian of one view: [9][N]."""
    proj = _f64(proj)
    N = proj.shape[1]
    W, H = cam["width"], cam["height"]
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    ranges_view = np.ascontiguousarray(ranges_view, dtype=np.uint32)
    g = _f64(dL_drgb).reshape(3, H, W)
    out = np.zeros((9, N))
    bgv = np.asarray(bg, dtype=np.float64)
    rc = lib().oracle_render_bwd(_p(proj), N, W, H, _p(ids) if ids.size else None, _p(ranges_view),
                                 _p(bgv), _p(g), _p(out))
    assert rc == 0
    return out


def project_bwd(P, cam: dict, dproj) -> np.ndarray:
    P = _f64(P)
    N = P.shape[1]
    dproj = _f64(dproj)
    grad = np.zeros((59, N))
    lib().oracle_project_bwd(_p(P), N, _p(pack_camera(cam)), _p(dproj), _p(grad))
    return grad


def adam(p, g, m, v, lr6, beta1: float, beta2: float, eps: float, batch: int, t: int) -> None:
    """In-place Adam step on [59][N] float64 arrays with the batch scaling rules."""
    for a in (p, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    N = p.shape[1]
    lr = np.asarray(lr6, dtype=np.float64)
    lib().oracle_adam(_p(p), _p(g), _p(m), _p(v), N, _p(lr), beta1, beta2, eps, batch, t)


def l1_loss(images: list, targets: list):
    """Mean absolute error over the 3HW values of each view, averaged over the
    views of the batch (the batch gradient is the mean of per-view gradients);
    returns (loss, [dL/dimage per view]) with sign(0) = 0."""
    V = len(images)
    loss, grads = 0.0, []
    for im, tg in zip(images, targets):
        d = _f64(im) - _f64(tg)
        loss += np.abs(d).mean() / V
        grads.append(np.sign(d) / (d.size * V))
    return loss, grads


# ----------------------------------------------------------------------------- L1 + D-SSIM loss
# The loss step of the paper's background section (step 3: L1 and SSIM over
# pixel windows). Readings: SSIM per colour channel with an 11x11 Gaussian
# window of standard deviation 1.5 (normalised), zero padding outside the
# image, C1 = 0.01^2, C2 = 0.03^2, averaged over the 3HW values of a view
# (window and constants as SSIM's definition: Wang, Bovik, Sheikh,
# Simoncelli, IEEE Trans. Image Processing 13(4), 2004); loss of a view =
# (1 - lam) L1 + lam (1 - SSIM), lam = 0.2 (the weight of Kerbl et al., ACM
# Trans. Graphics 42(4), 2023); batch loss = mean over the views.
SSIM_WIN, SSIM_SIGMA, SSIM_C1, SSIM_C2 = 11, 1.5, 0.01 ** 2, 0.03 ** 2


def ssim_window_1d() -> np.ndarray:
    k = np.arange(SSIM_WIN, dtype=np.float64) - SSIM_WIN // 2
    g = np.exp(-k * k / (2.0 * SSIM_SIGMA ** 2))
    return g / g.sum()


def _filter(img: np.ndarray) -> np.ndarray:
    """Window-weighted sum around every pixel of an [H, W] image, zero
    outside: out[y, x] = sum_ij g[i] g[j] img[y + i - 5, x + j - 5] (the
    2-D window is the outer product, so rows then columns)."""
    g, r = ssim_window_1d(), SSIM_WIN // 2
    H, W = img.shape
    pad = np.zeros((H + 2 * r, W + 2 * r))
    pad[r:r + H, r:r + W] = img
    rows = sum(g[j] * pad[:, j:j + W] for j in range(SSIM_WIN))      # [H + 2r, W]
    return sum(g[i] * rows[i:i + H, :] for i in range(SSIM_WIN))     # [H, W]


def ssim_map(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Per-pixel SSIM of two [H, W] images."""
    mx, my = _filter(x), _filter(y)
    sxx = _filter(x * x) - mx * mx
    syy = _filter(y * y) - my * my
    sxy = _filter(x * y) - mx * my
    return ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))


def ssim_grad(x: np.ndarray, y: np.ndarray, dS: np.ndarray) -> np.ndarray:
    """Gradient with respect to x of sum_p dS[p] SSIM[p]. SSIM depends on x
    through the filtered mean m = G x, the filtered square e = G x^2 and the
    filtered product f = G (x y) (with var = e - m^2, cov = f - m my); the
    filter is symmetric with zero padding, so its adjoint is itself and
    d/dx = G(dS dS/dm) + 2 x G(dS dS/de) + y G(dS dS/df)."""
    mx, my = _filter(x), _filter(y)
    sxx = _filter(x * x) - mx * mx
    syy = _filter(y * y) - my * my
    sxy = _filter(x * y) - mx * my
    A = 2 * mx * my + SSIM_C1
    B = 2 * sxy + SSIM_C2
    Cm = mx * mx + my * my + SSIM_C1
    D = sxx + syy + SSIM_C2
    S = A * B / (Cm * D)
    dS_dmx = 2 * my * B / (Cm * D) - S * 2 * mx / Cm      # through the means' terms only
    dS_dvar = -S / D
    dS_dcov = 2 * A / (Cm * D)
    d_m = dS * (dS_dmx + dS_dvar * (-2 * mx) + dS_dcov * (-my))
    d_e = dS * dS_dvar
    d_f = dS * dS_dcov
    return _filter(d_m) + 2 * x * _filter(d_e) + y * _filter(d_f)


def l1_dssim_loss(images: list, targets: list, lam: float = 0.2, with_grad: bool = True):
    """Batch loss mean_v [(1 - lam) mean|x - y| + lam (1 - mean SSIM)] over
    the views' [3, H, W] images, and dL/dimage per view (sign(0) = 0; None
    per view when with_grad is false)."""
    V = len(images)
    loss, grads = 0.0, []
    for im, tg in zip(images, targets):
        x, y = _f64(im), _f64(tg)
        n = x.size
        d = x - y
        S = np.stack([ssim_map(x[c], y[c]) for c in range(x.shape[0])])
        loss += ((1 - lam) * np.abs(d).mean() + lam * (1 - S.mean())) / V
        if not with_grad:
            grads.append(None)
            continue
        w = -lam / (n * V)                                 # dL/dSSIM[p] for every pixel and channel
        g = np.stack([ssim_grad(x[c], y[c], np.full(x.shape[1:], w)) for c in range(x.shape[0])])
        grads.append((1 - lam) * np.sign(d) / (n * V) + g)
    return loss, grads


# ----------------------------------------------------------------------------- densification
# Adaptive densification (the training process of section 2.1 and appendix
# A.1): Gaussians whose projected position gradient is large are cloned
# (small ones) or split (large ones, by a scale threshold); Gaussians of low
# opacity (or too large) are pruned; opacities are reset periodically. The
# paper names these steps and their hyperparameters, not their arithmetic;
# the readings follow the procedure of the 3D Gaussian splatting paper this
# one builds on (Kerbl et al., ACM Trans. Graphics 42(4), 2023):
#  - statistic: per (view, Gaussian) visible record, the norm of the loss
#    gradient w.r.t. the projected centre (u, v) in pixels, times `scale` (the
#    batch size, so it is the gradient of that view's own loss), summed per
#    Gaussian with a count of the visible records;
#  - selected: count > 0 and sum >= threshold * count (in FP64);
#  - split if selected and max log-scale > split_log_scale, else clone;
#  - pruned: opacity logit < prune_logit or max log-scale > prune_log_scale
#    (decided in the logit / log domain, exact on FP32 inputs);
#  - split children k = 0, 1: mean + R(q) (exp(log-scale) * noise[k]),
#    log-scale - log(1.6), every other parameter copied; a child is pruned by
#    the same rule (its max log-scale is the parent's minus log(1.6), decided
#    as parent's > prune_log_scale + log(1.6)); the split parent is removed;
#  - a clone is an exact copy; a pruned parent's clone is pruned too;
#  - output order: kept originals, clones, first children, second children,
#    each in index order; Adam moments are copied for kept originals and zero
#    for new Gaussians.
SPLIT_SHRINK = 1.6


def densify_stats(du, dv, visible, scale: float = 1.0):
    """du, dv, visible: [V][N]. Returns (sum [N] of scale * |(du, dv)| over
    visible records, count [N] of visible records)."""
    du, dv = _f64(du), _f64(dv)
    vis = np.asarray(visible, dtype=bool)
    norms = scale * np.sqrt(du * du + dv * dv)
    return np.where(vis, norms, 0.0).sum(axis=0), vis.sum(axis=0).astype(np.int64)


def quat_rotation(q: np.ndarray) -> np.ndarray:
    """Rotation matrices [N][3][3] of quaternions [4][N] = (w, x, y, z),
    normalised first."""
    q = _f64(q) / np.linalg.norm(_f64(q), axis=0)
    w, x, y, z = q
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def densify_classes(P, accum, denom, grad_thr, split_log_scale, prune_logit, prune_log_scale):
    """Boolean masks (kept original, kept clone, kept child 0 = child 1,
    split) per Gaussian, decided as described above."""
    P = _f64(P)
    accum, denom = _f64(accum), np.asarray(denom)
    maxls = P[3:6].max(axis=0)
    selected = (denom > 0) & (accum >= grad_thr * denom.astype(np.float64))
    big = maxls > split_log_scale
    pruned = (P[10] < prune_logit) | (maxls > prune_log_scale)
    child_pruned = (P[10] < prune_logit) | (maxls > prune_log_scale + np.log(SPLIT_SHRINK))
    split = selected & big
    return ~split & ~pruned, selected & ~big & ~pruned, split & ~child_pruned, split


def densify(P, m, v, accum, denom, noise, grad_thr, split_log_scale, prune_logit, prune_log_scale):
    """One densification: returns (P', m', v') [59][N'] in the output order
    above. noise: [2][3][N] standard normal draws (inputs, so that any
    implementation can be checked against this one)."""
    P, m, v = _f64(P), _f64(m), _f64(v)
    keep, clone, child, _ = densify_classes(P, accum, denom, grad_thr, split_log_scale, prune_logit,
                                            prune_log_scale)
    R = quat_rotation(P[6:10])
    s = np.exp(P[3:6])
    parts = [P[:, keep], P[:, clone]]
    for k in range(2):
        c = P.copy()
        c[0:3] = P[0:3] + np.einsum("nij,jn->in", R, s * _f64(noise[k]))
        c[3:6] = P[3:6] - np.log(SPLIT_SHRINK)
        parts.append(c[:, child])
    n_new = int(clone.sum() + 2 * child.sum())
    z = np.zeros((59, n_new))
    return (np.concatenate(parts, axis=1), np.concatenate([m[:, keep], z], axis=1),
            np.concatenate([v[:, keep], z], axis=1))


def reset_opacity(P, m, v, max_opacity: float = 0.01) -> None:
    """In place: opacity = min(opacity, max_opacity), as logits; the opacity
    row's Adam moments are zeroed."""
    cap = np.log(max_opacity / (1.0 - max_opacity))
    P[10] = np.minimum(P[10], cap)
    m[10] = 0.0
    v[10] = 0.0


# ----------------------------------------------------------------------------- pipelines
def rounded_for_binning(proj: np.ndarray):
    """FP32 copies of (u, v, radius, depth): binning decides in FP32."""
    return (proj[F_U].astype(np.float32), proj[F_V].astype(np.float32),
            proj[F_RADIUS].astype(np.float32), proj[F_DEPTH].astype(np.float32))


def forward(P, cams: list, bg=(0.0, 0.0, 0.0), fragile_tol: float = 0.0, pos_rel: float = 0.0,
            t_tol: float = 1e-5) -> dict:
    """Whole forward for a batch of views from the oracle's own projection.
    For comparison with another implementation's own projection, fragile_tol
    flags radii within that relative distance of an integer, pos_rel the
    centre's possible offset as a fraction of the image size, t_tol the
    transmittance threshold margin (flags only; the arithmetic is the same)."""
    projs = [project(P, c) for c in cams]
    parts = [rounded_for_binning(pr) for pr in projs]
    u, v, r, d = (np.stack([p[j] for p in parts]) for j in range(4))
    keys, ids, ranges = bin_sort(u, v, r, d, cams)
    base = tile_base(cams)
    views = []
    for vi, (pr, c) in enumerate(zip(projs, cams)):
        fragile = None
        if fragile_tol > 0.0:
            re = pr[F_REXACT]
            fragile = (np.abs(re - np.round(re)) <= fragile_tol * np.maximum(re, 1.0)).astype(np.uint8)
        views.append(render(pr, c, ids, ranges[base[vi]:base[vi + 1]], bg, fragile, depth_check=fragile_tol > 0.0,
                            pos_tol=pos_rel * max(c["width"], c["height"]), t_tol=t_tol))
    return {"proj": projs, "keys": keys, "ids": ids, "ranges": ranges, "views": views, "tile_base": base}


def backward(P, cams: list, fwd: dict, dL_drgb: list, bg=(0.0, 0.0, 0.0)):
    """Gradient of the loss w.r.t. the [59][N] parameters, summed over views;
    also returns the per-view [9][N] projected-space gradients."""
    P64 = _f64(P)
    grad = np.zeros_like(P64)
    dprojs = []
    base = fwd["tile_base"]
    for vi, c in enumerate(cams):
        dp = render_bwd(fwd["proj"][vi], c, fwd["ids"], fwd["ranges"][base[vi]:base[vi + 1]], dL_drgb[vi], bg)
        dprojs.append(dp)
        grad += project_bwd(P64, c, dp)
    return grad, dprojs
