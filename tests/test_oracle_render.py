"""Pins of the oracle's binning and composition (paper, section "Background on
3D Gaussian Training", step 2; 16x16 blocks of section "Pixel-wise
Distribution"): closed forms for one, two and stacked Gaussians, invariants,
brute force without tiles, and library sorts for the instance order."""
import math

import numpy as np
import pytest
import torch

import oracle
from synthetic import scenes


def _proj(entries, N=None):
    """Hand-made projected fields: entries = list of dicts with u, v, depth,
    conic (a, b, c), opacity, rgb, radius."""
    N = len(entries) if N is None else N
    pr = np.zeros((oracle.ONF, N))
    for i, e in enumerate(entries):
        pr[oracle.F_U, i], pr[oracle.F_V, i] = e["u"], e["v"]
        pr[oracle.F_DEPTH, i] = e.get("depth", 1.0 + i)
        pr[[oracle.F_A, oracle.F_B, oracle.F_C], i] = e["conic"]
        pr[oracle.F_OPAC, i] = e["o"]
        pr[[oracle.F_R, oracle.F_G, oracle.F_BL], i] = e["rgb"]
        pr[oracle.F_RADIUS, i] = e["r"]
        pr[oracle.F_REXACT, i] = e["r"]
    return pr


def _render(pr, cam, bg=(0.0, 0.0, 0.0)):
    u, v, r, d = oracle.rounded_for_binning(pr)
    keys, ids, ranges = oracle.bin_sort(u[None], v[None], r[None], d[None], [cam])
    return oracle.render(pr, cam, ids, ranges, bg)


def _cam(W, H):
    return {"width": W, "height": H}


# --------------------------------------------------------------------------- closed forms
def test_single_isotropic_gaussian_closed_form():
    W, H = 40, 36
    sig2, o, col, bg = 9.0, 0.8, [0.2, 0.5, 0.9], (0.1, 0.3, 0.05)
    u, v = 17.3, 20.6
    r = math.ceil(3 * math.sqrt(sig2))
    pr = _proj([{"u": u, "v": v, "conic": (1 / sig2, 0, 1 / sig2), "o": o, "rgb": col, "r": r}])
    out = _render(pr, _cam(W, H), bg)
    ys, xs = np.mgrid[0:H, 0:W]
    d2 = (xs + 0.5 - u) ** 2 + (ys + 0.5 - v) ** 2
    alpha = np.minimum(0.99, o * np.exp(-d2 / (2 * sig2)))
    alpha = np.where((d2 <= r * r) & (alpha >= 1 / 255), alpha, 0.0)
    for ch in range(3):
        np.testing.assert_allclose(out["rgb"][ch], alpha * col[ch] + (1 - alpha) * bg[ch], atol=1e-15)
    np.testing.assert_allclose(out["T"], 1 - alpha, atol=1e-15)
    assert (out["last"] == (alpha > 0)).all()


def test_two_gaussians_front_to_back():
    W = H = 32
    g1 = {"u": 15.5, "v": 16.2, "conic": (0.05, 0.01, 0.04), "o": 0.7, "rgb": [1, 0, 0], "r": 14, "depth": 2.0}
    g2 = {"u": 17.0, "v": 14.9, "conic": (0.03, -0.005, 0.06), "o": 0.9, "rgb": [0, 0.5, 1], "r": 15, "depth": 1.5}
    bg = np.array([0.2, 0.2, 0.2])
    out = _render(_proj([g1, g2]), _cam(W, H), tuple(bg))
    ys, xs = np.mgrid[0:H, 0:W]

    def alpha(g):
        dx, dy = xs + 0.5 - g["u"], ys + 0.5 - g["v"]
        a, b, c = g["conic"]
        al = np.minimum(0.99, g["o"] * np.exp(-0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy))
        return np.where((dx * dx + dy * dy <= g["r"] ** 2) & (al >= 1 / 255), al, 0.0)
    a1, a2 = alpha(g2), alpha(g1)          # g2 is nearer: it blends first
    c1, c2 = np.array(g2["rgb"]), np.array(g1["rgb"])
    ref = a1 * c1[:, None, None] + (1 - a1) * a2 * c2[:, None, None] + (1 - a1) * (1 - a2) * bg[:, None, None]
    np.testing.assert_allclose(out["rgb"], ref, atol=1e-14)


def test_transmittance_stop_excludes_crossing_gaussian():
    """Five co-centred Gaussians with alpha 0.95 at the centre pixel: T after
    three is 1.25e-4 (kept); a fourth would give 6.25e-6 < 1e-4, so it and all
    later ones are excluded and the last contributor is the third."""
    W = H = 16
    u = v = 8.5                                  # centre pixel (8, 8) sits on the mean
    cols = [[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1], [0.5, 0.5, 0.5]]
    ents = [{"u": u, "v": v, "conic": (0.5, 0, 0.5), "o": 0.95, "rgb": cols[i], "r": 4, "depth": 1 + i} for i in range(5)]
    out = _render(_proj(ents), _cam(W, H))
    assert out["T"][8, 8] == pytest.approx(0.05 ** 3, rel=1e-12)
    assert out["last"][8, 8] == 3 and out["ncontrib"][8, 8] == 3
    np.testing.assert_allclose(out["rgb"][:, 8, 8], [0.95, 0.05 * 0.95, 0.05 * 0.05 * 0.95], rtol=1e-12)


def test_alpha_clamped_at_099_and_skip_below_1_255():
    W = H = 16
    g_hi = {"u": 8.5, "v": 8.5, "conic": (0.1, 0, 0.1), "o": 1.0, "rgb": [1, 1, 1], "r": 9, "depth": 1.0}
    out = _render(_proj([g_hi]), _cam(W, H))
    assert out["T"][8, 8] == pytest.approx(0.01, rel=1e-12)
    o_lo = 0.999 / 255.0                         # peak alpha just below 1/255
    g_lo = {"u": 8.5, "v": 8.5, "conic": (0.1, 0, 0.1), "o": o_lo, "rgb": [1, 1, 1], "r": 9, "depth": 1.0}
    out = _render(_proj([g_lo]), _cam(W, H))
    assert (out["T"] == 1.0).all() and (out["last"] == 0).all()


def test_circle_test_is_the_intersection_predicate():
    """A pixel outside the radius circle gets nothing even where alpha would be large."""
    W = H = 32
    g = {"u": 16.0, "v": 16.0, "conic": (1e-4, 0, 1e-4), "o": 0.9, "rgb": [1, 1, 1], "r": 5, "depth": 1.0}
    out = _render(_proj([g]), _cam(W, H))
    ys, xs = np.mgrid[0:H, 0:W]
    inside = (xs + 0.5 - 16) ** 2 + (ys + 0.5 - 16) ** 2 <= 25
    assert (out["T"][~inside] == 1.0).all() and (out["T"][inside] < 0.2).all()


# --------------------------------------------------------------------------- binning
def _brute_tiles(u, v, r, W, H):
    """Tiles containing at least one pixel whose centre lies in the footprint's
    bounding box [u - r, u + r] x [v - r, v + r] (decided in FP32)."""
    u, v, r = np.float32(u), np.float32(v), np.float32(r)
    if not r > 0:
        return set()
    xs = np.arange(W, dtype=np.float32)
    ys = np.arange(H, dtype=np.float32)
    okx = (xs >= (u - r) - np.float32(0.5)) & (xs <= (u + r) - np.float32(0.5))
    oky = (ys >= (v - r) - np.float32(0.5)) & (ys <= (v + r) - np.float32(0.5))
    TX = (W + 15) // 16
    return {(int(y) // 16) * TX + int(x) // 16 for x in xs[okx] for y in ys[oky]}


@pytest.mark.parametrize("seed", [0, 1])
def test_binning_matches_brute_force_and_library_sort(seed):
    rng = np.random.default_rng(seed)
    cams = [{"width": 70, "height": 45}, {"width": 33, "height": 50}]
    N = 60
    u = rng.uniform(-10, 80, (2, N)).astype(np.float32)
    v = rng.uniform(-10, 60, (2, N)).astype(np.float32)
    r = np.where(rng.uniform(size=(2, N)) < 0.1, 0, rng.integers(1, 20, (2, N))).astype(np.float32)
    d = rng.uniform(0.5, 3, (2, N)).astype(np.float32)
    d[0, 5] = d[0, 6]                               # a depth tie: order by Gaussian index
    keys, ids, ranges = oracle.bin_sort(u, v, r, d, cams)
    base = oracle.tile_base(cams)
    # brute-force instance set, ordered by numpy's lexsort on (tile, depth bits, id)
    tiles, dbits, gids = [], [], []
    for vi, c in enumerate(cams):
        for i in range(N):
            for t in _brute_tiles(u[vi, i], v[vi, i], r[vi, i], c["width"], c["height"]):
                tiles.append(base[vi] + t)
                dbits.append(int(d[vi, i].view(np.uint32)))
                gids.append(i)
    tiles, dbits, gids = map(np.array, (tiles, dbits, gids))
    order = np.lexsort((gids, dbits, tiles))
    np.testing.assert_array_equal(ids, gids[order].astype(np.uint32))
    np.testing.assert_array_equal(keys, (tiles[order].astype(np.uint64) << np.uint64(32)) | dbits[order].astype(np.uint64))
    # ranges: [start, end) per tile from a library search over the sorted tiles
    st = tiles[order]
    for t in range(base[-1]):
        s, e = np.searchsorted(st, t, "left"), np.searchsorted(st, t, "right")
        exp = (s, e) if e > s else (0, 0)
        assert tuple(ranges[t]) == exp
    # torch's stable sort over (tile << 32 | depth bits) keeps emission (id) order on ties
    emit_keys = torch.tensor(((tiles.astype(np.int64) << 32) | dbits).tolist())
    perm = torch.sort(emit_keys, stable=True).indices.numpy()
    np.testing.assert_array_equal(ids, gids[perm].astype(np.uint32))


# --------------------------------------------------------------------------- invariants and brute force
@pytest.fixture(scope="module")
def small_scene():
    w = scenes.diff_check_small(dtype=torch.float64)
    return w


@pytest.mark.parametrize("which", ["single_view_256", "diff_check_64"])
def test_tiled_equals_brute_force(which):
    w = scenes.plain_single_view(torch.float64) if which == "single_view_256" else scenes.diff_check_small()
    cam = w.cameras[0]
    if which == "single_view_256":
        cam = dict(cam, width=96, height=80, cx=48.0, cy=40.0)   # keep brute force quick
    bg = (0.3, 0.1, 0.6)
    f = oracle.forward(w.params, [cam], bg)
    b = oracle.render_brute(f["proj"][0], cam, bg)
    v = f["views"][0]
    assert (v["rgb"] == b["rgb"]).all() and (v["T"] == b["T"]).all() and (v["ncontrib"] == b["ncontrib"]).all()
    assert v["blended"] > 100


def test_render_invariants(small_scene):
    w = small_scene
    cam = w.cameras[0]
    P = w.params.clone()
    P[11:14] = torch.rand(3, P.shape[1], dtype=torch.float64, generator=torch.Generator().manual_seed(3)) * 3
    # white Gaussians on black: weights + T = 1 gives C = 1 - T per channel
    Pw = P.clone()
    Pw[11:14] = (1.0 - 0.5) / (1.0 / (2.0 * math.sqrt(math.pi)))
    Pw[14:59] = 0.0
    v = oracle.forward(Pw, [cam])["views"][0]
    np.testing.assert_allclose(v["rgb"], np.broadcast_to(1.0 - v["T"], v["rgb"].shape), atol=1e-13)
    # colour within the hull of contributing colours and the background
    bg = (0.25, 0.5, 0.75)
    f = oracle.forward(P, [cam], bg)
    v = f["views"][0]
    rgb = f["proj"][0][[oracle.F_R, oracle.F_G, oracle.F_BL]]
    for ch in range(3):
        lo = min(rgb[ch][f["proj"][0][oracle.F_RADIUS] > 0].min(), bg[ch])
        hi = max(rgb[ch].max(), bg[ch])
        assert v["rgb"][ch].min() >= lo - 1e-12 and v["rgb"][ch].max() <= hi + 1e-12
    # T within (1e-4, 1] and non-increasing as the list is extended
    assert (v["T"] >= 1e-4).all() and (v["T"] <= 1).all()


def test_transmittance_monotone_along_the_list(small_scene):
    """Rendering with only the first k entries of every tile list gives a
    transmittance that is non-increasing in k."""
    w = small_scene
    cam = w.cameras[0]
    f = oracle.forward(w.params, [cam])
    ranges = f["ranges"].copy()
    prev = np.ones((cam["height"], cam["width"]))
    for k in range(0, 40, 3):
        rr = ranges.copy()
        rr[:, 1] = np.minimum(rr[:, 1], rr[:, 0] + k)
        T = oracle.render(f["proj"][0], cam, f["ids"], rr)["T"]
        assert (T <= prev + 1e-15).all()
        prev = T


def test_behind_near_plane_contributes_nothing(small_scene):
    w = small_scene
    cam = w.cameras[0]
    P = w.params.clone()
    base = oracle.forward(P, [cam])["views"][0]
    # add Gaussians between the camera (at x = 4) and the near plane, and behind it
    extra = P[:, :3].clone()
    extra[0, 0], extra[0, 1], extra[0, 2] = 3.85, 4.5, 10.0
    extra[1:3, :] = 0.0
    extra[3:6, :] = 0.0                              # big: scale 1
    P2 = torch.cat([P, extra], dim=1)
    f2 = oracle.forward(P2, [cam])
    v2 = f2["views"][0]
    assert (f2["proj"][0][oracle.F_RADIUS, -3:] == 0).all()
    assert (v2["rgb"] == base["rgb"]).all() and (v2["T"] == base["T"]).all()
    g = np.random.default_rng(0).normal(size=v2["rgb"].shape)
    grad, _ = oracle.backward(P2, [cam], f2, [g])
    assert (grad[:, -3:] == 0).all()


# --------------------------------------------------------------------------- near-threshold decisions
def test_alpha_threshold_margin_scales_with_the_exponent_terms():
    """A decision on alpha >= 1/255 is near-threshold within the FP32
    evaluation's rounding, which grows with S = |qa| + |qb| + |qc| (the terms
    of the exponent before they cancel), not with the exponent itself. A thin
    footprint (conic (k, -k(1-e), k), evaluated along its long axis) with
    S ~ 3200 whose alpha is 1e-3 above the threshold in the log domain is
    flagged; the same log distance on an isotropic footprint (S = |power|
    ~ 4.8) is not."""
    o, k, d = 0.5, 100.0, 4.0
    target = math.log(1.0 / (255.0 * o)) + 1e-3            # alpha a little above 1/255
    eps = -target / (k * d * d)
    u = v = 10.5 - d                                       # pixel (10, 10) at offset (d, d)
    thin = _proj([{"u": u, "v": v, "conic": (k, -k * (1 - eps), k), "o": o, "rgb": [1, 0, 0], "r": 8}])
    S = 0.5 * k * d * d + k * (1 - eps) * d * d + 0.5 * k * d * d
    assert S > 3000
    out = _render(thin, _cam(24, 24))
    assert out["amb"][10, 10] == 1
    # its other branch: the Gaussian skipped, so the background shows
    assert out["rgb"][0, 10, 10] > 0 and out["rgb_alt"][0, 10, 10] == 0
    # isotropic: power = -(d2 / 2) sig^-2 at the same log distance
    sig2 = 2 * d * d / (2 * -target)
    iso = _proj([{"u": u, "v": v, "conic": (1 / sig2, 0, 1 / sig2), "o": o, "rgb": [1, 0, 0], "r": 8}])
    out = _render(iso, _cam(24, 24))
    assert out["amb"][10, 10] == 0 and out["rgb"][0, 10, 10] > 0


def test_error_bound_covers_an_fp32_evaluation():
    """The per-pixel "bound" must cover what FP32 arithmetic does to the same
    walk: thin footprints (conics close to singular, so the exponent's terms
    cancel) rendered in FP64 by the oracle and with every step in FP32 here,
    one Gaussian over a background; no pixel may differ by more than its
    bound (plus the rounding of the final colour sum)."""
    rng = np.random.default_rng(5)
    f32 = np.float32
    W = H = 16
    ys, xs = np.mgrid[0:H, 0:W]
    worst = 0.0
    for trial in range(60):
        k = 10.0 ** rng.uniform(-1, 2)
        eps = 10.0 ** rng.uniform(-4, -1)
        th = rng.uniform(0, np.pi)
        # eigenvalues k and k*eps along a random direction
        cth, sth = math.cos(th), math.sin(th)
        a, b, c = (f32(k * (cth * cth + eps * sth * sth)), f32(k * (1 - eps) * cth * sth),
                   f32(k * (sth * sth + eps * cth * cth)))
        u, v = f32(rng.uniform(4, 12)), f32(rng.uniform(4, 12))
        o = f32(rng.uniform(0.3, 1.0))
        col = rng.uniform(0, 1, 3).astype(np.float32)
        bg = tuple(float(x) for x in rng.uniform(0, 1, 3).astype(np.float32))
        pr = _proj([{"u": float(u), "v": float(v), "conic": (float(a), float(-b), float(c)), "o": float(o),
                     "rgb": [float(x) for x in col], "r": 12}])
        out = _render(pr, _cam(W, H), bg)
        # FP32: the exponent from its three terms, then alpha and the blend
        dx = (xs.astype(f32) + f32(0.5)) - u
        dy = (ys.astype(f32) + f32(0.5)) - v
        power = -(f32(0.5) * a * dx * dx + f32(0.5) * c * dy * dy) - f32(-b) * dx * dy
        alpha = np.minimum(o * np.exp(power, dtype=f32), f32(0.99))
        use = (dx * dx + dy * dy <= f32(144)) & (power <= 0) & (alpha >= f32(1 / 255))
        ok = out["amb"] == 0                              # near-threshold pixels: either branch
        assert (use[ok] == (out["last"][ok] > 0)).all()
        for ch in range(3):
            c32 = np.where(use, col[ch] * alpha + (f32(1) - alpha) * f32(bg[ch]), f32(bg[ch]))
            err = np.abs(c32.astype(np.float64) - out["rgb"][ch])
            assert (err[ok] <= out["bound"][ok] + 2.4e-7).all(), trial
            worst = max(worst, float((err[ok] / (out["bound"][ok] + 2.4e-7)).max()))
    assert worst > 0.05             # and is not loose by orders of magnitude (measured 0.19)


def test_exponent_positive_only_within_rounding_of_zero():
    """The render kernels leave out the exponent-sign test (skip a pair whose
    exponent is positive). With a positive definite conic the exponent they
    form in FP32 -- na (dx dx) + dy (nb dx + nc dy), (na, nb, nc) the conic
    scaled by -log2(e) (1/2, 1, 1/2), two fused multiply-adds -- is positive
    only by rounding. Thin conics (eigenvalue ratio down to 3e-8) laid along
    the pixel grid, centres near a pixel centre: wherever that FP32 value is
    positive, the exact exponent is within 1e-6 S of zero (S = |qa| + |qb| +
    |qc|), the band in which the oracle takes either branch of its own sign
    test."""
    f32 = np.float32

    def fma32(a, b, c):   # one rounding: the FP64 product of two FP32 values is exact
        return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(f32)

    l2e = f32(1.4426950408889634)
    half_l2e = f32(-0.5) * l2e
    rng = np.random.default_rng(7)
    ys, xs = np.mgrid[100:141, 100:141]
    pxc, pyc = xs.astype(f32) + f32(0.5), ys.astype(f32) + f32(0.5)
    positive, worst = 0, 0.0
    for _ in range(1500):
        k, eps = 10.0 ** rng.uniform(-2, 2), 10.0 ** rng.uniform(-7.5, -3)
        th = rng.choice([0.0, math.pi / 4, math.pi / 2, 3 * math.pi / 4]) + rng.normal(0, 1e-4)
        cth, sth = math.cos(th), math.sin(th)
        a, b, c = (f32(k * (cth * cth + eps * sth * sth)), f32(-k * (1 - eps) * cth * sth),
                   f32(k * (sth * sth + eps * cth * cth)))
        assert float(a) * float(c) - float(b) * float(b) > 0          # positive definite as stored
        u, v = f32(120.5 + rng.normal(0, 1e-3)), f32(120.5 + rng.normal(0, 1e-3))
        na, nb, nc = half_l2e * a, -l2e * b, half_l2e * c
        dx, dy = pxc - u, pyc - v
        p2 = fma32(dy, fma32(np.full_like(dy, nc), dy, nb * dx), na * (dx * dx))
        dxe, dye = dx.astype(np.float64), dy.astype(np.float64)
        qa, qb, qc = 0.5 * float(a) * dxe * dxe, float(b) * dxe * dye, 0.5 * float(c) * dye * dye
        power, S = -(qa + qb + qc), np.abs(qa) + np.abs(qb) + np.abs(qc)
        m = p2 > 0
        if m.any():
            positive += int(m.sum())
            worst = max(worst, float((np.abs(power[m]) / S[m]).max()))
    assert positive > 20                     # the FP32 form does go positive (measured: 79 pixels)
    assert worst <= 1e-6, worst              # measured 7.8e-8, about 1.3 unit roundoffs
