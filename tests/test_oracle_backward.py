"""Pins of the oracle's hand-written backward (render and transformation) and
of its Adam with the batch scaling rules (paper, section "Scaling
Hyperparameters for Batched Training", eqs. "lambda" and "beta"):
torch FP64 autograd of an independent dense formulation, central finite
differences on branch-stable coordinates, a single-Gaussian closed form, and
torch.optim.Adam."""
import math

import numpy as np
import pytest
import torch

import oracle
from synthetic import scenes
from tests import dense_reference as dense


@pytest.fixture(scope="module")
def scene():
    w = scenes.diff_check_small(dtype=torch.float64)
    return w


def test_dense_forward_agrees_with_oracle(scene):
    cam = scene.cameras[0]
    f = oracle.forward(scene.params, [cam], (0.1, 0.2, 0.3))
    pr = dense.project(scene.params, cam)
    img, T = dense.render(pr, cam, (0.1, 0.2, 0.3))
    np.testing.assert_allclose(img.numpy(), f["views"][0]["rgb"], atol=1e-12)
    np.testing.assert_allclose(T.numpy(), f["views"][0]["T"], atol=1e-12)


def test_backward_matches_torch_autograd_of_dense_formulation(scene):
    cam = scene.cameras[0]
    bg = (0.1, 0.2, 0.3)
    P = scene.params.clone().requires_grad_(True)
    pr = dense.project(P, cam)
    img, _ = dense.render(pr, cam, bg)
    G = torch.from_numpy(np.random.default_rng(7).normal(size=img.shape))
    (img * G).sum().backward()
    f = oracle.forward(scene.params, [cam], bg)
    grad, _ = oracle.backward(scene.params, [cam], f, [G.numpy()], bg)
    ref = P.grad.numpy()
    groups = {"mean": slice(0, 3), "scale": slice(3, 6), "quat": slice(6, 10), "opacity": slice(10, 11),
              "sh": slice(11, 59)}
    for name, sl in groups.items():
        err = np.linalg.norm(grad[sl] - ref[sl]) / max(np.linalg.norm(ref[sl]), 1e-300)
        assert err < 1e-9, (name, err)


def _loss(P, cam, G, bg):
    f = oracle.forward(P, [cam], bg)
    v = f["views"][0]
    sig = (f["ids"].tobytes(), f["ranges"].tobytes(), v["last"].tobytes(), v["ncontrib"].tobytes(),
           f["proj"][0][oracle.F_RADIUS].tobytes())
    return float((v["rgb"] * G).sum()), sig


def test_backward_matches_central_finite_differences(scene):
    """Central differences with h = 1e-6 in FP64 on 120 coordinates; a
    coordinate counts only if every discrete decision (instance list, radius,
    last contributor and number blended per pixel) is the same at +h and -h."""
    cam = scene.cameras[0]
    bg = (0.0, 0.0, 0.0)
    P = scene.params.numpy().copy()
    G = np.random.default_rng(8).normal(size=(3, cam["height"], cam["width"]))
    f = oracle.forward(P, [cam], bg)
    grad, _ = oracle.backward(P, [cam], f, [G], bg)
    rng = np.random.default_rng(9)
    vis = np.nonzero(f["proj"][0][oracle.F_RADIUS] > 0)[0]
    checked = skipped = 0
    h = 1e-6
    for _ in range(120):
        i = int(rng.choice(vis))
        row = int(rng.integers(0, 59))
        Pp, Pm = P.copy(), P.copy()
        Pp[row, i] += h
        Pm[row, i] -= h
        lp, sp = _loss(Pp, cam, G, bg)
        lm, sm = _loss(Pm, cam, G, bg)
        if sp != sm:
            skipped += 1
            continue
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[row, i]) <= 1e-6 * max(1.0, abs(fd)), (row, i, fd, grad[row, i])
        checked += 1
    assert checked >= 100 and skipped <= 20


def guard_band_scene():
    """24 large Gaussians (log-scale -1) whose centres lie outside the guard
    band of a 64x64 view (|x/z| or |y/z| between 1.32 and 1.6 times
    tan(half field of view), so the Jacobian point is clamped) yet whose
    footprints reach into the image, and 16 inside it."""
    cam = scenes.orbit_camera(64, 64, 4.0, 0.4, 0.3)
    R, t = np.asarray(cam["R"]), np.asarray(cam["t"])
    tx, ty = 0.5 * cam["width"] / cam["fx"], 0.5 * cam["height"] / cam["fy"]
    rng = np.random.default_rng(31)
    P = scenes.uniform_cube_gaussians(40, 32, torch.float64).numpy()
    for i in range(40):
        z = rng.uniform(3.0, 4.5)
        if i < 24:
            far = rng.uniform(1.32, 1.6) * rng.choice([-1.0, 1.0])
            near = rng.uniform(-0.9, 0.9)
            xr, yr = (far * tx, near * ty) if i % 3 else (near * tx, far * ty)
            if i % 8 == 0:
                yr = rng.uniform(1.32, 1.5) * rng.choice([-1.0, 1.0]) * ty   # both axes clamped
            P[3:6, i] = rng.normal(-1.0, 0.1, 3)
        else:
            xr, yr = rng.uniform(-0.9, 0.9) * tx, rng.uniform(-0.9, 0.9) * ty
            P[3:6, i] = rng.normal(-2.5, 0.3, 3)
        P[0:3, i] = R.T @ (np.array([xr * z, yr * z, z]) - t)
    return P, cam, (1.3 * tx, 1.3 * ty)


def test_guard_band_scene_really_clamps():
    P, cam, (limx, limy) = guard_band_scene()
    R, t = np.asarray(cam["R"]), np.asarray(cam["t"])
    y = (R @ P[0:3]).T + t
    out = (np.abs(y[:, 0] / y[:, 2]) > limx) | (np.abs(y[:, 1] / y[:, 2]) > limy)
    f = oracle.forward(P, [cam], (0.1, 0.2, 0.3))
    shown = f["proj"][0][oracle.F_RADIUS] > 0
    tiles = oracle.tiles_touched(*(a[None] for a in oracle.rounded_for_binning(f["proj"][0])[:3]), [cam])[0]
    assert (out & (tiles > 0)).sum() >= 16 and (f["views"][0]["ncontrib"] > 0).mean() > 0.3
    assert shown.all()


def test_guard_band_gradient_matches_dense_autograd():
    """torch autograd of the dense formulation, whose torch.clamp passes no
    gradient through a clamped coordinate, on a scene where 24 Gaussians are
    clamped: 1e-9 per parameter group."""
    Pn, cam, _ = guard_band_scene()
    bg = (0.1, 0.2, 0.3)
    P = torch.from_numpy(Pn).clone().requires_grad_(True)
    pr = dense.project(P, cam)
    img, _ = dense.render(pr, cam, bg)
    G = torch.from_numpy(np.random.default_rng(33).normal(size=img.shape))
    (img * G).sum().backward()
    f = oracle.forward(Pn, [cam], bg)
    np.testing.assert_allclose(img.detach().numpy(), f["views"][0]["rgb"], atol=1e-12)
    grad, _ = oracle.backward(Pn, [cam], f, [G.numpy()], bg)
    ref = P.grad.numpy()
    for name, sl in {"mean": slice(0, 3), "scale": slice(3, 6), "quat": slice(6, 10), "opacity": slice(10, 11),
                     "sh": slice(11, 59)}.items():
        err = np.linalg.norm(grad[sl] - ref[sl]) / max(np.linalg.norm(ref[sl]), 1e-300)
        assert err < 1e-9, (name, err)


def test_guard_band_gradient_matches_central_differences():
    """Central differences (h = 1e-6, FP64, branch-stable coordinates) of
    the clamped Gaussians' positions: the clamped coordinate stays at the
    band's edge under the perturbation, so a gradient through it would show."""
    P, cam, (limx, limy) = guard_band_scene()
    bg = (0.0, 0.0, 0.0)
    G = np.random.default_rng(34).normal(size=(3, cam["height"], cam["width"]))
    f = oracle.forward(P, [cam], bg)
    grad, _ = oracle.backward(P, [cam], f, [G], bg)
    R, t = np.asarray(cam["R"]), np.asarray(cam["t"])
    y = (R @ P[0:3]).T + t
    out = np.nonzero((np.abs(y[:, 0] / y[:, 2]) > limx) | (np.abs(y[:, 1] / y[:, 2]) > limy))[0]
    h = 1e-6
    checked = 0
    for i in out:
        for row in (0, 1, 2, 3, 6):
            Pp, Pm = P.copy(), P.copy()
            Pp[row, i] += h
            Pm[row, i] -= h
            lp, sp = _loss(Pp, cam, G, bg)
            lm, sm = _loss(Pm, cam, G, bg)
            if sp != sm:
                continue
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grad[row, i]) <= 1e-6 * max(1.0, abs(fd)), (row, i, fd, grad[row, i])
            checked += abs(fd) > 1e-6
    assert checked >= 40


def test_single_gaussian_opacity_gradient_closed_form():
    """C = alpha c + (1 - alpha) bg with alpha = o G: dC/do = G (c - bg)."""
    W = H = 24
    pr = np.zeros((oracle.ONF, 1))
    pr[[oracle.F_U, oracle.F_V, oracle.F_DEPTH], 0] = [11.2, 12.7, 1.0]
    pr[[oracle.F_A, oracle.F_B, oracle.F_C], 0] = [0.1, 0.0, 0.1]
    pr[oracle.F_OPAC, 0] = 0.6
    pr[[oracle.F_R, oracle.F_G, oracle.F_BL], 0] = [0.9, 0.4, 0.1]
    pr[oracle.F_RADIUS, 0] = pr[oracle.F_REXACT, 0] = 10
    cam = {"width": W, "height": H}
    bg = (0.2, 0.3, 0.4)
    u, v, r, d = oracle.rounded_for_binning(pr)
    _, ids, ranges = oracle.bin_sort(u[None], v[None], r[None], d[None], [cam])
    g = np.zeros((3, H, W))
    g[1, 12, 11] = 1.0                                   # dL/dC_green at one pixel
    dp = oracle.render_bwd(pr, cam, ids, ranges, g, bg)
    dx, dy = 11.5 - 11.2, 12.5 - 12.7
    G = math.exp(-0.05 * (dx * dx + dy * dy))
    assert dp[5, 0] == pytest.approx(G * (0.4 - 0.3), rel=1e-12)
    assert dp[7, 0] == pytest.approx(0.6 * G, rel=1e-12)  # dC/dc = alpha


def test_batched_gradient_is_sum_over_views():
    """The batch gradient of the per-view-mean L1 is the mean of the per-view
    gradients (paper, derivation under the Independent Gradients Hypothesis,
    g = sum_k g_k / b)."""
    w = scenes.diff_check_small(dtype=torch.float64)
    cams = [scenes.orbit_camera(48, 40, 4.0, a, 0.3) for a in (0.0, 1.0, 2.5)]
    targets = [np.random.default_rng(k).uniform(size=(3, 40, 48)) for k in range(3)]
    f = oracle.forward(w.params, cams)
    loss, g = oracle.l1_loss([v["rgb"] for v in f["views"]], targets)
    grad, _ = oracle.backward(w.params, cams, f, g)
    acc = np.zeros_like(grad)
    for k, c in enumerate(cams):
        fk = oracle.forward(w.params, [c])
        lk, gk = oracle.l1_loss([fk["views"][0]["rgb"]], [targets[k]])
        gr, _ = oracle.backward(w.params, [c], fk, gk)
        acc += gr / 3.0
    np.testing.assert_allclose(grad, acc, rtol=1e-12, atol=1e-18)


# --------------------------------------------------------------------------- Adam
def test_scaling_rule_closed_forms():
    """At batch 16 the rules give lr x 4, beta1 0.9 -> 0.185302018885184 and
    beta2 0.999 -> 0.984119441815640 (eqs. "lambda", "beta"). One oracle step
    from zero moments shows them: m = (1 - beta1') g, v = (1 - beta2') g^2 and,
    after bias correction, every parameter moves by lr * 4 against sign(g)."""
    rng = np.random.default_rng(0)
    N = 5
    g = rng.normal(size=(59, N))
    p = np.zeros((59, N))
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    lr6 = [1e-3] * 6
    oracle.adam(p, g, m, v, lr6, 0.9, 0.999, 0.0, 16, 1)
    np.testing.assert_allclose(m, (1 - 0.185302018885184) * g, rtol=1e-13)
    np.testing.assert_allclose(v, (1 - 0.984119441815640) * g * g, rtol=1e-11)
    np.testing.assert_allclose(p, -4e-3 * np.sign(g), rtol=1e-11)


@pytest.mark.parametrize("batch", [1, 4, 16])
def test_adam_matches_torch_optim_adam(batch):
    rng = np.random.default_rng(batch)
    N = 37
    lr6 = [1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3, 2.5e-3 / 20]
    beta1, beta2, eps = 0.9, 0.999, 1e-15
    p = rng.normal(size=(59, N))
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    tp = torch.tensor(p.copy(), requires_grad=True)
    rows = [slice(0, 3), slice(3, 6), slice(6, 10), slice(10, 11), slice(11, 14), slice(14, 59)]
    views = [tp[s] for s in rows]
    params = [torch.nn.Parameter(x.detach().clone()) for x in views]
    opt = torch.optim.Adam([{"params": [pp], "lr": lr * math.sqrt(batch)} for pp, lr in zip(params, lr6)],
                           betas=(beta1 ** batch, beta2 ** batch), eps=eps)
    for t in range(1, 6):
        g = rng.normal(size=(59, N))
        g[:, 3] = 0.0                                   # a Gaussian with no gradient still moves by momentum
        oracle.adam(p, g, m, v, lr6, beta1, beta2, eps, batch, t)
        for pp, s in zip(params, rows):
            pp.grad = torch.tensor(g[s])
        opt.step()
    ref = torch.cat([pp.detach() for pp in params]).numpy()
    np.testing.assert_allclose(p, ref, rtol=1e-12, atol=1e-15)
