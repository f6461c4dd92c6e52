"""Pins of the oracle's L1 + D-SSIM loss (the loss step of the paper's
background section: L1 and SSIM over pixel windows). Each check comes from
outside the oracle's own formulas: a brute-force window sum, the closed form
for constant images, the identity SSIM(x, x) = 1 (a maximum, so a zero
gradient), central differences, and torch autograd of an independent
conv2d formulation."""
import math

import numpy as np
import pytest
import torch

import oracle


def test_window_is_a_normalised_gaussian():
    g = oracle.ssim_window_1d()
    assert g.shape == (11,) and abs(g.sum() - 1.0) < 1e-15
    assert np.allclose(g, g[::-1], rtol=0, atol=0)
    assert np.argmax(g) == 5
    assert abs(g[4] / g[5] - math.exp(-1.0 / (2 * 1.5 ** 2))) < 1e-15
    assert abs(g[0] / g[5] - math.exp(-25.0 / (2 * 1.5 ** 2))) < 1e-15


def test_filter_equals_brute_force_window_sum():
    rng = np.random.default_rng(1)
    img = rng.random((9, 7))
    g = oracle.ssim_window_1d()
    out = np.zeros_like(img)
    for y in range(9):
        for x in range(7):
            acc = 0.0
            for i in range(11):
                for j in range(11):
                    yy, xx = y + i - 5, x + j - 5
                    if 0 <= yy < 9 and 0 <= xx < 7:
                        acc += g[i] * g[j] * img[yy, xx]
            out[y, x] = acc
    assert np.max(np.abs(oracle._filter(img) - out)) < 1e-15


def test_identical_images_have_ssim_one_and_zero_gradient():
    rng = np.random.default_rng(2)
    x = rng.random((23, 19))
    assert np.max(np.abs(oracle.ssim_map(x, x) - 1.0)) < 1e-12
    g = oracle.ssim_grad(x, x, np.ones_like(x))
    assert np.max(np.abs(g)) < 1e-10


@pytest.mark.parametrize("a,b", [(0.2, 0.7), (0.5, 0.5), (0.9, 0.1), (0.0, 0.3)])
def test_constant_images_closed_form_away_from_the_border(a, b):
    x, y = np.full((30, 31), a), np.full((30, 31), b)
    S = oracle.ssim_map(x, y)
    C1 = 0.01 ** 2
    # interior: full window, means a and b, zero variances and covariance
    assert np.max(np.abs(S[5:-5, 5:-5] - (2 * a * b + C1) / (a * a + b * b + C1))) < 1e-12


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    x, y = rng.random((12, 11)), rng.random((12, 11))
    dS = rng.normal(size=x.shape)
    g = oracle.ssim_grad(x, y, dS)
    h = 1e-6
    for (r, c) in [(0, 0), (0, 10), (6, 5), (11, 3), (2, 9)]:
        xp, xm = x.copy(), x.copy()
        xp[r, c] += h
        xm[r, c] -= h
        fd = ((dS * oracle.ssim_map(xp, y)).sum() - (dS * oracle.ssim_map(xm, y)).sum()) / (2 * h)
        assert abs(fd - g[r, c]) <= 1e-6 * max(1.0, abs(fd)), (r, c, fd, g[r, c])


def _torch_l1_dssim(x, y, lam):
    """An independent formulation: 2-D Gaussian window by outer product,
    conv2d with zero padding, SSIM map from the moments, autograd for the
    gradient; x, y: [V][3, H, W] double tensors."""
    k = torch.arange(11, dtype=torch.float64) - 5
    g1 = torch.exp(-k * k / (2 * 1.5 ** 2))
    g1 = g1 / g1.sum()
    w = (g1[:, None] * g1[None, :])[None, None]
    total = 0.0
    for xi, yi in zip(x, y):
        X, Y = xi[:, None], yi[:, None]                      # channels as a batch
        f = lambda t: torch.nn.functional.conv2d(t, w, padding=5)
        mx, my = f(X), f(Y)
        vx, vy, cxy = f(X * X) - mx * mx, f(Y * Y) - my * my, f(X * Y) - mx * my
        c1, c2 = 0.01 ** 2, 0.03 ** 2
        S = ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))
        total = total + ((1 - lam) * (xi - yi).abs().mean() + lam * (1 - S.mean())) / len(x)
    return total


@pytest.mark.parametrize("lam", [0.2, 0.0, 1.0])
def test_loss_and_gradient_match_torch_autograd(lam):
    rng = np.random.default_rng(4)
    shapes = [(3, 17, 23), (3, 9, 6)]
    ims = [rng.random(s) for s in shapes]
    tgs = [rng.random(s) for s in shapes]
    loss, grads = oracle.l1_dssim_loss(ims, tgs, lam)
    xt = [torch.tensor(a, requires_grad=True) for a in ims]
    yt = [torch.tensor(a) for a in tgs]
    lt = _torch_l1_dssim(xt, yt, lam)
    lt.backward()
    assert abs(loss - lt.item()) <= 1e-12 * abs(lt.item())
    for g, t in zip(grads, xt):
        assert np.max(np.abs(g - t.grad.numpy())) <= 1e-12 * np.max(np.abs(t.grad.numpy()))


def test_lam_zero_is_the_l1_loss():
    rng = np.random.default_rng(5)
    ims = [rng.random((3, 8, 9))]
    tgs = [rng.random((3, 8, 9))]
    a, ga = oracle.l1_dssim_loss(ims, tgs, 0.0)
    b, gb = oracle.l1_loss(ims, tgs)
    assert abs(a - b) < 1e-15 and np.array_equal(ga[0], gb[0])
