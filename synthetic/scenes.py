"""Seeded synthetic scenes and cameras.

This module only draws inputs: Gaussian parameter sets, camera poses and
request streams. It holds none of the rasterizer's arithmetic, so both the
CPU oracle (``oracle/``) and the HIP path (``paper_2406_18533_amd``) can be
fed from it without sharing any code with each other.

Conventions of the inputs it produces
-------------------------------------
Gaussian parameters are one planar structure-of-arrays block ``[59][N]``
(float32, or float64 for the differentiation check), rows:

====== ===========================================================
rows   field
====== ===========================================================
0-2    mean x, y, z (world)
3-5    log-scale per axis (scale = exp)
6-9    rotation quaternion w, x, y, z (normalised inside the method)
10     opacity logit (opacity = sigmoid)
11-58  spherical-harmonic coefficients, row 11 + 3*k + c for
       coefficient k = l*l + l + m (degree 3, 16 coefficients) and
       colour channel c
====== ===========================================================

These are the four learnable quantities of a Gaussian (position, scale and
rotation, opacity, 48 SH values) of the paper's background section (3DGS
parameters paragraph).

Cameras are dictionaries ``{width, height, fx, fy, cx, cy, R (3x3 row-major
world->camera), t (3), znear}`` in the OpenCV frame (+x right, +y down, +z
forward); the camera centre is ``-R^T t``. Horizontal field of view is
60 degrees, square pixels, principal point at the image centre, and
``znear = 0.2``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

N_PARAM_ROWS = 59
ROW_MEAN = 0
ROW_LOG_SCALE = 3
ROW_QUAT = 6
ROW_OPACITY = 10
ROW_SH = 11
ZNEAR = 0.2
HFOV_DEG = 60.0


# --------------------------------------------------------------------------- cameras
def _look_at(eye, target, up):
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.asarray(up, dtype=np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])  # rows: camera axes in world coordinates
    t = -R @ eye
    return R, t


def make_camera(width: int, height: int, R, t, hfov_deg: float = HFOV_DEG, znear: float = ZNEAR) -> dict:
    fx = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    return {
        "width": int(width), "height": int(height),
        "fx": float(fx), "fy": float(fx),
        "cx": width / 2.0, "cy": height / 2.0,
        "R": np.asarray(R, dtype=np.float64).reshape(3, 3).copy(),
        "t": np.asarray(t, dtype=np.float64).reshape(3).copy(),
        "znear": float(znear),
    }


def orbit_camera(width: int, height: int, radius: float, az: float, el: float) -> dict:
    """Camera on a sphere around the origin looking at it, world up = +z."""
    eye = radius * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    R, t = _look_at(eye, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    return make_camera(width, height, R, t)


def aerial_camera(width: int, height: int, pos_xy, altitude: float, tilt: float, yaw: float) -> dict:
    """Camera at ``altitude`` above the ground patch, tilted ``tilt`` radians from
    nadir towards heading ``yaw``; the image top points along the heading."""
    h = np.array([math.cos(yaw), math.sin(yaw), 0.0])
    fwd = math.sin(tilt) * h + math.cos(tilt) * np.array([0.0, 0.0, -1.0])
    right = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    eye = np.array([pos_xy[0], pos_xy[1], altitude], dtype=np.float64)
    return make_camera(width, height, R, -R @ eye)


# --------------------------------------------------------------------------- gaussians
def _finish_params(gen, means: torch.Tensor, log_scale_mu: float, log_scale_sd: float, dtype) -> torch.Tensor:
    """Draws the non-position rows in a fixed order, in the output dtype:
    log-scales, quaternions, opacity logits, SH DC, SH rest."""
    n = means.shape[1]
    P = torch.empty(N_PARAM_ROWS, n, dtype=dtype)
    P[0:3] = means.to(dtype)
    P[3:6] = torch.randn(3, n, generator=gen, dtype=dtype).mul_(log_scale_sd).add_(log_scale_mu)
    q = torch.randn(4, n, generator=gen, dtype=dtype)
    P[6:10] = q / q.norm(dim=0, keepdim=True)
    P[10] = torch.randn(n, generator=gen, dtype=dtype)
    P[11:14] = torch.randn(3, n, generator=gen, dtype=dtype).mul_(0.2).add_(0.5)
    P[14:59] = torch.randn(45, n, generator=gen, dtype=dtype).mul_(0.05)
    return P


def uniform_cube_gaussians(n: int, seed: int, dtype=torch.float32) -> torch.Tensor:
    """Means uniform in [-1,1]^3, log-scales N(-4, 0.5), random unit
    quaternions, opacity logits N(0,1), SH DC N(0.5,0.2) and higher N(0,0.05)."""
    gen = torch.Generator().manual_seed(seed)
    means = 2.0 * torch.rand(3, n, generator=gen, dtype=torch.float64) - 1.0
    return _finish_params(gen, means, -4.0, 0.5, dtype)


def gmm_means(n: int, gen, n_comp: int = 64, box: float = 5.0) -> torch.Tensor:
    """Means from a mixture of isotropic Gaussians (component means uniform in
    [-box, box]^3, std U[0.2, 1.0], Dirichlet(1) weights); samples outside the
    box are redrawn from their component."""
    centres = (2.0 * torch.rand(n_comp, 3, generator=gen, dtype=torch.float64) - 1.0) * box
    stds = 0.2 + 0.8 * torch.rand(n_comp, generator=gen, dtype=torch.float64)
    w = -torch.log(torch.rand(n_comp, generator=gen, dtype=torch.float64))  # Dirichlet(1) via exponentials
    w = w / w.sum()
    comp = torch.multinomial(w, n, replacement=True, generator=gen)
    out = centres[comp] + stds[comp, None] * torch.randn(n, 3, generator=gen, dtype=torch.float64)
    bad = (out.abs() > box).any(dim=1)
    while bool(bad.any()):
        idx = bad.nonzero().squeeze(1)
        c = comp[idx]
        out[idx] = centres[c] + stds[c, None] * torch.randn(idx.numel(), 3, generator=gen, dtype=torch.float64)
        bad = (out.abs() > box).any(dim=1)
    return out.t().contiguous()


def clustered_gaussians(n: int, seed: int, dtype=torch.float32) -> torch.Tensor:
    gen = torch.Generator().manual_seed(seed)
    return _finish_params(gen, gmm_means(n, gen), -4.0, 0.5, dtype)


def aerial_gaussians(n: int, seed: int, dtype=torch.float32, patch: float = 1000.0,
                     tall_frac: float = 0.05, n_tall: int = 100) -> torch.Tensor:
    """Ground patch [-patch/2, patch/2]^2 with heights N(0, 5) and log-scales
    N(-1, 0.7); a ``tall_frac`` share sits in ``n_tall`` tall clusters
    (horizontal std 5 around a uniform centre, height U[0, 60])."""
    gen = torch.Generator().manual_seed(seed)
    half = patch / 2.0
    n_t = int(round(tall_frac * n))
    n_g = n - n_t
    means = torch.empty(3, n, dtype=torch.float64)
    means[0:2, :n_g] = (2.0 * torch.rand(2, n_g, generator=gen, dtype=torch.float64) - 1.0) * half
    means[2, :n_g] = 5.0 * torch.randn(n_g, generator=gen, dtype=torch.float64)
    centres = (2.0 * torch.rand(n_tall, 2, generator=gen, dtype=torch.float64) - 1.0) * half
    which = torch.randint(0, n_tall, (n_t,), generator=gen)
    means[0:2, n_g:] = (centres[which] + 5.0 * torch.randn(n_t, 2, generator=gen, dtype=torch.float64)).t()
    means[2, n_g:] = 60.0 * torch.rand(n_t, generator=gen, dtype=torch.float64)
    return _finish_params(gen, means, -1.0, 0.7, dtype)


def jittered(params: torch.Tensor, seed: int, sd: float = 0.02) -> torch.Tensor:
    """Copy of a scene with means moved by N(0, sd): the target scene."""
    gen = torch.Generator().manual_seed(seed)
    out = params.clone()
    out[0:3] += (sd * torch.randn(3, params.shape[1], generator=gen, dtype=torch.float64)).to(params.dtype)
    return out


def sphere_cameras(k: int, seed: int, width: int, height: int, radius: float = 8.0,
                   el_lo_deg: float = 10.0, el_hi_deg: float = 60.0) -> list:
    gen = torch.Generator().manual_seed(seed)
    az = 2.0 * math.pi * torch.rand(k, generator=gen, dtype=torch.float64)
    el = torch.deg2rad(el_lo_deg + (el_hi_deg - el_lo_deg) * torch.rand(k, generator=gen, dtype=torch.float64))
    return [orbit_camera(width, height, radius, float(a), float(e)) for a, e in zip(az, el)]


# --------------------------------------------------------------------------- workloads
@dataclass
class Workload:
    name: str
    params: torch.Tensor          # [59][N]
    cameras: list                 # list of camera dicts (one per view in the batch)
    target_params: torch.Tensor | None = None


def plain_single_view(dtype=torch.float32) -> Workload:
    """10,000 Gaussians (seed 0) in [-1,1]^3, one 256x256 view from distance 4."""
    P = uniform_cube_gaussians(10_000, 0, dtype)
    cam = orbit_camera(256, 256, 4.0, 0.0, 0.0)
    return Workload("single_view_256", P, [cam], jittered(P, 100))


def diff_check_small(dtype=torch.float64) -> Workload:
    """200 Gaussians (seed 1), one 64x64 view from distance 4."""
    P = uniform_cube_gaussians(200, 1, dtype)
    cam = orbit_camera(64, 64, 4.0, 0.0, 0.0)
    return Workload("diff_check_64", P, [cam], jittered(P, 101))


def diff_check_large(n: int = 1_000_000, dtype=torch.float32) -> Workload:
    """1M clustered Gaussians (seed 1), one 1920x1080 view on the radius-8 sphere."""
    P = clustered_gaussians(n, 1, dtype)
    cams = sphere_cameras(1, 11, 1920, 1080)
    return Workload("diff_check_1080p", P, cams, jittered(P, 102))


def batched_1080p(n: int = 1_000_000, views: int = 16, dtype=torch.float32) -> Workload:
    """1M clustered Gaussians, a batch of 16 views at 1920x1080, radius-8 sphere,
    azimuth U[0, 2pi), elevation U[10, 60] degrees."""
    P = clustered_gaussians(n, 1, dtype)
    cams = sphere_cameras(views, 12, 1920, 1080)
    return Workload(f"batched_{views}x1080p", P, cams, jittered(P, 103))


def aerial_4k(n: int = 20_000_000, dtype=torch.float32) -> Workload:
    """20M Gaussians over a 1000x1000 ground patch; 2 views at 4608x3456 and 2 at
    3840x2160, altitude U[150, 250], tilt U[0, 30] degrees, yaw U[0, 2pi)."""
    P = aerial_gaussians(n, 4, dtype)
    gen = torch.Generator().manual_seed(14)
    cams = []
    for (w, h) in [(4608, 3456), (4608, 3456), (3840, 2160), (3840, 2160)]:
        r = torch.rand(5, generator=gen, dtype=torch.float64)
        pos = ((2.0 * r[0:2] - 1.0) * 0.8 * 500.0).tolist()
        cams.append(aerial_camera(w, h, pos, 150.0 + 100.0 * float(r[2]),
                                  math.radians(30.0) * float(r[3]), 2.0 * math.pi * float(r[4])))
    return Workload("aerial_2x4608x3456_2x3840x2160", P, cams, jittered(P, 104))


SERVE_RESOLUTIONS = [(512, 512), (1280, 720), (1920, 1080), (3840, 2160)]


def serving_scene(n: int = 5_000_000, dtype=torch.float32) -> torch.Tensor:
    """Device-resident render-only model: 5M clustered Gaussians (seed 5)."""
    return clustered_gaussians(n, 5, dtype)


def serving_requests(k: int, qps: float, seed: int = 15) -> list:
    """Poisson arrivals at ``qps``; resolution uniform over SERVE_RESOLUTIONS;
    pose uniform on the radius-8 sphere (elevation 10-60 degrees).
    Returns a list of (arrival_seconds, camera)."""
    gen = torch.Generator().manual_seed(seed)
    gaps = -torch.log(torch.rand(k, generator=gen, dtype=torch.float64)) / qps
    arrivals = torch.cumsum(gaps, 0)
    res = torch.randint(0, len(SERVE_RESOLUTIONS), (k,), generator=gen)
    az = 2.0 * math.pi * torch.rand(k, generator=gen, dtype=torch.float64)
    el = torch.deg2rad(10.0 + 50.0 * torch.rand(k, generator=gen, dtype=torch.float64))
    out = []
    for j in range(k):
        w, h = SERVE_RESOLUTIONS[int(res[j])]
        out.append((float(arrivals[j]), orbit_camera(w, h, 8.0, float(az[j]), float(el[j]))))
    return out


def random_images(cameras: list, seed: int, dtype=torch.float32) -> torch.Tensor:
    """Concatenated per-view planar [3][H][W] images with values U[0,1]."""
    gen = torch.Generator().manual_seed(seed)
    total = sum(3 * c["width"] * c["height"] for c in cameras)
    return torch.rand(total, generator=gen, dtype=torch.float64).to(dtype)


def image_pair(cameras: list, seed: int, dtype=torch.float32, noise: float = 0.05):
    """A (rendered, target) pair of concatenated planar [3][H][W] images shaped
    like a training step's: the target a smooth colour field with fine noise,
    a flat rectangle and values clipped to [0, 1] (saturated areas); the
    rendered image the target plus independent noise of standard deviation
    `noise`, clipped the same way, and equal to it on the flat rectangle."""
    gen = np.random.default_rng(seed)
    rgb, tgt = [], []
    for c in cameras:
        W, H = c["width"], c["height"]
        yy, xx = np.meshgrid(np.arange(H) / max(H, 1), np.arange(W) / max(W, 1), indexing="ij")
        t = np.empty((3, H, W))
        for ch in range(3):
            f1, f2, ph = gen.uniform(1, 8), gen.uniform(1, 8), gen.uniform(0, 2 * math.pi)
            t[ch] = 0.5 + 0.6 * np.sin(f1 * 2 * math.pi * xx + ph) * np.cos(f2 * 2 * math.pi * yy)
        t += 0.03 * gen.standard_normal(t.shape)
        x0, y0 = int(gen.integers(0, max(W // 2, 1))), int(gen.integers(0, max(H // 2, 1)))
        flat = (slice(None), slice(y0, y0 + max(H // 4, 1)), slice(x0, x0 + max(W // 4, 1)))
        t[flat] = gen.uniform(0.1, 0.9)
        t = np.clip(t, 0.0, 1.0)
        r = np.clip(t + noise * gen.standard_normal(t.shape), 0.0, 1.0)
        r[flat] = t[flat]
        rgb.append(r.ravel())
        tgt.append(t.ravel())
    return (torch.from_numpy(np.concatenate(rgb)).to(dtype), torch.from_numpy(np.concatenate(tgt)).to(dtype))
