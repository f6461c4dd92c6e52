"""A dense, differentiable PyTorch formulation of the forward pass, used only
as a pin for the oracle's hand-written backward (torch autograd in FP64).

It is written independently of ``oracle/``: the projection is expressed with
torch tensor algebra, the harmonics with their textbook degree <= 3 polynomial
forms, and the composition runs every pixel against every Gaussian (no tiles)
in increasing (FP32 depth bits, index) order with masks for the footprint
circle, the 1/255 skip and the transmittance stop. Discrete decisions (radius,
masks, stop, order) are taken on detached values, exactly as piecewise-
constant quantities carry no gradient.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def sh_poly(d: torch.Tensor) -> torch.Tensor:
    """Real orthonormal harmonics l <= 3 (Condon-Shortley phase) of unit
    directions d [..., 3] -> [..., 16], index l*l + l + m."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    pi = math.pi
    c = lambda v: math.sqrt(v)
    out = [
        torch.full_like(x, c(1 / (4 * pi))),
        -c(3 / (4 * pi)) * y, c(3 / (4 * pi)) * z, -c(3 / (4 * pi)) * x,
        c(15 / (4 * pi)) * x * y, -c(15 / (4 * pi)) * y * z, c(5 / (16 * pi)) * (3 * z * z - 1),
        -c(15 / (4 * pi)) * x * z, c(15 / (16 * pi)) * (x * x - y * y),
        -c(35 / (32 * pi)) * (3 * x * x * y - y ** 3), c(105 / (4 * pi)) * x * y * z,
        -c(21 / (32 * pi)) * y * (5 * z * z - 1), c(7 / (16 * pi)) * (5 * z ** 3 - 3 * z),
        -c(21 / (32 * pi)) * x * (5 * z * z - 1), c(105 / (16 * pi)) * z * (x * x - y * y),
        -c(35 / (32 * pi)) * (x ** 3 - 3 * x * y * y),
    ]
    return torch.stack(out, dim=-1)


def quat_to_matrix(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrices [N,3,3] of quaternions (w,x,y,z) [4,N], normalised here."""
    q = q / q.norm(dim=0, keepdim=True)
    w, x, y, z = q
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def project(P: torch.Tensor, cam: dict):
    """Returns dict of per-Gaussian tensors for one view (float64)."""
    R = torch.tensor(np.asarray(cam["R"]), dtype=P.dtype)
    t = torch.tensor(np.asarray(cam["t"]), dtype=P.dtype)
    fx, fy, cx, cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    mean = P[0:3].t()                                   # [N,3]
    s = torch.exp(P[3:6]).t()                           # [N,3]
    Rq = quat_to_matrix(P[6:10])                        # [N,3,3]
    Msc = Rq * s[:, None, :]
    Sigma = Msc @ Msc.transpose(1, 2)
    opac = torch.sigmoid(P[10])
    y = mean @ R.t() + t                                # camera space
    z = y[:, 2]
    u = fx * y[:, 0] / z + cx
    v = fy * y[:, 1] / z + cy
    limx = 1.3 * 0.5 * cam["width"] / fx
    limy = 1.3 * 0.5 * cam["height"] / fy
    xi = torch.clamp(y[:, 0] / z, -limx, limx)
    eta = torch.clamp(y[:, 1] / z, -limy, limy)
    zero = torch.zeros_like(z)
    J = torch.stack([torch.stack([fx / z, zero, -fx * xi / z], -1),
                     torch.stack([zero, fy / z, -fy * eta / z], -1)], -2)   # [N,2,3]
    Tm = J @ R
    S2 = Tm @ Sigma @ Tm.transpose(1, 2) + 0.3 * torch.eye(2, dtype=P.dtype)
    A, B, C = S2[:, 0, 0], S2[:, 0, 1], S2[:, 1, 1]
    det = A * C - B * B
    conic = torch.stack([C / det, -B / det, A / det], 0)
    mid = 0.5 * (A + C)
    lmax = mid + torch.sqrt(torch.clamp(mid * mid - det, min=0.0))
    radius = torch.ceil(3.0 * torch.sqrt(lmax.detach()))
    centre = -(R.t() @ t)
    d = mean - centre
    dirs = d / d.norm(dim=1, keepdim=True)
    Y = sh_poly(dirs)                                    # [N,16]
    sh = P[11:59].reshape(16, 3, -1)                     # [16,3,N]
    raw = torch.einsum("nk,kcn->cn", Y, sh) + 0.5
    rgb = torch.clamp(raw, min=0.0)
    visible = (z > cam["znear"]).detach()
    radius = torch.where(visible, radius, torch.zeros_like(radius))
    return {"u": u, "v": v, "depth": z, "conic": conic, "opac": opac, "rgb": rgb, "radius": radius}


def render(pr: dict, cam: dict, bg=(0.0, 0.0, 0.0)):
    """Dense composition of one view: every pixel x every Gaussian."""
    W, H = cam["width"], cam["height"]
    dt = pr["u"].dtype
    depth32 = pr["depth"].detach().numpy().astype(np.float32).view(np.uint32).astype(np.int64)
    idx = np.arange(depth32.shape[0])
    keep = pr["radius"].detach().numpy() > 0
    order = np.lexsort((idx[keep], depth32[keep]))
    order = idx[keep][order]
    py, px = torch.meshgrid(torch.arange(H, dtype=dt), torch.arange(W, dtype=dt), indexing="ij")
    px = px.reshape(-1) + 0.5
    py = py.reshape(-1) + 0.5
    T = torch.ones(H * W, dtype=dt)
    Cacc = torch.zeros(3, H * W, dtype=dt)
    active = torch.ones(H * W, dtype=torch.bool)
    for i in order.tolist():
        dx = px - pr["u"][i]
        dy = py - pr["v"][i]
        a, b, c = pr["conic"][0][i], pr["conic"][1][i], pr["conic"][2][i]
        r = pr["radius"][i]
        power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
        og = pr["opac"][i] * torch.exp(power)
        alpha = torch.clamp(og, max=0.99)
        inside = ((dx * dx + dy * dy) <= r * r) & (power <= 0) & (alpha >= 1.0 / 255.0)
        inside = inside.detach() & active
        Tn = T * (1.0 - alpha)
        stop = inside & (Tn.detach() < 1e-4)
        active = active & ~stop
        blend = inside & ~stop
        Cacc = Cacc + torch.where(blend, pr["rgb"][:, i:i + 1] * alpha * T, torch.zeros_like(Cacc))
        T = torch.where(blend, Tn, T)
    bgt = torch.tensor(bg, dtype=dt)[:, None]
    return (Cacc + T * bgt).reshape(3, H, W), T.reshape(H, W)
