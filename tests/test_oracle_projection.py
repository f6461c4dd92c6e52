"""Pins of the oracle's Gaussian transformation (paper, section "Background on
3D Gaussian Training", step 1) against closed forms, library routines and
invariants: none of these re-types the oracle's own formulas."""
import math

import numpy as np
import pytest
import scipy.special as sps

import oracle
from synthetic import scenes


def _one(mean, log_scale, quat, logit=0.0, sh=None):
    P = np.zeros((59, 1))
    P[0:3, 0] = mean
    P[3:6, 0] = log_scale
    P[6:10, 0] = quat
    P[10, 0] = logit
    if sh is not None:
        P[11:59, 0] = sh
    return P


# --------------------------------------------------------------------------- harmonics
def _real_sh_scipy(l, m, theta, phi):
    """Real orthonormal harmonics from scipy's complex ones (Condon-Shortley
    phase included by scipy): m>0 -> sqrt2 Re Y_l^m, m<0 -> sqrt2 Im Y_l^|m|."""
    if hasattr(sps, "sph_harm_y"):
        Yc = sps.sph_harm_y(l, abs(m), theta, phi)
    else:  # older scipy argument order: (m, n, azimuth, polar)
        Yc = sps.sph_harm(abs(m), l, phi, theta)
    if m == 0:
        return Yc.real
    return math.sqrt(2.0) * (Yc.real if m > 0 else Yc.imag)


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.arctan2(d[:, 1], d[:, 0])
    Y = oracle.sh_basis(d)
    for l in range(4):
        for m in range(-l, l + 1):
            ref = _real_sh_scipy(l, m, theta, phi)
            np.testing.assert_allclose(Y[:, l * l + l + m], ref, atol=1e-12, rtol=0)


def test_sh_dc_constant():
    Y = oracle.sh_basis(np.array([[0.3, -0.4, math.sqrt(1 - 0.25)]]))
    assert Y[0, 0] == pytest.approx(1.0 / (2.0 * math.sqrt(math.pi)), abs=1e-15)


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi: exact for degree <= 6 products.
    zs, wz = np.polynomial.legendre.leggauss(8)
    phis = np.linspace(0.0, 2.0 * math.pi, 16, endpoint=False)
    Z, PH = np.meshgrid(zs, phis, indexing="ij")
    W = np.outer(wz, np.full(16, 2.0 * math.pi / 16))
    st = np.sqrt(1 - Z ** 2)
    d = np.stack([st * np.cos(PH), st * np.sin(PH), Z], -1).reshape(-1, 3)
    Y = oracle.sh_basis(d)
    G = (Y * W.reshape(-1, 1)).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_tangential_gradient_by_fd():
    rng = np.random.default_rng(1)
    d = rng.normal(size=(20, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    _, dY = oracle.sh_basis(d, with_grad=True)
    h = 1e-6
    for j in range(20):
        t = np.cross(d[j], rng.normal(size=3))
        t /= np.linalg.norm(t)
        dp = d[j] + h * t
        dm = d[j] - h * t
        fd = (oracle.sh_basis(dp / np.linalg.norm(dp)) - oracle.sh_basis(dm / np.linalg.norm(dm)))[0] / (2 * h)
        np.testing.assert_allclose(dY[j] @ t, fd, atol=1e-7)


# --------------------------------------------------------------------------- projection closed forms
def _axis_cam(W=256, H=256):
    return scenes.orbit_camera(W, H, 4.0, 0.0, 0.0)   # at (4,0,0) looking at the origin


def test_isotropic_on_axis_closed_form():
    cam = _axis_cam()
    s = 0.05
    P = _one([0, 0, 0], [math.log(s)] * 3, [1, 0, 0, 0], logit=0.7)
    pr = oracle.project(P, cam)[:, 0]
    f, dpt = cam["fx"], 4.0
    var = (f * s / dpt) ** 2 + 0.3
    assert pr[oracle.F_U] == pytest.approx(cam["cx"], abs=1e-12)
    assert pr[oracle.F_V] == pytest.approx(cam["cy"], abs=1e-12)
    assert pr[oracle.F_DEPTH] == pytest.approx(dpt, abs=1e-12)
    np.testing.assert_allclose(pr[[oracle.F_A, oracle.F_B, oracle.F_C]], [1 / var, 0, 1 / var], atol=1e-14, rtol=1e-12)
    assert pr[oracle.F_RADIUS] == math.ceil(3 * math.sqrt(var))
    assert pr[oracle.F_OPAC] == pytest.approx(1 / (1 + math.exp(-0.7)), abs=1e-15)


def test_anisotropic_rotated_about_view_axis():
    """On the optical axis the perspective Jacobian is (f/d) I on the first two
    camera axes, so the image covariance is (f/d)^2 times the top-left 2x2 of
    the camera-space covariance, plus 0.3 I. The rotation is built from the
    axis-angle form, not from the quaternion matrix."""
    cam = _axis_cam()
    sx, sy, sz = 0.02, 0.06, 0.015
    phi = 0.4
    q = [math.cos(phi / 2), math.sin(phi / 2), 0, 0]
    P = _one([0, 0, 0], [math.log(sx), math.log(sy), math.log(sz)], q)
    pr = oracle.project(P, cam)[:, 0]
    k = cam["fx"] / 4.0
    Rx = np.array([[1, 0, 0], [0, math.cos(phi), -math.sin(phi)], [0, math.sin(phi), math.cos(phi)]])
    Sw = Rx @ np.diag([sx * sx, sy * sy, sz * sz]) @ Rx.T
    Rc = np.asarray(cam["R"])
    S = k * k * (Rc @ Sw @ Rc.T)[:2, :2] + 0.3 * np.eye(2)
    Q = np.linalg.inv(S)
    assert abs(Q[0, 1]) > 1e-3          # the rotation really couples the axes
    np.testing.assert_allclose(pr[[oracle.F_A, oracle.F_B, oracle.F_C]], [Q[0, 0], Q[0, 1], Q[1, 1]], rtol=1e-11)
    lmax = np.linalg.eigvalsh(S).max()
    assert pr[oracle.F_REXACT] == pytest.approx(3 * math.sqrt(lmax), rel=1e-12)


def test_off_axis_matches_numerical_jacobian_of_pinhole():
    """EWA: image covariance = Jac(pinhole) Sigma_cam Jac^T + 0.3 I, with the
    Jacobian of (x, y, z) -> (fx x/z + cx, fy y/z + cy) taken numerically."""
    cam = scenes.orbit_camera(320, 240, 5.0, 0.3, 0.2)
    R, t = np.asarray(cam["R"]), np.asarray(cam["t"])
    rng = np.random.default_rng(3)
    for _ in range(10):
        mean = rng.uniform(-0.8, 0.8, 3)
        ls = rng.normal(-3.5, 0.4, 3)
        q = rng.normal(size=4)
        pr = oracle.project(_one(mean, ls, q), cam)[:, 0]
        y = R @ mean + t
        pin = lambda p: np.array([cam["fx"] * p[0] / p[2] + cam["cx"], cam["fy"] * p[1] / p[2] + cam["cy"]])
        np.testing.assert_allclose(pr[[oracle.F_U, oracle.F_V]], pin(y), rtol=1e-13)
        Jn = np.zeros((2, 3))
        for j in range(3):
            e = np.zeros(3)
            e[j] = 1e-5
            Jn[:, j] = (pin(y + e) - pin(y - e)) / 2e-5
        qn = q / np.linalg.norm(q)
        w, x, yq, z = qn
        # rotation from the axis-angle form (Rodrigues), independent of the quaternion matrix
        ang = 2 * math.atan2(np.linalg.norm(qn[1:]), w)
        ax = qn[1:] / np.linalg.norm(qn[1:])
        Kx = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
        Rq = np.eye(3) + math.sin(ang) * Kx + (1 - math.cos(ang)) * Kx @ Kx
        Sig = Rq @ np.diag(np.exp(2 * ls)) @ Rq.T
        S = Jn @ (R @ Sig @ R.T) @ Jn.T + 0.3 * np.eye(2)
        Q = np.linalg.inv(S)
        np.testing.assert_allclose(pr[[oracle.F_A, oracle.F_B, oracle.F_C]], [Q[0, 0], Q[0, 1], Q[1, 1]], rtol=1e-7)


def _pinhole_jacobian(cam, p):
    """Numerical Jacobian of (x, y, z) -> (fx x/z + cx, fy y/z + cy) at p."""
    pin = lambda q: np.array([cam["fx"] * q[0] / q[2] + cam["cx"], cam["fy"] * q[1] / q[2] + cam["cy"]])
    Jn = np.zeros((2, 3))
    for j in range(3):
        e = np.zeros(3)
        e[j] = 1e-5
        Jn[:, j] = (pin(p + e) - pin(p - e)) / 2e-5
    return Jn


def test_guard_band_evaluates_the_jacobian_at_the_clamped_point():
    """Reading of section 2.1 step 1 for Gaussians far off the optical axis:
    the perspective Jacobian of the EWA covariance is taken at the centre
    with x/z and y/z clamped to 1.3 tan(half field of view); the centre
    itself (u, v) is not clamped. Points just inside the band (1.25 tan)
    keep their own Jacobian, points beyond it (1.35 tan, 2 tan, on either
    side and on both axes) take it at the band's edge, so a wrong limit or a
    clamp applied to the centre fails."""
    cam = scenes.orbit_camera(320, 240, 5.0, 0.3, 0.2)
    R, t = np.asarray(cam["R"]), np.asarray(cam["t"])
    tx, ty = 0.5 * cam["width"] / cam["fx"], 0.5 * cam["height"] / cam["fy"]
    limx, limy = 1.3 * tx, 1.3 * ty
    rng = np.random.default_rng(21)
    cases = [(1.25 * tx, 0.1 * ty), (-1.25 * tx, 0.0), (0.0, 1.25 * ty), (1.35 * tx, 0.2 * ty), (-1.35 * tx, -0.3 * ty),
             (0.1 * tx, 1.35 * ty), (0.0, -2.0 * ty), (2.0 * tx, -1.5 * ty), (-1.6 * tx, 1.6 * ty)]
    clamped = 0
    for k, (xr, yr) in enumerate(cases):
        z = 3.0 + 0.5 * k
        y_cam = np.array([xr * z, yr * z, z])
        mean = R.T @ (y_cam - t)
        ls = rng.normal(-2.0, 0.3, 3)
        q = rng.normal(size=4)
        pr = oracle.project(_one(mean, ls, q), cam)[:, 0]
        # the centre projects without any clamp
        np.testing.assert_allclose(pr[[oracle.F_U, oracle.F_V]],
                                   [cam["fx"] * xr + cam["cx"], cam["fy"] * yr + cam["cy"]], rtol=1e-12)
        xi, eta = np.clip(xr, -limx, limx), np.clip(yr, -limy, limy)
        clamped += (xi != xr) or (eta != yr)
        Jn = _pinhole_jacobian(cam, np.array([xi * z, eta * z, z]))
        qn = q / np.linalg.norm(q)
        ang = 2 * math.atan2(np.linalg.norm(qn[1:]), qn[0])
        ax = qn[1:] / np.linalg.norm(qn[1:])
        Kx = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
        Rq = np.eye(3) + math.sin(ang) * Kx + (1 - math.cos(ang)) * Kx @ Kx
        Sc = R @ (Rq @ np.diag(np.exp(2 * ls)) @ Rq.T) @ R.T
        Q = np.linalg.inv(Jn @ Sc @ Jn.T + 0.3 * np.eye(2))
        np.testing.assert_allclose(pr[[oracle.F_A, oracle.F_B, oracle.F_C]], [Q[0, 0], Q[0, 1], Q[1, 1]], rtol=1e-7)
        if (xi, eta) != (xr, yr):
            # the unclamped Jacobian would give a clearly different footprint
            Ju = _pinhole_jacobian(cam, y_cam)
            Qu = np.linalg.inv(Ju @ Sc @ Ju.T + 0.3 * np.eye(2))
            assert np.max(np.abs(Qu - Q)) > 1e-3 * np.max(np.abs(Q))
    assert clamped == 6


def test_quaternion_sign_and_scale_invariance():
    cam = scenes.orbit_camera(128, 96, 4.0, 1.0, 0.5)
    rng = np.random.default_rng(4)
    q = rng.normal(size=4)
    base = oracle.project(_one([0.1, 0.2, -0.1], [-3, -3.5, -2.8], q, sh=rng.normal(0, 0.1, 48)), cam)
    for qq in (-q, 3.7 * q):
        other = oracle.project(_one([0.1, 0.2, -0.1], [-3, -3.5, -2.8], qq, sh=rng.normal(0, 0.1, 48) * 0 + 0), cam)
        np.testing.assert_allclose(other[:7], base[:7], rtol=1e-12, atol=1e-15)


def test_near_plane_cull_and_nonfinite():
    cam = _axis_cam()
    # a Gaussian behind the camera (x > 4) and one between camera and near plane
    for x in (5.0, 3.9):
        pr = oracle.project(_one([x, 0, 0], [-3] * 3, [1, 0, 0, 0]), cam)[:, 0]
        assert pr[oracle.F_RADIUS] == 0 and np.all(pr == 0)
    pr = oracle.project(_one([0, 0, 0], [-3] * 3, [0, 0, 0, 0]), cam)[:, 0]
    assert pr[oracle.F_RADIUS] == 0
    pr = oracle.project(_one([np.nan, 0, 0], [-3] * 3, [1, 0, 0, 0]), cam)[:, 0]
    assert pr[oracle.F_RADIUS] == 0


def test_dc_colour_and_clamp():
    cam = _axis_cam()
    sh = np.zeros(48)
    sh[0:3] = [0.5, -3.0, 1.0]
    pr = oracle.project(_one([0, 0, 0], [-3] * 3, [1, 0, 0, 0], sh=sh), cam)[:, 0]
    C0 = 1.0 / (2.0 * math.sqrt(math.pi))
    np.testing.assert_allclose(pr[[oracle.F_R, oracle.F_G, oracle.F_BL]], [C0 * 0.5 + 0.5, 0.0, C0 + 0.5], rtol=1e-14)


def test_view_dependent_colour_uses_world_direction():
    """Degree-1 coefficient on Y_1,0 (proportional to z): a camera above the
    Gaussian sees direction (camera -> Gaussian) pointing down, z < 0."""
    cam = scenes.orbit_camera(64, 64, 4.0, 0.0, math.radians(89.0))
    sh = np.zeros(48)
    sh[3 * 2 + 0] = 1.0
    pr = oracle.project(_one([0, 0, 0], [-3] * 3, [1, 0, 0, 0], sh=sh), cam)[:, 0]
    dz = -math.sin(math.radians(89.0))
    assert pr[oracle.F_R] == pytest.approx(max(0.0, math.sqrt(3 / (4 * math.pi)) * dz + 0.5), abs=1e-12)


def test_radius_cdf_shape_on_synthetic_scenes():
    """Workload-shape sanity: most radii are a small fraction of the image
    width (the paper reports 90% below 2% of the width on real scenes)."""
    w = scenes.plain_single_view(dtype=__import__("torch").float64)
    pr = oracle.project(w.params, w.cameras[0])
    r = pr[oracle.F_RADIUS]
    r = r[r > 0]
    assert np.quantile(r, 0.9) < 0.05 * w.cameras[0]["width"]
