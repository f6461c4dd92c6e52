"""Pins of the oracle's densification (appendix A.1: clone / split by the
position-gradient statistic and a scale threshold, prune by opacity, opacity
reset). Checks come from outside the oracle's formulas: a hand-worked
example, scipy's quaternion rotation, brute-force loops, and the equivalence
of the log / logit domain decisions with the direct ones."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle


def _params(n, rng):
    P = np.zeros((59, n))
    P[0:3] = rng.normal(size=(3, n))
    P[3:6] = rng.normal(-3.0, 0.7, size=(3, n))
    q = rng.normal(size=(4, n))
    P[6:10] = q / np.linalg.norm(q, axis=0)
    P[10] = rng.normal(size=n)
    P[11:59] = rng.normal(size=(48, n))
    return P


def test_rotation_matches_scipy():
    rng = np.random.default_rng(0)
    q = rng.normal(size=(4, 50)) * rng.uniform(0.5, 2.0, size=50)   # unnormalised on purpose
    R = oracle.quat_rotation(q)
    ref = Rotation.from_quat(np.stack([q[1], q[2], q[3], q[0]], -1)).as_matrix()
    assert np.max(np.abs(R - ref)) < 1e-14


def test_stats_equal_brute_force_loop():
    rng = np.random.default_rng(1)
    V, N = 4, 30
    du, dv = rng.normal(size=(V, N)), rng.normal(size=(V, N))
    vis = rng.random((V, N)) < 0.6
    acc, cnt = oracle.densify_stats(du, dv, vis, scale=4.0)
    for i in range(N):
        a, c = 0.0, 0
        for k in range(V):
            if vis[k, i]:
                a += 4.0 * math.hypot(du[k, i], dv[k, i])
                c += 1
        assert abs(acc[i] - a) <= 1e-13 * max(a, 1.0) and cnt[i] == c


def test_log_domain_decisions_equal_direct_rules():
    rng = np.random.default_rng(2)
    P = _params(2000, rng)
    min_op, pd_extent, big = 0.005, 0.05, 0.5
    _, _, _, split = oracle.densify_classes(P, np.ones(2000), np.ones(2000, int), 0.5, math.log(pd_extent),
                                            math.log(min_op / (1 - min_op)), math.log(big))
    keep, _, _, _ = oracle.densify_classes(P, np.zeros(2000), np.ones(2000, int), 0.5, math.log(pd_extent),
                                           math.log(min_op / (1 - min_op)), math.log(big))
    opac = 1.0 / (1.0 + np.exp(-P[10]))
    smax = np.exp(P[3:6]).max(axis=0)
    assert np.array_equal(split, smax > pd_extent)              # every Gaussian selected
    assert np.array_equal(keep, ~((opac < min_op) | (smax > big)))   # nothing selected


def test_hand_worked_example():
    """Six Gaussians, identity rotations, thresholds: grad 1.0, split above
    log-scale -2, prune below logit -4 or above log-scale 0."""
    P = np.zeros((59, 6))
    P[6] = 1.0                                    # w = 1: identity rotation
    P[0] = np.arange(6) * 10.0                    # distinct means along x
    P[3:6] = -3.0                                 # small
    P[3, 2] = -1.0                                # Gaussian 2 large (split)
    P[3, 3] = -1.5                                # Gaussian 3 large (split), low opacity: children pruned
    P[10] = 0.0
    P[10, 3] = -5.0
    P[10, 4] = -5.0                               # Gaussian 4 pruned, not selected
    P[3, 5] = 0.2                                 # Gaussian 5 too large: pruned (and selected: its split
    P[11:59] = np.arange(6)[None, :] + 100.0      # children have log-scale 0.2 - log 1.6 < 0: kept)
    m = np.full((59, 6), 7.0)
    v = np.full((59, 6), 9.0)
    accum = np.array([2.0, 0.5, 3.0, 3.0, 0.0, 5.0])
    denom = np.array([2, 1, 1, 1, 0, 1])          # averages 1.0 (>= threshold), 0.5, 3, 3, -, 5
    noise = np.zeros((2, 3, 6))
    noise[0, :, 2] = [1.0, 0.0, 0.0]
    noise[1, :, 2] = [0.0, -2.0, 0.0]
    noise[0, :, 5] = [0.0, 0.0, 1.0]
    noise[1, :, 5] = [0.0, 0.0, 0.0]
    Po, mo, vo = oracle.densify(P, m, v, accum, denom, noise, 1.0, -2.0, -4.0, 0.0)
    # kept originals 0, 1; clone of 0; first children of 2 and 5; second children of 2 and 5
    assert Po.shape == (59, 7)
    assert np.array_equal(Po[:, 0], P[:, 0]) and np.array_equal(Po[:, 1], P[:, 1])
    assert np.array_equal(Po[:, 2], P[:, 0])
    s2 = math.exp(-1.0)                           # largest axis of Gaussian 2
    assert np.allclose(Po[0:3, 3], [20.0 + s2, 0.0, 0.0], atol=1e-15)
    assert np.allclose(Po[0:3, 4], [50.0, 0.0, math.exp(-3.0)], atol=1e-15)
    assert np.allclose(Po[0:3, 5], [20.0, -2.0 * math.exp(-3.0), 0.0], atol=1e-15)
    assert np.allclose(Po[0:3, 6], [50.0, 0.0, 0.0], atol=1e-15)
    assert np.allclose(Po[3:6, 3], [-1.0 - math.log(1.6), -3.0 - math.log(1.6), -3.0 - math.log(1.6)])
    assert np.allclose(Po[3:6, 4], [0.2 - math.log(1.6), -3.0 - math.log(1.6), -3.0 - math.log(1.6)])
    assert np.array_equal(Po[6:59, 3], P[6:59, 2]) and np.array_equal(Po[6:59, 6], P[6:59, 5])
    assert np.all(mo[:, :2] == 7.0) and np.all(vo[:, :2] == 9.0)
    assert np.all(mo[:, 2:] == 0.0) and np.all(vo[:, 2:] == 0.0)


def test_split_children_match_scipy_and_counts_add_up():
    rng = np.random.default_rng(3)
    N = 400
    P = _params(N, rng)
    m, v = rng.normal(size=(59, N)), rng.random((59, N))
    accum, denom = rng.random(N) * 3, rng.integers(0, 4, N)
    noise = rng.normal(size=(2, 3, N))
    args = (0.6, -3.0, -1.5, -1.0)
    keep, clone, child, split = oracle.densify_classes(P, accum, denom, *args)
    Po, mo, vo = oracle.densify(P, m, v, accum, denom, noise, *args)
    nk, nc, nch = int(keep.sum()), int(clone.sum()), int(child.sum())
    assert Po.shape[1] == nk + nc + 2 * nch and 0 < nc and 0 < nch and nk < N
    idx = np.flatnonzero(child)
    rot = Rotation.from_quat(np.stack([P[7], P[8], P[9], P[6]], -1)[idx])
    for k in range(2):
        off = rot.apply((np.exp(P[3:6, idx]) * noise[k][:, idx]).T).T
        got = Po[:, nk + nc + k * nch: nk + nc + (k + 1) * nch]
        assert np.max(np.abs(got[0:3] - (P[0:3, idx] + off))) < 1e-13
        assert np.max(np.abs(got[3:6] - (P[3:6, idx] - math.log(1.6)))) < 1e-15
        assert np.array_equal(got[6:59], P[6:59, idx])
    assert np.array_equal(Po[:, :nk], P[:, keep]) and np.array_equal(Po[:, nk:nk + nc], P[:, clone])
    assert np.array_equal(mo[:, :nk], m[:, keep]) and not mo[:, nk:].any() and not vo[:, nk:].any()
    # the selection threshold is inclusive: a Gaussian exactly at it is selected
    a2 = np.array([1.2]); d2 = np.array([2])
    _, c2, _, _ = oracle.densify_classes(P[:, [0]], a2, d2, 0.6, 1e9, -1e9, 1e9)
    assert c2[0]


def test_opacity_reset_closed_form():
    rng = np.random.default_rng(4)
    P = _params(100, rng)
    m, v = rng.normal(size=(59, 100)), rng.random((59, 100))
    op = 1.0 / (1.0 + np.exp(-P[10]))
    P2, m2, v2 = P.copy(), m.copy(), v.copy()
    oracle.reset_opacity(P2, m2, v2, 0.01)
    assert np.allclose(1.0 / (1.0 + np.exp(-P2[10])), np.minimum(op, 0.01), rtol=1e-12, atol=0)
    assert not m2[10].any() and not v2[10].any()
    rows = [r for r in range(59) if r != 10]
    assert np.array_equal(P2[rows], P[rows]) and np.array_equal(m2[rows], m[rows])
