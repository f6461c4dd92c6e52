"""Parity of densification (gs_densify_stats / plan / apply, gs_reset_opacity,
through the C ABI) with the FP64 oracle. Classes, counts and output order
are integer results decided on the stored FP32 values and compared
bit-exactly; copied parameters and moments are bit-exact; split children's
means agree to 2e-6 of the offset's size plus 1e-6 of the mean's (FP32
rotation, exp and sums), their log-scales to 1e-6; the statistic to 1e-6
relative (FP32 sums of at most `views` norms)."""
import math

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_18533_amd import raster
    raster.init(0)


def _params(n, seed, dtype=torch.float32):
    g = torch.Generator().manual_seed(seed)
    P = torch.zeros(59, n, dtype=torch.float64)
    P[0:3] = torch.randn(3, n, generator=g)
    P[3:6] = torch.randn(3, n, generator=g) * 0.7 - 3.0
    q = torch.randn(4, n, generator=g)
    P[6:10] = q / q.norm(dim=0)
    P[10] = torch.randn(n, generator=g) * 1.5
    P[11:59] = torch.randn(48, n, generator=g)
    m, v = torch.randn(59, n, generator=g), torch.rand(59, n, generator=g)
    accum = (torch.rand(n, generator=g) * 3.0).float()
    count = torch.randint(0, 5, (n,), generator=g, dtype=torch.int32)
    noise = torch.randn(2, 3, n, generator=g)
    return P.to(dtype), m.to(dtype), v.to(dtype), accum, count, noise.to(dtype)


def _densify_gpu(P, m, v, accum, count, noise, hp):
    from paper_2406_18533_amd import raster as R
    n = P.shape[1]
    Pc, mc, vc = P.cuda().contiguous(), m.cuda().contiguous(), v.cuda().contiguous()
    plan = R.DensifyPlan(n)
    h = R.densify_hparams(*hp)
    R.gs_densify_plan(Pc, accum.cuda(), count.cuda(), h, plan)
    K, Cn, S = (int(x) for x in plan.counts.cpu())
    po, mo, vo = R.gs_densify_apply(Pc, mc, vc, noise.cuda().contiguous(), plan, K + Cn + 2 * S)
    torch.cuda.synchronize()
    return (K, Cn, S), po.cpu().double().numpy(), mo.cpu().double().numpy(), vo.cpu().double().numpy()


def _check(P, m, v, accum, count, noise, hp, fp64=False):
    counts, po, mo, vo = _densify_gpu(P, m, v, accum, count, noise, hp)
    Pn, mn, vn = P.double().numpy(), m.double().numpy(), v.double().numpy()
    an, cn = accum.double().numpy(), count.numpy()
    keep, clone, child, _ = oracle.densify_classes(Pn, an, cn, *hp)
    assert counts == (int(keep.sum()), int(clone.sum()), int(child.sum()))
    Po, Mo, Vo = oracle.densify(Pn, mn, vn, an, cn, noise.double().numpy(), *hp)
    assert po.shape == Po.shape
    K, C, S = counts
    assert np.array_equal(po[:, :K + C], Po[:, :K + C])                 # kept originals and clones: copies
    assert np.array_equal(mo, Mo) and np.array_equal(vo, Vo)
    ch, ref = po[:, K + C:], Po[:, K + C:]
    assert np.array_equal(ch[6:59], ref[6:59])
    tol_ls = 1e-12 if fp64 else 1e-6
    assert np.max(np.abs(ch[3:6] - ref[3:6]), initial=0.0) <= tol_ls
    if S:
        par = np.concatenate([np.flatnonzero(child)] * 2)
        off = np.abs(ref[0:3] - Pn[0:3, par]).max(axis=0)
        err = np.abs(ch[0:3] - ref[0:3]).max(axis=0)
        tol = (1e-12 if fp64 else 2e-6) * off + (1e-14 if fp64 else 1e-6) * np.abs(Pn[0:3, par]).max(axis=0)
        assert np.all(err <= tol), float((err - tol).max())
    return counts


@pytest.mark.parametrize("n", [1, 255, 256, 5000, 100_003])
def test_plan_and_apply_match_oracle(n):
    P, m, v, accum, count, noise = _params(n, 10 + n % 7)
    print(f"densify parity n={n}", flush=True)
    counts = _check(P, m, v, accum, count, noise, (0.6, -3.0, -1.5, -1.0))
    if n >= 5000:
        assert all(c > 0 for c in counts) and counts[0] < n


def test_fp64_path_matches_oracle():
    P, m, v, accum, count, noise = _params(3000, 3, torch.float64)
    _check(P, m, v, accum, count, noise, (0.6, -3.0, -1.5, -1.0), fp64=True)


def test_edge_cases():
    P, m, v, accum, count, noise = _params(4000, 4)
    # nothing selected, nothing pruned: the output is the input
    c = _check(P, m, v, accum, count, noise, (1e9, -3.0, -math.inf, math.inf))
    assert c == (4000, 0, 0)
    # everything pruned by opacity: empty output
    c = _check(P, m, v, accum, count, noise, (0.6, -3.0, math.inf, math.inf))
    assert c == (0, 0, 0)
    # every Gaussian selected and split (threshold 0 with count > 0)
    count = torch.ones_like(count)
    c = _check(P, m, v, accum, count, noise, (0.0, -math.inf, -math.inf, math.inf))
    assert c == (0, 0, 4000)
    # everything cloned
    c = _check(P, m, v, accum, count, noise, (0.0, math.inf, -math.inf, math.inf))
    assert c == (4000, 4000, 0)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_stats_match_oracle(dtype):
    from paper_2406_18533_amd import raster as R
    V, n = 5, 7001
    g = torch.Generator().manual_seed(5)
    proj = R.alloc_projected(n, V, dtype)
    tiles, _ = R.projected_side_arrays(proj)
    vis = torch.rand(V, n, generator=g) < 0.4
    tiles.copy_((vis.int() * torch.randint(1, 9, (V, n), generator=g, dtype=torch.int32)).cuda())
    dproj = torch.zeros(V, n, 12, dtype=dtype)
    dproj[..., 0] = (torch.randn(V, n, generator=g) * 1e-3).to(dtype)
    dproj[..., 1] = (torch.randn(V, n, generator=g) * 1e-3).to(dtype)
    dproj = dproj.cuda()
    accum = torch.full((n,), 0.25, device="cuda")
    count = torch.full((n,), 2, dtype=torch.int32, device="cuda")
    R.gs_densify_stats(proj, dproj, n, V, accum, count, scale=float(V))
    torch.cuda.synchronize()
    a, c = oracle.densify_stats(dproj[..., 0].cpu().double().numpy(), dproj[..., 1].cpu().double().numpy(),
                                vis.numpy(), scale=float(V))
    assert np.array_equal(count.cpu().numpy(), c + 2)
    assert np.allclose(accum.cpu().double().numpy(), a + 0.25, rtol=1e-6, atol=0)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_reset_opacity_matches_oracle(dtype):
    from paper_2406_18533_amd import raster as R
    P, m, v, *_ = _params(3001, 6, dtype)
    cap = float(np.float32(math.log(0.01 / 0.99)))            # representable: exact comparison
    Pc, mc, vc = P.cuda(), m.cuda(), v.cuda()
    R.gs_reset_opacity(Pc, mc, vc, cap)
    Pn, mn, vn = P.double().numpy(), m.double().numpy(), v.double().numpy()
    cap_op = 1.0 / (1.0 + math.exp(-cap))
    oracle.reset_opacity(Pn, mn, vn, cap_op)
    assert np.allclose(Pc.cpu().double().numpy(), Pn, rtol=0, atol=1e-12)
    assert np.array_equal(mc.cpu().double().numpy(), mn) and np.array_equal(vc.cpu().double().numpy(), vn)


def test_invalid_arguments_rejected():
    from paper_2406_18533_amd import raster as R
    from paper_2406_18533_amd._lib import GsError
    P, m, v, accum, count, noise = _params(100, 7)
    Pc = P.cuda()
    plan = R.DensifyPlan(100)
    with pytest.raises(GsError):
        R.gs_densify_plan(Pc, accum.cuda(), count.cuda(), R.densify_hparams(float("nan"), 0, 0), plan)
    plan.workspace = plan.workspace[:16]
    with pytest.raises(GsError):
        R.gs_densify_plan(Pc, accum.cuda(), count.cuda(), R.densify_hparams(0.5, 0, 0), plan)
    plan = R.DensifyPlan(100)
    R.gs_densify_plan(Pc, accum.cuda(), count.cuda(), R.densify_hparams(0.5, 0, 0), plan)
    with pytest.raises(GsError):
        R.gs_densify_apply(Pc, m.cuda(), v.cuda(), noise.cuda(), plan, 201)     # more than 2 n


def test_trainer_densifies_and_keeps_training():
    """Statistic accumulated inside the graph-captured step, then one
    densification: kept originals are the old columns bit for bit, the new
    size is K + C + 2 S, moments of new Gaussians are zero, and the step
    re-captures and runs at the new size."""
    from paper_2406_18533_amd import raster as R, train
    from synthetic import scenes
    P = scenes.clustered_gaussians(60_000, 3)
    cams = scenes.sphere_cameras(4, 21, 320, 240)
    tgt = scenes.random_images(cams, 4)
    tr = train.BatchedTrainer(P.cuda(), cams, tgt.cuda(), train.TrainConfig(graph=True))
    tr.enable_densify_stats()
    for _ in range(3):
        tr.step()
    torch.cuda.synchronize()
    acc, cnt = tr.stats[0].cpu().numpy(), tr.stats[1].cpu().numpy()
    assert cnt.max() <= 3 * len(cams) and (cnt > 0).sum() > 1000 and np.isfinite(acc).all()
    mean_stat = acc[cnt > 0] / cnt[cnt > 0]
    thr = float(np.quantile(mean_stat, 0.9))
    P0, m0 = tr.P.clone(), tr.m.clone()
    h = R.densify_hparams(thr, float(np.quantile(P0[3:6].max(dim=0).values.cpu().numpy(), 0.5)), -6.0)
    keep, clone, child, _ = oracle.densify_classes(P0.cpu().double().numpy(), acc, cnt, thr, h.split_log_scale,
                                                   -6.0, math.inf)
    K, C, S = tr.densify(h, seed=1)
    assert (K, C, S) == (int(keep.sum()), int(clone.sum()), int(child.sum())) and C > 0 and S > 0
    assert tr.n == K + C + 2 * S == tr.P.shape[1]
    assert torch.equal(tr.P[:, :K], P0[:, torch.from_numpy(np.flatnonzero(keep)).cuda()])
    assert torch.equal(tr.m[:, :K], m0[:, torch.from_numpy(np.flatnonzero(keep)).cuda()])
    assert not tr.m[:, K:].any() and not tr.v[:, K:].any()
    assert not tr.stats[0].any() and not tr.stats[1].any()
    for _ in range(2):
        tr.step()
    assert math.isfinite(tr.loss()) and not tr.check_overflow()
    tr.reset_opacity(0.01)
    assert float(tr.P[10].max()) <= math.log(0.01 / 0.99) + 1e-6 and not tr.m[10].any()
