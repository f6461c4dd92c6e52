"""gs_render_fwd_l1_noalloc (the entry point for callers that cannot
allocate: its loss scratch is the library's fixed per-device array) against
gs_render_fwd_l1 with a caller workspace: images, transmittance, last
positions, tile work, the L1 image gradient and the loss must be identical
(same kernels, same summation order). Two calls in a row, the second on a
smaller batch, so stale scratch contents from the first would show."""
import pytest
import torch

from synthetic import scenes

pytestmark = pytest.mark.gpu

BG = (0.1, 0.2, 0.3)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_18533_amd import raster
    raster.init(0)


def _prepare(P, cams_list, seed):
    from paper_2406_18533_amd import raster as R
    from tests import gpu_pipeline as gp
    cams = R.Cameras(cams_list)
    Pd = gp.to_dev(P)
    proj = R.gs_project(Pd, cams)
    bins = R.Bins(P.shape[1], cams, gp.estimate_capacity(proj))
    R.gs_bin_sort(proj, P.shape[1], cams, bins, check_capacity=True)
    target = scenes.random_images(cams_list, seed).cuda()
    return cams, proj, bins, target


def _run_both(P, cams_list, seed, scale):
    from paper_2406_18533_amd import raster as R
    cams, proj, bins, target = _prepare(P, cams_list, seed)
    n = P.shape[1]
    T_all = cams.total_tiles()
    Ptot = cams.total_pixels()
    dev = "cuda"
    # reference: the entry point with a caller-owned workspace
    buf = R.LossBuffers(cams)
    wf0 = torch.zeros(T_all, dtype=torch.int32, device=dev)
    wb0 = torch.zeros(T_all, dtype=torch.int32, device=dev)
    rgb0, T0, last0 = R.gs_render_fwd_l1(proj, n, bins, cams, target, buf, BG, tile_work_fwd=wf0, tile_work_bwd=wb0,
                                         scale=scale)
    # no-allocation variant: every output preallocated by the caller
    rgb1 = torch.full((3 * Ptot,), -7.0, device=dev)
    T1 = torch.full((Ptot,), -7.0, device=dev)
    last1 = torch.full((Ptot,), -7, dtype=torch.int32, device=dev)
    dL1 = torch.full((3 * Ptot,), -7.0, device=dev)
    loss1 = torch.full((1,), -7.0, dtype=torch.float64, device=dev)
    wf1 = torch.zeros(T_all, dtype=torch.int32, device=dev)
    wb1 = torch.zeros(T_all, dtype=torch.int32, device=dev)
    R.gs_render_fwd_l1_noalloc(proj, n, bins, cams, target, rgb1, T1, last1, dL1, loss1, BG, tile_work_fwd=wf1,
                               tile_work_bwd=wb1, scale=scale)
    torch.cuda.synchronize()
    assert torch.equal(rgb0, rgb1) and torch.equal(T0, T1) and torch.equal(last0, last1)
    assert torch.equal(wf0, wf1) and torch.equal(wb0, wb1)
    assert torch.equal(buf.dL, dL1)
    assert loss1.item() == buf.loss.item() and loss1.item() > 0.0
    print(f"noalloc: {len(cams_list)} views, {T_all} tiles, loss {loss1.item():.9g}", flush=True)


def test_noalloc_forward_equals_workspace_forward_twice():
    # first call: three ragged views, 20k Gaussians (more tiles)
    P = scenes.uniform_cube_gaussians(20_000, 7)
    cams = [scenes.orbit_camera(300, 170, 3.0, 0.3, 0.2), scenes.orbit_camera(200, 120, 4.0, 2.0, 0.5),
            scenes.orbit_camera(33, 50, 3.5, 4.0, -0.3)]
    _run_both(P, cams, 11, 1.0)
    # second call: one small view, fewer tiles than the first left in the scratch
    P2 = scenes.uniform_cube_gaussians(3_000, 8)
    _run_both(P2, [scenes.orbit_camera(70, 45, 3.0, 1.1, 0.1)], 12, 0.5)


def test_noalloc_rejects_more_tiles_than_its_scratch():
    from paper_2406_18533_amd import _lib
    from paper_2406_18533_amd import raster as R
    # 2^20 tiles in one 16384 x 16384 view plus one more tile: over the limit
    # (the check comes before any launch, so the buffers are never touched)
    cams = R.Cameras([scenes.orbit_camera(16384, 16384, 4.0, 0.0, 0.0), scenes.orbit_camera(16, 16, 4.0, 0.0, 0.0)])
    assert cams.total_tiles() == (1 << 20) + 1
    dummy = torch.zeros(16, device="cuda")
    bins = R.Bins(1, cams, 16)
    with pytest.raises(_lib.GsError) as ei:
        R.gs_render_fwd_l1_noalloc(dummy, 1, bins, cams, dummy, dummy, dummy, dummy.view(torch.int32), dummy,
                                   torch.zeros(1, dtype=torch.float64, device="cuda"))
    assert ei.value.status == _lib.GS_ERR_ARG
    assert "fixed scratch" in str(ei.value)
