"""CPU-side checks of the C ABI: the library loads, exports every entry point
that include/gs.h declares, and rejects bad arguments before touching a GPU."""
import os
import re

import pytest

from synthetic import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "gs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ["gs_project", "gs_bin_sort", "gs_render_fwd", "gs_render_bwd", "gs_adam_step"]:
        assert name in syms


def test_library_exports_every_declared_symbol():
    from paper_2406_18533_amd import _lib
    L = _lib.load()
    for name in declared_symbols():
        assert hasattr(L, name), name
    assert set(_lib.EXPORTS) == set(declared_symbols())
    assert L.gs_version().decode().startswith("gsmi")


def test_host_side_sizes_and_argument_checks():
    from paper_2406_18533_amd import _lib
    from paper_2406_18533_amd._lib import GsCamera
    import ctypes as C
    L = _lib.load()
    cams = (GsCamera * 2)()
    for k, (w, h) in enumerate([(1920, 1080), (70, 45)]):
        c = scenes.orbit_camera(w, h, 4.0, 0.0, 0.0)
        cams[k].width, cams[k].height = w, h
        cams[k].fx = cams[k].fy = c["fx"]
        cams[k].cx, cams[k].cy, cams[k].znear = c["cx"], c["cy"], c["znear"]
    p = C.cast(cams, C.POINTER(GsCamera))
    assert L.gs_total_tiles(p, 2) == 120 * 68 + 5 * 3
    assert L.gs_total_pixels(p, 2) == 1920 * 1080 + 70 * 45
    # records plus two uint32 and one uint64 side arrays per (view, Gaussian)
    assert L.gs_projected_bytes(_lib.GS_F32, 1000, 2) == 1000 * 2 * (12 * 4 + 16)
    assert L.gs_projected_bytes(_lib.GS_F64, 1000, 2) == 1000 * 2 * (12 * 8 + 16)
    assert L.gs_bin_workspace_bytes(1000, 2, 5000, 135) > 0
    # rejected before any device call
    assert L.gs_project(_lib.GS_F32, None, 10, None, p, 0, None, None) == _lib.GS_ERR_ARG
    assert L.gs_project(_lib.GS_F32, None, 10, None, p, 65, None, None) == _lib.GS_ERR_ARG
    assert L.gs_project(9, None, 10, None, p, 1, None, None) == _lib.GS_ERR_ARG
    assert L.gs_project(_lib.GS_F32, None, 10, None, p, 1, None, None) == _lib.GS_ERR_ARG
    assert b"null" in L.gs_last_error()
    assert L.gs_adam_step(_lib.GS_F32, None, None, None, None, 5, None, None, None, None, None) == _lib.GS_ERR_ARG
    cams[1].width, cams[1].height = 32768, 32768          # 2^22 tiles: the largest accepted view
    assert L.gs_total_tiles(p, 2) == 120 * 68 + 2048 * 2048
    cams[1].height = 32769                                  # one tile row more
    assert L.gs_total_tiles(p, 2) == -1
    assert b"2^22 tiles" in L.gs_last_error()
    cams[1].width, cams[1].height = 70, 45
    cams[1].fx = -1.0
    assert L.gs_total_tiles(p, 2) == -1


def test_product_path_has_no_fallback(monkeypatch):
    """Without libgs.so the binding raises instead of computing anything."""
    from paper_2406_18533_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/libgs.so")
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib.load()
