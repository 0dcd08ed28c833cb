"""Sort mode 2 (row binning: one item per non-empty tile row of each record,
a stable sort of the items by tile row, then each row's items placed into its
tiles) against the tile-key sort of mode 1: the sorted keys, values and tile
ranges must be identical bit for bit, and the sort must pass the same
structural check (a stable sort of exactly the emitted (record, tile) set).
Cases cover one and two row-sort passes, rows of up to 256 tiles, the scanned first pass of large capacities, slivers, uneven
resolutions, empty and culled scenes, a capacity overflow, the fallback to
mode 1 past 256 tiles per row or 1024 rows, and the 1M-Gaussian frame."""
import numpy as np
import pytest
import torch

import sgs_synth as S

from test_gpu_parity import _check_binning, _needles_config, _np, _render, _u32

pytestmark = pytest.mark.gpu


def _same(a, b, images=True):
    n = a.n_inst
    assert n == b.n_inst
    assert int(_u32(a.bufs["n_inst"])[0]) == int(_u32(b.bufs["n_inst"])[0])
    for k in ("keys", "vals"):
        np.testing.assert_array_equal(_np(a.bufs[k])[:n], _np(b.bufs[k])[:n], err_msg=k)
    np.testing.assert_array_equal(_np(a.bufs["ranges"]), _np(b.bufs["ranges"]), err_msg="ranges")
    if images:
        np.testing.assert_array_equal(_np(a.out_rgb), _np(b.out_rgb))
        np.testing.assert_array_equal(_np(a.out_T), _np(b.out_T))


def _modes(sc, poses, capacity=None, check=True, **opt):
    a = _render(sc, poses, capacity=capacity, sort_mode=1, **opt)
    b = _render(sc, poses, capacity=capacity, sort_mode=2, **opt)
    if check:
        _check_binning(b, sc.n * b.cams.n_views, b.cams)
    _same(a, b)
    return a, b


def test_tiny_scene():
    sc, pose = S.tiny_config()
    _modes(sc, pose)


def test_needles_slivers():
    sc, pose = _needles_config()
    _modes(sc, pose)


def test_enhanced_opacity():
    sc = S.blobs_scene(9, 3000, 1, enhanced=True)
    pose = S.Pose(S.look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), 160, 120)
    _modes(sc, pose)


def test_uneven_resolutions_one_launch():
    sc = S.blobs_scene(23, 5000, 1)
    poses = S.spline_poses(4, 4, resolutions=[(64, 48), (96, 64), (80, 80), (33, 17)])
    _modes(sc, poses)


def test_multiview_over_a_million_instances():
    sc = S.blobs_scene(21, 60_000, 0)
    a, b = _modes(sc, S.spline_poses(3, 3))
    assert a.n_inst > 1_000_000


@pytest.mark.parametrize("views,capacity", [(1, 2048 * 2048), (3, 4096 * 4096 + 12_345)])
def test_large_capacity_scanned_first_pass(views, capacity):
    """Unused capacity: 1024-item emission blocks (one view, about 2M
    instances), and above 4096 radix tiles of capacity (three views, about
    5.7M) 4096-item blocks whose scanned counts replace the first row pass's
    look-back."""
    sc = S.blobs_scene(21, 60_000, 0)
    poses = S.spline_poses(3, 3)[:views]
    a = _render(sc, poses, sort_mode=1)
    b = _render(sc, poses, sort_mode=2, capacity=capacity)
    assert int(_u32(b.bufs["n_inst"])[0]) == a.n_inst < capacity
    n = a.n_inst
    for k in ("keys", "vals"):
        np.testing.assert_array_equal(_np(a.bufs[k])[:n], _np(b.bufs[k])[:n], err_msg=k)
    np.testing.assert_array_equal(_np(a.bufs["ranges"]), _np(b.bufs["ranges"]))
    np.testing.assert_array_equal(_np(a.out_rgb), _np(b.out_rgb))


@pytest.mark.parametrize("views", [6, 24])
def test_two_row_passes_and_the_row_limit(views):
    """Six 720x720 views: 270 global tile rows, so the item sort takes two
    passes over 9 bits; 24 views: 1080 rows, past the 1024-row limit, so
    mode 1 sorts (same results)."""
    sc = S.blobs_scene(5, 20_000 if views == 6 else 3000, 0)
    poses = S.spline_poses(views, views, resolutions=[(720, 720)])
    _modes(sc, poses)


@pytest.mark.parametrize("width", [1000, 2400, 4100])
def test_wide_rows(width):
    """63, 150 and 257 tiles per row; past 256 tiles per row mode 2 falls
    back to mode 1 (same results)."""
    sc = S.blobs_scene(6, 8000, 0)
    pose = S.Pose(S.look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), width, 96)
    _modes(sc, pose)


def test_empty_and_culled():
    pose = S.Pose(S.look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), 40, 24, 60.0, 0.2, (0.1, 0.2, 0.3))
    sc = S.blobs_scene(1, 50, 0)
    a = _render(sc.subset(np.arange(0)), pose, sort_mode=2)
    assert a.n_inst == 0
    assert (_u32(a.bufs["ranges"]) == 0).all()
    behind = sc.subset(np.arange(50))
    behind.mean[2] = 20.0
    b = _render(behind, pose, sort_mode=2)
    assert b.n_inst == 0 and (_u32(b.bufs["ranges"]) == 0).all()
    np.testing.assert_array_equal(_np(b.out_T), 1.0)


def test_capacity_overflow_reports_the_count():
    """A capacity below the instance count: the count is still exact (the
    caller re-runs with it), every range stays within the capacity and
    nothing is written past it."""
    import ctypes as C
    import paper_2605_18334_amd as P
    from paper_2605_18334_amd.raster import _ptr
    sc = S.blobs_scene(21, 60_000, 0)
    poses = S.spline_poses(3, 3)
    full = _render(sc, poses, sort_mode=2)
    o = P.default_options(sort_mode=2)
    gs = P.GaussianSet.from_scene(sc)
    cams = P.CameraBatch.from_poses(poses, o)
    m = sc.n * cams.n_views
    geom, _ = P.raster.preprocess(gs, cams, o)
    cap = full.n_inst // 3
    lib = P.load()
    vals = torch.full((cap + 4096,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    ranges = torch.empty(2 * cams.total_tiles, dtype=torch.int32, device="cuda")
    n_inst = torch.zeros(1, dtype=torch.int32, device="cuda")
    sb = int(lib.sgs_bin_sort_scratch_bytes(m, cap, cams.total_tiles, C.byref(o)))
    scratch = torch.empty(sb, dtype=torch.uint8, device="cuda")
    st = lib.sgs_bin_sort(C.byref(geom), m, cams.host, _ptr(cams.dev), cams.n_views, C.byref(o), cap, None,
                          _ptr(vals), _ptr(ranges), _ptr(n_inst), None, _ptr(scratch), sb, None)
    assert st == 0
    torch.cuda.synchronize()
    assert int(_u32(n_inst)[0]) == full.n_inst
    assert (_u32(vals[cap:]) == 0x5A5A5A5A).all()
    assert (_u32(ranges) <= cap).all()


def test_million_gaussian_frame():
    """The 1M-Gaussian 1600x1064 frame (52M instances, 7.8M row items)."""
    sc, _, pose = S.diff_config()
    a = _render(sc, pose, sort_mode=1)
    b = _render(sc, pose, sort_mode=2)
    _same(a, b)
