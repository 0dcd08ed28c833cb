"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bars: images within 1e-4 max abs per channel on every pixel whose decisions
are not within the oracle's margins; sort keys, values and tile ranges
bit-exact; gradients within 1e-2 relative (per-tensor L2 and per element
where the gradient is not tiny).
"""
import math

import numpy as np
import pytest
import torch

import sgs_synth as S
from gradbar import compare_grads as _compare_grads
from imagebar import check_image_values
from oracle import sgs_oracle as O

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-4


def _P():
    import paper_2605_18334_amd as P
    P.load()
    return P


def _render(sc, poses, capacity=None, **opt):
    P = _P()
    o = P.default_options(**opt)
    gs = P.GaussianSet.from_scene(sc)
    cams = P.CameraBatch.from_poses(poses if isinstance(poses, list) else [poses], o)
    fr = P.render(gs, cams, o, keep_keys=True, capacity=capacity)
    torch.cuda.synchronize()
    return fr


def _np(t):
    return t.detach().cpu().numpy()


def _u32(t):
    return _np(t).view(np.uint32)


def _check_image(fr, ref, v=0, tol=IMG_TOL, max_amb=0.01, extra=None):
    img = _np(fr.image(v)).reshape(3, -1).T
    T = _np(fr.transmittance(v)).reshape(-1)
    return check_image_values(img[ref.pixels], T[ref.pixels], ref, tol, max_amb, extra)


# ------------------------------------------------------------------ stage K1
def _with_culled(sc, pose, k=60, seed=3):
    """The scene plus k Gaussians the extent must cull: a third too faint to
    reach alpha_min anywhere (peak opacity ~ 1e-3), a third beside the view
    (off screen), a third behind the near plane."""
    rng = np.random.default_rng(seed)
    extra = S.blobs_scene(seed, k, sc.sh_degree)
    extra.opa_logit[: k // 3] = -7.0
    extra.mean[0, k // 3: 2 * k // 3] += 30.0
    extra.mean[2, 2 * k // 3:] = rng.uniform(8.0, 12.0, k - 2 * k // 3)   # camera at z = 8 looking at -z
    cat = lambda a, b: None if a is None else np.ascontiguousarray(np.concatenate([a, b], -1))
    return S.Scene(cat(sc.mean, extra.mean), cat(sc.log_scale, extra.log_scale), cat(sc.quat, extra.quat),
                   cat(sc.skew, extra.skew), cat(sc.opa_logit, extra.opa_logit), cat(sc.sh, extra.sh),
                   sc.sh_degree)


def test_preprocess_matches_oracle_projection():
    sc, pose = S.tiny_config()
    sc = _with_culled(sc, pose)
    fr = _render(sc, pose)
    m = sc.n
    rec = _np(fr.bufs["rec"])[:16 * m].reshape(m, 4, 4).transpose(1, 0, 2)   # slot-major view
    tiles = _u32(fr.bufs["tiles"])[:m]
    ref = O.project_numpy(sc, pose)
    on = tiles > 0
    assert on.sum() > 0.5 * m
    assert ref["valid"][on].all()
    np.testing.assert_allclose(rec[0, on, 0], ref["mu2d"][on, 0], atol=2e-3)
    np.testing.assert_allclose(rec[0, on, 1], ref["mu2d"][on, 1], atol=2e-3)
    for k, col in ((0, (0, 2)), (1, (0, 3)), (2, (1, 0))):
        np.testing.assert_allclose(rec[col[0], on, col[1]], ref["conic"][on, k], rtol=2e-4,
                                   atol=2e-6 * np.abs(ref["conic"][on]).max())
    np.testing.assert_allclose(rec[1, on, 3], (ref["rho"] * ref["o1"])[on], rtol=2e-4, atol=1e-7)
    np.testing.assert_allclose(rec[1, on, 1:3], ref["beta2d"][on], rtol=2e-4,
                               atol=2e-5 * np.abs(ref["beta2d"][on]).max())
    np.testing.assert_allclose(rec[2, on, :3], ref["rgb"][on], atol=2e-6)
    # the depth key: the same float32 fma expression on both sides
    gd = _np(fr.bufs["depth"])[:m][on]
    rd = ref["z32"][on].astype(np.float32)
    ulps = np.abs(gd.view(np.int32).astype(np.int64) - rd.view(np.int32).astype(np.int64))
    print(f"depth keys: {int((ulps == 0).sum())} of {len(ulps)} bit-identical, max {int(ulps.max())} ulp", flush=True)
    assert ulps.max() <= 1 and (ulps == 0).mean() > 0.999
    # records the GPU culls (valid for the oracle, no tiles) reach alpha_min
    # at no pixel of the image: alpha~ stays below 1/255 everywhere
    off = np.nonzero(ref["valid"] & ~on)[0]
    assert len(off) >= 40          # the faint and the off-screen ones at least
    cam = O.camera_from_pose(pose)
    with torch.no_grad():
        pr = O.project(O.to_tensors(sc), 0, cam)
        _, pc = O.pixel_centres(cam, None)
        peak = O.alpha_tilde(pc, pr, torch.from_numpy(off), O.Options()).max(0).values.numpy()
    assert (np.minimum(peak, 0.99) < (1 / 255) * (1 + 1e-4)).all(), peak.max()
    # zero-skew Gaussians project to exactly zero 2D skew
    zero = (sc.skew == 0).all(0) & on
    assert zero.sum() > 0 and (rec[1, zero, 1:3] == 0).all()


# ------------------------------------------------------------------ K2-K4
def _check_binning(fr, m, cams):
    """The sorted instance list is exactly a stable sort of the emitted
    (record, tile) set: keys = (tile << 32 | depth bits of the record), keys
    non-decreasing, equal keys in ascending record order; each record emits
    tiles[record] distinct tiles, all inside its rect; ranges match keys."""
    n = int(_u32(fr.bufs["n_inst"])[0])
    assert n <= fr.n_inst          # the capacity
    keys = _np(fr.bufs["keys"])[:n].view(np.uint64)
    vals = _u32(fr.bufs["vals"])[:n]
    rect = _u32(fr.bufs["rect"])[:2 * m].reshape(m, 2)
    tiles = _u32(fr.bufs["tiles"])[:m]
    depth = _np(fr.bufs["depth"])[:m].view(np.uint32).astype(np.uint64)
    tile = (keys >> np.uint64(32)).astype(np.int64)
    assert n == int(tiles.astype(np.int64).sum())
    np.testing.assert_array_equal(keys & np.uint64(0xffffffff), depth[vals])
    assert (keys[1:] >= keys[:-1]).all()
    eq = keys[1:] == keys[:-1]
    assert (vals[1:][eq] > vals[:-1][eq]).all()
    np.testing.assert_array_equal(np.bincount(vals, minlength=m), tiles)
    pair = vals.astype(np.int64) * (1 << 32) + tile
    assert len(np.unique(pair)) == n
    nper = m // cams.n_views
    for v in range(cams.n_views):
        c = cams.view(v)
        sel = (vals // nper) == v
        lt = tile[sel] - c.tile_base
        tx, ty = lt % c.tiles_x, lt // c.tiles_x
        r = rect[vals[sel]]
        assert ((tx >= (r[:, 0] & 0xffff)) & (tx < (r[:, 1] & 0xffff)) &
                (ty >= (r[:, 0] >> 16)) & (ty < (r[:, 1] >> 16))).all()
    ranges = _u32(fr.bufs["ranges"]).reshape(-1, 2)
    starts = np.searchsorted(tile, np.arange(cams.total_tiles), "left")
    ends = np.searchsorted(tile, np.arange(cams.total_tiles), "right")
    has = ends > starts
    np.testing.assert_array_equal(ranges[has, 0], starts[has])
    np.testing.assert_array_equal(ranges[has, 1], ends[has])
    assert (ranges[~has, 0] == ranges[~has, 1]).all()


@pytest.mark.parametrize("mode", [0, 1])
def test_bin_sort_bit_exact(mode):
    sc, pose = S.tiny_config()
    fr = _render(sc, pose, sort_mode=mode)
    _check_binning(fr, sc.n, fr.cams)


def test_sort_modes_agree_on_large_multiview_input():
    sc = S.blobs_scene(21, 60_000, 0)
    poses = S.spline_poses(3, 3)
    a = _render(sc, poses, sort_mode=0)
    b = _render(sc, poses, sort_mode=1)
    _check_binning(b, sc.n * 3, b.cams)
    n = a.n_inst
    assert n == b.n_inst and n > 1_000_000
    np.testing.assert_array_equal(_np(a.bufs["keys"])[:n], _np(b.bufs["keys"])[:n])
    np.testing.assert_array_equal(_np(a.bufs["vals"])[:n], _np(b.bufs["vals"])[:n])
    np.testing.assert_array_equal(_np(a.bufs["ranges"]), _np(b.bufs["ranges"]))
    k = _np(a.bufs["keys"])[:n].view(np.uint64)
    assert (k[1:] >= k[:-1]).all()


@pytest.mark.parametrize("case", ["tiny", "multiview", "near0"])
def test_depth_digit_widths_give_identical_sorts(case):
    """The depth presort with 10-bit digits (3 passes over keys shifted
    by the near plane's bits to 30 bits) equals the 8-bit one (4 passes over
    the raw bits) bit for bit, and both equal the CPU stable sort; with a
    near plane at 0 the library falls back to 8-bit digits."""
    if case == "multiview":
        sc, poses = S.blobs_scene(21, 60_000, 0), S.spline_poses(3, 3)
    else:
        sc, pose = S.tiny_config()
        poses = [pose] if case == "tiny" else [S.Pose(pose.c2w_gl, pose.width, pose.height, pose.fovx_deg, 0.0)]
    a = _render(sc, poses, depth_digit_bits=8)
    b = _render(sc, poses, depth_digit_bits=10)
    _check_binning(b, sc.n * len(poses), b.cams)
    n = a.n_inst
    assert n == b.n_inst
    for k in ("keys", "vals", "ranges"):
        np.testing.assert_array_equal(_np(a.bufs[k])[:n] if k != "ranges" else _np(a.bufs[k]),
                                      _np(b.bufs[k])[:n] if k != "ranges" else _np(b.bufs[k]))
    np.testing.assert_array_equal(_np(a.out_rgb), _np(b.out_rgb))


@pytest.mark.parametrize("views,capacity", [(1, 2048 * 2048), (3, 4096 * 4096 + 12_345)])
def test_large_capacity_sort_is_identical(views, capacity):
    """Unused capacity is a long empty tail of the sort.  One view (about 2M
    instances) runs 1024-instance expansion blocks both ways; three views
    (about 5.7M) run them at the exact capacity, and at the larger capacity
    (above 4096 radix tiles of 4096 keys) 4096-instance blocks whose scanned
    first-digit counts replace the first pass's look-back.  Keys, values,
    ranges and the images equal the exact-capacity run."""
    sc = S.blobs_scene(21, 60_000, 0)
    poses = S.spline_poses(3, 3)[:views]
    a = _render(sc, poses, sort_mode=1)
    b = _render(sc, poses, sort_mode=1, capacity=capacity)
    n = a.n_inst
    assert int(_u32(b.bufs["n_inst"])[0]) == n and 100_000 < n < capacity
    _check_binning(b, sc.n * views, b.cams)
    np.testing.assert_array_equal(_np(a.bufs["keys"])[:n], _np(b.bufs["keys"])[:n])
    np.testing.assert_array_equal(_np(a.bufs["vals"])[:n], _np(b.bufs["vals"])[:n])
    np.testing.assert_array_equal(_np(a.bufs["ranges"]), _np(b.bufs["ranges"]))
    for v in range(views):
        np.testing.assert_array_equal(_np(a.image(v)), _np(b.image(v)))


def _needles_config(seed=7, n=400):
    """Long thin Gaussians (one axis 0.8-2.5, the others 0.004) at random
    orientations, high opacity, mostly small skew: their screen ellipses are
    slivers a few hundred pixels long, whose row extents and per-block
    x-ranges are far from the centre and of either sign."""
    sc = S.blobs_scene(seed, n, 0)
    rng = np.random.default_rng(seed + 100)
    sc.log_scale[:] = np.log(0.004)
    sc.log_scale[0] = np.log(rng.uniform(0.8, 2.5, n)).astype(np.float32)
    sc.opa_logit[:] = rng.uniform(1.0, 5.0, n).astype(np.float32)
    sc.skew[:] *= np.float32(0.02)
    return sc, S.Pose(S.look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), 256, 192)


@pytest.mark.parametrize("case", ["tiny", "needles"])
def test_extent_is_conservative(case):
    """Every (Gaussian, pixel) pair the oracle lets through (alpha above
    1/255 by a margin) has its (Gaussian, tile) instance in the sorted list."""
    sc, pose = S.tiny_config() if case == "tiny" else _needles_config()
    fr = _render(sc, pose)
    n = fr.n_inst
    keys = _np(fr.bufs["keys"])[:n].view(np.uint64)
    vals = _u32(fr.bufs["vals"])[:n].astype(np.int64)
    emitted = set((vals * (1 << 32) + (keys >> np.uint64(32)).astype(np.int64)).tolist())
    cam = O.camera_from_pose(pose)
    tx_n = (cam.W + 15) // 16
    with torch.no_grad():
        pr = O.project(O.to_tensors(sc), 0, cam)
        pix, pc = O.pixel_centres(cam, None)
        idx = torch.nonzero(pr.valid).flatten()
        bad = checked = 0
        for s in range(0, len(pix), 2048):
            at = O.alpha_tilde(pc[s:s + 2048], pr, idx, O.Options()).numpy()
            pp, gg = np.nonzero(at >= (1 / 255) * (1 + 1e-6))
            g = idx.numpy()[gg].astype(np.int64)
            t = (pix[s + pp] // cam.W // 16) * tx_n + (pix[s + pp] % cam.W) // 16
            for key in (g * (1 << 32) + t).tolist():
                checked += 1
                bad += key not in emitted
    assert checked > 10000 and bad == 0


# ------------------------------------------------------------------ images
@pytest.mark.parametrize("split", [0, 1 << 20])
def test_needles_image_matches_oracle(split):
    """Sliver-shaped ellipses against the oracle on every pixel, with whole
    tiles and with every tile split into quarters (4x4 wave blocks)."""
    sc, pose = _needles_config()
    fr = _render(sc, pose, split_tiles=split)
    ref = O.render(sc, pose)
    # float32 storage of the records moves alpha by up to a few ulps of the
    # exponent's terms, ~1e4 times the exponent along these slivers: the
    # tolerance adds the first-order effect of that on each pixel
    bound = O.float32_error_bound(sc, pose)
    assert bound[0].max() < 1e-3 and bound[1].max() < 1e-3
    _check_image(fr, ref, max_amb=0.02, extra=bound)


@pytest.mark.parametrize("mode", [0, 1])
def test_tiny_image_matches_oracle(mode):
    sc, pose = S.tiny_config()
    fr = _render(sc, pose, sort_mode=mode)
    ref = O.render(sc, pose)
    _check_image(fr, ref)
    # the last contributor of each pixel is the oracle's
    last = _u32(fr.out_last)
    vals = _u32(fr.bufs["vals"])
    ranges = _u32(fr.bufs["ranges"]).reshape(-1, 2)
    W = pose.width
    for p in np.nonzero(~ref.ambiguous)[0][::7]:
        pix = ref.pixels[p]
        t = (pix // W // 16) * ((W + 15) // 16) + (pix % W) // 16
        got = vals[ranges[t, 0] + last[pix] - 1] if last[pix] else -1
        assert got == ref.last[p]


@pytest.mark.parametrize("tile,batch", [((16, 8), 256), ((8, 8), 64), ((16, 16), 128), ((16, 16), 64)])
def test_tile_shapes_and_batches_give_identical_images(tile, batch):
    sc, pose = S.tiny_config()
    a = _render(sc, pose)
    b = _render(sc, pose, tile_w=tile[0], tile_h=tile[1], blend_batch=batch)
    np.testing.assert_array_equal(_np(a.out_rgb), _np(b.out_rgb))
    np.testing.assert_array_equal(_np(a.out_T), _np(b.out_T))


@pytest.mark.parametrize("case", ["tiny", "ragged_enhanced", "small_many"])
@pytest.mark.parametrize("tile,batch,sched", [((16, 16), 0, "split"), ((16, 16), 64, "order"),
                                              ((16, 16), 256, "persistent"), ((16, 8), 0, "order"),
                                              ((8, 8), 128, "none")])
def test_blend_lists_give_identical_outputs(case, tile, batch, sched):
    """Quarter lists (blend_lists 4) and wave lists (1) give every pixel the
    same records in the same order: colour, transmittance, last contributor
    and composited count agree bit for bit, for each tile shape, batch size
    and tile schedule (split tiles, a tile order, the persistent queue)."""
    P = _P()
    if case == "tiny":
        sc, pose = S.tiny_config()
    elif case == "ragged_enhanced":
        sc = S.blobs_scene(13, 1500, 1, enhanced=True)
        pose = S.Pose(S.look_at_gl((0.5, 0.3, 7.0), up=(0, 1, 0)), 97, 45)
    else:   # many small Gaussians: short quarter lists, several batches per tile
        sc = S.clusters_scene(21, 20000, 0)
        pose = S.Pose(S.look_at_gl((0.0, 0.0, 15.0), up=(0, 1, 0)), 160, 120)
    gs = P.GaussianSet.from_scene(sc)
    out = []
    for ql in (1, 4):
        o = P.default_options(tile_w=tile[0], tile_h=tile[1], blend_batch=batch, blend_lists=ql,
                              split_tiles=-1 if sched == "split" else 0)
        R = P.Renderer(gs, P.CameraBatch.from_poses([pose], o), o, count=True,
                       tile_order=sched != "none", persistent=sched == "persistent")
        R.forward()
        torch.cuda.synchronize()
        out.append([_np(x).copy() for x in (R.out_rgb, R.out_T, R.out_last, R.bufs["count"])])
    assert int(out[0][3].sum()) > 0
    for x, y in zip(*out):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("case", ["tiny", "ragged_enhanced"])
@pytest.mark.parametrize("split", [1, 5, 1 << 20])
def test_split_tiles_give_identical_outputs(case, split):
    """Heavy tiles blended as quarters with four lanes per pixel give the
    same colour, transmittance, last contributor and count, bit for bit."""
    P = _P()
    if case == "tiny":
        sc, pose = S.tiny_config()
    else:
        sc = S.blobs_scene(13, 1500, 1, enhanced=True)
        pose = S.Pose(S.look_at_gl((0.5, 0.3, 7.0), up=(0, 1, 0)), 97, 45)
    gs = P.GaussianSet.from_scene(sc)
    out, grads = [], []
    dL = None
    for st in (0, split):
        o = P.default_options(split_tiles=st)
        R = P.Renderer(gs, P.CameraBatch.from_poses([pose], o), o, tile_order=True, count=True)
        R.forward()
        torch.cuda.synchronize()
        # (the evaluated-pair counter is a work count: the quarters evaluate
        # up to three records past a pixel's stop, so it is not compared)
        out.append([_np(x).copy() for x in (R.out_rgb, R.out_T, R.out_last, R.bufs["count"])])
        if dL is None:
            dL = torch.from_numpy(np.random.default_rng(3).normal(size=tuple(R.out_rgb.shape))
                                  .astype(np.float32)).cuda()
        g = R.backward(dL)
        torch.cuda.synchronize()
        grads.append({k: _np(v).astype(np.float64) for k, v in g.items() if v is not None and k != "g2d"})
    for x, y in zip(*out):
        np.testing.assert_array_equal(x, y)
    # the backward sums per-pixel terms in another order: equal up to rounding
    for k, v in grads[0].items():
        np.testing.assert_allclose(grads[1][k], v, rtol=1e-4, atol=1e-6 * np.abs(v).max(), err_msg=k)


def test_zero_skew_is_bit_identical_to_symmetric_path():
    sc, pose = S.tiny_config()
    sc.skew[:] = 0.0
    a = _render(sc, pose)
    sym = S.Scene(sc.mean, sc.log_scale, sc.quat, None, sc.opa_logit, sc.sh, sc.sh_degree)
    b = _render(sym, pose)
    np.testing.assert_array_equal(_np(a.out_rgb), _np(b.out_rgb))
    np.testing.assert_array_equal(_np(a.out_T), _np(b.out_T))
    ref = O.render(sym, pose, opt=O.Options(symmetric=True))
    _check_image(b, ref)


def test_enhanced_opacity_image_matches_oracle():
    sc = S.blobs_scene(13, 1500, 1, enhanced=True)
    pose = S.tiny_config()[1]
    fr = _render(sc, pose)
    _check_image(fr, O.render(sc, pose))


def test_single_skewed_gaussian_matches_closed_form_tightly():
    """One strongly skewed Gaussian in front of the camera: the skew argument
    z spans about +-4 over the footprint, so the device 1 + erf(z) is checked
    against the FP64 oracle over its whole range (bound 1.5e-7 for the
    Abramowitz-Stegun formula, plus float32 rounding)."""
    pose = S.Pose(np.diag([1.0, -1.0, -1.0, 1.0]), 64, 64, 60.0, 0.2)
    q = np.array([[1.0], [0.0], [0.0], [0.0]], np.float32)
    sc = S.Scene(np.array([[0.05], [-0.02], [5.0]], np.float32),
                 np.array([[math.log(0.12)], [math.log(0.09)], [math.log(0.1)]], np.float32), q,
                 np.array([[25.0], [-14.0], [3.0]], np.float32), np.array([-0.5], np.float32),
                 np.array([[[0.4]], [[0.1]], [[-0.3]]], np.float32).reshape(1, 3, 1), 0)
    fr = _render(sc, pose)
    ref = O.render(sc, pose)
    img = _np(fr.image(0)).reshape(3, -1).T
    ok = ~ref.ambiguous
    assert ok.mean() > 0.99
    assert np.abs(img - ref.color)[ok].max() <= 2e-6
    pr = O.project_numpy(sc, pose)
    assert np.abs(pr["beta2d"][0]).max() * 12 > 4 * math.sqrt(2)   # |z| reaches ~4 in the footprint


def test_ragged_image_and_background():
    sc = S.blobs_scene(17, 800, 2)
    pose = S.Pose(S.look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), 97, 45, 60.0, 0.2, (0.2, 0.5, 0.9))
    fr = _render(sc, pose)
    _check_image(fr, O.render(sc, pose))


def test_empty_and_fully_culled_scenes():
    pose = S.Pose(S.look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), 40, 24, 60.0, 0.2, (0.1, 0.2, 0.3))
    sc = S.blobs_scene(1, 50, 0)
    empty = sc.subset(np.arange(0))
    fr = _render(empty, pose)
    img = _np(fr.image(0))
    np.testing.assert_allclose(img, np.broadcast_to(np.array([0.1, 0.2, 0.3], np.float32)[:, None, None], img.shape))
    behind = sc.subset(np.arange(50))
    behind.mean[2] = 20.0           # all behind the camera at z = 8 looking at -z
    fr = _render(behind, pose)
    assert fr.n_inst == 0
    np.testing.assert_array_equal(_np(fr.out_T), 1.0)


def test_multiview_batch_equals_single_views():
    sc = S.blobs_scene(23, 5000, 1)
    poses = S.spline_poses(4, 4, resolutions=[(64, 48), (96, 64), (80, 80), (33, 17)])
    batch = _render(sc, poses)
    for v, p in enumerate(poses):
        single = _render(sc, p)
        np.testing.assert_array_equal(_np(batch.image(v)), _np(single.image(0)))


# ------------------------------------------------------------------ gradients
def _grad_check(sc, pose, pixels=None, seed=0, rtol=1e-2, split=None):
    """split=None: render() and render_backward() (no tile order); else a
    Renderer with the tile order and that split_tiles (the launch
    configuration of the benchmark, default 256-record backward batches)."""
    P = _P()
    o = P.default_options() if split is None else P.default_options(split_tiles=split)
    gs = P.GaussianSet.from_scene(sc)
    cams = P.CameraBatch.from_poses([pose], o)
    Pn = pose.width * pose.height
    rng = np.random.default_rng(seed)
    g = np.zeros((3, Pn), np.float32)
    sel = np.arange(Pn) if pixels is None else pixels
    g[:, sel] = rng.normal(size=(3, len(sel))).astype(np.float32)
    if split is None:
        fr = P.render(gs, cams, o)
        grads = P.render_backward(fr, torch.from_numpy(g).cuda())
    else:
        R = P.Renderer(gs, cams, o, tile_order=True)
        R.forward()
        grads = R.backward(torch.from_numpy(g).cuda())
        torch.cuda.synchronize()
        assert not R.overflowed()
    ref = O.render_grad(sc, pose, g[:, sel].T.astype(np.float64), sel)
    return _compare_grads({k: _np(grads[k]) for k in ref}, ref, rtol, label=f"grad(split={split})")


def test_gradients_match_oracle_subscene():
    """64-Gaussian 64x64 subscene (blobs generator, SH3), L = sum g . C."""
    sc = S.blobs_scene(4, 64, 3)
    pose = S.Pose(S.look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), 64, 64)
    _grad_check(sc, pose)


def test_gradients_match_oracle_tiny_scene_with_background():
    sc = S.blobs_scene(31, 600, 2)
    pose = S.Pose(S.look_at_gl((1.0, 2.0, 7.0), up=(0, 1, 0)), 72, 56, 55.0, 0.2, (0.3, 0.1, 0.6))
    _grad_check(sc, pose, seed=3)


@pytest.mark.parametrize("split", [1 << 20, -1])
def test_gradients_match_oracle_through_the_tile_order(split):
    """The benchmark's launch configuration (tile order, split tiles, 256-
    record backward batches) against the oracle: every tile split into
    quarters (four lanes per pixel), and the default split count."""
    sc = S.blobs_scene(31, 600, 2)
    pose = S.Pose(S.look_at_gl((1.0, 2.0, 7.0), up=(0, 1, 0)), 72, 56, 55.0, 0.2, (0.3, 0.1, 0.6))
    _grad_check(sc, pose, seed=5, split=split)


def test_gradients_match_oracle_enhanced_opacity():
    sc = S.blobs_scene(9, 300, 1, enhanced=True)
    pose = S.Pose(S.look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), 64, 64)
    _grad_check(sc, pose, seed=2)


def _densify_check(sc, poses, seed, rtol=1e-2):
    """Densification statistics fused into the backward, over a batch of
    views, against the oracle's per-view statistics: uv sums over the views,
    z is the maximum, count the number of views that see the Gaussian."""
    P = _P()
    o = P.default_options()
    gs = P.GaussianSet.from_scene(sc)
    cams = P.CameraBatch.from_poses(poses, o)
    fr = P.render(gs, cams, o)
    Pt = sum(p.width * p.height for p in poses)
    g = np.random.default_rng(seed).normal(size=(3, Pt)).astype(np.float32)
    st = P.densify_stats(gs)
    P.render_backward(fr, torch.from_numpy(g).cuda(), densify=st)
    uv, z, cnt = (_np(st[k]).astype(np.float64) for k in ("uv", "z", "count"))
    ref_uv = np.zeros(sc.n)
    ref_z = np.zeros(sc.n)
    reach = np.zeros(sc.n, np.int64)
    valid = np.zeros(sc.n, np.int64)
    base = 0
    for p in poses:
        n_p = p.width * p.height
        r = O.densify_stats(sc, p, g[:, base:base + n_p].T.astype(np.float64))
        base += n_p
        ref_uv += np.where(r["valid"], r["uv"], 0.0)
        ref_z = np.maximum(ref_z, r["z"])
        reach += r["reach"]
        valid += r["valid"]
    # counts: every view where alpha reaches 1/255 sees the Gaussian (the
    # extent is conservative); a view sees only Gaussians it does not cull
    assert (cnt >= reach).all() and (cnt <= valid).all()
    assert (cnt > 0).sum() >= 10
    for name, gv, rv in (("uv", uv, ref_uv), ("z", z, ref_z)):
        rel = np.linalg.norm(gv - rv) / max(np.linalg.norm(rv), 1e-30)
        assert rel <= rtol, (name, rel)
        big = rv > 1e-2 * rv.max()
        e = np.abs(gv - rv)[big] / rv[big]
        assert np.quantile(e, 0.99) <= 5 * rtol, (name, np.quantile(e, 0.99))
    return st


def test_densify_stats_match_oracle_one_view():
    sc = S.blobs_scene(4, 64, 3)
    _densify_check(sc, [S.Pose(S.look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), 64, 48)], seed=7)


def test_densify_stats_accumulate_over_views():
    sc = S.blobs_scene(31, 400, 2)
    poses = [S.Pose(S.look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), 64, 48),
             S.Pose(S.look_at_gl((3.0, 1.0, 7.0), up=(0, 1, 0)), 40, 56)]
    st = _densify_check(sc, poses, seed=8)
    assert int(_np(st["count"]).max()) == 2


def test_autograd_function_matches_direct_backward():
    P = _P()
    sc = S.blobs_scene(4, 200, 1)
    pose = S.Pose(S.look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), 48, 40)
    o = P.default_options()
    cams = P.CameraBatch.from_poses([pose], o)
    gs = P.GaussianSet.from_scene(sc)
    leaves = {f: getattr(gs, f).clone().requires_grad_(True) for f in ("mean", "log_scale", "quat", "skew", "opa_logit", "sh")}
    img = P.rasterize(leaves["mean"], leaves["log_scale"], leaves["quat"], leaves["skew"],
                      leaves["opa_logit"], leaves["sh"], cams, o)
    target = torch.full_like(img, 0.3)
    loss = (img - target).abs().mean()
    loss.backward()
    fr = P.render(gs, cams, o)
    dL = torch.sign(fr.out_rgb - target) / img.numel()
    g = P.render_backward(fr, dL)
    for k, v in leaves.items():
        torch.testing.assert_close(v.grad, g[k], rtol=1e-5, atol=1e-7)


def test_autograd_gradient_matches_central_differences_of_gpu_forward():
    """Directional central differences of the FP32 GPU forward against the
    gradient of the autograd Function, for every parameter kind.  alpha_min
    and t_min are set near zero so that the image is continuous in the
    parameters (the skip and stop cut-offs of compositing otherwise make it
    jump), and the means move only across the view, which leaves every
    depth, and with it the compositing order, bit-unchanged for this
    axis-aligned camera.  What remains are the kinks of the alpha and colour
    clamps, whose effect on a central difference is of order h."""
    P = _P()
    sc = S.blobs_scene(4, 200, 1)
    W_, H_ = 48, 40
    pose = S.Pose(S.look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), W_, H_)
    o = P.default_options(alpha_min=1e-7, t_min=1e-9)
    cams = P.CameraBatch.from_poses([pose], o)
    gs = P.GaussianSet.from_scene(sc)
    names = ("mean", "log_scale", "quat", "skew", "opa_logit", "sh")
    base = {f: getattr(gs, f).clone() for f in names}
    w = torch.from_numpy(np.random.default_rng(21).normal(size=(3, W_ * H_))).cuda()

    def loss(p):
        with torch.no_grad():
            img = P.rasterize(*(p[f] for f in names), cams, o)
            return float((img.double() * w).sum())

    leaves = {f: v.clone().requires_grad_(True) for f, v in base.items()}
    img = P.rasterize(*(leaves[f] for f in names), cams, o)
    (img.double() * w).sum().backward()
    rng = np.random.default_rng(22)
    h = 4e-3
    for f in names:
        u = torch.from_numpy(rng.normal(size=tuple(base[f].shape)).astype(np.float32)).cuda()
        if f == "mean":
            u[2] = 0.0          # world z is the camera's depth axis here
        xp, xm = base[f] + h * u, base[f] - h * u
        fd = (loss({**base, f: xp}) - loss({**base, f: xm})) / (2 * h)
        an = float((leaves[f].grad.double() * (xp - xm).double()).sum()) / (2 * h)
        print(f"{f}: central difference {fd:.6f}, adjoint {an:.6f}", flush=True)
        assert abs(an) > 0.1, (f, an)
        assert abs(fd - an) <= 1e-2 * abs(an) + 1e-2, (f, fd, an)
