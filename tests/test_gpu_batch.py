"""GPU checks of the batched form: schedules, HIP-graph replay, launch
groups and the autotuner all give images bit-identical to the plain
single-view path."""
import json
import os

import numpy as np
import pytest
import torch

import sgs_synth as S

pytestmark = pytest.mark.gpu


def _P():
    import paper_2605_18334_amd as P
    P.load()
    return P


def _scene():
    return S.blobs_scene(41, 20_000, 1)


def _poses():
    return S.spline_poses(7, 5, resolutions=[(96, 64), (160, 120), (64, 64), (131, 77)])


def _len_bucket(n: int) -> int:
    """Quarter-octave length bucket of the documented tile order (0: empty)."""
    if n == 0:
        return 0
    lg = n.bit_length() - 1
    frac = (n >> (lg - 2)) & 3 if lg >= 2 else (n << (2 - lg)) & 3
    return min(127, 1 + 4 * lg + frac)


@pytest.mark.parametrize("order,persistent", [(True, False), (False, True), (True, True)])
def test_schedules_give_identical_images_and_gradients(order, persistent):
    P = _P()
    gs = P.GaussianSet.from_scene(_scene())
    o = P.default_options()
    cams = P.CameraBatch.from_poses(_poses(), o)
    a = P.Renderer(gs, cams, o, tile_order=False)
    b = P.Renderer(gs, cams, o, tile_order=order, persistent=persistent)
    ra, rb = a.forward().clone(), b.forward().clone()
    torch.cuda.synchronize()
    assert torch.equal(ra, rb)
    assert torch.equal(a.out_T, b.out_T)
    dL = torch.randn_like(ra)
    ga = {k: (None if v is None else v.clone()) for k, v in a.backward(dL).items()}
    gb = b.backward(dL)
    for k, v in ga.items():
        if v is None or k == "g2d":
            continue
        torch.testing.assert_close(gb[k], v, rtol=1e-4, atol=1e-6 * float(v.abs().max()))
    if order:
        to = b.bufs["tile_order"].cpu().numpy()
        assert sorted(to.tolist()) == list(range(cams.total_tiles))
        rg = b.bufs["ranges"].cpu().numpy().view(np.uint32).reshape(-1, 2)
        bk = np.array([_len_bucket(int(n)) for n in (rg[:, 1] - rg[:, 0])[to]])
        assert (bk[:-1] >= bk[1:]).all()


def test_graph_replays_match_eager_renders():
    """Replays (with eager work and a pose change between them) equal the
    eager render of the same state, bit for bit."""
    P = _P()
    gs = P.GaussianSet.from_scene(_scene())
    o = P.default_options()
    poses = _poses()
    cams = P.CameraBatch.from_poses(poses, o)
    R = P.Renderer(gs, cams, o, tile_order=True, persistent=True, headroom=2.0)
    ref = R.forward().clone()
    R.capture()
    other = P.Renderer(P.GaussianSet.from_scene(S.blobs_scene(5, 3000, 0)),
                       P.CameraBatch.from_poses([poses[0]], o), o)
    for k in range(3):
        other.forward()                       # eager work between replays
        torch.cuda.synchronize()
        out = R.replay().clone()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {k}"
    # move every camera a little, same layout: replay == fresh eager render
    moved = [S.Pose(p.c2w_gl @ np.array([[1, 0, 0, 0.05], [0, 1, 0, -0.03], [0, 0, 1, 0.02], [0, 0, 0, 1.0]]),
                    p.width, p.height, p.fovx_deg, p.near) for p in poses]
    for v, p in enumerate(moved):
        cams.host[v] = P.CameraBatch.camera_from_pose(p)
    import ctypes
    P.load().sgs_camera_layout(cams.host, cams.n_views, ctypes.byref(o), None, None)
    cams.upload()
    out = R.replay().clone()
    assert not R.overflowed()
    fresh = P.Renderer(gs, P.CameraBatch.from_poses(moved, o), o)
    assert torch.equal(out, fresh.forward())


def test_batch_renderer_groups_and_graph_match_single_views():
    P = _P()
    from paper_2605_18334_amd.batch import BatchRenderer, LaunchConfig
    sc = _scene()
    gs = P.GaussianSet.from_scene(sc)
    poses = _poses()
    br = BatchRenderer(gs, poses, LaunchConfig(16, 8, 128, 1, True, True, 2))
    br.capture()
    br.replay()
    torch.cuda.synchronize()
    o = P.default_options()
    for v, p in enumerate(poses):
        r = P.Renderer(gs, P.CameraBatch.from_poses([p], o), o)
        r.forward()
        assert torch.equal(br.image(v), r.image(0)), v


def test_autotune_picks_a_config_with_identical_images(tmp_path, monkeypatch):
    P = _P()
    from paper_2605_18334_amd.batch import BatchRenderer, LaunchConfig, autotune
    monkeypatch.setenv("SGS_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    gs = P.GaussianSet.from_scene(_scene())
    poses = _poses()
    cands = [LaunchConfig(16, 16, 256, 1, False, False, 5), LaunchConfig(8, 8, 64, 1, True, True, 2)]
    cfg, timings = autotune(gs, poses, candidates=cands, reps=2)
    assert cfg in cands and len(timings) == 2
    cached = json.load(open(tmp_path / "tune.json"))
    assert len(cached) == 1
    again, _ = autotune(gs, poses, candidates=cands)
    assert again == cfg
    a = BatchRenderer(gs, poses, cfg)
    b = BatchRenderer(gs, poses, LaunchConfig())
    a.forward()
    b.forward()
    for v in range(len(poses)):
        assert torch.equal(a.image(v), b.image(v))


def test_server_image_is_the_same_alone_and_in_the_mix():
    """A served request renders the same image alone and batched with other
    requests of both scenes under continuous batching (bitwise), and equal to
    the plain single-view render."""
    P = _P()
    from paper_2605_18334_amd.serve import GpuBackend, RenderServer, Request
    scA = S.blobs_scene(51, 30_000, 1)
    scB = S.clusters_scene(52, 20_000, 1, zero_skew=True)
    be = GpuBackend({"A": scA, "B": scB})
    target = S.Pose(S.look_at_gl((1.0, -7.0, 2.0)), 200, 150)
    srv = RenderServer(be, budget_bytes=4 << 30, max_batch=4, max_inflight=2)
    srv.start()
    alone = srv.submit(Request("A", target)).result(timeout=120).image.clone()
    import numpy as np
    rng = np.random.default_rng(3)
    futs = []
    for i in range(12):
        sc = "AB"[i % 2]
        p = S.Pose(S.look_at_gl(rng.normal(size=3) * 3 + np.array([0, -8.0, 0])), int(rng.integers(60, 220)),
                   int(rng.integers(40, 160)))
        futs.append(srv.submit(Request(sc, p)))
        if i == 5:
            mixed = srv.submit(Request("A", target))
    srv.stop(drain=True)
    assert all(f.done() and f.exception() is None for f in futs)
    res = mixed.result(timeout=0)
    assert res.batch_size >= 1
    assert torch.equal(res.image, alone)
    o = P.default_options()
    r = P.Renderer(P.GaussianSet.from_scene(scA), P.CameraBatch.from_poses([target], o), o)
    r.forward()
    assert torch.equal(r.image(0).cpu(), alone)
    assert max(x.batch_size for x in srv.results) > 1
