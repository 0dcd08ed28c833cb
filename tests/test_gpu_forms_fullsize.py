"""Oracle parity of the batched and served forms at their benchmark sizes,
against FP64 oracle values stored by tests/golden/make_oracle_samples.py
(only the seeded generators and the oracle; minutes per workload on the CPU).

  * the 16-view batch of 3M skew Gaussians (mixed resolutions), rendered as
    the benchmark does (BatchRenderer, launch groups of 4 views, one HIP
    graph): 1024 seeded pixels of views 0 and 9;
  * served requests on the resident 5M skew and 2M zero-skew scenes: two
    seeded requests per scene, each served alone and in a mix with other
    requests of both scenes; the served images equal, bit for bit, a plain
    single-view render of the same request, whose image and transmittance
    match the oracle at 512 seeded pixels."""
import importlib.util
import os
import types

import numpy as np
import pytest
import torch

import sgs_synth as S
from imagebar import check_image_values

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    return np.load(os.path.join(GOLD, name), allow_pickle=False)


def _ref(g, prefix):
    return types.SimpleNamespace(**{k: g[f"{prefix}_{k}"] for k in
                                    ("pixels", "color", "T", "ambiguous", "alt_start", "alt_rows")})


def _requests():
    spec = importlib.util.spec_from_file_location("mos", os.path.join(GOLD, "make_oracle_samples.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.serve_requests()


def test_batch16_3m_views_match_oracle():
    import paper_2605_18334_amd as P
    from paper_2605_18334_amd.batch import BatchRenderer, LaunchConfig
    g = _golden("batch16_3m_2views_1024px.npz")
    sc, poses = S.batch_config()
    gs = P.GaussianSet.from_scene(sc)
    del sc
    br = BatchRenderer(gs, poses, LaunchConfig(16, 16, 0, -1, True, False, 4))
    br.capture()
    br.replay()
    torch.cuda.synchronize()
    assert not br.overflowed()
    for v in g["views"]:
        v = int(v)
        ref = _ref(g, f"v{v}")
        gi, k = br.view_of[v]
        img = br.groups[gi].image(k).cpu().numpy().reshape(3, -1).T
        T = br.groups[gi].transmittance(k).cpu().numpy().reshape(-1)
        check_image_values(img[ref.pixels], T[ref.pixels], ref, max_amb=0.1)


def test_served_requests_match_oracle_alone_and_in_a_mix():
    import paper_2605_18334_amd as P
    from paper_2605_18334_amd.serve import GpuBackend, RenderServer, Request
    g = _golden("serve_5m2m_4requests_512px.npz")
    reqs = _requests()
    assert len(reqs) == int(g["n"])
    scA, scB = S.serve_scenes()
    be = GpuBackend({"A": scA, "B": scB})
    del scA, scB
    alone = []
    srv = RenderServer(be, budget_bytes=64 << 30, max_batch=1, max_inflight=1)
    srv.start()
    for name, pose in reqs:
        alone.append(srv.submit(Request(name, pose)).result(timeout=300).image.clone())
    srv.stop(drain=True)
    # the same requests among others of both scenes, batched
    rng = np.random.default_rng(77)
    srv = RenderServer(be, budget_bytes=64 << 30, max_batch=8, max_inflight=2)
    srv.start()
    futs, mixed = [], []
    for i, (name, pose) in enumerate(reqs):
        for _ in range(3):
            futs.append(srv.submit(Request("AB"[int(rng.integers(0, 2))], S.random_request_pose(rng))))
        mixed.append(srv.submit(Request(name, pose)))
    srv.stop(drain=True, timeout=300)
    assert all(f.done() and f.exception() is None for f in futs + mixed)
    assert max(r.batch_size for r in srv.results) > 1
    o = P.default_options()
    for i, (name, pose) in enumerate(reqs):
        assert torch.equal(mixed[i].result(timeout=0).image, alone[i]), f"request {i}: mix differs from alone"
        R = P.Renderer(be.scenes[name], P.CameraBatch.from_poses([pose], o), o)
        R.forward()
        torch.cuda.synchronize()
        assert not R.overflowed()
        assert torch.equal(R.image(0).cpu(), alone[i]), f"request {i}: served image differs from a plain render"
        ref = _ref(g, f"r{i}")
        img = alone[i].numpy().reshape(3, -1).T
        T = R.transmittance(0).cpu().numpy().reshape(-1)
        print(f"request {i} (scene {name}, {pose.width}x{pose.height})", flush=True)
        check_image_values(img[ref.pixels], T[ref.pixels], ref, max_amb=0.1)
        del R
