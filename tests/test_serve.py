"""Serving loop logic on the CPU: a fake backend with modelled durations and
a virtual clock drives the scheduler (admission by memory, continuous
batching, overlap, FIFO, failure handling, latency accounting)."""
import pytest

import sgs_synth as S
from paper_2605_18334_amd.serve import RenderServer, Request, ServerError


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeBackend:
    """Each batch costs `per_batch + per_view * views` seconds of virtual time
    and `bytes_per_view * views` bytes; batches run concurrently."""

    def __init__(self, clock, per_batch=1.0, per_view=0.5, bytes_per_view=100, fail_on=()):
        self.clock, self.per_batch, self.per_view = clock, per_batch, per_view
        self.bytes_per_view = bytes_per_view
        self.fail_on = set(fail_on)
        self.launches = []
        self.live = 0
        self.max_live = 0

    def bytes_for(self, scene, poses):
        return self.bytes_per_view * len(poses)

    def launch(self, scene, poses, want):
        k = len(self.launches)
        self.launches.append((scene, len(poses), self.clock()))
        if k in self.fail_on:
            raise RuntimeError("injected launch failure")
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        return {"end": self.clock() + self.per_batch + self.per_view * len(poses), "n": len(poses), "k": k}

    def done(self, h):
        return self.clock() >= h["end"]

    def results(self, h):
        return [f"img{h['k']}.{i}" for i in range(h["n"])]

    def release(self, h):
        self.live -= 1


def _req(scene, t):
    return Request(scene, S.Pose(None, 64, 48), t_arrival=t)


def _run(srv, clock, until, dt=0.25):
    while clock.t < until:
        srv.step()
        clock.t += dt
    srv.step()


def test_requests_of_one_scene_are_batched_in_arrival_order():
    c = Clock()
    be = FakeBackend(c)
    srv = RenderServer(be, budget_bytes=10_000, max_batch=4, max_inflight=1, clock=c)
    futs = [srv.submit(_req("A", 0.0)) for _ in range(6)]
    _run(srv, c, 10)
    assert [n for _, n, _ in be.launches] == [4, 2]
    assert [f.result().rid for f in futs] == list(range(6))
    assert all(f.result().batch_size in (4, 2) for f in futs)


def test_admission_respects_memory_budget():
    c = Clock()
    be = FakeBackend(c, bytes_per_view=100)
    srv = RenderServer(be, budget_bytes=250, max_batch=8, max_inflight=4, clock=c)
    for _ in range(7):
        srv.submit(_req("A", 0.0))
    srv.step()
    assert srv.in_use <= 250 and [n for _, n, _ in be.launches] == [2]
    _run(srv, c, 20)
    assert sum(n for _, n, _ in be.launches) == 7
    assert srv.in_use == 0


def test_request_larger_than_budget_fails_without_blocking_others():
    c = Clock()
    be = FakeBackend(c, bytes_per_view=100)
    srv = RenderServer(be, budget_bytes=50, max_batch=2, clock=c)
    f = srv.submit(_req("A", 0.0))
    _run(srv, c, 2)
    with pytest.raises(ServerError):
        f.result(timeout=0)
    be.bytes_per_view = 10
    g = srv.submit(_req("A", c.t))
    _run(srv, c, c.t + 5)
    assert g.result(timeout=0).image.startswith("img")


def test_continuous_batching_overlaps_new_arrivals_with_running_batches():
    """A request arriving while a batch is on the device starts at once on a
    second slot instead of waiting for the first batch to finish."""
    c = Clock()
    be = FakeBackend(c, per_batch=4.0, per_view=0.0)
    srv = RenderServer(be, budget_bytes=10_000, max_batch=8, max_inflight=2, clock=c)
    a = srv.submit(_req("A", 0.0))
    srv.step()
    c.t = 1.0
    b = srv.submit(_req("A", 1.0))
    srv.step()
    assert len(be.launches) == 2 and be.launches[1][2] == 1.0 and be.max_live == 2
    _run(srv, c, 10)
    assert a.result().latency == pytest.approx(4.0, abs=0.3)
    assert b.result().latency == pytest.approx(4.0, abs=0.3)


def test_fifo_one_at_a_time_is_the_degenerate_configuration():
    c = Clock()
    be = FakeBackend(c, per_batch=1.0, per_view=0.0)
    srv = RenderServer(be, budget_bytes=10_000, max_batch=1, max_inflight=1, clock=c)
    futs = [srv.submit(_req("A", 0.0)) for _ in range(4)]
    _run(srv, c, 10)
    lat = [f.result().latency for f in futs]
    assert lat == sorted(lat) and lat[-1] >= 4.0 and be.max_live == 1


def test_scenes_are_batched_separately_and_head_first():
    c = Clock()
    be = FakeBackend(c)
    srv = RenderServer(be, budget_bytes=10_000, max_batch=8, max_inflight=4, clock=c)
    for sc in "ABAB":
        srv.submit(_req(sc, 0.0))
    srv.step()
    assert [(s, n) for s, n, _ in be.launches] == [("A", 2), ("B", 2)]


def test_launch_failure_fails_that_batch_only():
    c = Clock()
    be = FakeBackend(c, fail_on={0})
    srv = RenderServer(be, budget_bytes=10_000, max_batch=1, max_inflight=1, clock=c)
    f1 = srv.submit(_req("A", 0.0))
    f2 = srv.submit(_req("A", 0.0))
    _run(srv, c, 5)
    with pytest.raises(ServerError):
        f1.result(timeout=0)
    assert f2.result(timeout=0).image == "img1.0"
    assert srv.in_use == 0 and srv.failed == 1


def test_latency_percentiles():
    c = Clock()
    be = FakeBackend(c, per_batch=1.0, per_view=0.0)
    srv = RenderServer(be, budget_bytes=10_000, max_batch=1, max_inflight=1, clock=c)
    for _ in range(10):
        srv.submit(_req("A", 0.0))
    _run(srv, c, 20)
    st = srv.stats()
    assert st["completed"] == 10 and st["batches"] == 10
    assert 5000 <= st["p50_ms"] <= 6500 and st["p99_ms"] >= 9000


def test_threaded_server_drains():
    be = FakeBackend(lambda: 0.0, per_batch=0.0, per_view=0.0)
    srv = RenderServer(be, budget_bytes=10_000, max_batch=4)
    srv.start()
    futs = [srv.submit(_req("AB"[i % 2], 0.0)) for i in range(20)]
    srv.stop(drain=True, timeout=10)
    assert all(f.done() and f.result().image.startswith("img") for f in futs)


def test_gpu_backend_memory_estimate_covers_what_a_renderer_allocates():
    """bytes_for of the GPU backend, from the library's size helpers, is at
    least the bytes of every buffer a Renderer of that batch allocates at the
    capacity the backend would give it (sized here with CPU tensors: building
    a Renderer with a fixed capacity touches no GPU)."""
    from paper_2605_18334_amd import _abi
    from paper_2605_18334_amd.raster import CameraBatch, GaussianSet, Renderer
    from paper_2605_18334_amd.serve import GpuBackend
    import numpy as np
    rng = np.random.default_rng(3)
    for enhanced, sh in ((False, 3), (True, 1)):
        sc = S.blobs_scene(2, 1000, sh, enhanced=enhanced)
        gs = GaussianSet.from_scene(sc, "cpu")
        be = object.__new__(GpuBackend)          # no streams: sizing only
        be.scenes, be.opt, be.ipp, be.headroom = {"A": gs}, _abi.default_options(), {"A": 11.0}, 1.3
        for views in (1, 3):
            poses = [S.random_request_pose(rng) for _ in range(views)]
            cams = CameraBatch.from_poses(poses, be.opt, device="cpu")
            R = Renderer(gs, cams, be.opt, capacity=be.capacity_for("A", cams.total_pixels))
            est = be.bytes_for("A", poses)
            assert est >= R.device_bytes() > 0
            assert est == R.device_bytes()        # the same expressions, nothing missed or extra
