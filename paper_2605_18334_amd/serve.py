"""Render server for the free-camera visualization engine.

The frontend sends camera requests (scene, OpenGL camera-to-world pose,
resolution, field of view) as in Alg. 3; the server keeps scenes resident on
the GPU, converts each pose with the CoordEngine (inside the library call
sgs_camera_from_gl), and renders.

Scheduling is continuous batching, not a queue: a scheduler step
  1. retires finished batches (their memory becomes free again),
  2. admits waiting requests in arrival order while their estimated device
     memory fits the budget, grouping requests of one scene into a batch of up
     to ``max_batch`` views (one launch per stage for the whole batch),
  3. launches the batch on a free stream while up to ``max_inflight`` batches
     run at once, so requests that arrive while others are on the GPU start
     as soon as memory and a stream free up, and their work overlaps.
A request that can never fit the budget is failed with an error instead of
blocking the queue; a batch whose launch raises fails its requests and the
server goes on.

Latency is completion minus arrival (completion includes the device-to-host
copy of the image when one is requested).
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    scene: str
    pose: object                 # sgs_synth.Pose-like: c2w_gl, width, height, fovx_deg, near, bg
    t_arrival: float = 0.0
    want_image: bool = True
    rid: int = -1


@dataclass
class Result:
    rid: int
    image: object                # [3, H, W] float32 (pinned host tensor, device tensor) or None
    t_arrival: float
    t_done: float
    batch_size: int

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class ServerError(RuntimeError):
    pass


@dataclass
class _Batch:
    scene: str
    reqs: list
    futures: list
    nbytes: int
    handle: object = None


class RenderServer:
    """Continuous-batching scheduler over a backend.

    A backend provides: ``bytes_for(scene, poses) -> int`` (device memory a
    batch needs), ``launch(scene, poses, want_images) -> handle`` (enqueues
    the batch, returns at once), ``done(handle) -> bool`` and
    ``results(handle) -> list`` (images, one per pose), ``release(handle)``.
    """

    def __init__(self, backend, budget_bytes: int, max_batch: int = 8, max_inflight: int = 2,
                 clock=time.perf_counter):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.max_inflight = int(max_inflight)
        self.clock = clock
        self.pending = collections.deque()      # (Request, Future)
        self.inflight: list[_Batch] = []
        self.in_use = 0
        self.lock = threading.Lock()
        self.results: list[Result] = []         # completed requests (timing only, no images)
        self.batches = 0
        self.failed = 0
        self.concurrency = []     # requests admitted and not yet done, after each launch
        self._next_id = 0
        self._thread = None
        self._stop = threading.Event()
        self._wake = threading.Event()

    # ------------------------------------------------------------ client side
    def submit(self, req: Request) -> Future:
        fut = Future()
        with self.lock:
            if req.rid < 0:
                req.rid = self._next_id
                self._next_id += 1
            if not req.t_arrival:
                req.t_arrival = self.clock()
            self.pending.append((req, fut))
        self._wake.set()
        return fut

    # ------------------------------------------------------------ scheduler
    def step(self) -> int:
        """One scheduling round; returns the number of batches launched."""
        self._retire()
        launched = 0
        while len(self.inflight) < self.max_inflight:
            b = self._admit()
            if b is None:
                break
            try:
                b.handle = self.backend.launch(b.scene, [r.pose for r in b.reqs],
                                               any(r.want_image for r in b.reqs))
            except Exception as e:          # launch failed: fail the batch, keep serving
                self.in_use -= b.nbytes
                self.failed += len(b.reqs)
                for f in b.futures:
                    f.set_exception(ServerError(f"batch launch failed: {e!r}"))
                continue
            self.inflight.append(b)
            self.batches += 1
            launched += 1
            self.concurrency.append(sum(len(x.reqs) for x in self.inflight))
        return launched

    def _retire(self):
        still = []
        for b in self.inflight:
            if not self.backend.done(b.handle):
                still.append(b)
                continue
            t = self.clock()
            try:
                imgs = self.backend.results(b.handle)
                err = None
            except Exception as e:
                imgs, err = None, e
            for k, (r, f) in enumerate(zip(b.reqs, b.futures)):
                if err is not None:
                    self.failed += 1
                    f.set_exception(ServerError(f"batch failed: {err!r}"))
                    continue
                res = Result(r.rid, imgs[k] if r.want_image else None, r.t_arrival, t, len(b.reqs))
                # the server keeps the timing only: the image goes to the
                # caller's future and lives as long as the caller keeps it
                self.results.append(Result(r.rid, None, r.t_arrival, t, len(b.reqs)))
                f.set_result(res)
            self.backend.release(b.handle)
            self.in_use -= b.nbytes
        self.inflight = still

    def _admit(self):
        with self.lock:
            if not self.pending:
                return None
            head, hfut = self.pending[0]
            scene = head.scene
            picked = []
            nbytes = 0
            # requests of the head's scene, in arrival order, while they fit
            for i, (r, f) in enumerate(self.pending):
                if r.scene != scene:
                    continue
                trial = self.backend.bytes_for(scene, [q.pose for q, _ in picked] + [r.pose])
                if self.in_use + trial > self.budget:
                    break
                picked.append((r, f))
                nbytes = trial
                if len(picked) >= self.max_batch:
                    break
            if not picked:
                alone = self.backend.bytes_for(scene, [head.pose])
                if alone > self.budget:
                    self.pending.popleft()
                    self.failed += 1
                    hfut.set_exception(ServerError(
                        f"request {head.rid} needs {alone} bytes, more than the budget {self.budget}"))
                return None                  # wait for memory to free up
            ids = {id(f) for _, f in picked}
            self.pending = collections.deque((r, f) for r, f in self.pending if id(f) not in ids)
        self.in_use += nbytes
        return _Batch(scene, [r for r, _ in picked], [f for _, f in picked], nbytes)

    # ------------------------------------------------------------ threaded use
    def start(self, idle_sleep: float = 50e-6):
        def loop():
            while not self._stop.is_set():
                n = self.step()
                if n == 0:
                    if self.inflight:
                        time.sleep(idle_sleep)
                    else:
                        self._wake.wait(0.01)
                        self._wake.clear()
        self._thread = threading.Thread(target=loop, name="sgs-render-server", daemon=True)
        self._thread.start()

    def stop(self, drain: bool = True, timeout: float = 60.0):
        if drain:
            t0 = time.perf_counter()
            while (self.pending or self.inflight) and time.perf_counter() - t0 < timeout:
                time.sleep(1e-3)
        self._stop.set()
        self._wake.set()
        if self._thread:
            self._thread.join(timeout)

    # ------------------------------------------------------------ statistics
    def stats(self) -> dict:
        lat = np.array([r.latency for r in self.results])
        if len(lat) == 0:
            return {"completed": 0, "failed": self.failed}
        t0 = min(r.t_arrival for r in self.results)
        t1 = max(r.t_done for r in self.results)
        return {"completed": len(lat), "failed": self.failed, "batches": self.batches,
                "mean_batch": float(np.mean([r.batch_size for r in self.results])),
                "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3), "span_s": float(t1 - t0),
                "admitted_concurrency_mean": float(np.mean(self.concurrency)) if self.concurrency else 0.0,
                "admitted_concurrency_max": int(max(self.concurrency, default=0)),
                "reruns": int(getattr(self.backend, "reruns", 0))}


# ------------------------------------------------------------------ GPU backend
class GpuBackend:
    """Scenes resident on the GPU; each batch renders on a stream of its own
    (streams of default priority), with a completion event polled by the
    scheduler.  Nothing here waits for the device: a batch's instance
    capacity comes from the instances per pixel learnt from earlier batches
    of its scene (with headroom), and its instance count and image are
    copied to pinned host memory on its stream.  When the batch's event has
    completed, done() reads the count: a batch that overflowed its capacity
    is rendered again alone on the same stream with exactly the count it
    reported (the library drops instances past the capacity and still
    reports the true count), and is done only when that finishes; a failed
    sort (0xffffffff) makes results() raise, and such a batch teaches the
    capacity model nothing."""

    def __init__(self, scenes: dict, opt=None, n_streams: int = 4, inst_per_pixel: float = 8.0,
                 headroom: float = 1.3):
        import torch
        from . import _abi
        from .raster import GaussianSet
        self.torch = torch
        self.scenes = {k: (v if isinstance(v, GaussianSet) else GaussianSet.from_scene(v))
                       for k, v in scenes.items()}
        self.opt = opt if opt is not None else _abi.default_options()
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.free_streams = list(range(n_streams))
        # instances per pixel, per scene: starts pessimistic, learnt from batches
        self.ipp = {k: inst_per_pixel for k in self.scenes}
        self.headroom = float(headroom)
        self.reruns = 0

    def capacity_for(self, scene, total_pixels: int) -> int:
        return int(self.ipp[scene] * total_pixels * self.headroom) + 4096

    def bytes_for(self, scene, poses) -> int:
        """Device bytes of the batch's renderer, from the library's size
        helpers at the capacity the batch will get."""
        from .raster import layout_totals, renderer_device_bytes
        gs = self.scenes[scene]
        tiles, pixels = layout_totals(poses, self.opt)
        return renderer_device_bytes(gs.n, len(poses), gs.enhanced, tiles, pixels,
                                     self.capacity_for(scene, pixels), self.opt)

    def _enqueue(self, scene, poses, want_images, capacity, si):
        torch = self.torch
        from .raster import CameraBatch, Renderer
        s = self.streams[si]
        with torch.cuda.stream(s):
            cams = CameraBatch.from_poses(poses, self.opt)
            if capacity is None:
                capacity = self.capacity_for(scene, cams.total_pixels)
            R = Renderer(self.scenes[scene], cams, self.opt, capacity=capacity)
            R.forward()
            n_host = torch.empty(1, dtype=torch.int32, pin_memory=True)
            n_host.copy_(R.bufs["n_inst"], non_blocking=True)
            host = None
            if want_images:
                host = torch.empty(R.out_rgb.shape, dtype=torch.float32, pin_memory=True)
                host.copy_(R.out_rgb, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s)
        return {"R": R, "ev": ev, "host": host, "n_host": n_host}

    def launch(self, scene, poses, want_images):
        if not self.free_streams:
            raise ServerError("no free stream")
        si = self.free_streams.pop()
        try:
            h = self._enqueue(scene, poses, want_images, None, si)
        except Exception:
            self.free_streams.append(si)
            raise
        h.update(si=si, poses=poses, scene=scene, want=want_images, rerun=False)
        return h

    def done(self, h) -> bool:
        if not h["ev"].query():
            return False
        n = int(h["n_host"][0]) & 0xFFFFFFFF
        if n != 0xFFFFFFFF and n > h["R"].capacity and not h["rerun"]:
            # overflow: render the batch again, sized exactly, on its stream
            self.reruns += 1
            h.update(self._enqueue(h["scene"], h["poses"], h["want"], n, h["si"]), rerun=True)
            return False
        return True

    def results(self, h):
        from .raster import check_instance_count
        R, host = h["R"], h["host"]
        n = int(h["n_host"][0]) & 0xFFFFFFFF
        check_instance_count(n, R.capacity)
        P = R.cams.total_pixels
        # a slowly decaying maximum: poses of one scene differ a lot in
        # instances per pixel, and an overflow costs a second render
        self.ipp[h["scene"]] = max(0.98 * self.ipp[h["scene"]], n / max(P, 1))
        out = []
        for v in range(len(h["poses"])):
            c = R.cams.view(v)
            if host is not None:      # pinned host tensor, kept alive by the result
                out.append(host[:, c.pix_base:c.pix_base + c.width * c.height].reshape(3, c.height, c.width))
            else:
                out.append(R.image(v))
        return out

    def release(self, h):
        self.free_streams.append(h["si"])
        h.clear()
