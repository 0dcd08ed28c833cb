"""Batched multi-view rendering and its autotuner.

BatchRenderer renders many views of one scene: the views are split into
launch groups of up to ``views_per_launch``; each group is one Renderer over
one global tile space (every stage is one launch for the whole group, with
uneven resolutions), and the kernels of all groups are captured in one HIP
graph, so a frame of the whole batch is a single graph launch.

autotune() times a small set of launch configurations (tile shape, LDS batch,
tile schedule, views per launch) on the actual workload and caches the
fastest per (GPU, Gaussian-count bucket, resolution multiset, SH degree).
Every configuration gives bit-identical images: they change the work
decomposition, never the per-pixel arithmetic or order.
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import asdict, dataclass

import torch

from . import _abi
from .raster import CameraBatch, GaussianSet, Renderer


@dataclass(frozen=True)
class LaunchConfig:
    tile_w: int = 16
    tile_h: int = 16
    blend_batch: int = 256
    sort_mode: int = -1            # -1: the library's choice by capacity; 1 tile keys; 2 row binning
    tile_order: bool = True
    persistent: bool = False
    views_per_launch: int = 16
    depth_digit_bits: int = 0      # radix digits of the depth presort: 8, 10 (0: the library's choice)

    def options(self) -> _abi.Options:
        return _abi.default_options(tile_w=self.tile_w, tile_h=self.tile_h,
                                    blend_batch=self.blend_batch, sort_mode=self.sort_mode,
                                    depth_digit_bits=self.depth_digit_bits)


class BatchRenderer:
    def __init__(self, gs: GaussianSet, poses, cfg: LaunchConfig = LaunchConfig(),
                 headroom: float = 1.15, count: bool = False):
        self.gs, self.cfg = gs, cfg
        self.poses = list(poses)
        opt = cfg.options()
        self.groups = []
        self.view_of = []          # global view -> (group, view within group)
        vpl = max(1, cfg.views_per_launch)
        for g0 in range(0, len(self.poses), vpl):
            ps = self.poses[g0:g0 + vpl]
            cams = CameraBatch.from_poses(ps, opt, gs.mean.device)
            r = Renderer(gs, cams, opt, headroom=headroom, tile_order=cfg.tile_order,
                         persistent=cfg.persistent, count=count)
            for k in range(len(ps)):
                self.view_of.append((len(self.groups), k))
            self.groups.append(r)
        self.graph = None

    @property
    def total_pixels(self) -> int:
        return sum(p.width * p.height for p in self.poses)

    def forward(self):
        for r in self.groups:
            r.forward()

    def capture(self):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.forward()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.forward()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    def image(self, v: int) -> torch.Tensor:
        gi, k = self.view_of[v]
        return self.groups[gi].image(k)

    def n_inst(self) -> int:
        return sum(r.n_inst() for r in self.groups)

    def overflowed(self) -> bool:
        return any(r.overflowed() for r in self.groups)


# ------------------------------------------------------------------ autotune
def _cache_path() -> str:
    base = os.environ.get("SGS_AUTOTUNE_CACHE")
    if base:
        return base
    root = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(root, "paper_2605_18334_amd", "autotune.json")


def tune_key(gs: GaussianSet, poses) -> str:
    name = torch.cuda.get_device_name(gs.mean.device)
    nb = 1 << max(0, math.ceil(math.log2(max(gs.n, 1))))
    res = sorted(f"{p.width}x{p.height}" for p in poses)
    return json.dumps([name, nb, res, gs.sh_degree, gs.enhanced, gs.skew is not None])


DEFAULT_CANDIDATES = [
    LaunchConfig(16, 16, 256, 1, False, False, 16),
    LaunchConfig(16, 16, 256, 1, True, False, 16),
    LaunchConfig(16, 16, 256, 1, True, True, 16),
    LaunchConfig(16, 16, 128, 1, True, False, 16),
    LaunchConfig(16, 8, 128, 1, True, False, 16),
    LaunchConfig(16, 8, 128, 1, True, False, 4),
    LaunchConfig(8, 8, 64, 1, True, False, 4),
    LaunchConfig(16, 16, 256, 1, True, False, 8),
    LaunchConfig(16, 16, 0, 1, True, False, 4),
    LaunchConfig(16, 16, 128, 1, True, False, 4),
    LaunchConfig(16, 16, 256, 1, True, False, 4),
    # radix digit width of the depth presort: 8-bit (4 passes) and 10-bit (3)
    LaunchConfig(16, 16, 0, 1, True, False, 4, 8),
    LaunchConfig(16, 16, 0, 1, True, False, 4, 10),
    LaunchConfig(16, 16, 0, 1, True, False, 16, 8),
    LaunchConfig(16, 16, 0, 1, True, False, 16, 10),
    # the sort: row binning (mode 2) against the tile-key sort above
    LaunchConfig(16, 16, 256, 2, True, False, 4),
    LaunchConfig(16, 16, 0, 2, True, False, 4),
    LaunchConfig(16, 16, 0, 2, True, False, 16),
    LaunchConfig(16, 8, 128, 2, True, False, 4),
]


def time_config(gs, poses, cfg: LaunchConfig, reps: int = 3) -> float:
    """Milliseconds per frame, or inf when the library rejects the
    configuration for this workload (for example, too many instances)."""
    try:
        br = BatchRenderer(gs, poses, cfg)
    except (_abi.SgsError, torch.cuda.OutOfMemoryError):
        torch.cuda.empty_cache()
        return float("inf")
    br.forward()
    torch.cuda.synchronize()
    if br.overflowed():
        return float("inf")
    t0 = time.perf_counter()
    for _ in range(reps):
        br.forward()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    del br
    torch.cuda.empty_cache()
    return ms


def autotune(gs: GaussianSet, poses, candidates=None, reps: int = 3, use_cache: bool = True,
             log=None) -> tuple[LaunchConfig, dict]:
    """Returns the fastest LaunchConfig for this workload and the timings."""
    key = tune_key(gs, poses)
    path = _cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return LaunchConfig(**cache[key]["config"]), cache[key]["ms"]
    cands = list(candidates or DEFAULT_CANDIDATES)
    cands = [c if c.views_per_launch <= len(poses) else LaunchConfig(**{**asdict(c), "views_per_launch": len(poses)})
             for c in cands]
    timings = {}
    for c in dict.fromkeys(cands):
        ms = time_config(gs, poses, c, reps)
        timings[json.dumps(asdict(c))] = ms
        if log:
            log(f"autotune {asdict(c)}: {ms:.3f} ms")
    if not any(v < float("inf") for v in timings.values()):
        raise _abi.SgsError("autotune: no candidate configuration fits this workload", 2)
    best = min(timings, key=timings.get)
    cfg = LaunchConfig(**json.loads(best))
    if use_cache:
        cache[key] = {"config": asdict(cfg), "ms": timings}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            json.dump(cache, open(path, "w"), indent=1)
        except OSError:
            pass
    return cfg, timings
