#!/usr/bin/env python3
"""Benchmark of the MI355X skew-Gaussian rasterizer.

Headline: Mpix/s of the forward render (preprocess + bin/sort + blend) of the
clustered workload: 300k skew Gaussians, SH degree 3, one 1280x720 view
(seeded synthetic scene standing in for the paper's trained scenes).  The
same JSON line carries forward+backward iterations/s at 1M Gaussians
(1600x1064, L1 loss), per-stage times, the roofline of the dominant kernel
and the FP64 CPU oracle timed on a bounded pixel sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-bwd]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# MI355X's published fp32 vector peak (packed FP32, an FMA counting 2 flops)
ALU_PEAK_TFLOPS = 157.3
# the rate without packed FP32 (which this build disables): 256 CUs x 4 SIMD
# x 16 lanes x 2.4 GHz = 39.3 T lane-ops/s, an FMA counting 2 -> 78.6 TFLOP/s
ALU_PEAK_NONPACKED_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
# flops of Alg. 1 per pair, exp and erf counted 1 each: evaluating alpha of a
# pair (offsets 2, quadratic form 9, exp 1, skew argument 4, erf 1, 1+erf 1,
# alpha product and clamp 2) = 20, for every pair past the exponent test;
# compositing a pair (T(1-alpha) 2, colour accumulation 7) = 9 more
FLOPS_EVAL = 20
FLOPS_COMPOSITE = 9
# backward per composited pair (the pairs Alg. 2 walks): the evaluation again
# (20) and the gradient terms: 1/(1-alpha), T and the weight 3, dL/dalpha 8,
# shared factors 6, the 11 record-gradient terms 27, colour-behind update 6,
# their sums over the tile's pixels 11 -> 20 + 61 flops; pairs skipped behind
# the last contributor are not counted (a lower bound of the work)
FLOPS_BWD_COMPOSITE = 81


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = {"k_blend_fwd": ["paper_2605_18334_amd/csrc/blend.hip",
                                  "paper_2605_18334_amd/csrc/sgs_dev.h"]}
TRAFFIC_PROFILE = "profiles/traffic_fwd_clustered300k_sh3_1280x720.md"


def source_hash(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE runs, scaled by a plain copy), or None
    when the kernel's source has changed since the counters were taken."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    want = source_hash(kernel)
    for line in open(path):
        if line.startswith(f"traffic {kernel} "):
            kv = dict(x.split("=", 1) for x in line.split()[2:])
            if kv.get("source_sha256") == want:
                return int(kv["read_bytes"]) + int(kv["write_bytes"])
    return None


def sh_bytes(deg: int) -> int:
    return 12 * (deg + 1) ** 2


def timed_forward(R, steps: int, warmup: int):
    """Warm-up (W frames, then at least 0.3 s of frames so that clocks have
    settled), a per-stage breakdown in a loop of its own (events between the
    stages), then the timed region: exactly `steps` whole frames between two
    synchronisations, with events around each blend launch only (its
    duration for the roofline; events between every stage would add ~5% to
    the step)."""
    import torch
    for _ in range(warmup):
        R.forward(count=False)
    torch.cuda.synchronize()
    t_w = time.perf_counter()
    while time.perf_counter() - t_w < 0.3:
        for _ in range(10):
            R.forward(count=False)
        torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for e in ev:
        e[0].record()
        R.preprocess()
        e[1].record()
        R.bin_sort()
        e[2].record()
        R.blend(count=False)
        e[3].record()
    torch.cuda.synchronize()
    stages = {"preprocess": float(np.mean([e[0].elapsed_time(e[1]) for e in ev])),
              "bin_sort": float(np.mean([e[1].elapsed_time(e[2]) for e in ev])),
              "blend_fwd": float(np.mean([e[2].elapsed_time(e[3]) for e in ev]))}
    bl = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(steps)]
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for b in bl:
        R.preprocess()
        R.bin_sort()
        b[0].record()
        R.blend(count=False)
        b[1].record()
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    blend_ms = float(np.mean([b[0].elapsed_time(b[1]) for b in bl]))
    return start.elapsed_time(end) / steps, wall, stages, blend_ms


def host_cpu() -> dict:
    """The host the CPU baseline ran on: logical CPUs, the affinity mask's
    size, OMP_NUM_THREADS, torch's thread count and the CPU model."""
    import torch
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "OMP_NUM_THREADS": os.environ.get("OMP_NUM_THREADS"), "torch_threads": torch.get_num_threads(),
            "cpu_model": model}


def cpu_baseline(sc, pose, target_s: float):
    """The FP64 oracle on a seeded pixel sample of the same workload, sized
    to take about target_s seconds; reported as sampled Mpix/s."""
    import torch
    import sgs_synth as S
    from oracle import sgs_oracle as O
    cores = torch.get_num_threads()
    n = 8
    t = 0.0
    while True:
        px = S.sample_pixels(99, pose.width, pose.height, n)
        t0 = time.perf_counter()
        O.render(sc, pose, pixels=px)
        t = time.perf_counter() - t0
        if t >= 0.6 * target_s or n >= 1 << 16:
            break
        n = int(min(max(2 * n, n * target_s / max(t, 1e-3)), 1 << 16))
    return {"value": n / t / 1e6, "unit": "Mpix/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} seeded tile-stratified pixels of the same 300k-Gaussian 1280x720 view, "
                      f"brute force over all Gaussians in FP64 ({t:.1f} s); the full-size parity tests "
                      f"use 4096 such pixels, computed beforehand",
            "host": host_cpu()}


def sort_stage_bytes(m: int, n_inst: int, total_tiles: int, depth_passes: int, mode: int = 1,
                     n_items: int = 0, item_passes: int = 1) -> dict:
    """Algorithmic HBM bytes of the bin/sort stage in the sort mode that ran
    (1: duplicate + tile-key sort; 2: row items + row sort + placement) and,
    for comparison, of the plain form the method describes (duplicate with
    64-bit (tile, depth) keys, LSD sort of 8-bit digits over all key bits)."""
    tb = max(1, math.ceil(math.log2(max(total_tiles, 2))))
    common = (m * (4 + depth_passes * 16)     # depth presort: histogram read, passes r+w key and id
              + m * 12                        # offsets: order, count in; offset out
              + m * 64)                       # expansion / emission: one record line per record
    if mode == 2:
        moved = (common
                 + n_items * 8                    # emission writes item key and record
                 + n_items * 16 * item_passes     # row passes: read + write key and record
                 + n_items * 4                    # piece counts: item keys
                 + n_items * 8 + n_inst * 4)      # placement: items in, record per instance out
    else:
        moved = (common
                 + n_inst * 8                     # expansion writes key and value
                 + n_inst * 16 * math.ceil(tb / 8))   # tile-key passes: read + write key and value
    passes64 = math.ceil((tb + 32) / 8)
    plain = m * (8 + 16) + n_inst * 12 + n_inst * (8 + passes64 * 24)
    return {"moved": moved, "plain_64bit_lsd": plain, "sort_mode": mode, "n_items": n_items}


def sort_info(R) -> dict:
    """The sort mode the library runs for a Renderer and, for mode 2, its row
    items (the non-empty tile rows of all records) and row-sort passes."""
    import ctypes as C
    lib = R.lib
    mode = int(lib.sgs_bin_sort_mode(C.byref(R.opt), R.capacity, R.cams.host, R.cams.n_views, 1))
    n_items = int(R.bufs["rows"][:R.m].to(torch_int64()).sum().item()) if mode == 2 else 0
    rows = sum(R.cams.view(v).tiles_y for v in range(R.cams.n_views))
    item_passes = 1 if rows <= 256 else 2
    return {"mode": mode, "n_items": n_items, "item_passes": item_passes}


def torch_int64():
    import torch
    return torch.int64


def stage_bandwidth(pre_bytes: int, sb: dict, stages: dict) -> dict:
    """Algorithmic HBM rates of the preprocess and bin/sort stages (all their
    kernels, whole-stage times); the bin/sort also as the rate at which the
    plain 64-bit-key LSD form's bytes would have to move to finish as soon."""
    out = {"preprocess": {"GB/s": pre_bytes / (stages["preprocess"] / 1e3) / 1e9},
           "bin_sort": {"GB/s": sb["moved"] / (stages["bin_sort"] / 1e3) / 1e9,
                        "plain_64bit_lsd_equivalent_GB/s": sb["plain_64bit_lsd"] / (stages["bin_sort"] / 1e3) / 1e9,
                        "sort_mode": sb["sort_mode"], "moved_MB": sb["moved"] / 1e6,
                        "row_items": sb["n_items"]}}
    for v in out.values():
        v["frac"] = v["GB/s"] / HBM_PEAK_GBS
    return out


def stage_times(R, reps: int = 20) -> dict:
    """Per-stage times of the forward (events between the stages, a loop of
    its own)."""
    import torch
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(reps)]
    for e in ev:
        e[0].record()
        R.preprocess()
        e[1].record()
        R.bin_sort()
        e[2].record()
        R.blend(count=False)
        e[3].record()
    torch.cuda.synchronize()
    return {"preprocess": float(np.mean([e[0].elapsed_time(e[1]) for e in ev])),
            "bin_sort": float(np.mean([e[1].elapsed_time(e[2]) for e in ev])),
            "blend_fwd": float(np.mean([e[2].elapsed_time(e[3]) for e in ev]))}


def fwd_bwd(steps: int, warmup: int):
    """Forward + L1 loss gradient + backward at 1M Gaussians, 1600x1064."""
    import torch
    import paper_2605_18334_amd as P
    import sgs_synth as S
    sc, tgt, pose = S.diff_config()
    opt = P.default_options(**OPT_OVER)
    cams = P.CameraBatch.from_poses([pose], opt)
    T = P.Renderer(P.GaussianSet.from_scene(tgt), cams, opt)
    target = T.forward().clone()
    del T
    R = P.Renderer(P.GaussianSet.from_scene(sc), cams, opt, count=True)   # (counts only when asked)
    npx = target.numel()

    def step():
        out = R.forward(count=False)
        dL = torch.sign(out - target).mul_(1.0 / npx)
        return R.backward(dL)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # steps back to back (a training loop does not wait per step); events at
    # the step boundaries give the forward / backward split
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    t0 = time.perf_counter()
    for e in ev:
        e[0].record()
        out = R.forward(count=False)
        e[1].record()
        dL = torch.sign(out - target).mul_(1.0 / npx)
        R.backward(dL, events=(e[3], e[4]))
        e[2].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev[0][0].elapsed_time(ev[-1][2])
    assert not R.overflowed()
    stages = stage_times(R)
    # backward roofline: the library call (blend backward + chain rule), the
    # composited pairs from a counting forward outside the timed loop
    bwd_ms = float(np.mean([e[3].elapsed_time(e[4]) for e in ev]))
    R.forward(count=True)
    torch.cuda.synchronize()
    pairs = int(R.bufs["count"].to(torch.int64).sum().item())
    achieved = pairs * FLOPS_BWD_COMPOSITE / (bwd_ms / 1e3) / 1e12
    roof_bwd = {"kernel": "k_blend_bwd + k_preprocess_bwd (sgs_render_bwd)", "bound": "alu",
                "achieved": achieved, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / ALU_PEAK_TFLOPS, "peak_nonpacked": ALU_PEAK_NONPACKED_TFLOPS,
                "frac_nonpacked": achieved / ALU_PEAK_NONPACKED_TFLOPS, "ms": bwd_ms,
                "units": f"{pairs} composited pairs x {FLOPS_BWD_COMPOSITE} flops, per call"}
    pre_bytes = sc.n * (56 + sh_bytes(sc.sh_degree)) + sc.n * 64
    si = sort_info(R)
    sbw = stage_bandwidth(pre_bytes, sort_stage_bytes(sc.n, R.n_inst(), cams.total_tiles, 4, si["mode"],
                                                      si["n_items"], si["item_passes"]), stages)
    return {"metric": "fwd+bwd iters/s at 1M Gaussians", "value": steps / (gpu_ms / 1e3), "unit": "iters/s",
            "stages_ms": stages, "stage_bandwidth": sbw, "roofline_bwd": roof_bwd,
            "wall_iters_s": steps / wall,
            "ms_fwd": float(np.mean([e[0].elapsed_time(e[1]) for e in ev])),
            "ms_bwd": float(np.mean([e[1].elapsed_time(e[2]) for e in ev])),
            "n_inst": R.n_inst(),
            "config": {"workload": "1M skew Gaussians (4-blob generator, SH0), one 1600x1064 view, "
                                   "L1 loss vs a separately seeded 1M target"}}


def train_multiview(steps: int, warmup: int):
    """Multi-view training step at 1M Gaussians: 4 views of 1600x1064 in one
    tile space, per-view L1 gradient, one backward accumulating all views,
    Adam; the whole step replayed as one HIP graph.  Beside it, the same
    work as 4 single-view forward/backward passes and one Adam step, eager."""
    import torch
    import paper_2605_18334_amd as P
    from paper_2605_18334_amd.train import Adam, MultiViewTrainer, l1_weights
    import sgs_synth as S
    sc, tgt, poses = S.train_config()
    opt = P.default_options(**OPT_OVER)
    cams = P.CameraBatch.from_poses(poses, opt)
    T = P.Renderer(P.GaussianSet.from_scene(tgt), cams, opt)
    target = T.forward().clone()
    del T, tgt
    tr = MultiViewTrainer(P.GaussianSet.from_scene(sc), poses, target, opt, headroom=1.25)
    tr.capture()
    for _ in range(warmup):
        tr.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tr.replay()
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) * 1e3 / steps
    assert not tr.overflowed()
    n_inst = tr.R.n_inst()
    del tr
    torch.cuda.empty_cache()
    # the same step as V single-view passes (eager), gradients summed, one Adam
    gs = P.GaussianSet.from_scene(sc)
    singles = []
    for v, p in enumerate(poses):
        c1 = P.CameraBatch.from_poses([p], opt)
        c = cams.view(v)
        singles.append((P.Renderer(gs, c1, opt, headroom=1.25), target[:, c.pix_base:c.pix_base + c.width * c.height],
                        l1_weights(c1, target.device)))
    ad = Adam(gs)
    total = {f: torch.zeros_like(getattr(gs, f)) for f in ad.names}

    def seq_step():
        for f in ad.names:
            total[f].zero_()
        for R, tv, w in singles:
            out = R.forward()
            g = R.backward(torch.sign(out - tv).mul_(w))
            for f in ad.names:
                total[f].add_(g[f])
        ad.step(total)

    for _ in range(warmup):
        seq_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        seq_step()
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) * 1e3 / steps
    assert not any(R.overflowed() for R, _, _ in singles)
    return {"metric": "multi-view training iters/s at 1M Gaussians", "value": 1e3 / ms_graph, "unit": "iters/s",
            "ms_step_graph": ms_graph, "ms_step_sequential": ms_seq, "speedup_vs_sequential": ms_seq / ms_graph,
            "views_per_s": len(poses) * 1e3 / ms_graph, "n_inst": n_inst,
            "config": {"workload": "1M skew Gaussians (4-blob generator, SH0), 4 spline views at 1600x1064, "
                                   "L1 loss vs a separately seeded 1M target, Adam; one HIP graph per step"}}


def batched(steps: int, warmup: int, small: bool = False):
    """16 views of mixed resolution of a 3M-Gaussian scene (small: 16
    640x480 views of the 300k clustered scene): one HIP-graph launch of the
    autotuned batch vs 16 sequential single-view renders."""
    import torch
    import paper_2605_18334_amd as P
    from paper_2605_18334_amd.batch import BatchRenderer, autotune
    import sgs_synth as S
    sc, poses = S.small_batch_config() if small else S.batch_config()
    gs = P.GaussianSet.from_scene(sc)
    del sc
    cfg, timings = autotune(gs, poses, reps=2, log=log)
    br = BatchRenderer(gs, poses, cfg)
    br.capture()
    for _ in range(warmup):
        br.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        br.replay()
    torch.cuda.synchronize()
    ms_b = (time.perf_counter() - t0) * 1e3 / steps
    assert not br.overflowed()
    o = P.default_options(**OPT_OVER)
    singles = [P.Renderer(gs, P.CameraBatch.from_poses([p], o), o) for p in poses]
    for _ in range(warmup):
        for r in singles:
            r.forward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for r in singles:
            r.forward()
    torch.cuda.synchronize()
    ms_s = (time.perf_counter() - t0) * 1e3 / steps
    same = all(torch.equal(br.image(v), singles[v].image(0)) for v in range(len(poses)))
    px = br.total_pixels
    out = {"metric": "Mpix/s render fwd, 16-view batch", "value": px / (ms_b / 1e3) / 1e6, "unit": "Mpix/s",
           "ms_batched": ms_b, "ms_sequential": ms_s, "speedup_vs_sequential": ms_s / ms_b,
           "sequential_mpix_s": px / (ms_s / 1e3) / 1e6, "bit_identical_to_single_views": same,
           "n_inst": br.n_inst(), "tuned": {k: v for k, v in cfg.__dict__.items()},
           "config": {"workload": ("300k skew Gaussians (32-cluster generator, SH3), 16 orbit views at 640x480"
                                   if small else
                                   "3M skew Gaussians (4-blob generator, SH0), 16 spline poses at "
                                   "640x480/1280x720/1600x1064/1920x1080 (4 each)")}}
    del br, singles
    torch.cuda.empty_cache()
    return out


SERVE_RATES = [60, 120, 240, 600]
OPT_OVER: dict = {}        # option overrides from the command line (--sort-mode, --blend-batch,
                           # --blend-lists, --split-tiles)


def serving(duration_s: float, rates):
    """Poisson request stream against resident 5M skew + 2M symmetric SH3
    scenes, continuous batching vs FIFO one-at-a-time."""
    import torch
    import paper_2605_18334_amd as P
    from paper_2605_18334_amd.serve import GpuBackend, RenderServer, Request
    import sgs_synth as S
    scA, scB = S.serve_scenes()
    be = GpuBackend({"A": scA, "B": scB})
    del scA, scB
    res = {}
    runs = [(f"batched@{r}", r, 8, 2) for r in rates] + [(f"fifo@{r}", r, 1, 1) for r in rates]
    for name, rate, mb, mi in runs:
        rng = np.random.default_rng(8)
        srv = RenderServer(be, budget_bytes=64 << 30, max_batch=mb, max_inflight=mi)
        # warm the backend (first launch allocates)
        srv.start()
        srv.submit(Request("A", S.random_request_pose(rng))).result(timeout=120)
        srv.submit(Request("B", S.random_request_pose(rng))).result(timeout=120)
        srv.results.clear()
        reruns0 = be.reruns
        t0 = time.perf_counter()
        t = 0.0
        n = 0
        pix = 0
        while t < duration_s:
            t += rng.exponential(1.0 / rate)
            now = time.perf_counter() - t0
            if t > now:
                time.sleep(t - now)
            pose = S.random_request_pose(rng)
            pix += pose.width * pose.height
            srv.submit(Request("AB"[int(rng.integers(0, 2))], pose, t_arrival=time.perf_counter()))
            n += 1
        srv.stop(drain=True, timeout=120)
        st = srv.stats()
        st["reruns"] = be.reruns - reruns0     # overflowed batches rendered again (this run)
        st["offered_req_s"] = rate
        st["mpix_s"] = pix / max(st.get("span_s", 1e-9), 1e-9) / 1e6
        res[name] = st
        log(f"serving {name}: {st}")
    return {"metric": "p50/p99 frame latency (served)", "unit": "ms",
            "config": {"workload": "resident 5M skew + 2M zero-skew Gaussians (32-cluster generator, SH3); "
                                   "Poisson arrivals; poses 50% orbit / 50% free flight; "
                                   "640x480/1280x720/1920x1080; images copied to host"},
            "runs": res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-bwd", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--no-train", action="store_true")
    ap.add_argument("--only", choices=["fwd", "fwdbwd", "train", "batch", "serve"], default=None,
                    help="run one workload only (for profiler runs)")
    ap.add_argument("--sort-mode", type=int, default=None, choices=[0, 1, 2],
                    help="override the library's default sort mode in every workload")
    ap.add_argument("--blend-batch", type=int, default=None, choices=[64, 128, 256],
                    help="override the records staged per LDS batch in the blends (default: "
                         "the library's, 128 forward and 256 backward)")
    ap.add_argument("--blend-lists", type=int, default=None, choices=[1, 4],
                    help="override the forward blend's record lists per wave (default: the "
                         "library's choice from the instance capacity per record)")
    ap.add_argument("--split-tiles", type=int, default=None,
                    help="override how many of the longest tiles the blends split into quarters "
                         "(default: the library's, total tiles / 128; 0: none)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size "
                         "kernel that scales hardware byte counters)")
    args = ap.parse_args()
    if args.sort_mode is not None:
        OPT_OVER["sort_mode"] = args.sort_mode
    if args.blend_batch is not None:
        OPT_OVER["blend_batch"] = args.blend_batch
    if args.blend_lists is not None:
        OPT_OVER["blend_lists"] = args.blend_lists
    if args.split_tiles is not None:
        OPT_OVER["split_tiles"] = args.split_tiles
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print("bench.py measures one GPU: this build renders on a single MI355X "
              "(multi-GPU sharding is a design note, not an implemented path)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2605_18334_amd as P
    import sgs_synth as S

    torch.cuda.set_device(0)
    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only == "fwdbwd":
        print(json.dumps(fwd_bwd(max(3, args.steps // 2), 2)), flush=True)
        return
    if args.only == "train":
        print(json.dumps(train_multiview(max(3, args.steps // 4), 2)), flush=True)
        return
    if args.only == "batch":
        print(json.dumps({"batched": batched(max(3, args.steps // 4), 1),
                          "batched_small": batched(max(10, args.steps // 2), 3, small=True)}), flush=True)
        return
    if args.only == "serve":
        print(json.dumps(serving(args.serve_seconds, SERVE_RATES)), flush=True)
        return
    sc, pose = S.clustered_config()
    opt = P.default_options(**OPT_OVER)
    gs = P.GaussianSet.from_scene(sc)
    cams = P.CameraBatch.from_poses([pose], opt)
    R = P.Renderer(gs, cams, opt, count=True)
    ms, wall, stages, blend_ms = timed_forward(R, args.steps, args.warmup)
    assert not R.overflowed()
    n_inst = R.n_inst()
    # the work counters run outside the timed region (the counting variant of
    # the blend has extra instructions)
    R.forward(count=True)
    pairs = int(R.bufs["count"].to(torch.int64).sum().item())
    evaluated = int(R.bufs["eval"].to(torch.int64).sum().item())
    npix = pose.width * pose.height
    mpix_s = npix / (ms / 1e3) / 1e6
    log(f"forward {ms:.3f} ms/step, stages {stages}, n_inst {n_inst}, pairs {pairs}")

    # roofline of the dominant kernel: the blend forward is the longest single
    # launch (bin/sort is a dozen kernels, each far shorter; see profiles/)
    flops = evaluated * FLOPS_EVAL + pairs * FLOPS_COMPOSITE
    achieved = flops / (blend_ms / 1e3) / 1e12
    roof = {"kernel": "k_blend_fwd", "bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / ALU_PEAK_TFLOPS,
            "traffic": measured_traffic("k_blend_fwd"),
            "peak_nonpacked": ALU_PEAK_NONPACKED_TFLOPS, "frac_nonpacked": achieved / ALU_PEAK_NONPACKED_TFLOPS,
            "units": f"{evaluated} evaluated pairs x {FLOPS_EVAL} + {pairs} composited pairs x "
                     f"{FLOPS_COMPOSITE} flops, per launch"}
    # algorithmic HBM rates of the other stages (whole stage, all its kernels)
    pre_bytes = sc.n * (56 + sh_bytes(sc.sh_degree)) + sc.n * 64
    si = sort_info(R)
    stage_bw = stage_bandwidth(pre_bytes, sort_stage_bytes(sc.n, n_inst, cams.total_tiles, 4, si["mode"],
                                                           si["n_items"], si["item_passes"]), stages)

    out = {
        "metric": "Mpix/s render fwd", "value": mpix_s, "unit": "Mpix/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "300k skew Gaussians (32-cluster generator), SH3, one 1280x720 view, "
                               "fov 60, radius-15 orbit; forward = preprocess + bin/sort + blend",
                   "global_batch": 1, "seq_len": None, "parallelism": "1 GPU"},
        "stages_ms": stages, "n_inst": n_inst, "composited_pairs": pairs, "evaluated_pairs": evaluated,
        "roofline": roof, "stage_bandwidth": stage_bw,
    }
    if not args.no_bwd and args.only is None:
        del R
        torch.cuda.empty_cache()
        out["fwd_bwd"] = fwd_bwd(max(3, args.steps // 2), 2)
        log(f"fwd+bwd {out['fwd_bwd']}")
    if not args.no_train and args.only is None:
        torch.cuda.empty_cache()
        out["train_multiview"] = train_multiview(max(3, args.steps // 4), 2)
        log(f"train {out['train_multiview']}")
    if not args.no_batch and args.only is None:
        torch.cuda.empty_cache()
        out["batched"] = batched(max(3, args.steps // 4), 1)
        torch.cuda.empty_cache()
        out["batched_small"] = batched(max(10, args.steps // 2), 3, small=True)
    if not args.no_serve and args.only is None:
        torch.cuda.empty_cache()
        out["served"] = serving(args.serve_seconds, SERVE_RATES)
    if not args.no_cpu and args.only is None:
        out["cpu_baseline"] = cpu_baseline(sc, pose, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
