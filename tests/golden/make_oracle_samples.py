"""Writes the FP64 oracle's expected values for the full-size parity tests.

    python tests/golden/make_oracle_samples.py [clustered] [blobs1m] [batch16] [serve]

The brute-force oracle takes minutes per workload at these sizes (every
Gaussian at every sampled pixel), so its results are stored once and read by
the GPU tests.  Only the seeded input generators (sgs_synth) and the oracle
are called; nothing here reads the HIP path.

clustered_300k_4096px.npz: the clustered workload (300k skew Gaussians, SH3,
  one 1280x720 view), 4096 seeded tile-stratified pixels: colour, final
  transmittance, the oracle's ambiguity flags (decisions within the margins
  where float32 may decide the other way) and, for ambiguous pixels, the
  colour and transmittance of every outcome of their uncertain decisions.

batch16_3m_2views_1024px.npz: the 16-view batch workload (3M skew Gaussians,
  4-blob generator, SH0, 16 spline poses of mixed resolution): 1024 seeded
  tile-stratified pixels of views 0 and 9, as for the clustered frame.

serve_5m2m_4requests_512px.npz: the serving scenes (5M skew and 2M zero-skew
  clustered SH3): two seeded requests per scene (the served-request pose
  generator), 512 seeded pixels of each.

blobs_1m_masked_4096px.npz: the differentiation workload (1M skew Gaussians,
  4-blob generator, SH0, one 1600x1064 view) with a masked loss
  L = sum_p w_p . C(p) over 4096 seeded tile-stratified pixels (w seeded
  normal, zero at the ambiguous pixels): colour, transmittance and
  ambiguity at those pixels; the gradient of L w.r.t. every parameter on a
  seeded sample of the Gaussians it reaches, plus per-tensor norms and
  maxima over all Gaussians and a bit mask of the Gaussians with a non-zero
  gradient.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import sgs_synth as S                      # noqa: E402
from oracle import sgs_oracle as O         # noqa: E402

N_PIX = 4096
PIXEL_SEED_CLUSTERED = 11
PIXEL_SEED_BLOBS = 41
WEIGHT_SEED = 43
SAMPLE_SEED = 47
N_SAMPLE = 16384
FIELDS = ("mean", "log_scale", "quat", "skew", "opa_logit", "sh")


def clustered(path: str) -> None:
    sc, pose = S.clustered_config()
    px = S.sample_pixels(PIXEL_SEED_CLUSTERED, pose.width, pose.height, N_PIX)
    t0 = time.time()
    r = O.render(sc, pose, pixels=px)
    print(f"clustered: {time.time() - t0:.0f} s, ambiguous {r.ambiguous.mean():.4f}", flush=True)
    np.savez_compressed(path, pixels=px, color=r.color, T=r.T, ambiguous=r.ambiguous, last=r.last,
                        alt_start=r.alt_start, alt_rows=r.alt_rows, ambiguous_grad=r.ambiguous_grad)


def blobs1m(path: str) -> None:
    sc, _, pose = S.diff_config()
    px = S.sample_pixels(PIXEL_SEED_BLOBS, pose.width, pose.height, N_PIX)
    t0 = time.time()
    r = O.render(sc, pose, pixels=px)
    print(f"blobs1m render: {time.time() - t0:.0f} s, ambiguous {r.ambiguous.mean():.4f}", flush=True)
    w = np.random.default_rng(WEIGHT_SEED).normal(size=(N_PIX, 3))
    w[r.ambiguous_grad] = 0.0        # the gradient is taken where every decision is clear
    w = w.astype(np.float32).astype(np.float64)     # the GPU test feeds the same float32 weights
    t0 = time.time()
    g = O.render_grad(sc, pose, w, px)
    print(f"blobs1m gradient: {time.time() - t0:.0f} s", flush=True)
    # per-Gaussian rows: [N, components] from the SoA shapes ([3][N], [N], [K][3][N])
    flat = {k: g[k].reshape(-1, sc.n).T for k in FIELDS}
    nonzero = np.zeros(sc.n, bool)
    for v in flat.values():
        nonzero |= (v != 0).any(1)
    reached = np.nonzero(nonzero)[0]
    rng = np.random.default_rng(SAMPLE_SEED)
    sample = np.sort(rng.choice(reached, size=min(N_SAMPLE, len(reached)), replace=False))
    out = {"pixels": px, "color": r.color, "T": r.T, "ambiguous": r.ambiguous, "weights": w.astype(np.float32),
           "alt_start": r.alt_start, "alt_rows": r.alt_rows, "ambiguous_grad": r.ambiguous_grad,
           "nonzero_bits": np.packbits(nonzero), "sample": sample.astype(np.int64)}
    for k, v in flat.items():
        out[f"g_{k}"] = v[sample].astype(np.float32)
        out[f"norm_{k}"] = np.linalg.norm(v)
        out[f"max_{k}"] = np.abs(v).max()
    np.savez_compressed(path, **out)
    print(f"blobs1m: {len(reached)} Gaussians reached, {len(sample)} sampled", flush=True)


BATCH_VIEWS = (0, 9)          # two of the 16 views (different resolutions)
N_PIX_BATCH = 1024
SERVE_SEED = 123
N_SERVE = 2                   # requests per scene
N_PIX_SERVE = 512


def batch16(path: str) -> None:
    sc, poses = S.batch_config()
    out = {}
    for v in BATCH_VIEWS:
        pose = poses[v]
        px = S.sample_pixels(PIXEL_SEED_BLOBS + v, pose.width, pose.height, N_PIX_BATCH)
        t0 = time.time()
        r = O.render(sc, pose, pixels=px)
        print(f"batch16 view {v} ({pose.width}x{pose.height}): {time.time() - t0:.0f} s, "
              f"ambiguous {r.ambiguous.mean():.4f}", flush=True)
        for k, val in (("pixels", px), ("color", r.color), ("T", r.T), ("ambiguous", r.ambiguous),
                       ("alt_start", r.alt_start), ("alt_rows", r.alt_rows)):
            out[f"v{v}_{k}"] = val
    np.savez_compressed(path, views=np.array(BATCH_VIEWS), **out)


def serve_requests():
    """The seeded requests the serving parity test sends: N_SERVE per scene,
    scene A first, poses from the served-request generator."""
    rng = np.random.default_rng(SERVE_SEED)
    return [(name, S.random_request_pose(rng)) for name in ("A",) * N_SERVE + ("B",) * N_SERVE]


def serve(path: str) -> None:
    scA, scB = S.serve_scenes()
    out = {}
    for i, (name, pose) in enumerate(serve_requests()):
        sc = scA if name == "A" else scB
        px = S.sample_pixels(SERVE_SEED + i, pose.width, pose.height, N_PIX_SERVE)
        t0 = time.time()
        r = O.render(sc, pose, pixels=px)
        print(f"serve request {i} (scene {name}, {pose.width}x{pose.height}): {time.time() - t0:.0f} s, "
              f"ambiguous {r.ambiguous.mean():.4f}", flush=True)
        for k, val in (("pixels", px), ("color", r.color), ("T", r.T), ("ambiguous", r.ambiguous),
                       ("alt_start", r.alt_start), ("alt_rows", r.alt_rows)):
            out[f"r{i}_{k}"] = val
    np.savez_compressed(path, n=np.array(len(serve_requests())), **out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["clustered", "blobs1m", "batch16", "serve"]
    if "clustered" in which:
        clustered(os.path.join(HERE, "clustered_300k_4096px.npz"))
    if "blobs1m" in which:
        blobs1m(os.path.join(HERE, "blobs_1m_masked_4096px.npz"))
    if "batch16" in which:
        batch16(os.path.join(HERE, "batch16_3m_2views_1024px.npz"))
    if "serve" in which:
        serve(os.path.join(HERE, "serve_5m2m_4requests_512px.npz"))
