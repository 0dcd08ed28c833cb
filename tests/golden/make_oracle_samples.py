"""Writes the FP64 oracle's expected values for the full-size parity tests.

    python tests/golden/make_oracle_samples.py [clustered] [blobs1m]

The brute-force oracle takes minutes per workload at these sizes (every
Gaussian at every sampled pixel), so its results are stored once and read by
the GPU tests.  Only the seeded input generators (sgs_synth) and the oracle
are called; nothing here reads the HIP path.

clustered_300k_4096px.npz: the clustered workload (300k skew Gaussians, SH3,
  one 1280x720 view), 4096 seeded tile-stratified pixels: colour, final
  transmittance, the oracle's ambiguity flags (decisions within the margins
  where float32 may decide the other way) and, for ambiguous pixels, the
  colour and transmittance of every outcome of their uncertain decisions.

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


if __name__ == "__main__":
    which = sys.argv[1:] or ["clustered", "blobs1m"]
    if "clustered" in which:
        clustered(os.path.join(HERE, "clustered_300k_4096px.npz"))
    if "blobs1m" in which:
        blobs1m(os.path.join(HERE, "blobs_1m_masked_4096px.npz"))
