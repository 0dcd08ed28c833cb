"""Seeded synthetic inputs for the skew-Gaussian rasterizer.

This module is the ONLY code shared by the HIP product path and the FP64
oracle.  It draws random numbers and builds camera poses; it holds none of
the method's arithmetic (no projection, no covariance, no skew mapping, no
compositing, no coordinate-convention change).  Everything here is an input:

* Gaussian parameter sets in the structure-of-arrays layout both sides read
  (mean[3][N], log_scale[3][N], quat[4][N] as (w,x,y,z), skew[3][N],
  opa_logit[N], optional opa2_logit[N] / opa_dir[3][N], sh[K][3][N]),
  all float32.
* Camera poses as the interactive frontend produces them: an OpenGL/Blender
  camera-to-world matrix (camera looks down -Z, +Y up), a resolution and a
  horizontal field of view.  Converting that pose to the rasterizer's OpenCV
  convention is the method's job (the paper's CoordEngine) and is done
  separately by each side.
* Seeded pixel samples for checks on large images.

Generators follow the workload descriptions of the benchmark configurations
(tiny blobs scene, clustered SH3 scene, 1M differentiation scene, 3M
batching scene, served 5M/2M scenes); the datasets the paper trains on
(Mip-NeRF 360, Tanks&Temples, Deep Blending) are not available and these
scenes stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Scene", "Pose", "uniform_quaternions", "blobs_scene", "clusters_scene",
    "look_at_gl", "orbit_pose", "spline_poses", "free_flight_pose",
    "sample_pixels", "tiny_config", "clustered_config", "diff_config",
    "batch_config", "serve_scenes", "random_request_pose",
]


@dataclass
class Scene:
    """Float32 structure-of-arrays Gaussian parameters (host numpy)."""
    mean: np.ndarray            # [3][N]
    log_scale: np.ndarray       # [3][N]
    quat: np.ndarray            # [4][N]  (w, x, y, z), not necessarily unit
    skew: np.ndarray | None     # [3][N]  or None for a purely symmetric scene
    opa_logit: np.ndarray       # [N]
    sh: np.ndarray              # [K][3][N], K = (sh_degree+1)^2
    sh_degree: int
    opa2_logit: np.ndarray | None = None   # [N] second base opacity logit
    opa_dir: np.ndarray | None = None      # [3][N] opacity split direction

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        pick = lambda a: None if a is None else np.ascontiguousarray(a[..., idx], dtype=np.float32)
        return Scene(pick(self.mean), pick(self.log_scale), pick(self.quat),
                     pick(self.skew), pick(self.opa_logit), pick(self.sh),
                     self.sh_degree, pick(self.opa2_logit), pick(self.opa_dir))


@dataclass
class Pose:
    """Frontend camera: OpenGL camera-to-world (4x4 float64), W, H, fov."""
    c2w_gl: np.ndarray
    width: int
    height: int
    fovx_deg: float = 60.0
    near: float = 0.2
    bg: tuple = (0.0, 0.0, 0.0)


def uniform_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random unit quaternions (Shoemake, Graphics Gems III, 1992),
    returned as [4][n] in (w, x, y, z) order."""
    u1, u2, u3 = rng.random((3, n))
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    x = a * np.sin(2 * np.pi * u2)
    y = a * np.cos(2 * np.pi * u2)
    z = b * np.sin(2 * np.pi * u3)
    w = b * np.cos(2 * np.pi * u3)
    return np.stack([w, x, y, z]).astype(np.float32)


def _sh_coeffs(rng, n, deg, dc_std=0.5, hi_std=0.1):
    k = (deg + 1) ** 2
    sh = np.empty((k, 3, n), np.float32)
    sh[0] = rng.normal(0.0, dc_std, (3, n))
    if k > 1:
        sh[1:] = rng.normal(0.0, hi_std, (k - 1, 3, n))
    return sh


def blobs_scene(seed: int, n: int, sh_degree: int = 0, enhanced: bool = False,
                zero_skew: bool = False) -> Scene:
    """Tiny-config generator: means from 4 isotropic blobs (sigma 1) kept
    inside [-3,3]^3, log-scales N(-2.5,0.5), uniform unit quaternions, skew
    N(0,1.5) per axis with a random 25% of Gaussians set exactly to zero,
    opacity logits N(0,1.5), SH DC N(0,0.5) (higher bands N(0,0.1)).

    Blob centres are uniform in [-2,2]^3 and points are redrawn until they
    fall inside the [-3,3]^3 cube.  ``enhanced`` adds a second opacity logit
    N(0,1.5) and a direction N(0,1) per Gaussian (enhanced opacity)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-2.0, 2.0, (4, 3))
    which = rng.integers(0, 4, n)
    pts = centres[which] + rng.normal(0.0, 1.0, (n, 3))
    bad = np.any(np.abs(pts) > 3.0, axis=1)
    while bad.any():
        m = int(bad.sum())
        pts[bad] = centres[which[bad]] + rng.normal(0.0, 1.0, (m, 3))
        bad = np.any(np.abs(pts) > 3.0, axis=1)
    mean = pts.T.astype(np.float32)
    log_scale = rng.normal(-2.5, 0.5, (3, n)).astype(np.float32)
    quat = uniform_quaternions(rng, n)
    skew = rng.normal(0.0, 1.5, (3, n)).astype(np.float32)
    zero = rng.permutation(n)[: n // 4]
    skew[:, zero] = 0.0
    if zero_skew:
        skew[:] = 0.0
    opa = rng.normal(0.0, 1.5, n).astype(np.float32)
    sh = _sh_coeffs(rng, n, sh_degree)
    opa2 = opa_dir = None
    if enhanced:
        opa2 = rng.normal(0.0, 1.5, n).astype(np.float32)
        opa_dir = rng.normal(0.0, 1.0, (3, n)).astype(np.float32)
    return _contig(Scene(mean, log_scale, quat, skew, opa, sh, sh_degree, opa2, opa_dir))


def _contig(sc: Scene) -> Scene:
    for f in ("mean", "log_scale", "quat", "skew", "opa_logit", "sh", "opa2_logit", "opa_dir"):
        a = getattr(sc, f)
        if a is not None:
            setattr(sc, f, np.ascontiguousarray(a, dtype=np.float32))
    return sc


def _random_rotations(rng, m):
    """m random rotation matrices from the QR factorisation of Gaussian
    matrices (sign-corrected so the distribution is uniform, det = +1)."""
    out = np.empty((m, 3, 3))
    for i in range(m):
        q, r = np.linalg.qr(rng.normal(size=(3, 3)))
        q = q * np.sign(np.diag(r))[None, :]
        if np.linalg.det(q) < 0:
            q[:, 0] = -q[:, 0]
        out[i] = q
    return out


def clusters_scene(seed: int, n: int, sh_degree: int = 3, zero_skew: bool = False,
                   chunk: int = 1 << 20) -> Scene:
    """Clustered-config generator: 80% of means from 32 anisotropic clusters
    (centres uniform in [-10,10]^3, covariance R diag(sigma^2) R^T with sigma
    ~ U(0.2,2) per axis), 20% uniform in [-10,10]^3; log-scales N(-4,1)
    clipped to [-9,0]; skew N(0,2) per axis (all zero if ``zero_skew``);
    opacity logits N(0,1.5); SH DC N(0,0.5), higher bands N(0,0.1)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-10.0, 10.0, (32, 3))
    rots = _random_rotations(rng, 32)
    sig = rng.uniform(0.2, 2.0, (32, 3))
    n_cl = int(round(0.8 * n))
    mean = np.empty((3, n), np.float32)
    which = rng.integers(0, 32, n_cl)
    for s in range(0, n_cl, chunk):
        w = which[s:s + chunk]
        z = rng.normal(0.0, 1.0, (len(w), 3)) * sig[w]
        p = centres[w] + np.einsum("nij,nj->ni", rots[w], z)
        mean[:, s:s + len(w)] = p.T
    mean[:, n_cl:] = rng.uniform(-10.0, 10.0, (3, n - n_cl))
    log_scale = np.clip(rng.normal(-4.0, 1.0, (3, n)), -9.0, 0.0).astype(np.float32)
    quat = uniform_quaternions(rng, n)
    skew = None
    if not zero_skew:
        skew = rng.normal(0.0, 2.0, (3, n)).astype(np.float32)
    opa = rng.normal(0.0, 1.5, n).astype(np.float32)
    sh = _sh_coeffs(rng, n, sh_degree)
    return _contig(Scene(mean, log_scale, quat, skew, opa, sh, sh_degree))


# ----------------------------------------------------------------- poses
def look_at_gl(eye, target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """OpenGL/Blender camera-to-world matrix for a camera at ``eye`` looking
    at ``target``: columns are right, up, back (= -forward) and position."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    upv = np.asarray(up, np.float64)
    if abs(float(np.dot(f, upv))) > 0.999 * np.linalg.norm(upv):
        upv = np.array([0.0, 1.0, 0.0]) if abs(f[1]) < 0.9 else np.array([1.0, 0.0, 0.0])
    r = np.cross(f, upv)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    m = np.eye(4)
    m[:3, 0], m[:3, 1], m[:3, 2], m[:3, 3] = r, u, -f, eye
    return m


def orbit_pose(radius, azimuth_rad, elevation_rad, W, H, fovx_deg=60.0, near=0.2) -> Pose:
    ce = math.cos(elevation_rad)
    eye = radius * np.array([ce * math.cos(azimuth_rad), ce * math.sin(azimuth_rad),
                             math.sin(elevation_rad)])
    return Pose(look_at_gl(eye), W, H, fovx_deg, near)


def _catmull_rom_closed(ctrl: np.ndarray, m: int) -> np.ndarray:
    k = len(ctrl)
    out = []
    for i in range(m):
        u = i * k / m
        j = int(math.floor(u))
        t = u - j
        p0, p1, p2, p3 = (ctrl[(j - 1) % k], ctrl[j % k], ctrl[(j + 1) % k], ctrl[(j + 2) % k])
        t2, t3 = t * t, t * t * t
        out.append(0.5 * ((2 * p1) + (-p0 + p2) * t + (2 * p0 - 5 * p1 + 4 * p2 - p3) * t2
                          + (-p0 + 3 * p1 - 3 * p2 + p3) * t3))
    return np.array(out)


BATCH_RESOLUTIONS = [(640, 480), (1280, 720), (1600, 1064), (1920, 1080)]


def spline_poses(seed: int, n_views: int = 16, radius: float = 8.0,
                 resolutions=BATCH_RESOLUTIONS, fovx_deg=60.0, near=0.2):
    """Poses on a closed Catmull-Rom spline through 6 seeded control points at
    radius 8 +- 1 around the origin, all looking at the origin; resolutions
    cycle through ``resolutions``."""
    rng = np.random.default_rng(seed)
    az = np.sort(rng.uniform(0, 2 * np.pi, 6))
    el = rng.uniform(-0.5, 0.6, 6)
    rad = radius + rng.uniform(-1.0, 1.0, 6)
    ctrl = np.stack([rad * np.cos(el) * np.cos(az), rad * np.cos(el) * np.sin(az),
                     rad * np.sin(el)], 1)
    eyes = _catmull_rom_closed(ctrl, n_views)
    poses = []
    for i, e in enumerate(eyes):
        W, H = resolutions[i % len(resolutions)]
        poses.append(Pose(look_at_gl(e), W, H, fovx_deg, near))
    return poses


def free_flight_pose(rng, W, H, fovx_deg=60.0, near=0.2, extent=12.0) -> Pose:
    """A camera anywhere in [-extent, extent]^3 with a random yaw and pitch."""
    eye = rng.uniform(-extent, extent, 3)
    yaw = rng.uniform(0, 2 * np.pi)
    pitch = rng.uniform(-0.6, 0.6)
    fwd = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw),
                    math.sin(pitch)])
    return Pose(look_at_gl(eye, eye + fwd), W, H, fovx_deg, near)


SERVE_RESOLUTIONS = [(640, 480), (1280, 720), (1920, 1080)]


def random_request_pose(rng) -> Pose:
    """Served-request pose: 50% orbit (radius U(12,18), looking at the
    origin), 50% free flight; resolution uniform over 640x480, 1280x720,
    1920x1080."""
    W, H = SERVE_RESOLUTIONS[int(rng.integers(0, len(SERVE_RESOLUTIONS)))]
    if rng.random() < 0.5:
        return orbit_pose(rng.uniform(12, 18), rng.uniform(0, 2 * np.pi),
                          rng.uniform(-0.4, 0.8), W, H)
    return free_flight_pose(rng, W, H)


def sample_pixels(seed: int, W: int, H: int, n: int, tile: int = 16) -> np.ndarray:
    """``n`` distinct pixel indices (row-major y*W+x), stratified over tiles:
    tiles are visited in a seeded random order and one random pixel is taken
    from each until ``n`` pixels are drawn (then a second round, ...)."""
    rng = np.random.default_rng(seed)
    tx, ty = -(-W // tile), -(-H // tile)
    n = min(n, W * H)
    chosen = set()
    out = []
    while len(out) < n:
        for t in rng.permutation(tx * ty):
            x0, y0 = (t % tx) * tile, (t // tx) * tile
            x = x0 + int(rng.integers(0, min(tile, W - x0)))
            y = y0 + int(rng.integers(0, min(tile, H - y0)))
            p = y * W + x
            if p not in chosen:
                chosen.add(p)
                out.append(p)
                if len(out) == n:
                    break
    return np.array(sorted(out), np.int64)


# --------------------------------------------------------- named workloads
def tiny_config(seed: int = 0):
    """2,000 skew Gaussians (blobs), SH0; one 128x128 camera, fov 60 deg, at
    distance 8 looking at the origin, near 0.2."""
    return blobs_scene(seed, 2000, 0), Pose(look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), 128, 128)


def clustered_config(seed: int = 1):
    """300k skew Gaussians (clusters), SH3; one 1280x720 camera on a radius-15
    orbit (elevation 20 deg, azimuth from the seed)."""
    sc = clusters_scene(seed, 300_000, 3)
    az = float(np.random.default_rng(seed + 1000).uniform(0, 2 * np.pi))
    return sc, orbit_pose(15.0, az, math.radians(20.0), 1280, 720)


def small_batch_config(seed: int = 1, n_views: int = 16):
    """The clustered 300k SH3 scene seen from n_views 640x480 cameras on the
    radius-15 orbit (elevation 20 deg, azimuths evenly spaced from the seed's):
    many small views, where one launch per view leaves the GPU mostly idle."""
    sc = clusters_scene(seed, 300_000, 3)
    az0 = float(np.random.default_rng(seed + 1000).uniform(0, 2 * np.pi))
    return sc, [orbit_pose(15.0, az0 + 2 * np.pi * k / n_views, math.radians(20.0), 640, 480)
                for k in range(n_views)]


def diff_config(seed: int = 2, target_seed: int = 3, n: int = 1_000_000):
    """1M skew Gaussians (blobs generator, SH0) at one 1600x1064 view from
    distance 8; the target image comes from a separately seeded 1M set."""
    pose = Pose(look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), 1600, 1064)
    return blobs_scene(seed, n, 0), blobs_scene(target_seed, n, 0), pose


def train_config(seed: int = 2, target_seed: int = 3, n: int = 1_000_000, n_views: int = 4,
                 pose_seed: int = 9):
    """Multi-view training: the 1M-Gaussian differentiation scene and its
    separately seeded target set, seen from n_views spline poses at
    1600x1064 (distance 8 +- 1, looking at the origin)."""
    poses = spline_poses(pose_seed, n_views, resolutions=[(1600, 1064)])
    return blobs_scene(seed, n, 0), blobs_scene(target_seed, n, 0), poses


def batch_config(seed: int = 5, n: int = 3_000_000, n_views: int = 16):
    """3M skew Gaussians (blobs generator) and 16 spline poses of mixed
    resolution."""
    return blobs_scene(seed, n, 0), spline_poses(seed, n_views)


def serve_scenes(seed_a: int = 6, seed_b: int = 7, n_a: int = 5_000_000, n_b: int = 2_000_000):
    """Scene A: clustered SH3 skew scene; scene B: clustered SH3 with all skew
    exactly zero (symmetric 3DGS)."""
    return clusters_scene(seed_a, n_a, 3), clusters_scene(seed_b, n_b, 3, zero_skew=True)
