"""Plain FP64 CPU oracle of the 3D skew-Gaussian rasterizer.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this module.  It shares no code with
the HIP product path (no kernels, headers, helpers, constants or tables); the
only module both sides read is ``sgs_synth`` (seeded random inputs).

Everything is computed in float64 with plain PyTorch CPU tensor operations,
so that gradients are the exact derivatives of the forward definition
(autograd), and brute force: every Gaussian is evaluated at every requested
pixel, Gaussians are ordered near to far by camera-space depth (ties by
ascending index) and composited front to back.  No tiles, extents or radix
sorts are used.

Paper passages followed (3D Skew Gaussian Splatting):
  * Sec. "Preliminary of 3D Gaussian Splatting": Gaussian G(x), covariance
    Sigma = R S S^T R^T from a quaternion and a scale, SH colour, affine
    (EWA) projection to a 2D covariance Sigma', front-to-back compositing.
  * Sec. "3D Skew Gaussian Kernel": S(x) = 2 G(x) Phi(beta^T (x - mu)),
    Phi(z) = (1 + erf(z / sqrt 2)) / 2, zero skew gives 3DGS.
  * Alg. 1 (forward pass) and the appendix "Forward Pass": 2D opacity
    alpha = d G'(x) (1 + erf(z)), z = (beta_x dx + beta_y dy) / sqrt 2,
    d = o sqrt(det Sigma' / det(Sigma' + sI)), (Sigma' + sI)^-1 = [[a,b],[b,c]].
  * Sec. "3D Skew Gaussian Rasterization and Splatting": compositing equation
    and the enhanced opacity o(x) = ((a1 + a2) + (a1 - a2) erf((beta + d)^T x
    / sqrt 2)) / 2.
  * Alg. 3 and Sec. "Decoupled Interactive Visual Analytics Engine": M_cv =
    M_gl T_align with T_align = diag(1,-1,-1,1); intrinsics K from (W, H, FoV).

Readings where the paper is silent or inconsistent (each is a parameter or a
documented convention here):
  * The 2D skew (beta_x, beta_y) consumed by the rasterizer is the exact
    skew-normal marginal of the 3D kernel under the same affine map A used for
    Sigma' and the same isotropic blur sI:
        v = A Sigma beta, kappa = beta^T Sigma beta, m = v^T Q v,
        beta_2D = Q v / sqrt(1 + kappa - m),   Q = (Sigma' + sI)^-1.
    (Selection representation of the multivariate skew-normal; Azzalini &
    Dalla Valle 1996, Azzalini & Capitanio 1999.)  Zero skew maps to zero.
  * Enhanced opacity: x is the 2D offset p - mu_2D and (beta + d) is mapped to
    2D by the same rule; with a1 = a2 it reduces to a scalar opacity.
  * alpha is clamped to 0.99, pairs with alpha < 1/255 are skipped and a pixel
    stops before the Gaussian that would take its transmittance below 1e-4.
  * Low-pass filter s = 0.3 px^2 with opacity compensation; Jacobian evaluated
    with x/z, y/z clamped to 1.3 tan(half FoV); Gaussians with z <= near are
    culled; pixel (i, j) is sampled at (i + 0.5, j + 0.5); fy = fx (square
    pixels, horizontal FoV); background colour defaults to black.
  * Real spherical harmonics with the Condon-Shortley phase, ordered m = -l..l
    (sin terms for m < 0), colour = max(0, sum + 0.5).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

F64 = torch.float64
SQRT2 = math.sqrt(2.0)

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4


@dataclass
class Options:
    filter_s: float = 0.3
    compensate: bool = True
    guard: float = 1.3
    alpha_min: float = ALPHA_MIN
    alpha_max: float = ALPHA_MAX
    t_min: float = T_MIN
    symmetric: bool = False   # drop the skew factor entirely (textbook 3DGS)


# ------------------------------------------------------------------ camera
T_ALIGN = np.diag([1.0, -1.0, -1.0, 1.0])


def coord_engine(c2w_gl: np.ndarray) -> np.ndarray:
    """OpenGL/Blender camera-to-world -> OpenCV camera-to-world,
    M_cv = M_gl T_align (Alg. 3, Sec. "Decoupled Interactive Visual Analytics
    Engine", coordinate-alignment equation)."""
    return np.asarray(c2w_gl, np.float64) @ T_ALIGN


def intrinsics(W: int, H: int, fovx_deg: float, fovy_deg: float | None = None) -> np.ndarray:
    """K = [[W/(2 tan(FoVx/2)), 0, W/2], [0, H/(2 tan(FoVy/2)), H/2], [0,0,1]]
    (Sec. "Decoupled Interactive Visual Analytics Engine", intrinsic mapping).
    With one FoV given it is horizontal and pixels are square."""
    fx = W / (2.0 * math.tan(math.radians(fovx_deg) / 2.0))
    fy = fx if fovy_deg is None else H / (2.0 * math.tan(math.radians(fovy_deg) / 2.0))
    return np.array([[fx, 0.0, W / 2.0], [0.0, fy, H / 2.0], [0.0, 0.0, 1.0]])


@dataclass
class Camera:
    W: int
    H: int
    K: np.ndarray       # 3x3
    w2c: np.ndarray     # 4x4 OpenCV world-to-camera
    near: float
    bg: np.ndarray      # [3]

    @property
    def position(self) -> np.ndarray:
        return np.linalg.inv(self.w2c)[:3, 3]


def camera_from_pose(pose) -> Camera:
    """Frontend pose (sgs_synth.Pose) -> rasterizer camera via CoordEngine."""
    m_cv = coord_engine(pose.c2w_gl)
    return Camera(int(pose.width), int(pose.height),
                  intrinsics(pose.width, pose.height, pose.fovx_deg),
                  np.linalg.inv(m_cv), float(pose.near), np.asarray(pose.bg, np.float64))


# ---------------------------------------------------------- spherical harm.
def _legendre_derivative_coeffs(l: int, m: int) -> np.ndarray:
    """Power-series coefficients of d^m/dz^m P_l(z)."""
    c = np.polynomial.legendre.leg2poly([0] * l + [1])
    return np.polynomial.polynomial.polyder(c, m) if m > 0 else c


def sh_basis(deg: int, d: torch.Tensor) -> torch.Tensor:
    """Real SH Y_lm at unit directions d [N,3] -> [N, (deg+1)^2].

    Y_l0 = N_l0 P_l(z); for m > 0 the cos/sin pair is
    sqrt(2) N_lm P_l^m(cos t) {cos m phi, sin m phi}, where
    P_l^m(cos t) {cos, sin}(m phi) = (-1)^m P_l^(m)(z) {Re, Im}((x + i y)^m)
    (Condon-Shortley phase) and N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
    Order within a band: m = -l..l, sin terms for m < 0."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    out = []
    for l in range(deg + 1):
        band = [None] * (2 * l + 1)
        re, im = torch.ones_like(x), torch.zeros_like(x)    # (x + i y)^0
        for m in range(0, l + 1):
            if m > 0:
                re, im = re * x - im * y, re * y + im * x
            coeffs = _legendre_derivative_coeffs(l, m)
            poly = torch.zeros_like(z)
            for k in reversed(range(len(coeffs))):
                poly = poly * z + float(coeffs[k])
            nlm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
            if m == 0:
                band[l] = nlm * poly
            else:
                s = ((-1) ** m) * math.sqrt(2.0) * nlm
                band[l + m] = s * poly * re
                band[l - m] = s * poly * im
        out.extend(band)
    return torch.stack(out, 1)


# ------------------------------------------------------------ depth key
def fma_f32(a, b, c) -> np.ndarray:
    """Correctly rounded float32 fused multiply-add a * b + c of float32
    arrays (IEEE 754 fusedMultiplyAdd, round to nearest even): the product
    of two float32 values is exact in float64; TwoSum (Knuth) gives the sum
    s + e exactly; rounding s to float32 is then correct except when s is a
    float32 midpoint, where the sign of e (or evenness, when e = 0) decides."""
    a = np.asarray(a, np.float32).astype(np.float64)
    b = np.asarray(b, np.float32).astype(np.float64)
    c = np.asarray(c, np.float32).astype(np.float64)
    p = a * b                                   # exact (48-bit significand)
    s = p + c
    bb = s - p
    e = (p - (s - bb)) + (c - bb)               # s + e == p + c exactly
    r = s.astype(np.float32)
    d = s - r.astype(np.float64)
    up = np.nextafter(r, np.float32(np.inf))
    dn = np.nextafter(r, np.float32(-np.inf))
    half_up = (up.astype(np.float64) - r.astype(np.float64)) / 2
    half_dn = (r.astype(np.float64) - dn.astype(np.float64)) / 2
    # s on a midpoint: r is the even neighbour; move if e points the other way
    mid_up = (d == half_up) & (half_up > 0)     # s = r + half ulp: tie broken downwards to r
    mid_dn = (d == -half_dn) & (half_dn > 0)    # s = r - half ulp: tie broken upwards to r
    r = np.where(mid_up & (e > 0), up, r)
    r = np.where(mid_dn & (e < 0), dn, r)
    return r.astype(np.float32)


def depth_key(mean_f32: np.ndarray, cam: Camera) -> np.ndarray:
    """Camera-space depth as the float32 key of ordering and near culling:
    z = fma(r20, x, fma(r21, y, fma(r22, z, t2))) in float32 from the float32
    means and the float32-rounded third row of w2c, every fma correctly
    rounded, so that any implementation of this expression gets the same bits
    (reading R17: order by camera z, ties by index)."""
    W = cam.w2c[2, :4].astype(np.float32)
    x, y, z = (np.asarray(mean_f32[k], np.float32) for k in range(3))
    return fma_f32(W[0], x, fma_f32(W[1], y, fma_f32(W[2], z, W[3])))


# ----------------------------------------------------------- per Gaussian
def quat_to_rotmat(q: torch.Tensor) -> torch.Tensor:
    """Unit-quaternion rotation matrix, q = (w, x, y, z) normalised first."""
    q = q / torch.linalg.norm(q, dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], 1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], 1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1),
    ], 1)


def skew_to_2d(g: torch.Tensor, sigma3: torch.Tensor, A: torch.Tensor, Q: torch.Tensor) -> torch.Tensor:
    """2D skew of the image of a 3D skew-normal under the affine map A with
    blur sI (Q = (A Sigma A^T + sI)^-1):  Q v / sqrt(1 + g^T Sigma g - v^T Q v),
    v = A Sigma g.  g [N,3], sigma3 [N,3,3], A [N,2,3], Q [N,2,2] -> [N,2]."""
    sg = torch.einsum("nij,nj->ni", sigma3, g)
    v = torch.einsum("nij,nj->ni", A, sg)
    qv = torch.einsum("nij,nj->ni", Q, v)
    kappa = (g * sg).sum(1)
    m = (v * qv).sum(1)
    return qv / torch.sqrt(1.0 + kappa - m)[:, None]


@dataclass
class Projected:
    mu2d: torch.Tensor      # [N,2] pixels
    conic: torch.Tensor     # [N,3] (a, b, c) of (Sigma' + sI)^-1
    rho: torch.Tensor       # [N]   sqrt(det Sigma' / det(Sigma' + sI)) (or 1)
    o1: torch.Tensor        # [N]
    o2: torch.Tensor        # [N]
    beta2d: torch.Tensor    # [N,2]
    w2d: torch.Tensor | None  # [N,2] enhanced-opacity direction in 2D
    rgb: torch.Tensor       # [N,3]
    depth: torch.Tensor     # [N] camera-space z
    valid: torch.Tensor     # [N] bool (not culled)
    z32: torch.Tensor | None = None   # [N] float32 depth key (ordering and near cull)


def to_tensors(scene, requires_grad=False, dtype=F64) -> dict:
    """Scene arrays (float32 SoA) -> float64 [N, ...] leaf tensors (float32
    with dtype=torch.float32: used only to size the decision margins)."""
    npt = np.float64 if dtype == F64 else np.float32
    def t(a, shape_fn):
        if a is None:
            return None
        x = torch.from_numpy(np.ascontiguousarray(shape_fn(np.asarray(a, npt))))
        return x.requires_grad_(requires_grad)
    return {
        "mean": t(scene.mean, lambda a: a.T),
        "log_scale": t(scene.log_scale, lambda a: a.T),
        "quat": t(scene.quat, lambda a: a.T),
        "skew": t(scene.skew, lambda a: a.T),
        "opa_logit": t(scene.opa_logit, lambda a: a),
        "opa2_logit": t(scene.opa2_logit, lambda a: a),
        "opa_dir": t(scene.opa_dir, lambda a: a.T),
        "sh": t(scene.sh, lambda a: a.transpose(2, 0, 1)),   # [N, K, 3]
    }


def project(P: dict, sh_degree: int, cam: Camera, opt: Options = Options(),
            mu2d_shift: torch.Tensor | None = None) -> Projected:
    """Per-Gaussian projection (Sec. "Preliminary of 3D Gaussian Splatting";
    appendix "Forward Pass"; 2D skew and enhanced-opacity readings above).
    ``mu2d_shift`` [N,2] (pixels) is added to the projected means: a handle
    for the gradient with respect to the 2D means, zero in every render."""
    mean = P["mean"]
    n = mean.shape[0]
    dt = mean.dtype
    # Sigma = R S S^T R^T
    s = torch.exp(P["log_scale"])
    R = quat_to_rotmat(P["quat"])
    M = R * s[:, None, :]
    sigma3 = M @ M.transpose(1, 2)
    # world -> camera (OpenCV)
    Wr = torch.from_numpy(cam.w2c[:3, :3].copy()).to(dt)
    tv = torch.from_numpy(cam.w2c[:3, 3].copy()).to(dt)
    t = mean @ Wr.T + tv
    tx, ty, tz = t.unbind(1)
    # order and near cull by the float32 depth key (the projection itself
    # uses the full-precision tz)
    z32 = torch.from_numpy(depth_key(mean.detach().numpy().T.astype(np.float32), cam).astype(np.float64))
    valid = (z32 > float(np.float32(cam.near))) & torch.isfinite(z32)
    fx, fy, cx, cy = cam.K[0, 0], cam.K[1, 1], cam.K[0, 2], cam.K[1, 2]
    tzs = torch.where(valid, tz, torch.ones_like(tz))      # culled rows: harmless values
    limx = opt.guard * (cam.W / (2.0 * fx))
    limy = opt.guard * (cam.H / (2.0 * fy))
    txc = torch.clamp(tx / tzs, -limx, limx) * tzs
    tyc = torch.clamp(ty / tzs, -limy, limy) * tzs
    zero = torch.zeros_like(tzs)
    J = torch.stack([
        torch.stack([fx / tzs, zero, -fx * txc / (tzs * tzs)], 1),
        torch.stack([zero, fy / tzs, -fy * tyc / (tzs * tzs)], 1),
    ], 1)
    A = J @ Wr
    sig2 = A @ sigma3 @ A.transpose(1, 2)
    eye = torch.eye(2, dtype=dt)
    sigf = sig2 + opt.filter_s * eye
    det2 = sig2[:, 0, 0] * sig2[:, 1, 1] - sig2[:, 0, 1] * sig2[:, 1, 0]
    detf = sigf[:, 0, 0] * sigf[:, 1, 1] - sigf[:, 0, 1] * sigf[:, 1, 0]
    valid = valid & (detf > 0)
    detf_s = torch.where(valid, detf, torch.ones_like(detf))
    Q = torch.linalg.inv(torch.where(valid[:, None, None], sigf, eye.expand(n, 2, 2)))
    conic = torch.stack([Q[:, 0, 0], Q[:, 0, 1], Q[:, 1, 1]], 1)
    if opt.compensate:
        rho = torch.sqrt(torch.clamp(det2, min=0.0) / detf_s)
    else:
        rho = torch.ones_like(detf_s)
    mu2d = torch.stack([fx * tx / tzs + cx, fy * ty / tzs + cy], 1)
    if mu2d_shift is not None:
        mu2d = mu2d + mu2d_shift
    o1 = torch.sigmoid(P["opa_logit"])
    o2 = torch.sigmoid(P["opa2_logit"]) if P.get("opa2_logit") is not None else o1
    if P.get("skew") is not None and not opt.symmetric:
        beta2d = skew_to_2d(P["skew"], sigma3, A, Q)
    else:
        beta2d = torch.zeros((n, 2), dtype=dt)
    w2d = None
    if P.get("opa2_logit") is not None:
        g = P["opa_dir"] if P.get("opa_dir") is not None else torch.zeros((n, 3), dtype=dt)
        if P.get("skew") is not None:
            g = g + P["skew"]
        w2d = skew_to_2d(g, sigma3, A, Q)
    # view-dependent colour from SH
    campos = torch.from_numpy(cam.position.copy()).to(dt)
    dvec = mean - campos
    dirs = dvec / torch.linalg.norm(dvec, dim=1, keepdim=True)
    Y = sh_basis(sh_degree, dirs)                           # [N, K]
    rgb = torch.clamp((Y[:, :, None] * P["sh"]).sum(1) + 0.5, min=0.0)
    return Projected(mu2d, conic, rho, o1, o2, beta2d, w2d, rgb, tz, valid, z32)


# ------------------------------------------------------------ per pixel
def pixel_centres(cam: Camera, pixels: np.ndarray | None) -> tuple[np.ndarray, torch.Tensor]:
    if pixels is None:
        pixels = np.arange(cam.W * cam.H, dtype=np.int64)
    px = (pixels % cam.W).astype(np.float64) + 0.5
    py = (pixels // cam.W).astype(np.float64) + 0.5
    return pixels, torch.from_numpy(np.stack([px, py], 1))


def alpha_tilde(pc: torch.Tensor, pr: Projected, idx: torch.Tensor, opt: Options):
    """Unclamped 2D opacity of Gaussians ``idx`` at pixel centres pc [P,2]:
    alpha~ = rho o(delta) G'(delta) (1 + erf(beta . delta / sqrt 2)), with
    G' = exp(-(a dx^2 + c dy^2)/2 - b dx dy) (Alg. 1).  Returns [P, len(idx)]."""
    pc = pc.to(pr.mu2d.dtype)
    mu = pr.mu2d[idx]
    dx = pc[:, None, 0] - mu[None, :, 0]
    dy = pc[:, None, 1] - mu[None, :, 1]
    a, b, c = pr.conic[idx].unbind(1)
    g = torch.exp(-0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy)
    bx, by = pr.beta2d[idx].unbind(1)
    if opt.symmetric:
        skew = torch.ones_like(g)
    else:
        skew = 1.0 + torch.erf((bx * dx + by * dy) / SQRT2)
    if pr.w2d is not None:
        wx, wy = pr.w2d[idx].unbind(1)
        o = 0.5 * ((pr.o1[idx] + pr.o2[idx]) + (pr.o1[idx] - pr.o2[idx]) * torch.erf((wx * dx + wy * dy) / SQRT2))
    else:
        o = pr.o1[idx]
    return pr.rho[idx] * o * g * skew


def power_terms(pc: torch.Tensor, pr: Projected, idx: torch.Tensor) -> torch.Tensor:
    """Magnitude of the terms of the exponent of G' at pixel centres pc:
    (|a| dx^2 + 2 |b dx dy| + |c| dy^2) / 2, [P, len(idx)].  A float32
    pipeline stores the 2D mean and conic rounded to float32, which moves
    the exponent by up to a few float32 ulps of this magnitude: for thin,
    long ellipses far from their centre the terms are 1e4 times the
    exponent itself.  Test infrastructure: it widens the ambiguity margins
    of render(), nothing else."""
    mu = pr.mu2d[idx]
    dx = pc[:, None, 0] - mu[None, :, 0]
    dy = pc[:, None, 1] - mu[None, :, 1]
    a, b, c = pr.conic[idx].unbind(1)
    return 0.5 * (a.abs() * dx * dx + 2.0 * (b * dx * dy).abs() + c.abs() * dy * dy)


def depth_order(pr: Projected) -> torch.Tensor:
    """Valid Gaussians sorted near to far by the float32 depth key, ties by
    index."""
    idx = torch.nonzero(pr.valid).flatten()
    key = (pr.z32 if pr.z32 is not None else pr.depth.detach())[idx].numpy()
    order = np.argsort(key, kind="stable")
    return idx[torch.from_numpy(order)]


def inclusion_with(at: torch.Tensor, opt: Options, keep: torch.Tensor) -> torch.Tensor:
    """The inclusion rule with the alpha_min decisions given (keep [P,K]):
    the pixel still stops before the first kept pair whose T_{k+1} would fall
    below t_min."""
    alpha = torch.clamp(at, max=opt.alpha_max)
    a = torch.where(keep, alpha, torch.zeros_like(alpha))
    live = torch.cumprod(1.0 - a, dim=1) >= opt.t_min
    return keep & live


def composite_pixel(at: np.ndarray, rgb: np.ndarray, bg: np.ndarray, opt: Options,
                    flip_keep=(), flip_stop=()) -> np.ndarray:
    """One pixel's front-to-back compositing written as the Alg. 1 loop (at
    [K] unclamped alpha in depth order, rgb [K,3]), with the alpha_min
    decision of the pairs in flip_keep and the stop decision of the pairs in
    flip_stop taken the other way.  Returns (C, T) as [4]."""
    T = 1.0
    C = np.zeros(3)
    for k in range(len(at)):
        a = min(opt.alpha_max, float(at[k]))
        if (a >= opt.alpha_min) == (k in flip_keep):
            continue
        Tn = T * (1.0 - a)
        if (Tn < opt.t_min) != (k in flip_stop):
            break
        C = C + rgb[k] * (a * T)
        T = Tn
    return np.concatenate([C + T * np.asarray(bg, np.float64), [T]])


def inclusion(at: torch.Tensor, opt: Options) -> torch.Tensor:
    """Which ordered pairs contribute (Alg. 1 loop with the thresholds of the
    readings): alpha = min(0.99, alpha~) must reach 1/255, and the pixel stops
    before the first Gaussian whose T_{k+1} = T_k (1 - alpha_k) would fall
    below t_min.  at [P,K] in depth order -> bool [P,K]."""
    alpha = torch.clamp(at, max=opt.alpha_max)
    keep = alpha >= opt.alpha_min
    a = torch.where(keep, alpha, torch.zeros_like(alpha))
    t_after = torch.cumprod(1.0 - a, dim=1)
    # T is non-increasing, so "not yet stopped" is a prefix of the list
    live = t_after >= opt.t_min
    return keep & live


def composite(at: torch.Tensor, rgb: torch.Tensor, bg: torch.Tensor, include: torch.Tensor,
              opt: Options):
    """Front-to-back compositing (compositing equation; Alg. 1 loop):
    C = sum_k c_k alpha_k T_k + T_final bg with T_k = prod_{j<k} (1 - alpha_j)
    over the included pairs.  at [P,K] unclamped alpha in depth order,
    rgb [K,3], include [P,K] fixed decisions.  Returns C [P,3], T_final [P]."""
    alpha = torch.clamp(at, max=opt.alpha_max)
    a = torch.where(include, alpha, torch.zeros_like(alpha))
    t_after = torch.cumprod(1.0 - a, dim=1)
    t_before = torch.cat([torch.ones_like(t_after[:, :1]), t_after[:, :-1]], 1)
    C = (a * t_before) @ rgb
    T_final = t_after[:, -1] if t_after.shape[1] else torch.ones(at.shape[0], dtype=F64)
    return C + T_final[:, None] * bg[None, :], T_final


@dataclass
class RenderResult:
    pixels: np.ndarray
    color: np.ndarray        # [P,3]
    T: np.ndarray            # [P]
    last: np.ndarray         # [P] index of the last contributing Gaussian (-1 if none)
    n_contrib: np.ndarray    # [P]
    ambiguous: np.ndarray    # [P] bool: a decision of the image within the margins below
    # ambiguous pixels whose only uncertain decisions are alpha >= alpha_min
    # (at most MAX_FLIPS of them): (C, T) of every combination of those
    # decisions, as rows [n_alt, 4] of alt_rows[alt_start[p]:alt_start[p+1]];
    # an empty range for pixels without alternatives
    alt_start: np.ndarray | None = None   # [P+1]
    alt_rows: np.ndarray | None = None    # [*, 4]
    # ambiguous for a gradient: also alpha~ within the margins of the 0.99
    # clamp, where the derivative of alpha jumps
    ambiguous_grad: np.ndarray | None = None


MAX_FLIPS = 4


def skew_factor(pc: torch.Tensor, pr: Projected, idx: torch.Tensor, opt: Options) -> torch.Tensor:
    """1 + erf(beta . delta / sqrt 2) of Gaussians ``idx`` at pixel centres
    pc [P,2] (1 in the symmetric mode).  Returns [P, len(idx)]."""
    pc = pc.to(pr.mu2d.dtype)
    mu = pr.mu2d[idx]
    dx = pc[:, None, 0] - mu[None, :, 0]
    dy = pc[:, None, 1] - mu[None, :, 1]
    if opt.symmetric:
        return torch.ones_like(dx)
    bx, by = pr.beta2d[idx].unbind(1)
    return 1.0 + torch.erf((bx * dx + by * dy) / SQRT2)


def _margins(at, order_depth, opt, rel, cond=None, pair_extra=None, detail=False):
    """Per-pixel flag: some decision of the definition lies within a relative
    margin of its threshold, where float32 evaluation may legitimately
    decide the other way (alpha vs 1/255 or vs the 0.99 clamp, T(1-alpha) vs
    the stop level, two reaching Gaussians at equal depth).  Alpha margins
    are on the log scale, |ln(alpha~ / threshold)| <= margin, and a pair's
    grows by rel["cond"] times its power_terms (cond): rounding the stored
    exponent's terms scales alpha~ by exp(+-rel["cond"] * power_terms).
    pair_extra [P,K]: a further per-pair margin on the same log scale.
    detail: also return the per-pair alpha_min flags [P,K] (pairs up to the
    stop point) and the per-pixel flag of the other kinds of ambiguity."""
    ra = rel["alpha"] if cond is None else rel["alpha"] + rel.get("cond", 0.0) * cond
    if pair_extra is not None:
        ra = ra + pair_extra
    la = torch.log(at.clamp_min(1e-300))
    alpha = torch.clamp(at, max=opt.alpha_max)
    a = torch.where(alpha >= opt.alpha_min, alpha, torch.zeros_like(alpha))
    ta = torch.cumprod(1.0 - a, 1)
    stopped = ta < opt.t_min
    upto = torch.cumsum(stopped.to(torch.int64), 1) <= 1     # up to the stop point
    flip = ((la - math.log(opt.alpha_min)).abs() <= ra) & upto
    tflip = ((ta - opt.t_min).abs() <= rel["T"] * opt.t_min) & (a > 0) & upto
    amb = flip.any(1) | tflip.any(1)
    other = torch.zeros_like(amb)
    # alpha near the 0.99 clamp changes no decision of the image (both sides'
    # alpha differ by the same rounding either way) but the derivative there
    # jumps: flagged for gradients only
    clamp = ((la - math.log(opt.alpha_max)).abs() <= ra).any(1)
    # depth keys: both sides order by the same float32 key and break equal
    # keys by index; two Gaussians that reach the pixel, consecutive among
    # those that do, whose keys differ by a few float32 ulps at most could
    # only swap if a key's bits differed between implementations (from w2c
    # rounded differently): flagged
    z = order_depth
    if z.numel() > 1 and rel.get("depth", 0.0) > 0:
        reach = (at >= opt.alpha_min * (1 - rel["alpha"])) & upto
        for p in torch.nonzero(reach.sum(1) > 1).flatten().tolist():
            zp = z[reach[p]]
            dz = (zp[1:] - zp[:-1]).abs()
            if bool(((dz > 0) & (dz <= rel["depth"] * zp[1:].abs())).any()):
                amb[p] = True
                other[p] = True
    return (amb, flip, tflip, other, amb | clamp) if detail else amb | clamp


# Margins where a float32 pipeline may decide a threshold the other way, on
# the log scale of alpha~ (reading R18):
#   "alpha": a floor (the blend's own rounding: exp2, products, the stored
#            log of the opacity factor: a few float32 ulps of an exponent <= 8)
#   "cond":  2^-23 (two float32 half-ulps) per unit of power_terms (rounding
#            of the stored mean and conic)
#   "fp32":  times |ln alpha~_f32 - ln alpha~|, the change when the same
#            projection and alpha are evaluated in float32 from the float32
#            inputs (the size of the projection's float32 error for this pair)
#   "erf":   an absolute error of 1 + erf(z) (a float32 erfc approximation with
#            |error| <= 1.5e-7 plus its own rounding), divided by 1 + erf(z)
# T: relative margin of T(1 - alpha) against t_min; depth: relative
# difference of two float32 depth keys (2 ulps) below which their order is
# flagged (see _margins).
DEFAULT_MARGINS = {"alpha": 1e-5, "cond": 2.0 ** -22, "fp32": 8.0, "erf": 3e-7,
                   "T": 2e-3, "depth": 0.0}


def render(scene, pose_or_cam, pixels: np.ndarray | None = None, opt: Options = Options(),
           chunk_elems: int = 1 << 19, margins=DEFAULT_MARGINS) -> RenderResult:
    """Brute-force FP64 render of ``pixels`` (row-major indices; all if None)."""
    cam = pose_or_cam if isinstance(pose_or_cam, Camera) else camera_from_pose(pose_or_cam)
    with torch.no_grad():
        P = to_tensors(scene)
        pr = project(P, scene.sh_degree, cam, opt)
        order = depth_order(pr)
        pixels, pc = pixel_centres(cam, pixels)
        bg = torch.from_numpy(cam.bg.astype(np.float64))
        rgb = pr.rgb[order]
        od = pr.z32[order]
        n_pix = pc.shape[0]
        # the same projection in float32 (margins only: it sizes how far a
        # float32 pipeline's alpha~ may sit from the FP64 value)
        pr32 = project(to_tensors(scene, dtype=torch.float32), scene.sh_degree, cam, opt) \
            if margins.get("fp32", 0.0) > 0 else None
        bad32 = None if pr32 is None else ~pr32.valid[order]
        col = np.zeros((n_pix, 3)); Tf = np.ones(n_pix)
        last = np.full(n_pix, -1, np.int64); ncon = np.zeros(n_pix, np.int64)
        amb = np.zeros(n_pix, bool)
        amb_grad = np.zeros(n_pix, bool)
        alts = {}
        step = max(1, chunk_elems // max(1, order.numel()))
        for s in range(0, n_pix, step):
            pcs = pc[s:s + step]
            at = alpha_tilde(pcs, pr, order, opt)
            inc = inclusion(at, opt)
            C, T = composite(at, rgb, bg, inc, opt)
            col[s:s + step] = C.numpy(); Tf[s:s + step] = T.numpy()
            cnt = inc.sum(1)
            ncon[s:s + step] = cnt.numpy()
            k = inc.shape[1]
            lastpos = torch.where(inc, torch.arange(k).expand_as(inc), torch.full_like(inc, -1, dtype=torch.int64)).max(1).values if k else torch.full((pcs.shape[0],), -1)
            last[s:s + step] = np.where(lastpos.numpy() >= 0, order.numpy()[np.maximum(lastpos.numpy(), 0)], -1)
            cond = power_terms(pcs, pr, order) if margins.get("cond", 0.0) > 0 else None
            # per-pair margins, on the pairs near a threshold only (far below
            # it neither term can move a decision, and float32 underflows)
            la = torch.log(at.clamp_min(1e-300))
            near = ((la - math.log(opt.alpha_min)).abs() < 0.5) | ((la - math.log(opt.alpha_max)).abs() < 0.5)
            extra = torch.zeros_like(la)
            if pr32 is not None:
                la32 = torch.log(alpha_tilde(pcs, pr32, order, opt).double().clamp_min(1e-300))
                dl = (la32 - la).abs().clamp_max(1e-2)
                # a Gaussian the float32 projection culls gets a wide margin
                dl = torch.where(bad32[None, :] | ~torch.isfinite(dl), torch.full_like(dl, 1e-2), dl)
                extra = extra + margins["fp32"] * dl
            if margins.get("erf", 0.0) > 0:
                extra = extra + (margins["erf"] / skew_factor(pcs, pr, order, opt).clamp_min(1e-300)).clamp_max(1e-2)
            extra = torch.where(near, extra, torch.zeros_like(extra))
            a_, flip, tflip, other, ag = _margins(at, od, opt, margins, cond, extra, detail=True)
            amb[s:s + step] = a_.numpy()
            amb_grad[s:s + step] = ag.numpy()
            # every outcome of the uncertain decisions of a pixel: each
            # alpha_min decision and each stop decision near its threshold
            # taken either way
            for q in torch.nonzero(a_ & ~other).flatten().tolist():
                fa = torch.nonzero(flip[q]).flatten().tolist()
                ft = torch.nonzero(tflip[q]).flatten().tolist()
                if len(fa) + len(ft) > MAX_FLIPS:
                    continue
                atq = at[q].numpy()
                rows = []
                for bits in range(1 << (len(fa) + len(ft))):
                    fa_set = {k for j, k in enumerate(fa) if (bits >> j) & 1}
                    ft_set = {k for j, k in enumerate(ft) if (bits >> (len(fa) + j)) & 1}
                    rows.append(composite_pixel(atq, rgb.numpy(), cam.bg, opt, fa_set, ft_set))
                alts[s + q] = np.array(rows)
    starts = np.zeros(n_pix + 1, np.int64)
    for q in range(n_pix):
        starts[q + 1] = starts[q] + (len(alts[q]) if q in alts else 0)
    rows = np.concatenate([alts[q] for q in sorted(alts)]) if alts else np.zeros((0, 4))
    return RenderResult(pixels, col, Tf, last, ncon, amb, starts, rows, amb_grad)


def float32_error_bound(scene, pose_or_cam, pixels: np.ndarray | None = None, opt: Options = Options(),
                        u: float = 2.0 ** -22, chunk_elems: int = 1 << 19):
    """First-order bound of the image and transmittance error that a float32
    pipeline may incur from storing each pair's 2D mean and conic rounded:
    with every alpha~ of an included pair off by a relative u * power_terms,
    |dC_p| <= sum_k |dC_p/d alpha~_pk| alpha~_pk u power_terms_pk (same for
    T).  The derivatives come from autograd through the same compositing
    definition as render(), with the inclusion decisions held fixed.  Test
    infrastructure: it sizes tolerances for ill-conditioned inputs (thin,
    long ellipses), and is negligible for ordinary ones.  Returns
    (bound_C [P,3], bound_T [P])."""
    cam = pose_or_cam if isinstance(pose_or_cam, Camera) else camera_from_pose(pose_or_cam)
    with torch.no_grad():
        P = to_tensors(scene)
        pr = project(P, scene.sh_degree, cam, opt)
        order = depth_order(pr)
        pixels, pc = pixel_centres(cam, pixels)
        bg = torch.from_numpy(cam.bg.astype(np.float64))
        rgb = pr.rgb[order]
    n_pix = pc.shape[0]
    bC = np.zeros((n_pix, 3)); bT = np.zeros(n_pix)
    step = max(1, chunk_elems // max(1, order.numel()))
    for s in range(0, n_pix, step):
        pcs = pc[s:s + step]
        with torch.no_grad():
            at0 = alpha_tilde(pcs, pr, order, opt)
            inc = inclusion(at0, opt)
            e = u * power_terms(pcs, pr, order) * at0
        at = at0.clone().requires_grad_(True)
        C, T = composite(at, rgb, bg, inc, opt)
        for ch in range(4):
            out = T if ch == 3 else C[:, ch]
            g, = torch.autograd.grad(out.sum(), at, retain_graph=ch < 3)
            b = (g.abs() * e).sum(1).detach().numpy()
            if ch == 3:
                bT[s:s + step] = b
            else:
                bC[s:s + step, ch] = b
    return bC, bT


def project_numpy(scene, pose_or_cam, opt: Options = Options()) -> dict:
    """Per-Gaussian projected quantities as float64 numpy arrays."""
    cam = pose_or_cam if isinstance(pose_or_cam, Camera) else camera_from_pose(pose_or_cam)
    with torch.no_grad():
        pr = project(to_tensors(scene), scene.sh_degree, cam, opt)
    out = {k: (None if v is None else v.numpy()) for k, v in pr.__dict__.items()}
    return out


def render_grad(scene, pose_or_cam, dL_dC: np.ndarray, pixels: np.ndarray | None = None,
                opt: Options = Options(), chunk_elems: int = 1 << 19) -> dict:
    """Gradient of L = sum_p dL_dC[p] . C(p) w.r.t. every Gaussian parameter,
    by reverse-mode differentiation of the FP64 forward definition.  The set
    of included pairs and the stopping point are held fixed (the function is
    piecewise smooth); clamped alpha and clamped colour channels have zero
    derivative.  Returns float64 numpy arrays in the scene's SoA shapes."""
    cam = pose_or_cam if isinstance(pose_or_cam, Camera) else camera_from_pose(pose_or_cam)
    P = to_tensors(scene, requires_grad=True)
    pr = project(P, scene.sh_degree, cam, opt)
    # chain rule in two stages (memory stays bounded for large scenes): the
    # gradient of L with respect to the projected quantities, accumulated over
    # pixel chunks, then pulled back through the projection once
    names = [f for f in ("mu2d", "conic", "rho", "o1", "o2", "beta2d", "w2d", "rgb")
             if getattr(pr, f) is not None and getattr(pr, f).requires_grad]
    det = {f: getattr(pr, f).detach().requires_grad_(True) for f in names}
    prd = Projected(**{**{k: v for k, v in pr.__dict__.items()}, **det})
    acc = {f: torch.zeros_like(det[f]) for f in names}
    order = depth_order(pr)
    pixels, pc = pixel_centres(cam, pixels)
    g = torch.from_numpy(np.asarray(dL_dC, np.float64).reshape(-1, 3))
    bg = torch.from_numpy(cam.bg.astype(np.float64))
    step = max(1, chunk_elems // max(1, order.numel()))
    for s in range(0, pc.shape[0], step):
        pcs = pc[s:s + step]
        with torch.no_grad():     # decisions on the full ordered list
            inc = inclusion(alpha_tilde(pcs, prd, order, opt), opt)
            cols = torch.nonzero(inc.any(0)).flatten()
        if cols.numel() == 0:
            continue
        # pairs never included have no value and no derivative: keep only the
        # Gaussians included at some pixel of the chunk, with the same decisions
        sub = order[cols]
        at = alpha_tilde(pcs, prd, sub, opt)
        C, _ = composite(at, prd.rgb[sub], bg, inc[:, cols], opt)
        lc = (C * g[s:s + step]).sum()
        gr = torch.autograd.grad(lc, [det[f] for f in names], allow_unused=True)
        for f, v in zip(names, gr):
            if v is not None:
                acc[f] += v
    total = sum((getattr(pr, f) * acc[f]).sum() for f in names)
    leaves = {k: v for k, v in P.items() if v is not None}
    grads = torch.autograd.grad(total, list(leaves.values()), allow_unused=True)
    out = {}
    for (k, v), gr in zip(leaves.items(), grads):
        gr = torch.zeros_like(v) if gr is None else gr
        a = gr.detach().numpy()
        out[k] = a.transpose(1, 2, 0) if k == "sh" else (a.T if a.ndim == 2 else a)
    return out


def _loss_graph(P: dict, sh_degree: int, cam: Camera, dL_dC, pixels, opt: Options,
                chunk_elems: int, mu2d_shift: torch.Tensor | None = None):
    """L = sum_p dL_dC[p] . C(p) as a differentiable graph of the leaves in P
    (and of mu2d_shift), with the included pairs and stop points held fixed
    at their values.  Returns (L, Projected)."""
    pr = project(P, sh_degree, cam, opt, mu2d_shift)
    order = depth_order(pr)
    pixels, pc = pixel_centres(cam, pixels)
    g = torch.from_numpy(np.asarray(dL_dC, np.float64).reshape(-1, 3))
    bg = torch.from_numpy(cam.bg.astype(np.float64))
    n_pix = pc.shape[0]
    step = max(1, chunk_elems // max(1, order.numel()))
    total = torch.zeros((), dtype=F64)
    for s in range(0, n_pix, step):
        pcs = pc[s:s + step]
        with torch.no_grad():     # decisions on the full ordered list
            inc = inclusion(alpha_tilde(pcs, pr, order, opt), opt)
            cols = torch.nonzero(inc.any(0)).flatten()
        # pairs never included have no value and no derivative: keep only the
        # Gaussians included at some pixel of the chunk, with the same decisions
        sub = order[cols]
        at = alpha_tilde(pcs, pr, sub, opt)
        C, _ = composite(at, pr.rgb[sub], bg, inc[:, cols], opt)
        total = total + (C * g[s:s + step]).sum()
    return total, pr


def densify_stats(scene, pose_or_cam, dL_dC: np.ndarray, pixels: np.ndarray | None = None,
                  opt: Options = Options(), chunk_elems: int = 1 << 19) -> dict:
    """Per-Gaussian densification statistics of one view for the loss
    L = sum_p dL_dC[p] . C(p) (Sec. "Depth-Aware Densification Strategy",
    Eq. depth_grad, with the 2D statistic of 3DGS beside it):
      uv[i]    = || (dL/dmu2d_x * W/2, dL/dmu2d_y * H/2) ||, the gradient with
                 respect to the projected mean in NDC units (mu2d held as a
                 variable of its own: conic, skew and colour fixed);
      z[i]     = | r . dL/dmean_i |, r the camera's depth axis (third row of
                 w2c): the derivative of L when the centre moves in depth,
                 through every path (projection, footprint, SH direction);
      reach[i] = alpha reaches alpha_min at some requested pixel;
      valid[i] = not culled (in front of the near plane, invertible 2D
                 covariance).
    Float64 numpy arrays [N] (bool for reach and valid)."""
    cam = pose_or_cam if isinstance(pose_or_cam, Camera) else camera_from_pose(pose_or_cam)
    P = to_tensors(scene, requires_grad=True)
    shift = torch.zeros((scene.n, 2), dtype=F64, requires_grad=True)
    total, pr = _loss_graph(P, scene.sh_degree, cam, dL_dC, pixels, opt, chunk_elems, shift)
    g_mean, g_shift = torch.autograd.grad(total, [P["mean"], shift], allow_unused=True)
    g_mean = torch.zeros((scene.n, 3), dtype=F64) if g_mean is None else g_mean
    g_shift = torch.zeros((scene.n, 2), dtype=F64) if g_shift is None else g_shift
    ndc = g_shift.detach().numpy() * np.array([0.5 * cam.W, 0.5 * cam.H])
    r = cam.w2c[2, :3]
    z = np.abs(g_mean.detach().numpy() @ r)
    with torch.no_grad():
        pr0 = project(to_tensors(scene), scene.sh_degree, cam, opt)
        idx = torch.nonzero(pr0.valid).flatten()
        _, pc = pixel_centres(cam, pixels)
        reach = np.zeros(scene.n, bool)
        step = max(1, chunk_elems // max(1, idx.numel()))
        for s in range(0, pc.shape[0], step):
            at = alpha_tilde(pc[s:s + step], pr0, idx, opt)
            hit = (torch.clamp(at, max=opt.alpha_max) >= opt.alpha_min).any(0)
            reach[idx[hit].numpy()] = True
    return {"uv": np.sqrt((ndc * ndc).sum(1)), "z": z, "reach": reach,
            "valid": pr0.valid.numpy().copy(), "dL_dmu2d": g_shift.detach().numpy()}


# ------------------------------------------------------------ densification
@dataclass
class DensifyOptions:
    tau_uv: float = 0.001        # the appendix's threshold of the 2D gradient statistic
    tau_z: float = 0.001         # reading: the same threshold for the depth gradient g_z
    dense_scale: float = 0.01    # 3DGS: Gaussians larger than this are split, smaller cloned
    split_shrink: float = 1.6    # 3DGS: child scale = parent scale / 1.6


def densify_decisions(log_scale: np.ndarray, uv_sum, view_count, z_max,
                      opt: DensifyOptions = DensifyOptions()) -> np.ndarray:
    """Clone / split selection of Sec. "Depth-Aware Densification Strategy":
    a Gaussian is densified when its mean screen-space gradient norm (the
    accumulated g_uv over the views that saw it, divided by their number)
    reaches tau_uv, or when its depth gradient g_z (Eq. depth_grad) reaches
    tau_z; it is split when its largest scale exceeds dense_scale, else
    cloned.  The comparisons are float decisions that pick an integer, so
    they are taken in float32 (the kernel's precision).  log_scale [3][N];
    returns int8 [N]: 0 keep, 1 clone, 2 split."""
    n = log_scale.shape[1]
    f32 = np.float32
    sel = np.zeros(n, bool)
    if uv_sum is not None:
        cnt = np.asarray(view_count).astype(f32)
        with np.errstate(divide="ignore", invalid="ignore"):
            avg = np.where(cnt > 0, np.asarray(uv_sum, f32) / np.where(cnt > 0, cnt, f32(1)), f32(0))
        sel |= avg >= f32(opt.tau_uv)
    if z_max is not None:
        sel |= np.asarray(z_max, f32) >= f32(opt.tau_z)
    big = np.asarray(log_scale, f32).max(0) > f32(math.log(opt.dense_scale))
    return np.where(sel, np.where(big, 2, 1), 0).astype(np.int8)


def skew_normal_moments(sigma3: np.ndarray, beta: np.ndarray):
    """Mean offset and covariance of the normalised 3D skew-normal density
    2 phi(x; 0, Sigma) Phi(beta^T x) (the paper's kernel, normalised):
    delta = Sigma beta / sqrt(1 + beta^T Sigma beta), mean sqrt(2/pi) delta,
    covariance Sigma - (2/pi) delta delta^T (Azzalini & Dalla Valle 1996)."""
    sb = sigma3 @ beta
    delta = sb / math.sqrt(1.0 + float(beta @ sb))
    return math.sqrt(2.0 / math.pi) * delta, sigma3 - (2.0 / math.pi) * np.outer(delta, delta), delta


def densify(scene, decisions: np.ndarray, opt: DensifyOptions = DensifyOptions()) -> dict:
    """The new Gaussian set of a densification step (float64): in input order,
    kept Gaussians once, cloned ones twice, split ones as two children.
    Reading of the split (the paper's split figure: along the largest axis,
    children's scales adjusted to the skew): child scale along the largest
    axis e is s_max / split_shrink, every other attribute the parent's; the
    two children are placed on e so that, as equal-weight skew-normal
    densities, they have the parent's mean and the parent's variance along
    e.  Returns SoA arrays like the scene's plus the parent index."""
    n = scene.n
    ls = scene.log_scale.astype(np.float64)
    R = quat_to_rotmat(torch.from_numpy(scene.quat.T.astype(np.float64))).numpy()
    outs = {k: [] for k in ("mean", "log_scale", "parent")}
    for i in range(n):
        d = int(decisions[i])
        mu = scene.mean[:, i].astype(np.float64)
        if d != 2:
            for _ in range(2 if d == 1 else 1):
                outs["mean"].append(mu)
                outs["log_scale"].append(ls[:, i])
                outs["parent"].append(i)
            continue
        s = np.exp(ls[:, i])
        k = int(np.argmax(ls[:, i]))           # first largest
        e = R[i][:, k]
        sc = s.copy()
        sc[k] = s[k] / opt.split_shrink
        beta = np.zeros(3) if scene.skew is None else scene.skew[:, i].astype(np.float64)
        m_p, cov_p, _ = skew_normal_moments(R[i] @ np.diag(s * s) @ R[i].T, beta)
        m_c, cov_c, _ = skew_normal_moments(R[i] @ np.diag(sc * sc) @ R[i].T, beta)
        a = math.sqrt(max(float(e @ cov_p @ e) - float(e @ cov_c @ e), 0.0))
        lc = ls[:, i].copy()
        lc[k] = math.log(sc[k])
        for sign in (1.0, -1.0):
            outs["mean"].append(mu + m_p - m_c + sign * a * e)
            outs["log_scale"].append(lc)
            outs["parent"].append(i)
    parent = np.array(outs["parent"], np.int64)
    res = {"mean": np.array(outs["mean"]).T.reshape(3, -1), "log_scale": np.array(outs["log_scale"]).T.reshape(3, -1),
           "parent": parent}
    for f in ("quat", "skew", "opa_logit", "opa2_logit", "opa_dir", "sh"):
        v = getattr(scene, f)
        res[f] = None if v is None else v[..., parent].astype(np.float64)
    return res
