"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (tests/golden/), closed forms derived by hand, numerical
integration of the paper's 3D kernel, textbook/library routines for the
special cases, invariants of compositing, and central finite differences of
the forward definition.  No GPU is needed.
"""
import math
import os

import numpy as np
import pytest
import scipy.integrate
import scipy.special
import scipy.stats
import torch

import sgs_synth as S
from oracle import sgs_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#")[0].strip()
        if line:
            rows.append([float(v) for v in line.split()])
    return np.array(rows)


# ------------------------------------------------------------------ erf / Phi
def test_erf_matches_paper_taylor_series():
    """Appendix "Forward Pass": erf(z) = 2/sqrt(pi) sum_n (-1)^n z^(2n+1) /
    (n! (2n+1)).  The printed leading coefficients pin the general term, the
    series pins the erf the oracle evaluates."""
    gold = _golden("erf_taylor.txt")
    for n, (power, num, den) in enumerate(gold):
        assert power == 2 * n + 1
        assert num / den == pytest.approx((-1) ** n / (math.factorial(n) * (2 * n + 1)), rel=0, abs=1e-15)
    z = torch.linspace(-2.0, 2.0, 81, dtype=torch.float64)
    series = sum(((-1) ** n) * z ** (2 * n + 1) / (float(math.factorial(n)) * (2 * n + 1)) for n in range(45))
    series = series * 2.0 / math.sqrt(math.pi)
    assert torch.max(torch.abs(series - torch.erf(z))).item() < 1e-13


def test_phi_zero_is_half_and_erf_derivative():
    """Sec. "3D Skew Gaussian Kernel": Phi(0) = 1/2 with
    Phi(z) = (1 + erf(z/sqrt 2))/2; appendix: d erf/dz = 2/sqrt(pi) e^{-z^2}."""
    z0 = torch.zeros(1, dtype=torch.float64)
    assert (0.5 * (1 + torch.erf(z0 / math.sqrt(2)))).item() == 0.5
    z = torch.linspace(-3, 3, 61, dtype=torch.float64)
    h = 1e-6
    fd = (torch.erf(z + h) - torch.erf(z - h)) / (2 * h)
    assert torch.max(torch.abs(fd - 2 / math.sqrt(math.pi) * torch.exp(-z * z))).item() < 1e-9


# ------------------------------------------------------------------ camera
def test_coord_engine_t_align_and_intrinsics():
    """T_align = diag(1,-1,-1,1) (printed), an involution; K from (W,H,FoV)."""
    gold = _golden("t_align.txt")
    np.testing.assert_array_equal(O.T_ALIGN, gold)
    np.testing.assert_array_equal(O.T_ALIGN @ O.T_ALIGN, np.eye(4))
    K = O.intrinsics(1280, 720, 60.0)
    assert K[0, 0] == pytest.approx(1280 / (2 * math.tan(math.radians(30))), rel=1e-15)
    assert K[1, 1] == K[0, 0]
    assert (K[0, 2], K[1, 2]) == (640.0, 360.0)
    K2 = O.intrinsics(1280, 720, 60.0, fovy_deg=40.0)
    assert K2[1, 1] == pytest.approx(720 / (2 * math.tan(math.radians(20))), rel=1e-15)


def test_coord_engine_axis_conventions():
    """OpenGL (right, up, back) pose -> OpenCV (right, down, forward):
    the look-at target lands on the principal point, the frontend's right is
    +x in the image and its up is -y (Sec. "Camera Trajectories and Format
    Standardization")."""
    eye = np.array([3.0, -5.0, 4.0])
    pose = S.Pose(S.look_at_gl(eye, (0.5, 0.2, -0.1)), 640, 480)
    cam = O.camera_from_pose(pose)
    K = cam.K

    def proj(x):
        t = cam.w2c[:3, :3] @ x + cam.w2c[:3, 3]
        return np.array([K[0, 0] * t[0] / t[2] + K[0, 2], K[1, 1] * t[1] / t[2] + K[1, 2]]), t[2]

    p, z = proj(np.array([0.5, 0.2, -0.1]))
    np.testing.assert_allclose(p, [320, 240], atol=1e-9)
    assert z == pytest.approx(np.linalg.norm(eye - [0.5, 0.2, -0.1]), rel=1e-12)
    right, up = pose.c2w_gl[:3, 0], pose.c2w_gl[:3, 1]
    pr, _ = proj(np.array([0.5, 0.2, -0.1]) + 0.1 * right)
    pu, _ = proj(np.array([0.5, 0.2, -0.1]) + 0.1 * up)
    assert pr[0] > 320 and abs(pr[1] - 240) < 1e-9
    assert pu[1] < 240 and abs(pu[0] - 320) < 1e-9
    np.testing.assert_allclose(cam.position, eye, atol=1e-12)


# ------------------------------------------------------------------ SH
def test_sh_orthonormal_by_quadrature():
    """Real SH are orthonormal on the sphere (Gauss-Legendre x uniform phi)."""
    nt, nphi = 24, 48
    xg, wg = np.polynomial.legendre.leggauss(nt)
    phi = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = torch.from_numpy(np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3))
    Y = O.sh_basis(3, d).numpy()
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_matches_library_associated_legendre():
    """Same basis built from scipy's associated Legendre functions (with the
    Condon-Shortley phase) and cos/sin of the azimuth; Y00 = 1/(2 sqrt pi)."""
    rng = np.random.default_rng(3)
    v = rng.normal(size=(50, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    Y = O.sh_basis(3, torch.from_numpy(v)).numpy()
    th = np.arccos(v[:, 2])
    ph = np.arctan2(v[:, 1], v[:, 0])
    col = 0
    for l in range(4):
        for m in range(-l, l + 1):
            am = abs(m)
            N = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            P = scipy.special.lpmv(am, l, np.cos(th))
            if m == 0:
                ref = N * P
            elif m > 0:
                ref = math.sqrt(2) * N * P * np.cos(am * ph)
            else:
                ref = math.sqrt(2) * N * P * np.sin(am * ph)
            np.testing.assert_allclose(Y[:, col], ref, atol=1e-12)
            col += 1
    np.testing.assert_allclose(Y[:, 0], 1 / (2 * math.sqrt(math.pi)), rtol=1e-15)


# ------------------------------------------------------------------ kernel
def _identity_pose(W=64, H=64, fov=60.0):
    # M_gl = T_align gives M_cv = I: camera at the origin looking down +z
    return S.Pose(np.diag([1.0, -1.0, -1.0, 1.0]), W, H, fov, 0.2)


def _one_gaussian(mean, sigma, skew, opa_logit=2.0, dc=(0.3, -0.1, 0.2)):
    q = np.array([[1.0], [0.0], [0.0], [0.0]], np.float32)
    return S.Scene(np.array(mean, np.float32).reshape(3, 1),
                   np.full((3, 1), math.log(sigma), np.float32), q,
                   np.array(skew, np.float32).reshape(3, 1),
                   np.array([opa_logit], np.float32),
                   np.array(dc, np.float32).reshape(1, 3, 1), 0)


def test_single_gaussian_closed_form():
    """Isotropic Gaussian at (0,0,Z) in front of the camera, no filter, skew
    (bx, by, 0): by hand, Sigma' = (f sigma/Z)^2 I and the 2D skew is
    (Z/f)(bx, by), so C(p) = rgb min(0.99, o exp(-|d|^2 / (2 sigma_p^2))
    (1 + erf((Z/f)(bx dx + by dy)/sqrt 2))), rgb = 0.5 + DC/(2 sqrt pi)."""
    Z, sig, bx, by = 6.0, 0.05, 7.0, -4.0
    pose = _identity_pose()
    sc = _one_gaussian([0.0, 0.0, Z], sig, [bx, by, 0.0])
    opt = O.Options(filter_s=0.0, compensate=False)
    r = O.render(sc, pose, opt=opt)
    f = 64 / (2 * math.tan(math.radians(30)))
    Zf, bxf, byf = (float(np.float32(v)) for v in (Z, bx, by))
    sf = math.exp(float(np.float32(math.log(sig))))
    sp = f * sf / Zf
    o = 1 / (1 + math.exp(-2.0))
    rgb = 0.5 + np.array([0.3, -0.1, 0.2], np.float32).astype(np.float64) / (2 * math.sqrt(math.pi))
    px = (np.arange(64 * 64) % 64) + 0.5 - 32
    py = (np.arange(64 * 64) // 64) + 0.5 - 32
    a = o * np.exp(-(px ** 2 + py ** 2) / (2 * sp ** 2)) * (1 + scipy.special.erf((Zf / f) * (bxf * px + byf * py) / math.sqrt(2)))
    a = np.minimum(a, 0.99)
    a = np.where(a >= 1 / 255, a, 0.0)
    np.testing.assert_allclose(r.color, a[:, None] * rgb[None, :], atol=1e-12)
    np.testing.assert_allclose(r.T, 1 - a, atol=1e-12)
    pr = O.project_numpy(sc, pose, opt)
    np.testing.assert_allclose(pr["beta2d"][0], [Zf / f * bxf, Zf / f * byf], rtol=1e-12)


def test_skew_along_view_ray_projects_to_zero():
    """Isotropic Gaussian on the optical axis with skew parallel to the ray:
    the marginal is symmetric, so the image equals the zero-skew image."""
    pose = _identity_pose()
    a = O.render(_one_gaussian([0, 0, 5.0], 0.08, [0, 0, 9.0]), pose)
    b = O.render(_one_gaussian([0, 0, 5.0], 0.08, [0, 0, 0.0]), pose)
    np.testing.assert_allclose(a.color, b.color, atol=1e-13)


def test_zero_skew_reduces_exactly_to_3dgs():
    """beta = 0 gives Phi(0) = 1/2, S = G (Sec. "3D Skew Gaussian Kernel"):
    the image equals the textbook 3DGS image, which drops the skew factor
    entirely, bit for bit."""
    sc, pose = S.tiny_config()
    sc = sc.subset(np.arange(400))
    sc.skew[:] = 0.0
    a = O.render(sc, pose)
    b = O.render(sc, pose, opt=O.Options(symmetric=True))
    np.testing.assert_array_equal(a.color, b.color)
    np.testing.assert_array_equal(a.T, b.T)


def test_gaussian_falloff_matches_library_normal_pdf():
    """G'(delta) = exp(-delta^T (Sigma'+sI)^-1 delta / 2) equals the bivariate
    normal density with covariance Sigma'+sI times 2 pi sqrt(det)."""
    sc, pose = S.tiny_config()
    sc = sc.subset(np.arange(5))
    cam = O.camera_from_pose(pose)
    with torch.no_grad():
        pr = O.project(O.to_tensors(sc), 0, cam, O.Options(symmetric=True))
    pix, pc = O.pixel_centres(cam, np.arange(0, 128 * 128, 97))
    idx = torch.arange(5)
    at = O.alpha_tilde(pc, pr, idx, O.Options(symmetric=True)).numpy()
    for i in range(5):
        a, b, c = pr.conic[i].numpy()
        cov = np.linalg.inv(np.array([[a, b], [b, c]]))
        g = scipy.stats.multivariate_normal(pr.mu2d[i].numpy(), cov).pdf(pc.numpy()) * 2 * math.pi * math.sqrt(np.linalg.det(cov))
        d = (pr.rho[i] * pr.o1[i]).item()
        np.testing.assert_allclose(at[:, i], d * g, rtol=1e-10, atol=1e-300)


def _rand_spd(rng, n, scale=1.0):
    B = rng.normal(size=(n, n)) * scale
    return B @ B.T + 0.3 * np.eye(n)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_skew_projection_equals_line_integral_of_3d_kernel(seed):
    """The 2D skew used by the rasterizer is pinned to the paper's 3D kernel
    S(x) = 2 G(x) Phi(beta^T x): integrating the normalised 3D density along
    the null direction n of the affine map A gives, for every image point y,
    |det[A; n^T]|^-1 times the integral, which must equal
    2 N(y; A Sigma A^T) Phi(beta_2D . y) (no blur)."""
    rng = np.random.default_rng(seed)
    Sig = _rand_spd(rng, 3, 0.8)
    beta = rng.normal(size=3) * 1.5
    A = rng.normal(size=(2, 3))
    n = np.cross(A[0], A[1]); n /= np.linalg.norm(n)
    Sig2 = A @ Sig @ A.T
    Q = np.linalg.inv(Sig2)
    b2 = O.skew_to_2d(torch.from_numpy(beta[None]), torch.from_numpy(Sig[None]),
                      torch.from_numpy(A[None]), torch.from_numpy(Q[None]))[0].numpy()
    mvn3 = scipy.stats.multivariate_normal(np.zeros(3), Sig)
    mvn2 = scipy.stats.multivariate_normal(np.zeros(2), Sig2)
    jac = abs(np.linalg.det(np.vstack([A, n])))
    pinv = A.T @ np.linalg.inv(A @ A.T)
    for y in rng.normal(size=(6, 2)) * 1.2:
        x0 = pinv @ y
        f = lambda t: 2 * mvn3.pdf(x0 + t * n) * scipy.stats.norm.cdf(beta @ (x0 + t * n))
        num, _ = scipy.integrate.quad(f, -np.inf, np.inf, epsabs=0, epsrel=1e-12, limit=200)
        closed = 2 * mvn2.pdf(y) * scipy.stats.norm.cdf(b2 @ y)
        assert num / jac == pytest.approx(closed, rel=1e-8)


def test_skew_projection_with_blur_equals_convolution():
    """With the low-pass filter the 2D density is the (no-blur) marginal
    convolved with N(0, sI); 2D Gauss-Hermite quadrature of that convolution
    must equal 2 N(y; A Sigma A^T + sI) Phi(beta_2D . y) with beta_2D from
    Q = (A Sigma A^T + sI)^-1."""
    rng = np.random.default_rng(7)
    Sig = _rand_spd(rng, 3, 0.9)
    beta = rng.normal(size=3) * 2.0
    A = rng.normal(size=(2, 3))
    s = 0.3
    Sig2 = A @ Sig @ A.T
    Q0 = np.linalg.inv(Sig2)
    Qf = np.linalg.inv(Sig2 + s * np.eye(2))
    tb = lambda Q: O.skew_to_2d(torch.from_numpy(beta[None]), torch.from_numpy(Sig[None]),
                                torch.from_numpy(A[None]), torch.from_numpy(Q[None]))[0].numpy()
    b0, bf = tb(Q0), tb(Qf)
    h, w = np.polynomial.hermite.hermgauss(60)
    E = np.sqrt(2 * s) * np.stack(np.meshgrid(h, h, indexing="ij"), -1).reshape(-1, 2)
    W = (w[:, None] * w[None, :]).reshape(-1) / math.pi
    mvn0 = scipy.stats.multivariate_normal(np.zeros(2), Sig2)
    mvnf = scipy.stats.multivariate_normal(np.zeros(2), Sig2 + s * np.eye(2))
    for y in rng.normal(size=(5, 2)):
        pts = y[None, :] - E
        conv = np.sum(W * 2 * mvn0.pdf(pts) * scipy.stats.norm.cdf(pts @ b0))
        closed = 2 * mvnf.pdf(y) * scipy.stats.norm.cdf(bf @ y)
        assert conv == pytest.approx(closed, rel=1e-9)


def test_dalpha_dbeta_matches_paper_closed_form():
    """Eq. for dS/dbeta (Sec. "3D Skew Gaussian Kernel"), in 2D with the
    opacity factor: d alpha~/d beta = d G'(x) (2/sqrt pi) e^{-(beta.delta/
    sqrt2)^2} delta / sqrt 2."""
    sc, pose = S.tiny_config()
    sc = sc.subset(np.arange(40))
    cam = O.camera_from_pose(pose)
    with torch.no_grad():
        pr = O.project(O.to_tensors(sc), 0, cam)
    beta = pr.beta2d.clone().requires_grad_(True)
    pr.beta2d = beta
    pix, pc = O.pixel_centres(cam, np.arange(0, 128 * 128, 211))
    idx = torch.arange(40)
    at = O.alpha_tilde(pc, pr, idx, O.Options())
    gx, = torch.autograd.grad(at.sum(), beta)
    with torch.no_grad():
        dx = pc[:, None, 0] - pr.mu2d[None, :, 0]
        dy = pc[:, None, 1] - pr.mu2d[None, :, 1]
        a, b, c = pr.conic.unbind(1)
        G = torch.exp(-0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy)
        z = (beta[:, 0] * dx + beta[:, 1] * dy) / math.sqrt(2)
        common = (pr.rho * pr.o1) * G * (2 / math.sqrt(math.pi)) * torch.exp(-z * z) / math.sqrt(2)
        ref = torch.stack([(common * dx).sum(0), (common * dy).sum(0)], 1)
    np.testing.assert_allclose(gx.numpy(), ref.numpy(), rtol=1e-12, atol=1e-300)


# ------------------------------------------------------------------ compositing
def test_compositing_hand_expanded_and_rules():
    """Compositing equation expanded by hand for three Gaussians, plus the
    skip (alpha < 1/255), clamp (0.99) and stop (T < 1e-4) rules."""
    opt = O.Options()
    rgb = torch.tensor([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.2, 0.3, 0.4]], dtype=torch.float64)
    bg = torch.tensor([0.1, 0.2, 0.3], dtype=torch.float64)
    at = torch.tensor([[0.3, 0.5, 0.25]], dtype=torch.float64)
    C, T = O.composite(at, rgb, bg, O.inclusion(at, opt), opt)
    a1, a2, a3 = 0.3, 0.5, 0.25
    ref = (a1 * rgb[0] + a2 * (1 - a1) * rgb[1] + a3 * (1 - a1) * (1 - a2) * rgb[2]
           + (1 - a1) * (1 - a2) * (1 - a3) * bg)
    np.testing.assert_allclose(C[0].numpy(), ref.numpy(), atol=1e-15)
    at = torch.tensor([[0.003, 1.7, 0.5]], dtype=torch.float64)  # skip, clamp, stop
    inc = O.inclusion(at, opt)
    assert inc.tolist() == [[False, True, True]]
    C, T = O.composite(at, rgb, bg, inc, opt)
    np.testing.assert_allclose(C[0].numpy(), (0.99 * rgb[1] + 0.5 * 0.01 * rgb[2] + 0.005 * bg).numpy(), atol=1e-15)
    at = torch.tensor([[0.99, 0.99, 0.6, 0.9]], dtype=torch.float64)
    inc = O.inclusion(at, opt)   # T: 1 -> .01 -> 1e-4 (kept, not below) -> stop
    assert inc.tolist() == [[True, True, False, False]]


def test_compositing_partition_of_unity_and_monotone_T():
    """sum_k alpha_k T_k + T_final = 1, 0 <= T <= 1 and T non-increasing."""
    sc, pose = S.tiny_config()
    sc.sh[:] = 0.0
    sc.sh[0] = 0.5 * 2 * math.sqrt(math.pi)     # rgb = 1 exactly on all channels
    r = O.render(sc, pose)
    np.testing.assert_allclose(r.color[:, 0] + r.T, 1.0, atol=1e-12)
    assert (r.T >= 0).all() and (r.T <= 1).all()
    cam = O.camera_from_pose(pose)
    with torch.no_grad():
        pr = O.project(O.to_tensors(sc), 0, cam)
        order = O.depth_order(pr)
        _, pc = O.pixel_centres(cam, np.arange(0, 128 * 128, 53))
        at = O.alpha_tilde(pc, pr, order, O.Options())
        inc = O.inclusion(at, O.Options())
        a = torch.where(inc, torch.clamp(at, max=0.99), torch.zeros_like(at))
        T = torch.cumprod(1 - a, 1)
    assert bool((T[:, 1:] <= T[:, :-1]).all())


def test_equal_depth_ties_break_by_index():
    """Two Gaussians at the same depth: the lower index is composited first."""
    pose = _identity_pose()
    sc = _one_gaussian([0, 0, 5.0], 0.1, [0, 0, 0])
    sc2 = _one_gaussian([0, 0, 5.0], 0.1, [0, 0, 0], dc=(-1.0, 1.0, 0.0))
    both = S.Scene(*(np.concatenate([getattr(sc, f), getattr(sc2, f)], -1) for f in
                     ("mean", "log_scale", "quat", "skew", "opa_logit", "sh")), 0)
    r = O.render(both, pose, pixels=np.array([32 * 64 + 32]))
    assert r.last[0] == 1 and r.n_contrib[0] == 2
    cam = O.camera_from_pose(pose)
    pr = O.project_numpy(both, cam)
    ca, cb, cc = pr["conic"][0]
    dx = dy = 0.5                # pixel centre (32.5, 32.5), mean at (32, 32)
    a = min(0.99, pr["rho"][0] * pr["o1"][0] * math.exp(-0.5 * (ca * dx * dx + cc * dy * dy) - cb * dx * dy))
    ref = a * pr["rgb"][0] + a * (1 - a) * pr["rgb"][1]
    np.testing.assert_allclose(r.color[0], ref, atol=1e-12)


# ------------------------------------------------------------------ enhanced opacity
def test_enhanced_opacity_reduces_to_scalar_when_equal():
    """o(x) = ((a1+a2) + (a1-a2) erf(...))/2 equals a1 when a1 = a2."""
    sc = S.blobs_scene(11, 300, 1, enhanced=True)
    sc.opa2_logit[:] = sc.opa_logit
    pose = S.tiny_config()[1]
    a = O.render(sc, pose)
    sc2 = S.Scene(sc.mean, sc.log_scale, sc.quat, sc.skew, sc.opa_logit, sc.sh, sc.sh_degree)
    b = O.render(sc2, pose)
    np.testing.assert_allclose(a.color, b.color, atol=1e-15)


# ------------------------------------------------------------------ gradients
def _param_list(sc):
    names = ["mean", "log_scale", "quat", "skew", "opa_logit", "sh", "opa2_logit", "opa_dir"]
    return [n for n in names if getattr(sc, n) is not None]


def _fd_check(sc, pose, pix, g, n_coords, seed, h=1e-6, rtol=1e-6):
    import copy
    grads = O.render_grad(sc, pose, g, pix)
    rng = np.random.default_rng(seed)
    cam = O.camera_from_pose(pose)

    def loss(s):
        with torch.no_grad():
            P = O.to_tensors(s)
            pr = O.project(P, s.sh_degree, cam)
            order = O.depth_order(pr)
            _, pc = O.pixel_centres(cam, pix)
            at = O.alpha_tilde(pc, pr, order, O.Options())
            inc = O.inclusion(at, O.Options())
            C, _ = O.composite(at, pr.rgb[order], torch.zeros(3, dtype=torch.float64), inc, O.Options())
            return float((C.numpy() * g).sum()), (order.numpy().tobytes(), inc.numpy().tobytes(),
                                                  (pr.rgb > 0).numpy().tobytes(), (at < 0.99).numpy().tobytes())
    checked = 0
    for _ in range(n_coords * 3):
        if checked >= n_coords:
            break
        name = _param_list(sc)[rng.integers(0, len(_param_list(sc)))]
        arr = getattr(sc, name)
        flat = int(rng.integers(0, arr.size))
        vals = []
        for sgn in (1, -1):
            s2 = copy.deepcopy(sc)
            a64 = np.array(getattr(s2, name), dtype=np.float64, order="C")
            a64.reshape(-1)[flat] += sgn * h
            setattr(s2, name, a64)
            vals.append(loss(s2))
        if vals[0][1] != vals[1][1]:
            continue   # a decision flips within +-h: the derivative is not defined there
        fd = (vals[0][0] - vals[1][0]) / (2 * h)
        an = grads[name].reshape(-1)[flat]
        scale = max(1e-6, np.abs(grads[name]).max())
        assert abs(fd - an) <= rtol * scale + 1e-6 * abs(an) + 1e-9, (name, flat, fd, an)
        checked += 1
    assert checked >= n_coords // 2


def test_gradient_matches_central_differences_subscene():
    """64-Gaussian subscene (blobs generator, SH3) on a 64x64 view: FP64
    central differences (h = 1e-6) of L = sum dL/dC . C agree with the
    oracle's reverse-mode gradient for every parameter kind."""
    sc = S.blobs_scene(4, 64, 3)
    pose = S.Pose(S.look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), 64, 64)
    g = np.random.default_rng(1).normal(size=(64 * 64, 3))
    _fd_check(sc, pose, None, g, n_coords=60, seed=5)


def test_gradient_matches_central_differences_enhanced():
    sc = S.blobs_scene(9, 24, 1, enhanced=True)
    pose = S.Pose(S.look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), 48, 48)
    g = np.random.default_rng(2).normal(size=(48 * 48, 3))
    _fd_check(sc, pose, None, g, n_coords=40, seed=6)


def test_densify_stats_match_central_differences():
    """Densification statistics (Sec. "Depth-Aware Densification Strategy"):
    g_z is pinned by central differences of L when one centre moves along the
    camera's depth axis, g_uv by central differences of L in that Gaussian's
    projected mean (scaled to NDC units by W/2, H/2).  Coordinates whose
    decisions flip within +-h are skipped."""
    sc = S.blobs_scene(4, 64, 3)
    W_, H_ = 64, 48
    pose = S.Pose(S.look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), W_, H_)
    g = np.random.default_rng(11).normal(size=(W_ * H_, 3))
    st = O.densify_stats(sc, pose, g)
    cam = O.camera_from_pose(pose)
    r = cam.w2c[2, :3]
    opt = O.Options()

    def loss(s, shift=None):
        with torch.no_grad():
            pr = O.project(O.to_tensors(s), s.sh_degree, cam, opt, shift)
            order = O.depth_order(pr)
            _, pc = O.pixel_centres(cam, None)
            at = O.alpha_tilde(pc, pr, order, opt)
            inc = O.inclusion(at, opt)
            C, _ = O.composite(at, pr.rgb[order], torch.zeros(3, dtype=torch.float64), inc, opt)
            sig = (order.numpy().tobytes(), inc.numpy().tobytes(), (pr.rgb > 0).numpy().tobytes(),
                   (at < opt.alpha_max).numpy().tobytes())
            return float((C.numpy() * g).sum()), sig

    assert st["reach"].sum() >= 20
    assert not (st["reach"] & ~st["valid"]).any()
    h = 1e-6
    cand = np.flatnonzero(st["reach"])
    checked_z = checked_uv = 0
    for i in cand[:24]:
        # depth axis
        vals = []
        for sgn in (1, -1):
            s2 = sc.subset(np.arange(sc.n))
            m = np.array(s2.mean, dtype=np.float64, order="C")
            m[:, i] += sgn * h * r
            s2.mean = m
            vals.append(loss(s2))
        if vals[0][1] == vals[1][1]:
            fd = (vals[0][0] - vals[1][0]) / (2 * h)
            assert abs(abs(fd) - st["z"][i]) <= 1e-6 * max(1.0, st["z"][i]), (i, fd, st["z"][i])
            checked_z += 1
        # projected mean, both axes
        comp = []
        for ax in range(2):
            vals = []
            for sgn in (1, -1):
                sh = torch.zeros((sc.n, 2), dtype=torch.float64)
                sh[i, ax] = sgn * h
                vals.append(loss(sc, sh))
            if vals[0][1] != vals[1][1]:
                break
            comp.append((vals[0][0] - vals[1][0]) / (2 * h))
        if len(comp) == 2:
            uv = math.hypot(comp[0] * W_ / 2, comp[1] * H_ / 2)
            assert abs(uv - st["uv"][i]) <= 1e-6 * max(1.0, st["uv"][i]), (i, uv, st["uv"][i])
            checked_uv += 1
    assert checked_z >= 16 and checked_uv >= 16
    # the statistics are not trivially zero
    assert st["z"][cand].max() > 0 and st["uv"][cand].max() > 0


def test_power_terms_bound_the_exponent():
    """power_terms (the scale of the float32 rounding margin) bounds |log G'|
    by the triangle inequality, with equality for an axis-aligned conic, and
    a 100:1 sliver along its long axis has terms (L/w)^2 = 1e4 times the
    exponent."""
    rng = np.random.default_rng(3)
    n = 50
    a_, c_ = rng.uniform(0.01, 0.3, n), rng.uniform(0.01, 0.3, n)
    pr = O.Projected(
        mu2d=torch.from_numpy(rng.uniform(40, 60, (n, 2))),
        conic=torch.from_numpy(np.stack([a_, rng.uniform(-0.9, 0.9, n) * np.sqrt(a_ * c_), c_], 1)),
        rho=torch.ones(n, dtype=torch.float64), o1=torch.ones(n, dtype=torch.float64),
        o2=torch.ones(n, dtype=torch.float64), beta2d=torch.zeros(n, 2, dtype=torch.float64),
        w2d=None, rgb=torch.zeros(n, 3, dtype=torch.float64), depth=torch.ones(n, dtype=torch.float64),
        valid=torch.ones(n, dtype=torch.bool))
    pc = torch.from_numpy(rng.uniform(35, 65, (30, 2)))
    idx = torch.arange(n)
    at = O.alpha_tilde(pc, pr, idx, O.Options(symmetric=True))
    terms = O.power_terms(pc, pr, idx)
    assert (terms >= -torch.log(at) * (1 - 1e-12)).all()
    pr.conic[:, 1] = 0.0
    at = O.alpha_tilde(pc, pr, idx, O.Options(symmetric=True))
    np.testing.assert_allclose(O.power_terms(pc, pr, idx).numpy(), -torch.log(at).numpy(), rtol=1e-12)
    # conic of a 100:1 ellipse at 45 degrees, 120 px along the long axis
    s = 1 / np.sqrt(2)
    R = np.array([[s, -s], [s, s]])
    Q = R @ np.diag([1 / 50.0 ** 2, 1 / 0.5 ** 2]) @ R.T
    pr.conic[0] = torch.tensor([Q[0, 0], Q[0, 1], Q[1, 1]])
    p = pr.mu2d[0:1] + torch.tensor([[120 * s, 120 * s]])
    t = float(O.power_terms(p, pr, idx[:1])[0, 0])
    e = float(-torch.log(O.alpha_tilde(p, pr, idx[:1], O.Options(symmetric=True)))[0, 0])
    assert abs(e - 0.5 * (120 / 50) ** 2) < 1e-9 and abs(t / e - 1e4) < 1e-3 * 1e4


# ------------------------------------------------------------------ projection chain
def _hamilton(p, q):
    """Quaternion product p q, (w, x, y, z) order."""
    pw, px, py, pz = p
    qw, qx, qy, qz = q
    return np.array([pw * qw - px * qx - py * qy - pz * qz,
                     pw * qx + px * qw + py * qz - pz * qy,
                     pw * qy - px * qz + py * qw + pz * qx,
                     pw * qz + px * qy - py * qx + pz * qw])


def test_rotation_matrix_equals_quaternion_sandwich():
    """Sec. "Preliminary of 3D Gaussian Splatting": R is the rotation of the
    (normalised) quaternion q, i.e. R v is the vector part of q (0, v) q*,
    computed here by Hamilton products; also equal to scipy's rotation of
    the same quaternion (scalar-last order there)."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(41)
    q = rng.normal(size=(24, 4)) * rng.uniform(0.3, 3.0, (24, 1))      # not unit length
    R = O.quat_to_rotmat(torch.from_numpy(q)).numpy()
    for i in range(len(q)):
        qn = q[i] / np.linalg.norm(q[i])
        qc = qn * np.array([1.0, -1.0, -1.0, -1.0])
        for v in [*np.eye(3), rng.normal(size=3)]:
            rv = _hamilton(_hamilton(qn, np.concatenate([[0.0], v])), qc)
            assert abs(rv[0]) < 1e-13
            np.testing.assert_allclose(R[i] @ v, rv[1:], atol=1e-13)
    np.testing.assert_allclose(R, Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix(), atol=1e-13)


def _perspective_jacobian_fd(cam, t):
    """Central differences of the pinhole map pi(t) = (fx tx/tz + cx,
    fy ty/tz + cy) at camera-space point t: a 2x3 matrix."""
    fx, fy, cx, cy = cam.K[0, 0], cam.K[1, 1], cam.K[0, 2], cam.K[1, 2]
    pi = lambda u: np.array([fx * u[0] / u[2] + cx, fy * u[1] / u[2] + cy])
    J = np.zeros((2, 3))
    for k in range(3):
        h = 1e-5 * max(1.0, abs(t[k]))
        e = np.zeros(3)
        e[k] = h
        J[:, k] = (pi(t + e) - pi(t - e)) / (2 * h)
    return J, pi(t)


def test_ewa_projection_matches_perspective_map_off_axis():
    """Sec. "Preliminary of 3D Gaussian Splatting" (affine approximation of
    the viewing transform) and the appendix "Forward Pass": Sigma' = A Sigma
    A^T with A the Jacobian of the pinhole map at the camera-space centre
    times the world-to-camera rotation; the Jacobian is taken at the centre
    with x/z and y/z clamped to +-1.3 tan(FoV/2) (reading R15).  Sigma comes
    from scipy's rotation of the quaternion and the scales; A from central
    differences of the pinhole map at the clamped point.  Means lie off the
    axis inside and beyond the clamp, under a general camera pose; the conic
    (Sigma' + sI)^-1, rho and the 2D mean are compared."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(43)
    pose = S.Pose(S.look_at_gl((2.0, -3.0, 7.0), (0.3, 0.1, -0.2)), 160, 96, 60.0, 0.2)
    cam = O.camera_from_pose(pose)
    c2w = np.linalg.inv(cam.w2c)
    fx, fy = cam.K[0, 0], cam.K[1, 1]
    limx, limy = 1.3 * (cam.W / 2) / fx, 1.3 * (cam.H / 2) / fy
    # camera-space targets: ratios x/z, y/z inside and beyond the clamp
    ratios = [(0.2, -0.1), (-0.6, 0.3), (0.9 * limx, -0.8 * limy), (1.4 * limx, 0.2),
              (-1.7 * limx, 1.5 * limy), (0.1, -2.0 * limy), (-0.5, 0.95 * limy)]
    n = len(ratios)
    tcam = np.array([[rx * z, ry * z, z] for (rx, ry), z in zip(ratios, rng.uniform(3.0, 9.0, n))])
    mean = (c2w[:3, :3] @ tcam.T).T + c2w[:3, 3]
    q = rng.normal(size=(n, 4))
    ls = rng.uniform(-3.0, -0.5, (n, 3))
    sc = S.Scene(mean.T.astype(np.float32), ls.T.astype(np.float32), q.T.astype(np.float32),
                 np.zeros((3, n), np.float32), np.zeros(n, np.float32),
                 np.zeros((1, 3, n), np.float32), 0)
    s_f = 0.3
    pr = O.project_numpy(sc, pose, O.Options(filter_s=s_f))
    beyond = 0
    for i in range(n):
        m64 = sc.mean[:, i].astype(np.float64)
        t = cam.w2c[:3, :3] @ m64 + cam.w2c[:3, 3]
        rx, ry = t[0] / t[2], t[1] / t[2]
        tc = np.array([np.clip(rx, -limx, limx) * t[2], np.clip(ry, -limy, limy) * t[2], t[2]])
        beyond += (abs(rx) > limx) or (abs(ry) > limy)
        J, _ = _perspective_jacobian_fd(cam, tc)
        _, mu = _perspective_jacobian_fd(cam, t)
        A = J @ cam.w2c[:3, :3]
        Rq = Rotation.from_quat(sc.quat[[1, 2, 3, 0], i].astype(np.float64)).as_matrix()
        s = np.exp(sc.log_scale[:, i].astype(np.float64))
        sig3 = Rq @ np.diag(s * s) @ Rq.T
        sig2 = A @ sig3 @ A.T
        Q = np.linalg.inv(sig2 + s_f * np.eye(2))
        rho = math.sqrt(np.linalg.det(sig2) / np.linalg.det(sig2 + s_f * np.eye(2)))
        np.testing.assert_allclose(pr["conic"][i], [Q[0, 0], Q[0, 1], Q[1, 1]], rtol=1e-7,
                                   atol=1e-9 * np.abs(Q).max(), err_msg=f"conic {i}")
        assert pr["rho"][i] == pytest.approx(rho, rel=1e-7), i
        np.testing.assert_allclose(pr["mu2d"][i], mu, rtol=1e-12, atol=1e-9)
    assert beyond >= 3


def test_filter_and_compensation_closed_form():
    """Appendix "Forward Pass": d = o sqrt(det Sigma' / det(Sigma' + sI)).
    For an isotropic Gaussian of scale sigma at (0, 0, Z) in front of the
    camera Sigma' = sigma_p^2 I with sigma_p = f sigma / Z, so by hand
    rho = sigma_p^2 / (sigma_p^2 + s) and, without skew, C(p) = rgb min(0.99,
    o rho exp(-|delta|^2 / (2 (sigma_p^2 + s)))) with s = 0.3."""
    Z, sig, s_f = 6.0, 0.07, 0.3
    pose = _identity_pose()
    sc = _one_gaussian([0.0, 0.0, Z], sig, [0.0, 0.0, 0.0], opa_logit=3.0)
    opt = O.Options(filter_s=s_f, compensate=True)
    f = 64 / (2 * math.tan(math.radians(30)))
    Zf = float(np.float32(Z))
    sf = math.exp(float(np.float32(math.log(sig))))
    sp2 = (f * sf / Zf) ** 2
    rho = sp2 / (sp2 + s_f)
    assert 0.3 < rho < 0.9                         # the filter matters here
    pr = O.project_numpy(sc, pose, opt)
    assert pr["rho"][0] == pytest.approx(rho, rel=1e-12)
    o = 1 / (1 + math.exp(-3.0))
    rgb = 0.5 + np.array([0.3, -0.1, 0.2], np.float32).astype(np.float64) / (2 * math.sqrt(math.pi))
    px = (np.arange(64 * 64) % 64) + 0.5 - 32
    py = (np.arange(64 * 64) // 64) + 0.5 - 32
    a = np.minimum(o * rho * np.exp(-(px ** 2 + py ** 2) / (2 * (sp2 + s_f))), 0.99)
    a = np.where(a >= 1 / 255, a, 0.0)
    r = O.render(sc, pose, opt=opt)
    np.testing.assert_allclose(r.color, a[:, None] * rgb[None, :], atol=1e-12)


def _needle_scene(seed=7, n=60):
    sc = S.blobs_scene(seed, n, 0)
    rng = np.random.default_rng(seed + 100)
    sc.log_scale[:] = np.log(0.004)
    sc.log_scale[0] = np.log(rng.uniform(0.8, 2.5, n)).astype(np.float32)
    sc.opa_logit[:] = rng.uniform(1.0, 5.0, n).astype(np.float32)
    sc.skew[:] *= np.float32(0.02)
    # a mid-grey background gives derivatives of both signs along a pixel
    return sc, S.Pose(S.look_at_gl((0.0, 0.0, 8.0), up=(0, 1, 0)), 96, 72, 60.0, 0.2, (0.5, 0.5, 0.5))


def _composite_by_hand(alpha_t, rgb, bg, amax):
    """Front-to-back compositing of one pixel's included pairs (in order),
    written out: returns colour [3] and T."""
    T, C = 1.0, np.zeros(3)
    for at, c in zip(alpha_t, rgb):
        a = min(amax, at)
        C += c * a * T
        T *= 1.0 - a
    return C + T * bg, T


def test_float32_error_bound_covers_rounding_and_is_first_order_tight():
    """float32_error_bound sizes the tolerance on ill-conditioned inputs: it
    must (1) cover the change of the FP64 image when every conic is rounded
    to float32 (exponent terms off by at most 2^-24 of power_terms, a
    quarter of the u = 2^-22 the bound assumes), with the decisions held,
    and (2) equal, pixel by pixel, the first-order effect of the worst-case
    perturbation alpha~ -> alpha~ (1 +- u power_terms), here obtained by
    central differences of compositing written out by hand."""
    sc, pose = _needle_scene()
    opt = O.Options()
    bC, bT = O.float32_error_bound(sc, pose)
    cam = O.camera_from_pose(pose)
    with torch.no_grad():
        pr = O.project(O.to_tensors(sc), 0, cam, opt)
        order = O.depth_order(pr)
        pix, pc = O.pixel_centres(cam, None)
        at = O.alpha_tilde(pc, pr, order, opt)
        inc = O.inclusion(at, opt)
        bg = torch.from_numpy(cam.bg)
        C0, T0 = O.composite(at, pr.rgb[order], bg, inc, opt)
        pr.conic = pr.conic.float().double()
        at32 = O.alpha_tilde(pc, pr, order, opt)
        C1, T1 = O.composite(at32, pr.rgb[order], bg, inc, opt)
        pt = O.power_terms(pc, pr, order).numpy()
    dC = (C1 - C0).abs().numpy()
    dT = (T1 - T0).abs().numpy()
    assert bC.max() > 1e-7                         # the needles make the bound matter
    assert (dC <= bC * (1 + 1e-6) + 1e-15).all() and (dT <= bT * (1 + 1e-6) + 1e-15).all()
    assert dC.max() > 0.05 * bC.max()              # and the rounding is of its order
    # first-order tightness on the pixels with the largest bounds and on
    # those where most pairs overlap (derivatives of mixed sign)
    u = 2.0 ** -22
    atn, incn, rgb = at.numpy(), inc.numpy(), pr.rgb[order].numpy()
    many = np.argsort(-(incn.sum(1) + 1e-3 * (bC.max(1) > 1e-9)))[:12]
    assert incn.sum(1)[many].min() >= 3
    for p in np.concatenate([np.argsort(-bC.max(1))[:12], many]):
        ks = np.nonzero(incn[p])[0]
        a_p, c_p = atn[p, ks], rgb[ks]
        tight = np.zeros(4)
        for j, k in enumerate(ks):
            if a_p[j] >= opt.alpha_max:
                continue                              # clamped: no derivative
            h = 1e-7 * a_p[j]
            up, dn = a_p.copy(), a_p.copy()
            up[j] += h
            dn[j] -= h
            Cu, Tu = _composite_by_hand(up, c_p, cam.bg, opt.alpha_max)
            Cd, Td = _composite_by_hand(dn, c_p, cam.bg, opt.alpha_max)
            d = np.concatenate([(Cu - Cd), [Tu - Td]]) / (2 * h)
            tight += np.abs(d) * a_p[j] * u * pt[p, k]
        np.testing.assert_allclose(np.concatenate([bC[p], [bT[p]]]), tight, rtol=1e-5,
                                   atol=1e-9 * tight.max())


# ------------------------------------------------------------ densification
def test_densify_decisions_by_hand():
    """Thresholds of the selection (mean uv statistic, depth gradient) and the
    clone / split choice by the largest scale, on hand-made statistics."""
    ls = np.log(np.array([[0.005, 0.02, 0.005, 0.02, 0.005, 0.02],
                          [0.001, 0.001, 0.009, 0.001, 0.001, 0.001],
                          [0.002, 0.003, 0.001, 0.004, 0.001, 0.001]], np.float32))
    uv = np.array([0.003, 0.003, 0.0, 0.0019, 0.0, 0.0], np.float32)
    cnt = np.array([2, 3, 0, 2, 0, 5], np.uint32)
    z = np.array([0.0, 0.0, 0.0, 0.0, 0.002, 0.0005], np.float32)
    d = O.densify_decisions(ls, uv, cnt, z)
    # 0: mean 0.0015 >= 1e-3, small -> clone; 1: mean 1e-3 (float32) >= 1e-3, large -> split;
    # 2: unseen -> keep; 3: mean 0.00095 -> keep; 4: g_z -> clone; 5: below both -> keep
    np.testing.assert_array_equal(d, [1, 2, 0, 0, 1, 0])
    np.testing.assert_array_equal(O.densify_decisions(ls, None, None, z), [0, 0, 0, 0, 1, 0])


@pytest.mark.parametrize("b", [-3.0, 0.7, 5.0])
def test_skew_normal_moments_match_scipy_on_an_axis(b):
    """Diagonal Sigma and skew along one axis: the marginal is the 1D skew
    normal 2 phi(x; s) Phi(b x), whose mean and variance scipy gives."""
    from scipy.stats import skewnorm
    s = np.array([0.3, 0.8, 0.5])
    beta = np.array([0.0, b, 0.0])
    mean, cov, _ = O.skew_normal_moments(np.diag(s * s), beta)
    ref = skewnorm(b * s[1], scale=s[1])
    assert mean[1] == pytest.approx(ref.mean(), rel=1e-12)
    assert cov[1, 1] == pytest.approx(ref.var(), rel=1e-12)
    assert mean[0] == 0.0 and mean[2] == 0.0 and cov[0, 0] == pytest.approx(s[0] ** 2)


def _sample_skew_normal(rng, mu, sigma3, beta, n):
    """Azzalini's stochastic representation of 2 phi(x - mu; Sigma) Phi(beta.(x - mu)):
    x = mu + delta |u0| + v, v ~ N(0, Sigma - delta delta^T)."""
    _, _, delta = O.skew_normal_moments(sigma3, beta)
    L = np.linalg.cholesky(sigma3 - np.outer(delta, delta) + 1e-15 * np.eye(3))
    return mu + np.abs(rng.normal(size=(n, 1))) * delta + rng.normal(size=(n, 3)) @ L.T


def test_split_children_keep_the_parents_mean_and_axis_variance():
    """Samples of the two children (equal weights) against samples of the
    parent: same 3D mean, same variance along the split axis, the split axis
    being the parent's largest; with zero skew the children sit at
    +- s sqrt(1 - 1/1.6^2) on that axis with scale s / 1.6."""
    rng = np.random.default_rng(7)
    sc = S.blobs_scene(3, 4, 0)
    sc.log_scale[:] = np.log(np.array([[0.4, 0.1, 0.2, 0.3], [0.1, 0.5, 0.2, 0.1], [0.2, 0.1, 0.6, 0.1]], np.float32))
    sc.skew[:, 3] = 0.0
    d = np.full(4, 2, np.int8)
    out = O.densify(sc, d)
    assert out["mean"].shape == (3, 8) and (out["parent"] == np.repeat(np.arange(4), 2)).all()
    R = O.quat_to_rotmat(torch.from_numpy(sc.quat.T.astype(np.float64))).numpy()
    n = 400_000
    for i in range(4):
        s = np.exp(sc.log_scale[:, i].astype(np.float64))
        k = int(np.argmax(s))
        e = R[i][:, k]
        beta = sc.skew[:, i].astype(np.float64)
        par = _sample_skew_normal(rng, sc.mean[:, i].astype(np.float64), R[i] @ np.diag(s * s) @ R[i].T, beta, n)
        kids = []
        for c in (2 * i, 2 * i + 1):
            sk = np.exp(out["log_scale"][:, c])
            assert sk[k] == pytest.approx(s[k] / 1.6) and np.delete(sk, k) == pytest.approx(np.delete(s, k))
            kids.append(_sample_skew_normal(rng, out["mean"][:, c], R[i] @ np.diag(sk * sk) @ R[i].T, beta, n // 2))
        kids = np.concatenate(kids)
        se = np.sqrt(np.diag(np.cov(par.T)) / n).max()
        np.testing.assert_allclose(kids.mean(0), par.mean(0), atol=6 * se)
        vp, vk = (par @ e).var(), (kids @ e).var()
        assert vk == pytest.approx(vp, rel=0.02)
        if i == 3:   # zero skew: the textbook symmetric split
            a = s[k] * math.sqrt(1 - 1 / 1.6 ** 2)
            np.testing.assert_allclose(out["mean"][:, 6] - sc.mean[:, 3], a * e, atol=1e-6)
            np.testing.assert_allclose(out["mean"][:, 7] - sc.mean[:, 3], -a * e, atol=1e-6)


def test_densify_keeps_and_clones_copy_the_attributes():
    sc = S.blobs_scene(5, 6, 1)
    d = np.array([0, 1, 0, 1, 0, 0], np.int8)
    out = O.densify(sc, d)
    assert (out["parent"] == [0, 1, 1, 2, 3, 3, 4, 5]).all()
    np.testing.assert_array_equal(out["mean"], sc.mean[:, out["parent"]].astype(np.float64))
    np.testing.assert_array_equal(out["sh"], sc.sh[..., out["parent"]].astype(np.float64))


# ------------------------------------------------------------ depth key and margins
def _round_f32_exact(fr):
    """Correct round-to-nearest-even of a Fraction to float32 (by comparing
    the three float32 neighbours of the double nearest to it)."""
    from fractions import Fraction
    if fr == 0:
        return np.float32(0)
    f = np.float32(float(fr))
    best = None
    for cand in (np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))):
        d = abs(Fraction(float(cand)) - fr)
        even = (int(np.float32(cand).view(np.uint32)) & 1) == 0
        if best is None or d < best[0] or (d == best[0] and even):
            best = (d, cand)
    return best[1]


def test_fma_f32_is_correctly_rounded():
    """Against exact rational arithmetic, on random triples and on triples
    whose exact result is a rounding error (c = -fl(a b)) or sits on a
    float32 midpoint."""
    from fractions import Fraction
    rng = np.random.default_rng(0)
    n = 3000
    a = rng.normal(size=n).astype(np.float32)
    b = rng.normal(size=n).astype(np.float32)
    c = rng.normal(size=n).astype(np.float32) * np.float32(4.0)
    c[::3] = -(a[::3].astype(np.float64) * b[::3]).astype(np.float32)
    # midpoints: a = 1 + 2^-12, b = 1 + 2^-12: a b = 1 + 2^-11 + 2^-24, c = 0 ties-to-even on the 2^-24 bit
    a[1::7] = np.float32(1 + 2 ** -12)
    b[1::7] = np.float32(1 + 2 ** -12)
    c[1::7] = np.float32(0.0)
    got = O.fma_f32(a, b, c)
    for i in range(n):
        ref = _round_f32_exact(Fraction(float(a[i])) * Fraction(float(b[i])) + Fraction(float(c[i])))
        assert got[i] == ref, (i, a[i], b[i], c[i], got[i], ref)


def test_depth_key_is_the_camera_depth_in_float32():
    sc, pose = S.tiny_config()
    cam = O.camera_from_pose(pose)
    z32 = O.depth_key(sc.mean, cam)
    z64 = (cam.w2c[2, :3] @ sc.mean.astype(np.float64)) + cam.w2c[2, 3]
    assert z32.dtype == np.float32
    np.testing.assert_allclose(z32, z64, rtol=4 * 2.0 ** -24, atol=1e-6)


def test_composite_pixel_equals_vectorised_compositing_and_flips_one_decision():
    """The per-pixel loop (used for the outcomes of uncertain decisions)
    against the vectorised compositing, and a flipped alpha_min decision
    against compositing with that pair's decision negated."""
    rng = np.random.default_rng(3)
    opt = O.Options()
    for _ in range(30):
        K = 12
        at = rng.uniform(0, 1.2, K) * (rng.uniform(size=K) > 0.3)
        at[rng.integers(0, K)] = 1 / 255 * (1 + 1e-9)
        rgb = rng.uniform(0, 1, (K, 3))
        bg = rng.uniform(0, 1, 3)
        att = torch.from_numpy(at[None, :])
        inc = O.inclusion(att, opt)
        C, T = O.composite(att, torch.from_numpy(rgb), torch.from_numpy(bg), inc, opt)
        got = O.composite_pixel(at, rgb, bg, opt)
        np.testing.assert_allclose(got, np.concatenate([C.numpy()[0], T.numpy()]), rtol=1e-12, atol=1e-15)
        k = int(rng.integers(0, K))
        keep = torch.clamp(att, max=opt.alpha_max) >= opt.alpha_min
        keep[0, k] = ~keep[0, k]
        C2, T2 = O.composite(att, torch.from_numpy(rgb), torch.from_numpy(bg), O.inclusion_with(att, opt, keep), opt)
        np.testing.assert_allclose(O.composite_pixel(at, rgb, bg, opt, flip_keep={k}),
                                   np.concatenate([C2.numpy()[0], T2.numpy()]), rtol=1e-12, atol=1e-15)


def test_ambiguous_pixels_list_their_outcomes():
    """On the tiny scene every ambiguous pixel lists the outcomes of its
    uncertain decisions, the first being the oracle's own colour."""
    sc, pose = S.tiny_config()
    r = O.render(sc, pose)
    assert r.ambiguous.mean() < 1e-3
    for q in np.nonzero(r.ambiguous)[0]:
        rows = r.alt_rows[r.alt_start[q]:r.alt_start[q + 1]]
        assert len(rows) >= 2
        np.testing.assert_allclose(rows[0, :3], r.color[q], atol=1e-12)
