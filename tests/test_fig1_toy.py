"""The 1D square-wave experiment of Fig. 1 (CPU): the kernel against its
closed forms, the analytic Jacobian against central differences, and the
paper's claim that five skew-normal kernels fit a square wave more closely
than five normal kernels."""
import math

import numpy as np
import pytest
from scipy.stats import skewnorm

from paper_2605_18334_amd import fig1_toy as F


def test_zero_skew_is_the_normal_kernel():
    x = np.linspace(-3, 5, 401)
    p = np.array([0.7, 1.1, math.log(0.4), 0.0])
    ref = 0.7 * np.exp(-0.5 * ((x - 1.1) / 0.4) ** 2)
    np.testing.assert_array_equal(F.kernel_sum(p, x, True), F.kernel_sum(p[:3], x, False))
    np.testing.assert_allclose(F.kernel_sum(p, x, True), ref, rtol=1e-15, atol=1e-300)


@pytest.mark.parametrize("beta", [-6.0, -0.5, 2.0, 9.0])
def test_kernel_is_a_scaled_skew_normal_density(beta):
    """w 2 exp(-z^2/2) Phi(beta sigma z) = w sqrt(2 pi) sigma skewnorm(a = beta sigma)."""
    mu, sig, w = 0.3, 0.6, 1.7
    x = np.linspace(-3, 3, 301)
    got = F.kernel_sum(np.array([w, mu, math.log(sig), beta]), x, True)
    ref = w * math.sqrt(2 * math.pi) * sig * skewnorm.pdf(x, beta * sig, loc=mu, scale=sig)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("skew", [False, True])
def test_jacobian_matches_central_differences(skew):
    rng = np.random.default_rng(5)
    k = 4 if skew else 3
    p = np.stack([rng.uniform(0.3, 1.0, 3), rng.uniform(0, 4, 3), np.log(rng.uniform(0.2, 0.6, 3))]
                 + ([rng.normal(0, 3, 3)] if skew else []), 1).ravel()
    x = np.linspace(0, 4, 97)
    J = F.kernel_jacobian(p, x, skew)
    h = 1e-6
    for i in range(3 * k):
        e = np.zeros_like(p)
        e[i] = h
        fd = (F.kernel_sum(p + e, x, skew) - F.kernel_sum(p - e, x, skew)) / (2 * h)
        np.testing.assert_allclose(J[:, i], fd, rtol=1e-6, atol=1e-8)


def test_square_wave():
    x = np.array([0.0, 0.49, 0.5, 1.0, 1.49, 1.5, 2.49, 2.5, 3.49, 3.5])
    np.testing.assert_array_equal(F.square_wave(x), [0, 0, 1, 1, 1, 0, 0, 1, 1, 0])


def test_five_skew_normals_fit_the_square_wave_better_than_five_normals():
    r = F.fit_square_wave(n_kernels=5, starts=6, seed=0)
    print(f"RMSE normal {r['rmse_normal']:.4f}, skew-normal {r['rmse_skew']:.4f}")
    assert r["rmse_skew"] <= r["rmse_normal"]          # the skew family contains the normal one
    assert r["rmse_skew"] < 0.5 * r["rmse_normal"]     # and its edges are much sharper
    assert r["rmse_normal"] > 0.1
