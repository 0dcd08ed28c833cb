"""The 1D expressiveness experiment of the paper's Fig. 1: a square wave
fitted by a sum of five skew-normal kernels and by a sum of five normal
kernels (Introduction, Fig. 1 (b) and (c)).

The 1D form of the paper's kernel (Sec. "3D Skew Gaussian Kernel",
S(x) = 2 G(x) Phi(beta^T (x - mu))) with an unnormalised Gaussian of width
sigma and a weight w:

    S(x) = w * 2 exp(-(x - mu)^2 / (2 sigma^2)) * Phi(beta (x - mu)),

Phi the standard normal CDF; beta = 0 gives w * exp(-(x - mu)^2 / (2 sigma^2))
(Phi(0) = 1/2), the normal kernel.  The fit is plain least squares on a
dense grid (scipy's trust-region reflective solver), from seeded starting
points; the skew fit also starts from the best normal fit with beta = 0, so
its residual can only be smaller or equal.  CPU only: the experiment has no
data and no GPU work.

    python -m paper_2605_18334_amd.fig1_toy
"""
from __future__ import annotations

import math
import time

import numpy as np
from scipy.optimize import least_squares
from scipy.special import ndtr


def square_wave(x: np.ndarray, period: float = 2.0, duty: float = 0.5, phase: float = 0.5) -> np.ndarray:
    """1 on the first `duty` fraction of each period (shifted by `phase`), else 0."""
    return (np.mod(x - phase, period) < duty * period).astype(np.float64)


def kernel_sum(params: np.ndarray, x: np.ndarray, skew: bool) -> np.ndarray:
    """Sum of kernels; params rows (w, mu, log sigma[, beta])."""
    p = params.reshape(-1, 4 if skew else 3)
    w, mu, s = p[:, 0], p[:, 1], np.exp(p[:, 2])
    d = x[:, None] - mu[None, :]
    g = np.exp(-0.5 * (d / s[None, :]) ** 2)
    if skew:
        g = 2.0 * g * ndtr(p[None, :, 3] * d)
    return (g * w[None, :]).sum(1)


def kernel_jacobian(params: np.ndarray, x: np.ndarray, skew: bool) -> np.ndarray:
    """d kernel_sum / d params, [len(x), params.size] (same parameter order)."""
    k = 4 if skew else 3
    p = params.reshape(-1, k)
    w, mu, s = p[:, 0], p[:, 1], np.exp(p[:, 2])
    d = x[:, None] - mu[None, :]
    g = np.exp(-0.5 * (d / s[None, :]) ** 2)
    J = np.empty((len(x), p.shape[0], k))
    if skew:
        beta = p[None, :, 3]
        Phi = ndtr(beta * d)
        phi = np.exp(-0.5 * (beta * d) ** 2) / math.sqrt(2.0 * math.pi)
        J[:, :, 0] = 2.0 * g * Phi
        J[:, :, 1] = w * 2.0 * g * (Phi * d / s ** 2 - phi * beta)
        J[:, :, 2] = w * 2.0 * g * Phi * d * d / s ** 2
        J[:, :, 3] = w * 2.0 * g * phi * d
    else:
        J[:, :, 0] = g
        J[:, :, 1] = w * g * d / s ** 2
        J[:, :, 2] = w * g * d * d / s ** 2
    return J.reshape(len(x), -1)


# parameter bounds: weight, centre (slack of one unit around the interval),
# width 0.02..2 (the wave's period is 2: a wider kernel is no longer local)
# and |beta| <= 50 (a slope of at least 1/50 of the interval per unit of
# the CDF's argument)
W_MAX, SIG_MIN, SIG_MAX, BETA_MAX = 3.0, 0.02, 2.0, 50.0


def _bounds(n: int, skew: bool, lo: float, hi: float):
    low = [-W_MAX, lo - 1.0, math.log(SIG_MIN)] + ([-BETA_MAX] if skew else [])
    high = [W_MAX, hi + 1.0, math.log(SIG_MAX)] + ([BETA_MAX] if skew else [])
    return np.tile(low, n), np.tile(high, n)


def _fit(x, y, p0, skew):
    k = 4 if skew else 3
    lb, ub = _bounds(len(p0) // k, skew, float(x[0]), float(x[-1]))
    p0 = np.clip(p0, lb + 1e-9, ub - 1e-9)
    r = least_squares(lambda p: kernel_sum(p, x, skew) - y, p0, bounds=(lb, ub),
                      jac=lambda p: kernel_jacobian(p, x, skew), method="trf", max_nfev=400)
    return r.x, float(np.sqrt(np.mean(r.fun ** 2)))


def fit_square_wave(n_kernels: int = 5, starts: int = 12, seed: int = 0, lo: float = 0.0,
                    hi: float = 4.0, n_grid: int = 801) -> dict:
    """Best least-squares fits of the square wave on [lo, hi] by n normal
    and by n skew-normal kernels over seeded starts.  Returns the RMSEs,
    the parameters and the grid."""
    x = np.linspace(lo, hi, n_grid)
    y = square_wave(x)
    rng = np.random.default_rng(seed)
    best_n = (None, math.inf)
    best_s = (None, math.inf)
    t0 = time.perf_counter()
    inits = []
    for _ in range(starts):
        mu = np.sort(rng.uniform(lo, hi, n_kernels))
        sig = np.log(rng.uniform(0.1, 0.5, n_kernels))
        w = rng.uniform(0.5, 1.0, n_kernels)
        inits.append((w, mu, sig))
        pn, en = _fit(x, y, np.stack([w, mu, sig], 1).ravel(), False)
        if en < best_n[1]:
            best_n = (pn, en)
    # skew starts: the same random starts with random skews, and the best
    # normal fit with random skews (beta = 0 among them: the skew family
    # contains the normal one, so the skew fit is never worse)
    pn = best_n[0].reshape(-1, 3)
    for k, (w, mu, sig) in enumerate(inits):
        beta = np.zeros(n_kernels) if k == 0 else rng.normal(0.0, 4.0, n_kernels)
        for p0 in (np.stack([w, mu, sig, beta], 1), np.concatenate([pn, beta[:, None]], 1)):
            ps, es = _fit(x, y, p0.ravel(), True)
            if es < best_s[1]:
                best_s = (ps, es)
    return {"x": x, "y": y, "rmse_normal": best_n[1], "rmse_skew": best_s[1],
            "params_normal": best_n[0].reshape(-1, 3), "params_skew": best_s[0].reshape(-1, 4),
            "seconds": time.perf_counter() - t0}


if __name__ == "__main__":
    r = fit_square_wave()
    print(f"square wave on [0, 4], 5 kernels: RMSE normal {r['rmse_normal']:.4f}, "
          f"skew-normal {r['rmse_skew']:.4f} ({r['seconds']:.1f} s)")
