"""Statistics helpers for the tests (closed forms and chi-square machinery).

The a0 density is fixed by Sec. 2 of the paper: p(a0) ~ sqrt(1 - a0^2) exp(alpha a0)
on [-1, 1], alpha = beta k.  Its CDF is evaluated here by adaptive quadrature
(scipy), independently of any sampler under test.
"""
import functools
import json
import os

import numpy as np
from scipy import integrate, optimize, special, stats

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@functools.lru_cache(maxsize=None)
def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def a0_pdf(x, alpha):
    z = np.pi * special.ive(1, alpha) / alpha  # Z e^{-alpha}
    return np.sqrt(np.clip(1 - x * x, 0, None)) * np.exp(alpha * (x - 1)) / z


def a0_cdf(x, alpha):
    if x <= -1:
        return 0.0
    if x >= 1:
        return 1.0
    z = np.pi * special.ive(1, alpha) / alpha
    f = lambda t: np.sqrt(max(1 - t * t, 0.0)) * np.exp(alpha * (t - 1))
    lo = max(-1.0, 1.0 - 60.0 / alpha) if alpha > 1 else -1.0
    if x <= lo:
        return 0.0
    return integrate.quad(f, lo, x, limit=400, epsabs=1e-15, epsrel=1e-12)[0] / z


def a0_cdf_vec(x, alpha, nodes=128):
    """a0_cdf for arrays of (x, alpha) pairs: with t = -cos(phi) the integral
    over [-1, x] becomes int_0^arccos(-x) sin^2(phi) exp(-alpha (1 + cos phi))
    dphi, a smooth integrand, taken by Gauss-Legendre quadrature per pair."""
    x = np.clip(np.asarray(x, dtype=np.float64), -1.0, 1.0)
    alpha = np.asarray(alpha, dtype=np.float64)
    g, w = np.polynomial.legendre.leggauss(nodes)
    top = np.arccos(-x)[..., None]
    phi = 0.5 * top * (g + 1.0)
    f = np.sin(phi) ** 2 * np.exp(-alpha[..., None] * (1.0 + np.cos(phi)))
    integral = 0.5 * top[..., 0] * (f * w).sum(axis=-1)
    return integral / (np.pi * special.ive(1, alpha) / alpha)


@functools.lru_cache(maxsize=None)
def a0_quantile_edges(alpha, nbins):
    edges = [-1.0]
    for q in np.arange(1, nbins) / nbins:
        edges.append(optimize.brentq(lambda x: a0_cdf(x, alpha) - q, -1.0, 1.0, xtol=1e-14))
    edges.append(1.0)
    return np.array(edges)


def chi2_equiprobable(samples, alpha, nbins=50):
    """Chi-square of a0 samples against p(.; alpha) with equiprobable bins.
    Returns (chi2, dof, p-value)."""
    edges = a0_quantile_edges(float(alpha), nbins)
    counts, _ = np.histogram(np.clip(samples, -1, 1), bins=edges)
    n = len(samples)
    expected = n / nbins
    chi2 = float(((counts - expected) ** 2 / expected).sum())
    dof = nbins - 1
    return chi2, dof, float(stats.chi2.sf(chi2, dof))


def bessel_moments(alpha):
    i1, i2 = special.ive(1, alpha), special.ive(2, alpha)
    return i2 / i1, 1 - 3 * i2 / (alpha * i1)


def semicircle_moments():
    """Haar measure on SU(2): a0 density (2/pi) sqrt(1 - a0^2)."""
    return 0.0, 0.25


def tau_int(x, c=6.0):
    """Integrated autocorrelation time with Madras-Sokal automatic windowing."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    x = x - x.mean()
    var = x.var()
    if var == 0 or n < 8:
        return 0.5
    f = np.fft.rfft(x, 2 * n)
    acf = np.fft.irfft(f * np.conj(f))[:n] / (var * np.arange(n, 0, -1))
    tau = 0.5
    for w in range(1, n):
        tau += acf[w]
        if w >= c * tau:
            break
    return max(tau, 0.5)


def mean_err(x):
    """Mean and tau_int-corrected standard error."""
    x = np.asarray(x, dtype=np.float64)
    t = tau_int(x)
    return float(x.mean()), float(np.sqrt(2 * t * x.var(ddof=1) / len(x)))
