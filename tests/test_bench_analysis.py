"""Host-side pins of the benchmark's scale-setting analysis: the Creutz ratio
recovers the string tension of an exact area-plus-perimeter law, the
deconfinement coupling of a smooth step is found within half a grid spacing,
and the T/Tc map is exact for an exponential string tension and equals 1 at
beta_c; the learned-vs-plain statistics (jackknife error of a mean, tau_int
and its Madras-Sokal error) reproduce closed forms."""
import numpy as np
import pytest

import bench


def test_creutz_ratio_of_area_and_perimeter_law():
    sigma, p, c = 0.137, 0.29, 0.05
    R = np.arange(1, 5)
    W = np.exp(-sigma * np.outer(R, R) - p * (R[:, None] + R[None, :]) - c)
    for r in (2, 3, 4):
        assert bench.creutz(W, r) == pytest.approx(sigma, abs=1e-13)


def test_beta_c_of_a_smooth_step():
    b = np.array(bench.POLYAKOV_BETAS)
    for b0 in (2.21, 2.33, 2.47, 2.56):
        absL = 0.01 + 0.3 * (1 + np.tanh((b - b0) / 0.03)) / 2
        assert abs(bench.beta_c(b, absL) - b0) <= 0.025 + 1e-12


def test_t_over_tc_exponential_string_tension():
    b = np.array(bench.POLYAKOV_BETAS)
    k = 4.0
    sigma = 0.5 * np.exp(-k * (b - 2.0))
    bc = 2.325
    x = bench.t_over_tc(b, sigma, bc, b)
    np.testing.assert_allclose(x, np.exp(0.5 * k * (b - bc)), rtol=1e-12)
    assert bench.t_over_tc(b, sigma, bc, [bc])[0] == pytest.approx(1.0, abs=1e-14)
    assert np.all(np.diff(x) > 0)


def test_jackknife_of_a_mean_is_its_standard_error():
    """For the mean, the leave-one-out jackknife error equals the textbook
    standard error s / sqrt(n) exactly."""
    x = np.random.default_rng(3).normal(2.0, 0.7, 64)
    m, e = bench.jackknife_mean(x)
    assert m == pytest.approx(x.mean(), rel=1e-15)
    assert e == pytest.approx(x.std(ddof=1) / np.sqrt(len(x)), rel=1e-12)


def test_tau_int_of_known_processes():
    """White noise has tau_int = 1/2; an AR(1) chain x_t = rho x_(t-1) + noise has
    tau_int = (1 + rho) / (2 (1 - rho)) (= 2.0 at rho = 0.6); the Madras-Sokal
    error formula matches tau sqrt(2 (2 c tau + 1) / n)."""
    rng = np.random.default_rng(7)
    n = 200_000
    assert bench.tau_int(rng.normal(size=n)) == pytest.approx(0.5, abs=0.03)
    rho = 0.6
    e = rng.normal(size=n)
    x = np.empty(n)
    x[0] = e[0]
    for i in range(1, n):
        x[i] = rho * x[i - 1] + e[i]
    want = (1 + rho) / (2 * (1 - rho))
    got = bench.tau_int(x)
    assert got == pytest.approx(want, rel=0.05)
    assert abs(got - want) < 4 * bench.tau_int_err(want, n)
    assert bench.tau_int_err(2.0, 1000) == pytest.approx(2.0 * np.sqrt(2 * 25.0 / 1000))
