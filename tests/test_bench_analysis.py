"""Host-side pins of the benchmark's scale-setting analysis: the Creutz ratio
recovers the string tension of an exact area-plus-perimeter law, the
deconfinement coupling of a smooth step is found within half a grid spacing,
and the T/Tc map is exact for an exponential string tension and equals 1 at
beta_c."""
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
