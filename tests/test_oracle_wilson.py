"""Pins of the oracle's rectangular Wilson loops (scale setting: the string
tension from Creutz ratios gives the lattice spacing the T/Tc axis of the
Polyakov-loop figure needs): the cold start, W(1,1) = the plaquette, the
symmetry W(R,T) = W(T,R) of the average over the 12 ordered planes, gauge
invariance, invariance under the centre transformation of a time slice, and
the strong-coupling area law W(R,T) = u^(RT) + O(u^(RT+4)), u = I2(beta)/I1(beta),
on an oracle Monte Carlo ensemble at beta = 0.5."""
import numpy as np
import pytest
from scipy import special

from tests import inputs


def test_cold_start_and_plaquette(orc):
    d = [4, 4, 6, 4]
    np.testing.assert_array_equal(orc.wilson_loops(d, orc.init(d, 0, 1), 2, 2), np.ones((2, 2)))
    U = inputs.as_f64(inputs.random_links(d, 3, spread=0.5))
    W = orc.wilson_loops(d, U, 2, 3)
    assert W[0, 0] == pytest.approx(orc.plaquette(d, U), abs=1e-14)


def test_symmetric_gauge_and_centre_invariant(orc):
    d = [6, 4, 4, 6]
    U = inputs.as_f64(inputs.random_links(d, 5, spread=0.7))
    W = orc.wilson_loops(d, U, 3, 3)
    np.testing.assert_allclose(W, W.T, atol=1e-14, rtol=0)
    G = U.copy()
    orc.gauge_transform(d, G, 11)
    np.testing.assert_allclose(orc.wilson_loops(d, G, 3, 3), W, atol=1e-13, rtol=0)
    # negate U_3 on the time slice t = 2: every contractible loop crosses it
    # an even number of times
    Z = U.reshape(d[3], -1, 4, 4).copy()
    Z[2, :, 3, :] *= -1
    np.testing.assert_allclose(orc.wilson_loops(d, Z.reshape(-1, 4, 4), 3, 3), W, atol=1e-14,
                               rtol=0)


def test_strong_coupling_area_law(orc):
    """beta = 0.5: u = I2/I1 = 0.1237; W(1,1) ~ u, W(1,2) ~ u^2, W(2,2) ~ u^4,
    each within three standard errors of the ensemble mean (configurations 2
    sweeps apart) plus five times the first correction u^(RT+4)."""
    d, beta = [6, 6, 6, 6], 0.5
    u = special.iv(2, beta) / special.iv(1, beta)
    U = orc.init(d, 1, 21)
    orc.sweeps(d, U, 40, 0, beta, 21)
    samples = []
    for k in range(150):
        orc.sweeps(d, U, 2, 40 + 2 * k, beta, 21)
        samples.append(orc.wilson_loops(d, U, 2, 2))
    S = np.array(samples)
    mean, err = S.mean(axis=0), S.std(axis=0, ddof=1) / np.sqrt(len(S))
    for (R, T) in ((1, 1), (1, 2), (2, 1), (2, 2)):
        want = u ** (R * T)
        tol = 3 * err[R - 1, T - 1] + 5 * u ** (R * T + 4)
        assert abs(mean[R - 1, T - 1] - want) < tol, (R, T, mean[R - 1, T - 1], want, tol)
    # the 1x2 loop is resolved: several standard errors above zero
    assert mean[0, 1] > 5 * err[0, 1]
