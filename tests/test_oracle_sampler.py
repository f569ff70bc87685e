"""Pins of the oracle's exact a0 sampler and single-link heat bath (Sec. 2).

The target density p(a0) ~ sqrt(1 - a0^2) exp(alpha a0) is checked by a
chi-square test against its exact CDF (quadrature), by the Bessel-ratio
moments, and by the acceptance rate of each branch (Kennedy-Pendleton for
alpha >= 1, semicircle rejection below), all closed forms in tests/golden.
"""
import numpy as np
import pytest

from tests import inputs, stats

ROWS = stats.golden("sampler_moments.json")["rows"]


@pytest.mark.parametrize("row", ROWS, ids=lambda r: f"alpha{r['alpha']}")
def test_sampler_distribution_moments_and_acceptance(orc, row):
    alpha = row["alpha"]
    n = 120_000
    delta, trials, margin = orc.sample_delta(np.full(n, alpha), seed=2024,
                                             site=np.arange(n, dtype=np.uint32), sweep=3, mu=1)
    a0 = 1 - delta
    assert np.all(np.abs(a0) <= 1)
    chi2, dof, p = stats.chi2_equiprobable(a0, alpha, nbins=60)
    assert p > 1e-4, (chi2, dof)
    m1, m2 = a0.mean(), (a0 * a0).mean()
    s1 = a0.std() / np.sqrt(n)
    s2 = (a0 * a0).std() / np.sqrt(n)
    assert abs(m1 - row["mean_a0"]) < 5 * s1
    assert abs(m2 - row["mean_a0_sq"]) < 5 * s2
    acc = row["accept_kp"] if alpha >= 1.0 else row["accept_semicircle"]
    mean_trials = trials.mean()
    # trials ~ geometric(acc): mean 1/acc, var (1-acc)/acc^2
    sig = np.sqrt((1 - acc) / acc ** 2 / n)
    assert abs(mean_trials - 1 / acc) < 5 * sig + 1e-12
    assert np.all(margin >= 0)


def test_sampler_is_keyed_by_counter(orc):
    a = np.full(64, 3.0)
    d1, _, _ = orc.sample_delta(a, 9, np.arange(64, dtype=np.uint32), 5, 2)
    d2, _, _ = orc.sample_delta(a, 9, np.arange(64, dtype=np.uint32), 5, 2)
    np.testing.assert_array_equal(d1, d2)
    for kw in ({"seed": 10}, {"sweep": 6}, {"mu": 3}, {"replica": 1}):
        args = dict(seed=9, sweep=5, mu=2, replica=0)
        args.update(kw)
        d3, _, _ = orc.sample_delta(a, args["seed"], np.arange(64, dtype=np.uint32),
                                    args["sweep"], args["mu"], args["replica"])
        assert np.mean(d3 != d1) > 0.9


def _frame(V):
    k = np.linalg.norm(V)
    return V / k, k


@pytest.mark.parametrize("vseed", [1, 2, 3])
def test_heatbath_link_distribution(orc, vseed):
    """U' = X U~^+ with X ~ exp(beta k x0) dHaar: X = U' U~ has a0 with the Bessel
    moments of alpha = beta k and an isotropic vector part; |U'| = 1."""
    V = inputs.random_staples(1, vseed, kmin=0.5, kmax=5.0)[0].astype(np.float64)
    beta = 1.7
    Ut, k = _frame(V)
    n = 40_000
    X = np.empty((n, 4))
    for i in range(n):
        out, _ = orc.heatbath_link(V, beta, seed=77, site=i, sweep=0, mu=2)
        assert abs(np.linalg.norm(out) - 1) < 1e-13
        X[i] = orc.qmul(out, Ut)[0]
    m1, m2 = stats.bessel_moments(beta * k)
    assert abs(X[:, 0].mean() - m1) < 5 * X[:, 0].std() / np.sqrt(n)
    assert abs((X[:, 0] ** 2).mean() - m2) < 5 * (X[:, 0] ** 2).std() / np.sqrt(n)
    for c in (1, 2, 3):
        assert abs(X[:, c].mean()) < 5 * X[:, c].std() / np.sqrt(n)
        want = (1 - m2) / 3
        assert abs((X[:, c] ** 2).mean() - want) < 5 * (X[:, c] ** 2).std() / np.sqrt(n)
    # the weight exp(beta/2 Tr(U'V)) = exp(beta k x0): check the mean of (1/2)Tr(U'V)
    tr = np.array([orc.qmul(orc.heatbath_link(V, beta, 78, i, 0, 2)[0], V)[0][0]
                   for i in range(4000)])
    assert abs(tr.mean() - k * m1) < 5 * tr.std() / np.sqrt(4000)


def test_heatbath_direction_is_isotropic(orc):
    """The vector part of X is uniform on the sphere: cos(theta) = X3/|X| and
    phi = atan2(X2, X1) are uniform; their 18-bit uniforms come from the low
    bits of the first trial's Philox words."""
    V = np.array([2.0, 0.3, -0.4, 0.1])
    Ut, k = _frame(V)
    n = 30_000
    X = np.array([orc.qmul(orc.heatbath_link(V, 1.3, 5, i, 2, 1)[0], Ut)[0] for i in range(n)])
    v = X[:, 1:] / np.linalg.norm(X[:, 1:], axis=1, keepdims=True)
    from scipy import stats as st
    assert st.kstest(v[:, 2], "uniform", args=(-1, 2)).pvalue > 1e-4
    phi = np.arctan2(v[:, 1], v[:, 0])
    assert st.kstest(phi, "uniform", args=(-np.pi, 2 * np.pi)).pvalue > 1e-4
    # the direction is independent of a0
    assert abs(np.corrcoef(X[:, 0], v[:, 2])[0, 1]) < 5 / np.sqrt(n)
    w = np.array([0, 511, 0x1FF00], dtype=np.uint32)
    u = [orc._load().orc_uniform18(int(m)) for m in w]
    assert u[0] == 2.0 ** -19 and 0 < min(u) and max(u) < 1


def test_heatbath_zero_staple_is_haar(orc):
    n = 40_000
    a0 = np.array([orc.heatbath_link(np.zeros(4), 2.0, 5, i, 0, 0)[0][0] for i in range(n)])
    assert abs(a0.mean()) < 5 * 0.5 / np.sqrt(n)
    assert abs((a0 ** 2).mean() - 0.25) < 5 * 0.2 / np.sqrt(n)
