"""Pins of the oracle's learned proposal: the rational-quadratic spline
(Durkan et al. 2019) against its defining properties, the FP64 NLL gradient
against central finite differences, the table against direct evaluation, and
the independence-Metropolis step against the heat-bath distribution of Sec. 2
(chi-square) and against its acceptance rate computed by quadrature."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import nn_oracle as nn
from tests import inputs, stats


def random_params(seed, scale=0.4):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(nn.NPARAM) * scale).astype(np.float32)


def identity_params(seed=0):
    p = random_params(seed)
    p[1120:1120 + 1504] = 0.0
    p[2624:] = nn.identity_raw_bias()
    return p


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_spline_properties(orc, seed):
    rng = np.random.default_rng(seed)
    raw = rng.standard_normal(47) * 2.0
    kn = orc.spline_from_raw(raw)
    x, y, d = kn
    assert x[0] == -1 and x[16] == 1 and y[0] == -1 and y[16] == 1
    assert np.all(np.diff(x) >= 2e-3 - 1e-15) and np.all(np.diff(y) >= 2e-3 - 1e-15)
    assert d[0] == 1 and d[16] == 1 and np.all(d[1:16] > 1e-3)
    assert orc.spline_fwd(kn, -1.0)[0] == pytest.approx(-1, abs=1e-15)
    assert orc.spline_fwd(kn, 1.0)[0] == pytest.approx(1, abs=1e-15)
    xs = np.linspace(-1, 1, 2001)
    g = np.array([orc.spline_fwd(kn, v)[0] for v in xs])
    assert np.all(np.diff(g) > 0)
    # knots are interpolated: g(x_k) = y_k
    for k in range(17):
        assert orc.spline_fwd(kn, x[k])[0] == pytest.approx(y[k], abs=1e-13)
    # inverse, derivative vs finite differences, normalisation of q = g'/2
    for v in rng.uniform(-0.999, 0.999, 200):
        gv, ld = orc.spline_fwd(kn, v)
        xi, ld2 = orc.spline_inv(kn, gv)
        assert xi == pytest.approx(v, abs=1e-12) and ld2 == pytest.approx(ld, abs=1e-9)
        h = 1e-6
        if np.min(np.abs(x - v)) < 10 * h:
            continue  # g'' jumps at a knot; the stencil needs a smooth interval
        G = lambda t: orc.spline_fwd(kn, v + t * h)[0]
        fd = (-G(2) + 8 * G(1) - 8 * G(-1) + G(-2)) / (12 * h)  # fourth-order stencil
        assert math.log(fd) == pytest.approx(ld, abs=1e-6)
    q = lambda v: 0.5 * math.exp(orc.spline_fwd(kn, v)[1])
    tot = sum(integrate.quad(q, x[k], x[k + 1], epsabs=1e-13)[0] for k in range(16))
    assert tot == pytest.approx(1.0, abs=1e-10)


def test_identity_spline(orc):
    p = identity_params()
    for a in (0.5, 3.0, 30.0):
        kn = orc.spline_from_raw(orc.nn_forward(p, orc.nn_feature(a)))
        for v in np.linspace(-1, 1, 17):
            g, ld = orc.spline_fwd(kn, v)
            # FP32 parameters: the boundary-derivative bias is exact to ~1e-8
            assert g == pytest.approx(v, abs=1e-7) and ld == pytest.approx(0, abs=1e-7)


def test_torch_nll_matches_c_forward(orc):
    p = random_params(4)
    al = inputs.log_uniform(300, 0.5, 30, 5)
    a0 = np.random.default_rng(6).uniform(-0.999, 0.999, 300)
    loss, _ = nn.loss_and_grad(p, al, a0)
    ld = [orc.spline_fwd(orc.spline_from_raw(orc.nn_forward(p, orc.nn_feature(a))), x)[1]
          for a, x in zip(al, a0)]
    assert loss == pytest.approx(-(math.log(0.5) + np.mean(ld)), abs=1e-12)
    assert nn.feature(np.array([0.5, 30.0])).numpy() == pytest.approx([-1, 1], abs=1e-15)


def test_gradient_matches_finite_differences():
    p = random_params(7).astype(np.float64)
    al = inputs.log_uniform(64, 0.5, 30, 8)
    a0 = np.random.default_rng(9).uniform(-0.995, 0.995, 64)
    _, g = nn.loss_and_grad(p, al, a0)
    idx = [0, 5, 31, 32, 40, 64, 500, 1087, 1088, 1119, 1120, 1200, 1700, 2600, 2623, 2624,
           2640, 2656, 2670]
    import torch
    def L(i, t):
        q = p.copy()
        q[i] += t
        return float(nn.nll(torch.tensor(q), al, a0))

    for i in idx:
        h = 1e-4  # fourth-order stencil: truncation ~h^4, rounding ~1e-16/h
        fd = (-L(i, 2 * h) + 8 * L(i, h) - 8 * L(i, -h) + L(i, -2 * h)) / (12 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9), i


def test_table_rows(orc):
    p = random_params(10)
    t = orc.nn_table(p)
    last = orc.NN_ROWS - 1
    assert t.shape == (orc.NN_ROWS, 48)
    for j in (0, 17, 32, last):
        f = -1 + 2 * j / last
        x, y, d = orc.spline_from_raw(orc.nn_forward(p, f))
        np.testing.assert_allclose(t[j, :16], x[1:], atol=0)
        np.testing.assert_allclose(t[j, 16:32], y[1:], atol=0)
        np.testing.assert_allclose(t[j, 32:48], d[1:], atol=0)
    assert orc.table_row(0.5)[0] == 0 and orc.table_row(30.0)[0] == last
    a_mid = 0.5 * 60 ** (0.5 / last)  # halfway between rows 0 and 1
    assert orc.table_row(a_mid * 1.001)[0] == 1 and orc.table_row(a_mid / 1.001)[0] == 0


def _chain(orc, table, V, beta, n, seed):
    k = np.linalg.norm(V)
    Ut = V / k
    U = np.array([1.0, 0, 0, 0])
    xs, acc = np.empty(n), 0
    for t in range(n):
        U, _, a = orc.learned_link(V, U, table, beta, seed, 0, t, 0)
        acc += a == 1
        xs[t] = orc.qmul(U, Ut)[0][0]
    return xs, acc / n


def test_mh_chain_is_stationary_and_acceptance_matches_quadrature(orc):
    """Identity spline = uniform proposal q = 1/2: the independence sampler's
    acceptance is (1/2) int int min(p(x), p(y)) dx dy by quadrature."""
    table = orc.nn_table(identity_params())
    V = np.array([0.9, 0.3, -0.2, 0.1])
    beta = 1.0
    alpha = beta * np.linalg.norm(V)
    xs, acc = _chain(orc, table, V, beta, 60_000, 3)
    chi2, dof, p = stats.chi2_equiprobable(xs[1000:][::3], alpha, nbins=40)
    assert p > 1e-4, (chi2, dof)
    grid = np.linspace(-1, 1, 4001)
    pd = stats.a0_pdf(grid, alpha)
    A = 0.5 * np.trapezoid([np.trapezoid(np.minimum(pi, pd), grid) for pi in pd], grid)
    assert acc == pytest.approx(A, abs=0.01)


def test_mh_chain_random_net_stationary(orc):
    """An arbitrary (untrained, non-uniform) proposal still leaves the exact
    distribution stationary; only the acceptance rate depends on the net."""
    table = orc.nn_table(random_params(11, scale=0.15))
    V = np.array([2.5, -1.0, 0.4, 0.8])
    beta = 2.0
    xs, acc = _chain(orc, table, V, beta, 80_000, 4)
    assert 0.1 < acc < 1.0
    chi2, dof, p = stats.chi2_equiprobable(xs[2000:][::8], beta * np.linalg.norm(V), nbins=30)
    assert p > 1e-4, (chi2, dof)


def test_mh_fallback_outside_range_is_heat_bath(orc):
    table = orc.nn_table(random_params(12))
    V = np.array([20.0, 3.0, 0.0, 0.0])  # alpha = 2 * |V| > 30
    Uold = np.array([1.0, 0, 0, 0])
    out, m, a = orc.learned_link(V, Uold, table, 2.0, 5, 7, 3, 1)
    assert m[1] == np.inf and m[2] > 0
    want, _ = orc.heatbath_link(V, 2.0, 5, 7, 3, 1)
    assert a == -1
    np.testing.assert_array_equal(out, want)


# ------------------------------------------------------ over-relaxed proposal
def _links_with_a0(x, Ut, seed):
    """Links U with (U U~)_0 = x and a random direction of the vector part."""
    rng = np.random.default_rng(seed)
    n = rng.standard_normal((len(x), 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    X = np.concatenate([x[:, None], np.sqrt(1 - x * x)[:, None] * n], axis=1)
    Utd = np.broadcast_to(Ut * np.array([1, -1, -1, -1]), X.shape)
    return orc_qmul(X, Utd)


def orc_qmul(a, b):
    from oracle import su2_oracle
    return su2_oracle.qmul(a, b)


def _one_step(orc, table, V, beta, x, width, seed):
    """One over-relaxed learned update of links whose a0 in the staple frame is
    x; returns the new a0 values and the acceptance fraction."""
    Ut = V / np.linalg.norm(V)
    U = _links_with_a0(x, Ut, seed)
    out, acc = np.empty(len(x)), 0
    for i in range(len(x)):
        Un, _, a = orc.learned_link(V, U[i], table, beta, seed, i, 0, 0, or_width=width)
        acc += a == 1
        out[i] = orc.qmul(Un, Ut)[0][0]
    return out, acc / len(x)


@pytest.mark.parametrize("width", [0.0, 0.3])
def test_or_step_keeps_the_exact_distribution(orc, width):
    """Starting from exact draws of p(a0) ~ sqrt(1 - a0^2) exp(alpha a0) (Sec.
    2), one over-relaxed Metropolis step with a non-uniform learned proposal
    leaves the distribution exact (chi-square against the quadrature CDF).  A
    wrong reflection, a missing Jacobian or a proposal that is not symmetric in
    the flow coordinate would bias it (accepting with p(a0')/p(x_old) alone,
    i.e. without the proposal densities, gives p ~ 0 here)."""
    params = identity_params()  # a non-uniform spline: perturbed output biases
    params[2624:] += np.random.default_rng(3).normal(0, 0.6, 47).astype(np.float32)
    table = orc.nn_table(params)
    V = np.array([1.2, 0.3, -0.4, 0.2])
    beta = 1.0
    alpha = beta * np.linalg.norm(V)
    n = 100_000
    x = 1.0 - orc.sample_delta(np.full(n, alpha), 77, np.arange(n), 0, 0)[0]
    xn, acc = _one_step(orc, table, V, beta, x, width, 21)
    assert 0.2 < acc < 1.0
    assert np.mean(np.abs(xn - x) > 1e-9) > 0.2  # the step moves most links
    chi2, dof, p = stats.chi2_equiprobable(xn, alpha, nbins=40)
    assert p > 1e-4, (chi2, dof)


def test_or_identity_spline_reflects_a0_and_acceptance_matches_quadrature(orc):
    """With the identity spline (u = a0) and no noise the proposal is a0' = -a0,
    accepted with min(1, p(-x)/p(x)) = min(1, exp(-2 alpha x)); from exact
    draws the acceptance is E_p[min(1, exp(-2 alpha x))] by quadrature."""
    table = orc.nn_table(identity_params())
    V = np.array([0.9, 0.3, -0.2, 0.1])
    beta = 1.5
    alpha = beta * np.linalg.norm(V)
    n = 40_000
    x = 1.0 - orc.sample_delta(np.full(n, alpha), 5, np.arange(n), 0, 0)[0]
    xn, acc = _one_step(orc, table, V, beta, x, 0.0, 6)
    moved = np.abs(xn - x) > 1e-9
    np.testing.assert_allclose(xn[moved], -x[moved], atol=2e-7)  # FP32 table knots
    grid = np.linspace(-1, 1, 20001)
    A = np.trapezoid(stats.a0_pdf(grid, alpha) * np.minimum(1.0, np.exp(-2 * alpha * grid)), grid)
    assert acc == pytest.approx(A, abs=0.01)


def test_or_reflection_is_an_involution(orc):
    """Without noise the proposal map a0 -> g^{-1}(-g(a0)) applied twice
    returns the starting a0 (accepted steps of the same staple)."""
    params = identity_params()
    params[2624:] += np.random.default_rng(13).normal(0, 0.6, 47).astype(np.float32)
    table = orc.nn_table(params)
    V = np.array([1.2, 0.3, -0.4, 0.2])
    beta = 0.6
    Ut = V / np.linalg.norm(V)
    x0 = np.random.default_rng(14).uniform(-0.9, 0.99, 300)
    U0 = _links_with_a0(x0, Ut, 15)
    checked = 0
    for i in range(len(x0)):
        U1, _, a1 = orc.learned_link(V, U0[i], table, beta, 3, i, 0, 0, or_width=0.0)
        U2, _, a2 = orc.learned_link(V, U1, table, beta, 3, i, 1, 0, or_width=0.0)
        if a1 == 1 and a2 == 1:
            x1 = orc.qmul(U1, Ut)[0][0]
            x2 = orc.qmul(U2, Ut)[0][0]
            assert abs(x1 - x0[i]) > 1e-6
            assert x2 == pytest.approx(x0[i], abs=1e-9)
            checked += 1
    assert checked > 60


def _training_data_checks(alpha, a0, lo, hi):
    """p-values of the checks on training pairs: ln(alpha) uniform on
    [ln lo, ln hi] (KS), and the probability integral transform F(a0; alpha)
    of Sec. 2's a0 density uniform (KS) and uniform within each of five alpha
    bins (chi-square, 20 equal bins)."""
    from scipy import stats as sst
    p_alpha = sst.kstest(np.log(alpha / lo) / np.log(hi / lo), "uniform").pvalue
    u = stats.a0_cdf_vec(a0, alpha)
    p_pit = sst.kstest(u, "uniform").pvalue
    edges = np.quantile(alpha, np.linspace(0, 1, 6))
    p_bins = []
    for b in range(5):
        sel = (alpha >= edges[b]) & (alpha <= edges[b + 1])
        counts, _ = np.histogram(u[sel], bins=20, range=(0, 1))
        exp = sel.sum() / 20
        p_bins.append(sst.chi2.sf(((counts - exp) ** 2 / exp).sum(), 19))
    return p_alpha, p_pit, min(p_bins)


def test_training_data_distribution(orc):
    """orc_nn_data, the proposal's training pairs: alpha log-uniform on [0.5, 30]
    and each a0 an exact draw from sqrt(1 - a0^2) exp(alpha a0) at its own alpha
    (Sec. 2).  The same statistics reject a linear-in-alpha map and a0 paired with
    alpha off by 10 % (their power, shown on the oracle's own samples)."""
    n = 120_000
    a, x = orc.nn_data(n, 0.5, 30.0, seed=77)
    assert a.min() >= 0.5 and a.max() <= 30.0 and np.all(np.abs(x) <= 1.0)
    p_alpha, p_pit, p_bin = _training_data_checks(a, x, 0.5, 30.0)
    assert p_alpha > 1e-3 and p_pit > 1e-3 and p_bin > 1e-4, (p_alpha, p_pit, p_bin)
    # power: a uniform (not log-uniform) alpha map, and a0 judged at 1.1 alpha
    lin = 0.5 + (np.log(a / 0.5) / np.log(60.0)) * 29.5
    assert _training_data_checks(lin, x, 0.5, 30.0)[0] < 1e-10
    assert min(_training_data_checks(a * 1.1, x, 0.5, 30.0)[1:]) < 1e-6
    # other seeds give other pairs; the same seed the same pairs
    a2, x2 = orc.nn_data(1000, 0.5, 30.0, seed=77)
    np.testing.assert_array_equal(a2, a[:1000])
    np.testing.assert_array_equal(x2, x[:1000])
    a3, _ = orc.nn_data(1000, 0.5, 30.0, seed=78)
    assert np.mean(a3 != a[:1000]) > 0.99


def test_training_data_range_argument(orc):
    """The range arguments are honoured: log-uniform on [2, 8]."""
    a, x = orc.nn_data(40_000, 2.0, 8.0, seed=5)
    assert a.min() >= 2.0 and a.max() <= 8.0
    p_alpha, p_pit, p_bin = _training_data_checks(a, x, 2.0, 8.0)
    assert p_alpha > 1e-3 and p_pit > 1e-3 and p_bin > 1e-4, (p_alpha, p_pit, p_bin)
