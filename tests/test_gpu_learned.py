"""Learned a0 proposal on the GPU against the FP64 oracle: training data,
NLL gradient, spline table, the Metropolis link update, the fused learned pass,
stationarity of the chain, and what training gains over the untrained
(uniform) proposal."""
import numpy as np
import pytest

from oracle import nn_oracle as nn
from tests import inputs, stats
from tests.gpu_util import announce, learned_flagged, max_flags, max_learned_flags, parities

pytestmark = pytest.mark.gpu


def random_params(seed, scale=0.3):
    return (np.random.default_rng(seed).standard_normal(nn.NPARAM) * scale).astype(np.float32)


def test_training_data_matches_oracle(su2, orc):
    announce("nn training data parity")
    n = 20000
    with su2.NN(seed=1) as net:
        net.sample_data(n, 0.5, 30.0, seed=77)
        a, x = net.data()
    oa, ox = orc.nn_data(n, 0.5, 30.0, 77)
    np.testing.assert_allclose(a, oa, rtol=2e-6)
    bad = np.abs(x - ox) > 1e-5
    assert bad.sum() <= max_flags(n), bad.sum()


@pytest.mark.parametrize("batch", [1000, 4096])
def test_loss_and_gradient_match_oracle(su2, batch):
    announce(f"nn gradient parity batch={batch}")
    p = random_params(3)
    al = inputs.log_uniform(batch, 0.5, 30.0, 4).astype(np.float32)
    x = np.random.default_rng(5).uniform(-0.999, 0.999, batch).astype(np.float32)
    with su2.NN(params=p) as net:
        net.set_data(al, x)
        loss, g = net.loss_grad(0, batch)
    wl, wg = nn.loss_and_grad(p.astype(np.float64), al.astype(np.float64), x.astype(np.float64))
    assert loss == pytest.approx(wl, rel=1e-5)
    # per tensor relative error of the FP32 gradient
    for lo, hi in ((0, 32), (32, 64), (64, 1088), (1088, 1120), (1120, 2624), (2624, 2671)):
        err = np.linalg.norm(g[lo:hi] - wg[lo:hi]) / np.linalg.norm(wg[lo:hi])
        assert err < 1e-3, (lo, hi, err)


def test_table_matches_oracle(su2, orc):
    announce("nn table parity")
    p = random_params(6)
    with su2.NN(params=p) as net:
        net.build_table()
        t = net.table()
    w = orc.nn_table(p)
    np.testing.assert_allclose(t[:, :32], w[:, :32], atol=2e-6)
    np.testing.assert_allclose(t[:, 32:], w[:, 32:], rtol=2e-5)


def test_learned_link_updates_match_oracle(su2, orc):
    announce("learned link parity")
    p = random_params(7, scale=0.2)
    n = 6000
    V = inputs.random_staples(n, 8, kmin=0.1, kmax=8.0)
    Uold = np.random.default_rng(10).standard_normal((n, 4))
    Uold = (Uold / np.linalg.norm(Uold, axis=1, keepdims=True)).astype(np.float32)
    beta = 2.1
    table = orc.nn_table(p)
    with su2.NN(params=p) as net:
        net.build_table()
        got, acc = net.test_links(V, Uold, beta, seed=11, sweep=4, mu=2, replica=1)
    nflag = 0
    kinds = {-1: 0, 0: 0, 1: 0}
    for i in range(n):
        want, m, a = orc.learned_link(V[i].astype(np.float64), Uold[i].astype(np.float64), table,
                                      beta, 11, i, 4, 2, 1)
        if learned_flagged(m)[0]:
            nflag += 1
            continue
        assert acc[i] == a, (i, acc[i], a, m)
        assert np.abs(got[i] - want).max() < 1e-5, (i, got[i], want)
        kinds[a] += 1
    assert nflag <= max_learned_flags(n)
    assert min(kinds.values()) > 50, kinds  # all three outcomes exercised


@pytest.mark.parametrize("dims", [[4, 4, 4, 4], [8, 6, 4, 6]], ids=lambda d: "x".join(map(str, d)))
def test_learned_pass_matches_oracle(su2, orc, dims):
    announce(f"learned pass parity dims={dims}")
    p = random_params(12, scale=0.2)
    table = orc.nn_table(p)
    beta, seed = 2.2, 99
    links = inputs.random_links(dims, 13, spread=0.7)
    par_of = parities(orc, dims)
    with su2.NN(params=p) as net, su2.Lattice(dims, beta, seed) as lat:
        net.build_table()
        lat.set_proposal(net)
        lat.set_links(links)
        lat.set_sweep(5)
        total_flag = 0
        for mu in range(4):
            for par in range(2):
                U = lat.get_links().astype(np.float64)
                margin, acc = orc.learned_pass(dims, U, table, mu, par, 5, beta, seed)
                lat.test_pass(mu, par, su2.SU2_LEARNED)
                got = lat.get_links()
                upd = par_of == par
                flag = learned_flagged(margin)
                ok = upd & ~flag
                total_flag += int((upd & flag).sum())
                assert np.abs(got[ok, mu] - U[ok, mu]).max() < 1e-5, (mu, par)
        assert total_flag <= max_learned_flags(4 * int(np.prod(dims)))


def test_learned_chain_is_stationary(su2):
    """4096 independent single-link chains with one fixed staple, iterated on
    the GPU: after burn-in, a0 = (U U~)_0 follows sqrt(1-a0^2) exp(alpha a0)."""
    announce("learned chain stationarity")
    p = random_params(14, scale=0.15)
    V = np.array([1.2, 0.5, -0.3, 0.2], np.float32)
    beta = 2.5
    alpha = beta * float(np.linalg.norm(V.astype(np.float64)))
    Ut = V.astype(np.float64) / np.linalg.norm(V.astype(np.float64))
    n = 4096
    Vs = np.tile(V, (n, 1))
    U = np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1))
    samples = []
    with su2.NN(params=p) as net:
        net.build_table()
        accs = 0
        for t in range(120):
            U, acc = net.test_links(Vs, U, beta, seed=15, sweep=t, mu=0)
            accs += (acc == 1).sum()
            if t >= 40:
                Ud = U.astype(np.float64)
                samples.append(Ud[:, 0] * Ut[0] - Ud[:, 1:] @ Ut[1:])
    x = np.concatenate(samples[::4])
    chi2, dof, pv = stats.chi2_equiprobable(x, alpha, nbins=50)
    assert pv > 1e-4, (chi2, dof)
    assert 0.05 < accs / (120 * n) < 1.0


def test_training_reduces_nll_and_raises_acceptance(su2, orc):
    """Train on exact-sampler draws; the trained proposal must beat the
    untrained (uniform) one in NLL and in Metropolis acceptance on a
    thermalised lattice."""
    announce("nn training gain")
    with su2.NN(seed=3) as net:
        net.sample_data(400_000, 0.5, 30.0, seed=5)
        l0, _ = net.loss_grad(0, 50_000)
        hist = net.train(600, 4096, 3e-3)
        l1, _ = net.loss_grad(0, 50_000)
        assert hist[-50:].mean() < hist[:50].mean()
        assert l1 < l0 - 0.5, (l0, l1)
        net.build_table()
        dims = [8, 8, 8, 8]
        rates = {}
        with su2.NN(seed=3) as untrained:
            untrained.build_table()
            for name, model in (("untrained", untrained), ("trained", net)):
                with su2.Lattice(dims, 2.3, 21, su2.SU2_HOT) as lat:
                    lat.heatbath_sweep(30)
                    lat.set_proposal(model)
                    lat.accept_stats(reset=True)
                    lat.heatbath_sweep(10, su2.SU2_LEARNED)
                    prop, acc = lat.accept_stats()
                    rates[name] = acc / prop
                    assert prop > 0.9 * 10 * 4 * 8 ** 4
        assert rates["trained"] > rates["untrained"] + 0.3, rates
        assert rates["trained"] > 0.8, rates


def test_learned_and_exact_ensembles_agree(su2):
    """Same lattice and beta: plaquette means of the learned-Metropolis chain and
    the exact heat-bath chain agree within their tau_int-corrected errors."""
    announce("learned vs exact ensembles")
    dims, beta = [8, 8, 8, 8], 2.3
    with su2.NN(seed=3) as net:
        net.sample_data(200_000, 0.5, 30.0, seed=6)
        net.train(400, 4096, 3e-3)
        net.build_table()
        means = []
        for mode, seed in ((su2.SU2_KP, 31), (su2.SU2_LEARNED, 32)):
            with su2.Lattice(dims, beta, seed, su2.SU2_HOT) as lat:
                lat.set_proposal(net)
                lat.heatbath_sweep(100, mode)
                h = lat.sweep_measure(1500, mode=mode).cpu().numpy()[:, 0]
                means.append(stats.mean_err(h))
    (m1, e1), (m2, e2) = means
    assert abs(m1 - m2) < 3 * np.hypot(e1, e2), means


def test_cosine_schedule_with_equal_ends_is_constant_lr(su2):
    announce("cosine schedule")
    params = []
    for cos in (False, True):
        with su2.NN(seed=4) as net:
            net.sample_data(50_000, 0.5, 30.0, seed=8)
            h = net.train(30, 1024, 2e-3, lr_end=2e-3 if cos else None)
            params.append(net.params)
            assert np.all(np.isfinite(h))
    np.testing.assert_array_equal(params[0], params[1])
