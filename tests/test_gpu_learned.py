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
    # element by element, per tensor (W1, b1, W2, b2, W3, b3): the FP32 gradient
    # within 1e-3 relative of the FP64 one, with an absolute floor of 1e-4 times
    # the tensor's norm for entries that nearly cancel over the batch
    for lo, hi in ((0, 32), (32, 64), (64, 1088), (1088, 1120), (1120, 2624), (2624, 2671)):
        w = wg[lo:hi]
        bound = 1e-3 * np.abs(w) + 1e-4 * np.linalg.norm(w)
        excess = np.abs(g[lo:hi] - w) / bound
        print(f"[gpu-test] gradient [{lo}:{hi}] worst error / bound {excess.max():.3f}",
              flush=True)
        assert np.all(excess <= 1.0), (lo, hi, int(np.argmax(excess)), excess.max())
        err = np.linalg.norm(g[lo:hi] - w) / np.linalg.norm(w)
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


@pytest.mark.parametrize("width", [-1.0, 0.0, 0.25], ids=["independence", "reflect", "or0.25"])
def test_learned_link_updates_match_oracle(su2, orc, width):
    announce(f"learned link parity or_width={width}")
    p = random_params(7, scale=0.2)
    n = 6000
    V = inputs.random_staples(n, 8, kmin=0.1, kmax=8.0)
    Uold = np.random.default_rng(10).standard_normal((n, 4))
    Uold = (Uold / np.linalg.norm(Uold, axis=1, keepdims=True)).astype(np.float32)
    beta = 2.1
    table = orc.nn_table(p)
    with su2.NN(params=p) as net:
        net.build_table()
        got, acc = net.test_links(V, Uold, beta, seed=11, sweep=4, mu=2, replica=1,
                                  or_width=width)
    nflag = 0
    kinds = {-1: 0, 0: 0, 1: 0}
    for i in range(n):
        want, m, a = orc.learned_link(V[i].astype(np.float64), Uold[i].astype(np.float64), table,
                                      beta, 11, i, 4, 2, 1, or_width=width)
        if learned_flagged(m)[0]:
            nflag += 1
            continue
        assert acc[i] == a, (i, acc[i], a, m)
        assert np.abs(got[i] - want).max() < 1e-5, (i, got[i], want)
        kinds[a] += 1
    assert nflag <= max_learned_flags(n)
    assert min(kinds.values()) > 50, kinds  # all three outcomes exercised


@pytest.mark.parametrize("width", [-1.0, 0.1], ids=["independence", "or0.1"])
@pytest.mark.parametrize("dims", [[4, 4, 4, 4], [8, 6, 4, 6]], ids=lambda d: "x".join(map(str, d)))
def test_learned_pass_matches_oracle(su2, orc, dims, width):
    announce(f"learned pass parity dims={dims} or_width={width}")
    p = random_params(12, scale=0.2)
    table = orc.nn_table(p)
    beta, seed = 2.2, 99
    links = inputs.random_links(dims, 13, spread=0.7)
    par_of = parities(orc, dims)
    with su2.NN(params=p) as net, su2.Lattice(dims, beta, seed) as lat:
        net.build_table()
        lat.set_proposal(net)
        lat.set_overrelax(width)
        lat.set_sweep(5)
        total_flag = 0
        for mu in range(4):
            for par in range(2):
                lat.set_links(links)
                U = links.astype(np.float64)
                margin, acc = orc.learned_pass(dims, U, table, mu, par, 5, beta, seed,
                                               or_width=width)
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


@pytest.mark.parametrize("width", [0.0, 0.3])
def test_overrelaxed_steps_keep_the_exact_distribution(su2, width):
    """Links drawn from the exact heat bath (GPU sampler, pinned to the
    quadrature CDF elsewhere) stay exactly distributed under repeated
    over-relaxed learned updates with the same staple (chi-square of every
    step's a0).  The flow is a non-uniform spline (perturbed identity), so the
    Metropolis ratio's proposal densities matter."""
    announce(f"over-relaxed steps stationary width={width}")
    p = random_params(14, scale=0.15)
    p[1120:2624] = 0.0
    p[2624:] = (nn.identity_raw_bias() +
                np.random.default_rng(3).normal(0, 0.6, 47)).astype(np.float32)
    V = np.array([1.2, 0.3, -0.4, 0.2], np.float32)
    beta = 1.0
    Vd = V.astype(np.float64)
    alpha = beta * float(np.linalg.norm(Vd))
    Ut = Vd / np.linalg.norm(Vd)
    n = 16384
    Vs = np.tile(V, (n, 1))
    U = su2.su2_test_heatbath_links(Vs, beta, 21, 0, 1)
    samples = []
    with su2.NN(params=p) as net:
        net.build_table()
        accs = 0
        for t in range(8):
            U, acc = net.test_links(Vs, U, beta, seed=22, sweep=t, mu=0, or_width=width)
            accs += (acc == 1).sum()
            Ud = U.astype(np.float64)
            samples.append(Ud[:, 0] * Ut[0] - Ud[:, 1:] @ Ut[1:])
    for x in samples:
        chi2, dof, pv = stats.chi2_equiprobable(x, alpha, nbins=40)
        assert pv > 1e-4, (chi2, dof)
    assert 0.1 < accs / (8 * n) < 1.0


def test_overrelaxed_ensemble_matches_heat_bath(su2):
    """Batched lattices (32 replicas of 8^4, beta 2.3, hot start): the
    over-relaxed learned update (trained flow, noise half-width 0.05) and the
    exact heat bath give the same mean plaquette (both chains are exact; the
    heat bath is pinned to the oracle elsewhere).  Replica chain means give the
    error bars."""
    announce("over-relaxed ensemble == heat bath")
    import torch
    n, therm, meas = 32, 150, 400
    dims = [[8, 8, 8, 8]] * n
    means = {}
    with su2.NN(seed=3) as net:
        net.sample_data(1_000_000, 0.5, 30.0, seed=3)
        net.train(3000, 8192, 3e-3, lr_end=1e-4)
        net.build_table()
        for name, mode, width in (("kp", su2.SU2_KP, -1.0), ("or", su2.SU2_LEARNED, 0.05)):
            with su2.Batch(dims, [2.3] * n, [1] * n, seed=11 if name == "kp" else 12) as b:
                b.set_proposal(net)
                b.set_overrelax(width)
                b.sweep(therm, mode)
                h = b.sweep_measure(meas, mode, meas=su2.SU2_MEAS_PLAQ).cpu().numpy()
                means[name] = h[:, :, 0].mean(axis=0)
                if name == "or":
                    prop, acc = b.accept_stats()
                    assert acc.sum() / prop.sum() > 0.9
    d = means["or"].mean() - means["kp"].mean()
    err = np.sqrt(means["or"].var(ddof=1) / n + means["kp"].var(ddof=1) / n)
    assert abs(d) < 3.5 * err, (d, err)
    torch.cuda.synchronize()


def test_training_gain_over_untrained_proposal(su2):
    """What training buys, measured on the GPU: the trained flow's NLL of
    exact-sampler draws falls well below the untrained (identity spline,
    uniform proposal) value ln 2, its Metropolis acceptance on a batch of
    thermalised lattices rises from ~0.15 to > 0.95, and the plaquette's
    integrated autocorrelation time drops by a large factor, so the trained
    proposal delivers several times more independent samples per sweep.  The
    untrained chains have tau_int of tens of sweeps, so they run 4000 sweeps:
    a windowed estimate from a run only ~15 tau long comes out biased low."""
    announce("learned: training gain")
    n, dims, beta = 16, [8, 8, 8, 8], 2.3
    res = {}
    with su2.NN(seed=3) as trained, su2.NN(seed=3) as untrained:
        trained.sample_data(1_000_000, 0.5, 30.0, seed=3)
        untrained.sample_data(1_000_000, 0.5, 30.0, seed=3)
        nll0, _ = untrained.loss_grad(0, 16384)
        trained.train(3000, 8192, 3e-3, lr_end=1e-4)
        nll1, _ = trained.loss_grad(0, 16384)
        for name, net in (("untrained", untrained), ("trained", trained)):
            net.build_table()
            with su2.Batch([dims] * n, [beta] * n, [1] * n, seed=4) as b:
                b.set_proposal(net)
                b.sweep(150)  # heat-bath thermalisation
                b.accept_stats(reset=True)
                h = b.sweep_measure(4000, su2.SU2_LEARNED, meas=su2.SU2_MEAS_PLAQ).cpu().numpy()
                prop, acc = b.accept_stats()
            taus = [stats.tau_int(h[:, r, 0]) for r in range(n)]
            res[name] = (acc.sum() / prop.sum(), float(np.mean(taus)))
    assert nll0 == pytest.approx(np.log(2.0), abs=1e-3)
    assert nll1 < nll0 - 0.5, (nll0, nll1)
    (a0, t0), (a1, t1) = res["untrained"], res["trained"]
    assert a0 < 0.3 and a1 > 0.95, res
    assert t0 > 4 * t1, res


def test_proposal_cannot_be_destroyed_while_attached(su2):
    """A context or batch holds its learned proposal: su2_nn_destroy refuses
    (SU2_ESTATE, nothing freed) while any of them has it attached, and
    succeeds once they have detached or been destroyed.  The binding keeps the
    network alive while attached, so dropping the caller's reference is safe."""
    announce("proposal lifetime")
    import gc
    with su2.NN(seed=4) as net:
        net.build_table()
        lat = su2.Lattice([4, 4, 4, 4], 2.3, 1, su2.SU2_HOT)
        b = su2.Batch([[4, 4, 4, 4], [6, 4, 4, 4]], [2.0, 2.5], [1, 1], 2)
        lat.set_proposal(net)
        b.set_proposal(net)
        for holders in (2, 1):
            with pytest.raises(su2.SU2Error) as e:
                su2.su2_nn_destroy(net.h)
            assert e.value.code == su2.SU2_ESTATE
            assert f"{holders} lattice" in str(e.value)
            if holders == 2:
                lat.set_proposal(None)  # detach
        b.close()  # destroying the batch detaches it
        net2 = su2.NN(seed=5)
        net2.build_table()
        lat.set_proposal(net2)
        del net2
        gc.collect()
        lat.heatbath_sweep(2, su2.SU2_LEARNED)  # the lattice kept net2 alive
        assert np.all(np.isfinite(lat.get_links()))
        lat.close()
    # net was destroyed by the context manager: nothing held it any more
    assert net.h is None
