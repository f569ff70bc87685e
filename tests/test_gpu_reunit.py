"""Reunitarisation fused into the passes (su2_set_reunit_fused).

In a reunitarisation sweep the last pass stage stores every link as U/|U|
(|U|^2 in FP64) and the plaquette stays fused into the odd passes.  In exact
arithmetic a heat-bath link is unit and the reunitarisation is the identity,
so against the FP64 oracle (which reunitarises after the sweep) every link
must agree to the one-sweep tolerance; against the separate
reunitarisation pass the links differ by rounding only.  Captured graphs,
batches, the over-relaxed compound sweep and the LDS-staged pass follow the
same schedule bit for bit."""
import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import MARGIN_FLAG, announce, max_flags

pytestmark = pytest.mark.gpu

PLAQ = 1
DIMS = [[4, 4, 4, 4], [6, 4, 8, 2], [8, 8, 8, 8], [4, 6, 2, 8], [10, 8, 6, 4], [12, 12, 12, 12]]
BETAS = [2.3, 1.9, 2.6, 0.7, 3.0, 2.1]
STARTS = [1, 0, 1, 1, 0, 1]


def norm_dev(links):
    """max | |U|^2 - 1 | over the links, in FP64."""
    n2 = (links.astype(np.float64) ** 2).sum(axis=-1)
    return float(np.abs(n2 - 1.0).max())


def oracle_sweep(orc, dims, U, sweep, n_or, beta, seed):
    """One (compound) sweep of the oracle with the reunitarisation after it;
    returns the number of heat-bath decisions within the flag margin."""
    nflag = 0
    for mu in range(4):
        for p in range(2):
            m = orc.do_pass(dims, U, mu, p, sweep, beta, seed, want_margin=True)
            nflag += int((m < MARGIN_FLAG).sum())
    for _ in range(n_or):
        for mu in range(4):
            for p in range(2):
                orc.or_pass(dims, U, mu, p)
    orc.reunitarize(dims, U)
    return nflag


@pytest.mark.parametrize("n_or", [0, 1], ids=["kp", "kp-or1"])
@pytest.mark.parametrize("dims", [[4, 6, 2, 8], [16, 16, 16, 16]],
                         ids=lambda d: "x".join(map(str, d)))
def test_fused_reunitarisation_sweep_matches_oracle(su2, orc, dims, n_or):
    """Sweep 9 with reunit_every 5 is a reunitarisation sweep: every link is
    unit to FP32 rounding afterwards, every link agrees with the oracle's
    sweep-then-reunitarise within (1 + n_or) 1e-5 outside the cones of
    flagged decisions, and the fused plaquette equals the oracle's and the
    standalone one on the final configuration."""
    announce(f"fused reunitarisation vs oracle dims={dims} n_or={n_or}")
    beta, seed, sw = 2.4, 23, 9
    links = inputs.random_links(dims, 130 + dims[1], spread=0.6)
    mode = su2.SU2_KP_OR if n_or else su2.SU2_KP
    with su2.Lattice(dims, beta, seed) as lat:
        lat.set_reunit_fused(True)
        lat.set_hb_overrelax(n_or)
        lat.set_links(links)
        lat.set_sweep(sw)
        h = lat.sweep_measure(1, mode, reunit_every=5, meas=PLAQ).cpu().numpy()
        got = lat.get_links()
        standalone = lat.plaquette()
    U = links.astype(np.float64)
    nflag = oracle_sweep(orc, dims, U, sw, n_or, beta, seed)
    V = int(np.prod(dims))
    tol = (1 + n_or) * 1e-5
    d = np.abs(got - U).max(axis=2)
    bad = int((d > tol).sum())
    announce(f"  max |gpu - oracle| {d.max():.2e}; off by > {tol}: {bad}; flagged {nflag}; "
             f"max ||U|^2 - 1| {norm_dev(got):.2e}")
    assert norm_dev(got) < 3e-7
    assert nflag <= max_flags(4 * V)
    assert bad <= 500 * nflag, (bad, nflag)
    assert abs(standalone - h[0, 0]) < 1e-6
    if bad == 0:
        assert abs(h[0, 0] - orc.plaquette(dims, U)) < 2e-6


def test_fused_reunitarisation_learned_sweep_matches_oracle(su2, orc):
    """The learned-proposal sweep (independence Metropolis with a random
    network's table) on a reunitarisation sweep with the fused
    reunitarisation, against the oracle's learned passes followed by its
    reunitarisation: links unit to FP32 rounding, within 1e-5 of the oracle's
    outside the cones of flagged Metropolis decisions."""
    from tests.gpu_util import learned_flagged
    announce("fused reunitarisation, learned proposal, vs oracle")
    dims, beta, seed, sw = [4, 6, 2, 8], 2.2, 41, 4
    params = (np.random.default_rng(16).standard_normal(orc.NN_NPARAM) * 0.2).astype(np.float32)
    table = orc.nn_table(params)
    links = inputs.random_links(dims, 151, spread=0.6)
    with su2.NN(params=params) as net, su2.Lattice(dims, beta, seed) as lat:
        net.build_table()
        lat.set_proposal(net)
        lat.set_reunit_fused(True)
        lat.set_links(links)
        lat.set_sweep(sw)
        h = lat.sweep_measure(1, su2.SU2_LEARNED, reunit_every=5, meas=PLAQ).cpu().numpy()
        got = lat.get_links()
        proposed, accepted = lat.accept_stats()
    U = links.astype(np.float64)
    nflag = 0
    for mu in range(4):
        for p in range(2):
            margin, _ = orc.learned_pass(dims, U, table, mu, p, sw, beta, seed)
            nflag += int(learned_flagged(margin).sum())
    orc.reunitarize(dims, U)
    d = np.abs(got - U).max(axis=2)
    bad = int((d > 1e-5).sum())
    announce(f"  max |gpu - oracle| {d.max():.2e}; off by > 1e-5: {bad}; flagged {nflag}; "
             f"accepted {int(np.sum(accepted))} of {int(np.sum(proposed))}; "
             f"max ||U|^2 - 1| {norm_dev(got):.2e}")
    assert int(np.sum(proposed)) > 0 and 0 < int(np.sum(accepted)) < int(np.sum(proposed))
    assert norm_dev(got) < 3e-7
    assert bad <= 500 * nflag, (bad, nflag)
    if bad == 0:
        assert abs(h[0, 0] - orc.plaquette(dims, U)) < 2e-6


def test_fused_and_separate_reunitarisation_differ_by_rounding(su2, orc):
    """The same reunitarisation sweep both ways from the same links: links
    within 2e-6 when the oracle takes no decision of the sweep within the
    flag margin (a flipped decision would move a cone of links), both unit to
    FP32 rounding, plaquettes within 1e-7; off the reunitarisation sweeps the
    two forms are the same kernels, bit for bit."""
    announce("fused vs separate reunitarisation")
    dims, beta, seed = [12, 12, 12, 12], 2.5, 31
    links = inputs.random_links(dims, 77, spread=0.5)
    U = links.astype(np.float64)
    nflag = oracle_sweep(orc, dims, U, 3, 0, beta, seed)
    with su2.Lattice(dims, beta, seed) as a, su2.Lattice(dims, beta, seed) as b:
        b.set_reunit_fused(True)
        for x in (a, b):
            x.set_links(links)
            x.set_sweep(3)
        ha = a.sweep_measure(1, reunit_every=4, meas=PLAQ).cpu().numpy()
        hb = b.sweep_measure(1, reunit_every=4, meas=PLAQ).cpu().numpy()
        la, lb = a.get_links(), b.get_links()
        diff = float(np.abs(la - lb).max())
        announce(f"  max |fused - separate| {diff:.2e}; |dP| {abs(ha[0, 0] - hb[0, 0]):.2e}; "
                 f"norms {norm_dev(la):.2e} / {norm_dev(lb):.2e}; flagged {nflag}")
        assert norm_dev(la) < 3e-7 and norm_dev(lb) < 3e-7
        if nflag == 0:
            assert diff < 2e-6
            assert abs(ha[0, 0] - hb[0, 0]) < 1e-7
        # sweeps 4..6 hold no reunitarisation: identical kernels on both
        for x in (a, b):
            x.set_links(lb)
        ha = a.sweep_measure(3, reunit_every=4, meas=PLAQ).cpu().numpy()
        hb = b.sweep_measure(3, reunit_every=4, meas=PLAQ).cpu().numpy()
        np.testing.assert_array_equal(a.get_links(), b.get_links())
        np.testing.assert_array_equal(ha, hb)


@pytest.mark.parametrize("n_or", [0, 2], ids=["kp", "kp-or2"])
def test_fused_capture_replay_equals_direct(su2, n_or):
    """Graph replays of captured fused-reunitarisation sweeps give the links and
    history rows of direct sweeps, bit for bit."""
    announce(f"fused reunitarisation capture/replay n_or={n_or}")
    import torch
    dims, beta, seed = [12, 10, 8, 6], 2.3, 8
    mode = su2.SU2_KP_OR if n_or else su2.SU2_KP
    side = torch.cuda.Stream()  # capture needs a non-null stream
    with torch.cuda.stream(side):
        with su2.Lattice(dims, beta, seed, su2.SU2_HOT) as a, \
                su2.Lattice(dims, beta, seed, su2.SU2_HOT) as g:
            for x in (a, g):
                x.set_reunit_fused(True)
                x.set_hb_overrelax(n_or)
            ha = a.sweep_measure(10, mode, reunit_every=5, meas=3).cpu().numpy()
            hg = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
            g.capture(5, mode, reunit_every=5, meas=3, hist=hg)
            g.replay(2)
            g.synchronize()
            np.testing.assert_array_equal(g.get_links(), a.get_links())
            np.testing.assert_array_equal(hg.cpu().numpy(), ha)
            assert norm_dev(a.get_links()) < 3e-7


def test_fused_batch_matches_single_lattices(su2):
    """Replica r of a batch with fused reunitarisation follows the single
    lattice run as replica r bit for bit (per-pass launches on both sides)."""
    announce("fused reunitarisation batch == single lattices")
    seed = 44
    with su2.Batch(DIMS, BETAS, STARTS, seed) as b0:
        inits = [b0.get_links(r) for r in range(len(DIMS))]
    with su2.Batch(DIMS, BETAS, STARTS, seed) as b:
        b.set_reunit_fused(True)
        h = b.sweep_measure(6, meas=3, reunit_every=2).cpu().numpy()
        bl = [b.get_links(r) for r in range(len(DIMS))]
    for r, (d, beta) in enumerate(zip(DIMS, BETAS)):
        with su2.Lattice(d, beta, seed, su2.SU2_COLD) as lat:
            lat.set_replica(r)
            lat.set_reunit_fused(True)
            lat.set_links(inits[r])
            hs = lat.sweep_measure(6, meas=3, reunit_every=2).cpu().numpy()
            np.testing.assert_array_equal(lat.get_links(), bl[r])
        np.testing.assert_allclose(h[:, r, 0], hs[:, 0], atol=1e-12, rtol=0)
        np.testing.assert_allclose(h[:, r, 1:], hs[:, 1:], atol=1e-6, rtol=0)
        assert norm_dev(bl[r]) < 3e-7


def test_fused_with_lds_staged_pass(su2):
    """With the LDS-staged pass configured, the reunitarising stage runs on the
    plain pass kernel and the others on the staged one: the same links as
    plain per-pass launches, bit for bit."""
    announce("fused reunitarisation with the LDS-staged pass")
    dims = [16, 16, 16, 16]
    with su2.Lattice(dims, 2.4, 5, su2.SU2_HOT) as plain, \
            su2.Lattice(dims, 2.4, 5, su2.SU2_HOT) as lat:
        plain.set_launch(256, 1 | 4, 8, 8, 0)
        lat.set_launch(256, 1 | 4 | 128, 8, 4, 0)
        for x in (plain, lat):
            x.set_reunit_fused(True)
        ha = plain.sweep_measure(4, reunit_every=2, meas=3).cpu().numpy()
        hb = lat.sweep_measure(4, reunit_every=2, meas=3).cpu().numpy()
        np.testing.assert_array_equal(plain.get_links(), lat.get_links())
        np.testing.assert_allclose(ha, hb, atol=1e-9, rtol=0)


def test_fused_reunitarisation_arguments(su2):
    """on must be 0 or 1; FP64 contexts refuse it; without reunitarisation
    sweeps the setting changes nothing."""
    dims = [8, 8, 8, 8]
    with su2.Lattice(dims, 2.2, 3, su2.SU2_HOT) as a, su2.Lattice(dims, 2.2, 3, su2.SU2_HOT) as b:
        for bad in (2, -1):
            with pytest.raises(su2.SU2Error) as e:
                a.set_reunit_fused(bad)
            assert e.value.code == su2.SU2_EINVAL
        with su2.Batch(DIMS[:2], BETAS[:2], STARTS[:2], 1) as bt:
            with pytest.raises(su2.SU2Error) as e:
                bt.set_reunit_fused(3)
            assert e.value.code == su2.SU2_EINVAL
        b.set_reunit_fused(True)
        ha = a.sweep_measure(3, meas=3).cpu().numpy()
        hb = b.sweep_measure(3, meas=3).cpu().numpy()
        np.testing.assert_array_equal(a.get_links(), b.get_links())
        np.testing.assert_array_equal(ha, hb)
    with su2.Lattice64(dims, 2.2, 3) as l64:
        l64.set_reunit_fused(False)
        with pytest.raises(su2.SU2Error) as e:
            l64.set_reunit_fused(True)
        assert e.value.code == su2.SU2_ESTATE
