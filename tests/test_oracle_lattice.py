"""Pins of the oracle's lattice code: indexing, init, staples, observables and
the checkerboard pass, against exact invariants of the model (Sec. 2, Sec. 4).
"""
import numpy as np
import pytest

from tests import inputs, stats

D4 = [4, 4, 4, 4]
DR = [4, 6, 2, 8]  # ragged, anisotropic


def test_dims_validation(orc):
    assert orc.check_dims([4, 4, 4, 4]) and orc.check_dims([2, 2, 2, 2])
    for bad in ([3, 4, 4, 4], [4, 4, 4, 5], [0, 4, 4, 4], [4, 4, 1, 4]):
        assert not orc.check_dims(bad)


@pytest.mark.parametrize("dims", [D4, DR])
def test_shift_and_parity(orc, dims):
    V = inputs.volume(dims)
    for s in range(0, V, 7):
        for mu in range(4):
            f = orc.shift(dims, s, mu, 1)
            assert orc.parity(dims, f) != orc.parity(dims, s)
            assert orc.shift(dims, f, mu, -1) == s
    # periodic wrap along t: (0,0,0,Nt-1) + t -> origin
    last = (dims[3] - 1) * dims[0] * dims[1] * dims[2]
    assert orc.shift(dims, last, 3, 1) == 0
    assert orc.shift(dims, 0, 0, -1) == dims[0] - 1


def test_cold_start_observables_exact(orc):
    U = orc.init(DR, 0, 1)
    assert orc.plaquette(DR, U) == 1.0
    assert orc.polyakov(DR, U) == (1.0, 1.0)
    np.testing.assert_array_equal(U[:, :, 0], 1.0)


def test_hot_start_is_haar(orc):
    dims = [8, 8, 8, 8]
    U = orc.init(dims, 1, 5)
    a = U.reshape(-1, 4)
    n = a.shape[0]
    np.testing.assert_allclose(np.linalg.norm(a, axis=1), 1.0, atol=1e-14)
    for c in range(4):
        assert abs(a[:, c].mean()) < 5 * 0.5 / np.sqrt(n)
        assert abs((a[:, c] ** 2).mean() - 0.25) < 5 * 0.22 / np.sqrt(n)
    # a0 density (2/pi) sqrt(1 - a0^2) is the alpha -> 0 limit of the a0 density
    chi2, dof, p = stats.chi2_equiprobable(a[:, 0], 1e-9, nbins=40)
    assert p > 1e-4


@pytest.mark.parametrize("dims", [D4, DR])
def test_staple_plaquette_identity(orc, dims):
    """sum_{s,mu} (1/2)Tr(U_mu(s) V(s,mu)) = 4 * 6V * P: every plaquette sits in
    the staples of its four links."""
    U = inputs.as_f64(inputs.random_links(dims, 3))
    V = inputs.volume(dims)
    assert np.isclose(orc.staple_action(dims, U), 24 * V * orc.plaquette(dims, U),
                      rtol=1e-12, atol=1e-11)


def test_staple_single_plaquette_by_hand(orc):
    """On a lattice where only U_1 at the origin differs from 1, the staple of
    U_0(origin) contains that link in exactly one forward term (nu = 1):
    U_1(s+0)=1, U_0(s+1)^+ = 1, U_1(s)^+ -> V = 5 + U_1(0)^+ (+ backward terms = 1)."""
    dims = [4, 4, 4, 4]
    U = orc.init(dims, 0, 0)
    q = np.array([0.6, 0.0, 0.8, 0.0])
    U[0, 1] = q
    V = orc.staple(dims, U, 0, 0)
    np.testing.assert_allclose(V, np.array([5.0, 0, 0, 0]) + q * [1, -1, -1, -1], atol=1e-15)
    # staple of U_1(origin) with mu=1 is unaffected by the link itself
    np.testing.assert_allclose(orc.staple(dims, U, 0, 1), [6, 0, 0, 0], atol=1e-15)
    # plaquette: one of 6V plaquettes is (1/2)Tr(q^+) = 0.6 ... it appears in planes (0,1),(1,2),(1,3)
    # at the origin and in the backward plaquettes (0,1) at s-0 etc.: 6 plaquettes contain U_1(0)
    P = orc.plaquette(dims, U)
    Vol = inputs.volume(dims)
    assert np.isclose(P, (6 * Vol - 6 + 6 * 0.6) / (6 * Vol), atol=1e-15)


@pytest.mark.parametrize("dims", [D4, DR])
def test_gauge_invariance(orc, dims):
    U = inputs.as_f64(inputs.random_links(dims, 4))
    P0, L0 = orc.plaquette(dims, U), orc.polyakov(dims, U)[0]
    U2 = U.copy()
    orc.gauge_transform(dims, U2, seed=99)
    assert np.abs(U2 - U).max() > 0.1
    assert abs(orc.plaquette(dims, U2) - P0) < 1e-13
    assert abs(orc.polyakov(dims, U2)[0] - L0) < 1e-13
    assert abs(orc.staple_action(dims, U2) - orc.staple_action(dims, U)) < 1e-10


def test_center_symmetry(orc):
    dims = DR
    U = inputs.as_f64(inputs.random_links(dims, 5))
    P0, (L0, A0) = orc.plaquette(dims, U), orc.polyakov(dims, U)
    U2 = U.copy()
    Ns3 = dims[0] * dims[1] * dims[2]
    U2[Ns3 * 1:Ns3 * 2, 3, :] *= -1  # U_3 on the time slice t = 1
    assert abs(orc.plaquette(dims, U2) - P0) < 1e-14
    L2, A2 = orc.polyakov(dims, U2)
    assert L2 == -L0 and A2 == A0


def test_polyakov_order_matters(orc):
    """Ordered product, t = 0 leftmost: with non-commuting links reversing the
    time order changes L(x) per site but the trace of a product of 2 is cyclic;
    use Nt = 4 and compare against a hand-built product."""
    dims = [2, 2, 2, 4]
    U = inputs.as_f64(inputs.random_links(dims, 6))
    Ns3 = 8
    want = 0.0
    for xs in range(Ns3):
        P = np.array([[1.0, 0, 0, 0]])
        for t in range(4):
            P = orc.qmul(P, U[xs + Ns3 * t, 3])
        want += P[0, 0]
    assert np.isclose(orc.polyakov(dims, U)[0], want / Ns3, atol=1e-15)


@pytest.mark.parametrize("dims", [D4, DR])
def test_pass_order_independence(orc, dims):
    """Within one (mu, parity) pass no link read is written, and the randoms are
    keyed by (site, sweep, mu): every visiting order gives identical links."""
    U0 = inputs.as_f64(inputs.random_links(dims, 7))
    outs = []
    for order in (0, 1, 2, 3):
        U = U0.copy()
        orc.do_pass(dims, U, mu=2, par=1, sweep=4, beta=2.2, seed=8, order=order, order_seed=3)
        outs.append(U)
    for U in outs[1:]:
        np.testing.assert_array_equal(U, outs[0])


def test_pass_touches_only_its_links(orc):
    dims = DR
    U0 = inputs.as_f64(inputs.random_links(dims, 8))
    U = U0.copy()
    orc.do_pass(dims, U, mu=1, par=0, sweep=0, beta=2.0, seed=1)
    V = inputs.volume(dims)
    par = np.array([orc.parity(dims, s) for s in range(V)])
    changed = np.any(U != U0, axis=2)
    assert not changed[:, [0, 2, 3]].any()
    assert not changed[par == 1, 1].any()
    assert changed[par == 0, 1].all()


def test_pass_equals_link_update_on_old_staples(orc):
    dims = D4
    U0 = inputs.as_f64(inputs.random_links(dims, 9))
    U = U0.copy()
    orc.do_pass(dims, U, mu=3, par=0, sweep=11, beta=2.5, seed=21)
    for s in range(0, inputs.volume(dims), 5):
        if orc.parity(dims, s) != 0:
            continue
        V = orc.staple(dims, U0, s, 3)
        want, _ = orc.heatbath_link(V, 2.5, 21, s, 11, 3)
        np.testing.assert_array_equal(U[s, 3], want)


def test_openmp_sweeps_bitidentical(orc):
    dims = DR
    U1 = orc.init(dims, 1, 3)
    U2 = U1.copy()
    p1, _ = orc.sweeps(dims, U1, 3, 0, 2.3, 3, nthreads=1, measure=True)
    p2, _ = orc.sweeps(dims, U2, 3, 0, 2.3, 3, nthreads=4, measure=True)
    np.testing.assert_array_equal(U1, U2)
    np.testing.assert_array_equal(p1, p2)


def test_resume_is_bitidentical(orc):
    dims = D4
    U1 = orc.init(dims, 1, 4)
    U2 = U1.copy()
    orc.sweeps(dims, U1, 6, 0, 2.1, 4, reunit_every=4)
    orc.sweeps(dims, U2, 3, 0, 2.1, 4, reunit_every=4)
    orc.sweeps(dims, U2, 3, 3, 2.1, 4, reunit_every=4)
    np.testing.assert_array_equal(U1, U2)


def test_unitarity_and_reunitarize(orc):
    dims = D4
    U = orc.init(dims, 1, 6)
    orc.sweeps(dims, U, 5, 0, 2.3, 6)
    n = np.linalg.norm(U, axis=2)
    assert np.abs(n - 1).max() < 1e-13
    U *= 1.01
    orc.reunitarize(dims, U)
    assert np.abs(np.linalg.norm(U, axis=2) - 1).max() < 1e-15


def test_hot_link_and_staple_without_the_lattice(orc):
    """The per-link hot start and the hot-start staple equal the full
    lattice's (used where the lattice is too large to hold on the host)."""
    dims = [4, 6, 2, 8]
    U = orc.init(dims, 1, 13, replica=2)
    rng = np.random.default_rng(1)
    for s in rng.integers(0, orc.volume(dims), 20):
        for mu in range(4):
            np.testing.assert_array_equal(orc.hot_link(s, mu, 13, 2), U[s, mu])
            np.testing.assert_allclose(orc.hot_staple(dims, s, mu, 13, 2),
                                       orc.staple(dims, U, s, mu), atol=1e-15, rtol=0)


def test_sweep_margins_are_the_pass_margins(orc):
    """orc.sweeps(want_margin=True) reports, per link, the smallest decision
    margin of the single-link heat bath over the sweeps' updates of it, the
    same numbers the passes report one at a time; reunitarisation and the
    measurements leave them alone."""
    dims = D4
    U1 = orc.init(dims, 1, 8)
    U2 = U1.copy()
    ph, lh, m = orc.sweeps(dims, U1, 2, 5, 2.2, 8, reunit_every=2, measure=True,
                           want_margin=True)
    want = np.full((orc.volume(dims), 4), np.inf)
    for sw in (5, 6):
        for mu in range(4):
            for p in range(2):
                pm = orc.do_pass(dims, U2, mu, p, sw, 2.2, 8, want_margin=True)
                want[:, mu] = np.minimum(want[:, mu], pm)
        if (sw + 1) % 2 == 0:
            orc.reunitarize(dims, U2)
    np.testing.assert_array_equal(U1, U2)
    np.testing.assert_array_equal(m, want)
    assert np.all(np.isfinite(m)) and np.all(m >= 0)
    # a margin is the distance of an accept test from its threshold: some
    # decisions of 2 x 4 x V updates land close to it, none below zero
    assert m.min() < 1e-2
    assert orc.sweeps(dims, U2.copy(), 1, 7, 2.2, 8, want_margin=True).shape == (orc.volume(dims), 4)
