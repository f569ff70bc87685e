"""Pins of the oracle's microcanonical over-relaxation (the baseline the
learned proposal is compared with; not in the paper): the link map keeps
(1/2)Tr(U V), hence the heat-bath weight of Sec. 2, stays in SU(2), is its own
inverse and keeps the Haar measure (checked with 2x2 complex matrices and
samples, independently of the oracle's quaternion code); a pass keeps the
plaquette sum exactly, because no plaquette holds two links of one pass; and
heat bath plus over-relaxation sweeps reproduce the strong-coupling
plaquette."""
import numpy as np
import pytest
from scipy import stats as sst

from tests import inputs, stats

SIG = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]),
       np.array([[1, 0], [0, -1]], complex)]


def mat(q):
    """U = a0 + i a.sigma as a 2x2 complex matrix."""
    q = np.asarray(q, dtype=np.float64)
    return q[0] * np.eye(2) + 1j * sum(q[k + 1] * SIG[k] for k in range(3))


def test_link_map_properties(orc):
    rng = np.random.default_rng(3)
    V = inputs.random_staples(200, 4, kmin=0.05, kmax=6.0).astype(np.float64)
    U = inputs.random_links([200, 1, 1, 1], 5)[:, 0].astype(np.float64)
    U /= np.linalg.norm(U, axis=1, keepdims=True)  # unit in FP64
    moved = 0
    for v, u in zip(V, U):
        w = orc.overrelax_link(v, u)
        Mw, Mu, Mv = mat(w), mat(u), mat(v)
        # the weight's argument (1/2) Re Tr(U V) is kept
        assert np.trace(Mw @ Mv).real == pytest.approx(np.trace(Mu @ Mv).real, abs=1e-12)
        # SU(2): unitary with unit determinant
        assert np.abs(Mw @ Mw.conj().T - np.eye(2)).max() < 1e-12
        assert np.linalg.det(Mw) == pytest.approx(1.0, abs=1e-12)
        # an involution
        np.testing.assert_allclose(orc.overrelax_link(v, w), u, atol=1e-12, rtol=0)
        moved += np.abs(w - u).max() > 1e-3
    assert moved > 190  # it moves the link (the identity would pass the checks above)
    # V = 0 leaves the link alone
    np.testing.assert_array_equal(orc.overrelax_link(np.zeros(4), U[0]), U[0])


def test_link_map_keeps_haar_measure(orc):
    """For a fixed staple, Haar-distributed links stay Haar-distributed: every
    component of U' has the semicircle law of a Haar SU(2) element."""
    v = np.array([0.3, -1.2, 0.5, 2.0])
    U = inputs.random_links([20000, 1, 1, 1], 9)[:, 0].astype(np.float64)
    W = np.array([orc.overrelax_link(v, u) for u in U])
    semicircle_cdf = lambda x: 0.5 + (x * np.sqrt(1 - x * x) + np.arcsin(x)) / np.pi
    for c in range(4):
        assert sst.kstest(W[:, c], semicircle_cdf).pvalue > 1e-3, c


def test_pass_keeps_the_plaquette_and_is_an_involution(orc):
    dims = [4, 6, 2, 8]
    U0 = inputs.as_f64(inputs.random_links(dims, 12))
    p0 = orc.plaquette(dims, U0)
    for mu in range(4):
        for par in range(2):
            U = U0.copy()
            orc.or_pass(dims, U, mu, par)
            assert orc.plaquette(dims, U) == pytest.approx(p0, abs=1e-13)
            changed = np.abs(U - U0).max(axis=2) > 1e-9
            parity = np.array([orc.parity(dims, s) for s in range(U.shape[0])])
            assert np.all(changed[:, mu] == (parity == par))
            assert not changed[:, [m for m in range(4) if m != mu]].any()
            orc.or_pass(dims, U, mu, par)
            np.testing.assert_allclose(U, U0, atol=1e-13, rtol=0)


def test_compound_sweeps(orc):
    """The compound sweep is the heat-bath sweep followed by n_or
    over-relaxation sweeps, then the reunitarisation schedule; n_or = 0 is the
    plain heat bath."""
    dims = [4, 4, 4, 4]
    U1 = orc.init(dims, 1, 4)
    U2 = U1.copy()
    U3 = U1.copy()
    ph, _ = orc.sweeps_or(dims, U1, 3, 2, 5, 2.2, 4, reunit_every=2, measure=True)
    for j in (5, 6, 7):
        orc.sweeps(dims, U2, 1, j, 2.2, 4)
        for _ in range(2):
            for mu in range(4):
                for p in range(2):
                    orc.or_pass(dims, U2, mu, p)
        if (j + 1) % 2 == 0:
            orc.reunitarize(dims, U2)
    np.testing.assert_array_equal(U1, U2)
    assert ph[-1] == orc.plaquette(dims, U1)
    orc.sweeps_or(dims, U3, 2, 0, 0, 2.2, 4)
    U4 = orc.init(dims, 1, 4)
    orc.sweeps(dims, U4, 2, 0, 2.2, 4)
    np.testing.assert_array_equal(U3, U4)


@pytest.mark.parametrize("beta", [0.25, 0.5])
def test_strong_coupling_plaquette_with_overrelaxation(orc, beta):
    row = [r for r in stats.golden("sampler_moments.json")["strong_coupling"]
           if r["beta"] == beta][0]
    u = row["u"]
    dims = [8, 8, 8, 8]
    U = orc.init(dims, 1, 41)
    orc.sweeps_or(dims, U, 10, 1, 0, beta, 41, nthreads=4)
    ph, _ = orc.sweeps_or(dims, U, 100, 1, 10, beta, 41, nthreads=4, measure=True)
    m, e = stats.mean_err(ph)
    assert abs(m - u) < 3 * e + 5 * u ** 5, (m, e, u)
    assert e < u / 20
