"""Pins of the FP64 SU(3) oracle (Cabibbo-Marinari heat bath built on the SU(2)
heat bath of Sec. 2) against facts that do not come from the oracle itself:
Haar moments of SU(3), closed-form plaquettes and Polyakov loops of abelian
fields, the Weyl integration formula at strong coupling, lattice perturbation
theory at weak coupling, an independent Haar sampler (QR of complex Gaussian
matrices) reweighted to the single-link distribution, and QR for the
reunitarisation.  CPU only.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle import su2_oracle as o2
from oracle import su3_oracle as o3


def haar_su3(n, rng):
    """Haar SU(3) from the QR decomposition of complex Gaussian matrices
    (phases of R's diagonal moved into Q, then det divided out by a cube root;
    multiplying by a centre element keeps the measure)."""
    z = (rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))) / np.sqrt(2)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    return q * (np.linalg.det(q) ** (-1.0 / 3.0))[:, None, None]


def su3_defects(U):
    M = U.reshape(-1, 3, 3)
    unit = np.abs(M @ np.conj(np.swapaxes(M, 1, 2)) - np.eye(3)).max()
    det = np.abs(np.linalg.det(M) - 1.0).max()
    return unit, det


def tau_err(x):
    """Mean and error from 50 batch means."""
    x = np.asarray(x)
    b = x[: len(x) // 50 * 50].reshape(50, -1).mean(axis=1)
    return x.mean(), b.std(ddof=1) / np.sqrt(50)


def test_hot_start_is_haar_su3():
    """Haar SU(3): <Tr U> = 0, <|Tr U|^2> = 1, <(Tr U)^3> = 1 (the singlet in
    3 x 3 x 3; it is 0 for U(3), so this pins det U = 1)."""
    dims = [8, 8, 8, 8]
    U = o3.init(dims, 1, 2024)
    unit, det = su3_defects(U)
    assert unit < 1e-13 and det < 1e-13
    t = np.trace(U.reshape(-1, 3, 3), axis1=1, axis2=2)
    n = t.size
    assert abs(t.mean()) < 5 * np.sqrt(1.0 / n)
    assert abs(np.mean(np.abs(t) ** 2) - 1.0) < 5 * np.sqrt(1.0 / n)
    assert abs(np.mean(t ** 3) - 1.0) < 5 * np.sqrt(6.0 / n)
    cold = o3.init(dims, 0, 1)
    assert np.array_equal(cold.reshape(-1, 3, 3), np.broadcast_to(np.eye(3), (cold.size // 9, 3, 3)))


def test_abelian_fields_closed_form():
    """Diagonal (abelian) fields: U_0(x) = diag(e^{i th y}, e^{-i th y}, 1) with
    th = 2 pi k / Ny gives plaquettes diag(e^{-i th}, e^{i th}, 1) in the (0, 1)
    planes and 1 elsewhere, so <P> = (5 + (1 + 2 cos th)/3) / 6; a constant
    U_3 = diag(e^{i ph}, e^{i ph}, e^{-2 i ph}) gives Tr L / 3 =
    (2 e^{i Nt ph} + e^{-2 i Nt ph}) / 3 at every site."""
    dims = [4, 6, 4, 8]
    V = o2.volume(dims)
    U = o3.init(dims, 0, 0)
    th, ph = 2 * np.pi * 1 / dims[1], 0.37
    for s in range(V):
        y = (s // dims[0]) % dims[1]
        U[s, 0] = np.diag([np.exp(1j * th * y), np.exp(-1j * th * y), 1.0])
        U[s, 3] = np.diag([np.exp(1j * ph), np.exp(1j * ph), np.exp(-2j * ph)])
    assert o3.plaquette(dims, U) == pytest.approx((5 + (1 + 2 * np.cos(th)) / 3) / 6, abs=1e-14)
    re, im, mag = o3.polyakov(dims, U)
    L = (2 * np.exp(1j * dims[3] * ph) + np.exp(-2j * dims[3] * ph)) / 3
    assert re == pytest.approx(L.real, abs=1e-13) and im == pytest.approx(L.imag, abs=1e-13)
    assert mag == pytest.approx(abs(L), abs=1e-13)


def test_staples_count_every_plaquette_four_times_and_are_gauge_covariant():
    """sum_{s,mu} Re Tr(U_mu(s) A_mu(s)) = 4 * 3 * 6V <P>: each plaquette holds
    four links.  A wrong staple orientation or neighbour breaks it.  Plaquette,
    Polyakov loop and this sum are invariant under a random gauge transformation."""
    dims = [4, 4, 6, 4]
    V = o2.volume(dims)
    U = o3.init(dims, 1, 77)
    o3.sweeps(dims, U, 2, 0, 5.0, 77)  # away from Haar, where <P> = 0
    P = o3.plaquette(dims, U)
    assert P > 0.2
    S = o3.staple_action(dims, U)
    assert S == pytest.approx(4 * 3 * 6 * V * P, rel=1e-12)
    pl = o3.polyakov(dims, U)
    G = U.copy()
    o3.gauge_transform(dims, G, 99)
    assert np.abs(G - U).max() > 0.1
    assert o3.plaquette(dims, G) == pytest.approx(P, abs=1e-13)
    assert o3.staple_action(dims, G) == pytest.approx(S, abs=1e-10)
    assert np.allclose(o3.polyakov(dims, G), pl, atol=1e-13)


@pytest.mark.parametrize("scale,beta", [(1.5, 2.0), (2.5, 2.0)])
def test_single_link_chain_matches_haar_reweighting(scale, beta):
    """With a fixed staple A the link's stationary law is
    exp[(beta/3) Re Tr(U A)] dU.  Its moments from independent Haar matrices
    (QR of Gaussians) reweighted by that factor agree with the oracle's chain of
    Cabibbo-Marinari updates; beta -> 3 beta / 4 (the SU(2) normalisation), a
    wrong quaternion projection or a transposed subgroup matrix moves them by
    many standard errors."""
    rng = np.random.default_rng(5)
    A = scale * haar_su3(3, rng).sum(axis=0)
    H = haar_su3(1_000_000, np.random.default_rng(6))
    twa = np.einsum("nij,ji->n", H, A)
    tu = np.trace(H, axis1=1, axis2=2)
    lw = beta / 3.0 * twa.real
    w = np.exp(lw - lw.max())
    w /= w.sum()
    _, obs = o3.link_chain(A, beta, 300_000, 31 + int(10 * scale))
    obs = obs[1000:]
    for exact_vals, chain in ((twa.real, obs[:, 0].real), (twa.imag, obs[:, 0].imag),
                              (tu.real, obs[:, 1].real), (tu.imag, obs[:, 1].imag)):
        mu_w = np.sum(w * exact_vals)
        err_w = np.sqrt(np.sum(w ** 2 * (exact_vals - mu_w) ** 2))  # self-normalised IS error
        mu_c, err_c = tau_err(chain)
        assert abs(mu_w - mu_c) < 4.5 * np.hypot(err_w, err_c), (mu_w, err_w, mu_c, err_c)


def weyl_plaquette(beta):
    """u(beta) = <Re Tr U / 3> under exp[(beta/3) Re Tr U] dU by the Weyl
    integration formula (eigenphases t1, t2, -t1-t2; Haar density |Vandermonde|^2)."""

    def f(t1, t2, moment):
        z = np.exp(1j * np.array([t1, t2, -t1 - t2]))
        vd = abs((z[0] - z[1]) * (z[0] - z[2]) * (z[1] - z[2])) ** 2
        rt = z.sum().real
        return vd * np.exp(beta / 3.0 * rt) * (rt / 3.0 if moment else 1.0)

    num = integrate.dblquad(lambda a, b: f(a, b, 1), -np.pi, np.pi, -np.pi, np.pi,
                            epsabs=1e-12)[0]
    den = integrate.dblquad(lambda a, b: f(a, b, 0), -np.pi, np.pi, -np.pi, np.pi,
                            epsabs=1e-12)[0]
    return num / den


def test_weyl_formula_small_beta_expansion():
    """The quadrature itself: u = beta/18 + beta^2/216 + O(beta^3) (Haar:
    <(Re Tr U)^2> = 1/2, <(Re Tr U)^3> = 1/4)."""
    b = 0.1
    assert weyl_plaquette(b) == pytest.approx(b / 18 + b * b / 216, abs=2e-6)


def test_strong_coupling_plaquette_matches_weyl_integral():
    """At strong coupling the 4D plaquette equals the single-plaquette value
    u(beta) up to O(u^5) (the smallest closed surface is a cube):
    at beta = 1, u^5 ~ 1e-6, far below the statistical error."""
    dims, beta = [6, 6, 6, 6], 1.0
    U = o3.init(dims, 1, 11)
    ph, _ = o3.sweeps(dims, U, 220, 0, beta, 11, nthreads=8, history=True)
    m, e = tau_err(ph[20:])
    assert abs(m - weyl_plaquette(beta)) < 4 * e, (m, e)
    assert e < 4e-4


def test_weak_coupling_plaquette_matches_perturbation_theory():
    """Lattice perturbation theory: 1 - <P> = (N^2 - 1)/(8N) g^2 + O(g^4) with
    g^2 = 2N/beta, i.e. 2/beta for SU(3); the next order adds about +1.5% at
    beta = 40.  A heat bath with the SU(2) normalisation beta/2 would give
    8/(3 beta), 33% higher."""
    dims, beta = [4, 4, 4, 4], 40.0
    U = o3.init(dims, 0, 12)
    ph, _ = o3.sweeps(dims, U, 400, 0, beta, 12, reunit_every=10, nthreads=8, history=True)
    m, e = tau_err(1.0 - ph[50:])
    assert e < 2e-4
    assert abs(m / (2.0 / beta) - 1.0) < 0.03, m


def test_pass_updates_only_its_links_and_sites_are_independent():
    """A pass changes exactly the links of its direction and parity; the order
    of its sites does not matter (serial and 8-thread passes agree bit for
    bit); every updated link stays in SU(3)."""
    dims = [4, 6, 4, 4]
    V = o2.volume(dims)
    U0 = o3.init(dims, 1, 5)
    par = np.array([o2.parity(dims, s) for s in range(V)])
    for mu, p in ((0, 0), (2, 1), (3, 1)):
        a, b = U0.copy(), U0.copy()
        o3.pass_(dims, a, mu, p, 3, 5.5, 5, nthreads=1)
        o3.pass_(dims, b, mu, p, 3, 5.5, 5, nthreads=8)
        assert np.array_equal(a, b)
        changed = np.abs(a - U0).reshape(V, 4, -1).max(axis=2) > 0
        expect = np.zeros((V, 4), dtype=bool)
        expect[par == p, mu] = True
        assert np.array_equal(changed, expect)
        unit, det = su3_defects(a)
        assert unit < 1e-13 and det < 1e-13


def test_reunitarize_is_gram_schmidt():
    """Rows 0, 1 of the result are the Q factor of the QR decomposition of the
    first two rows (transposed), with a positive diagonal of R; row 2 is the
    conjugate cross product, so the result is in SU(3)."""
    dims = [2, 2, 2, 2]
    U = o3.init(dims, 1, 8)
    rng = np.random.default_rng(3)
    U += 1e-3 * (rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape))
    R = U.copy()
    o3.reunitarize(dims, R)
    for M, out in zip(U.reshape(-1, 3, 3), R.reshape(-1, 3, 3)):
        q, r = np.linalg.qr(M[:2].T)
        q = q * (np.diag(r) / np.abs(np.diag(r)))[None, :]
        assert np.allclose(out[:2], q.T, atol=1e-14)
        assert np.allclose(out[2], np.conj(np.cross(out[0], out[1])), atol=1e-14)
    unit, det = su3_defects(R)
    assert unit < 1e-14 and det < 1e-14
    again = R.copy()
    o3.reunitarize(dims, again)
    assert np.abs(again - R).max() < 1e-15


def test_overrelaxation_keeps_the_action_and_moves_the_link():
    """Microcanonical over-relaxation: each subgroup step r = (v^+)^2 leaves
    Re Tr(U A) unchanged (checked here with numpy), keeps U in SU(3) and moves
    it by O(1); over a whole lattice an over-relaxation pass leaves the total
    action (the staple sum) unchanged."""
    rng = np.random.default_rng(21)
    for trial in range(20):
        U = haar_su3(1, rng)[0]
        A = (1.0 + trial / 10) * haar_su3(6, rng).sum(axis=0)
        Up = o3.overrelax_link(U, A)
        assert abs(np.trace(Up @ A).real - np.trace(U @ A).real) < 1e-12
        assert np.abs(Up @ Up.conj().T - np.eye(3)).max() < 1e-13
        assert abs(np.linalg.det(Up) - 1.0) < 1e-13
        assert np.abs(Up - U).max() > 0.05
    dims = [4, 4, 6, 4]
    L = o3.init(dims, 1, 5)
    o3.sweeps(dims, L, 2, 0, 5.5, 5)
    S0, P0 = o3.staple_action(dims, L), o3.plaquette(dims, L)
    before = L.copy()
    for mu in range(4):
        for p in range(2):
            o3.or_pass(dims, L, mu, p)
    assert o3.staple_action(dims, L) == pytest.approx(S0, abs=1e-9)
    assert o3.plaquette(dims, L) == pytest.approx(P0, abs=1e-13)
    assert np.abs(L - before).max() > 0.1


def test_overrelaxed_chain_keeps_the_plaquette_distribution():
    """Over-relaxation steps preserve the Boltzmann weight and the Haar measure,
    so chains of one heat-bath and three over-relaxation sweeps sample the same
    plaquette distribution as pure heat bath (4^4 at beta = 5.7, 6 + 6 chains)."""
    dims, beta = [4, 4, 4, 4], 5.7
    hb, orl = [], []
    for r in range(6):
        U = o3.init(dims, 0, 0)
        ph, _ = o3.sweeps(dims, U, 400, 0, beta, 40 + r, reunit_every=10, nthreads=8, history=True)
        hb.append(ph[50:].mean())
        U = o3.init(dims, 0, 0)
        ph, _ = o3.sweeps_or(dims, U, 400, 3, 0, beta, 60 + r, reunit_every=10, nthreads=8,
                             history=True)
        orl.append(ph[50:].mean())
    hb, orl = np.array(hb), np.array(orl)
    err = np.hypot(hb.std(ddof=1), orl.std(ddof=1)) / np.sqrt(6)
    assert abs(hb.mean() - orl.mean()) < 4 * err, (hb.mean(), orl.mean(), err)


def test_hot_link_and_staple_without_the_lattice():
    """The per-link hot start and the hot-start staple equal the full lattice's."""
    dims = [4, 2, 6, 4]
    U = o3.init(dims, 1, 17, replica=1)
    rng = np.random.default_rng(2)
    for s in rng.integers(0, o2.volume(dims), 15):
        for mu in range(4):
            np.testing.assert_array_equal(o3.hot_link(s, mu, 17, 1), U[s, mu])
            np.testing.assert_allclose(o3.hot_staple(dims, s, mu, 17, 1), o3.staple(dims, U, s, mu),
                                       atol=1e-14, rtol=0)
