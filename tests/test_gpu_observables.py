"""GPU observables and auxiliary kernels vs the oracle on identical links."""
import numpy as np
import pytest

from tests import inputs, stats
from tests.gpu_util import announce, parities

pytestmark = pytest.mark.gpu


# (x, y)-plane half-sites 2, 12, 24 and 128, then 192 (workgroups of 192), 170
# (256 with a ragged last tile) and 512 (two full tiles of 256); Nt 2 to 10
@pytest.mark.parametrize("dims", [[2, 2, 2, 2], [4, 6, 2, 8], [8, 6, 8, 10], [16, 16, 16, 16],
                                  [24, 16, 4, 6], [34, 10, 6, 4], [32, 32, 4, 2]],
                         ids=lambda d: "x".join(map(str, d)))
def test_plaquette_polyakov_on_identical_links(su2, orc, dims):
    announce(f"observables dims={dims}")
    links = inputs.random_links(dims, 5, spread=0.5)
    U = links.astype(np.float64)
    with su2.Lattice(dims, 2.0, 1) as lat:
        assert lat.plaquette() == 1.0 and lat.polyakov() == (1.0, 1.0)  # cold start
        lat.set_links(links)
        assert abs(lat.plaquette() - orc.plaquette(dims, U)) < 1e-6
        ls, la = lat.polyakov()
        ws, wa = orc.polyakov(dims, U)
        assert abs(ls - ws) < 1e-6 and abs(la - wa) < 1e-6


def test_gauge_and_center_invariance_on_gpu(su2, orc):
    announce("gauge/centre invariance")
    dims = [6, 4, 8, 4]
    links = inputs.random_links(dims, 8)
    with su2.Lattice(dims, 2.0, 1) as lat:
        lat.set_links(links)
        P0, (L0, _) = lat.plaquette(), lat.polyakov()
        lat.test_gauge_transform(seed=4)
        g = lat.get_links()
        want = links.astype(np.float64)
        orc.gauge_transform(dims, want, 4)
        assert np.abs(g - want).max() < 1e-5
        assert abs(lat.plaquette() - P0) < 2e-6
        assert abs(lat.polyakov()[0] - L0) < 2e-6
        flipped = links.copy()
        ns3 = dims[0] * dims[1] * dims[2]
        flipped[ns3:2 * ns3, 3] *= -1
        lat.set_links(flipped)
        assert abs(lat.plaquette() - P0) < 1e-7
        assert abs(lat.polyakov()[0] + L0) < 1e-7


def test_reunitarize(su2, orc):
    announce("reunitarize")
    dims = [4, 4, 6, 4]
    links = inputs.random_links(dims, 9) * np.float32(1.003)
    with su2.Lattice(dims, 2.0, 1) as lat:
        lat.set_links(links)
        lat.reunitarize()
        g = lat.get_links()
    want = links.astype(np.float64)
    orc.reunitarize(dims, want)
    assert np.abs(g - want).max() < 1e-7
    assert np.abs(np.linalg.norm(g.astype(np.float64), axis=2) - 1).max() < 2e-7


def test_fused_plaquette_equals_standalone_and_reunit_schedule(su2, orc):
    announce("fused plaquette + reunit schedule")
    dims = [8, 8, 8, 8]
    with su2.Lattice(dims, 2.3, 7, su2.SU2_HOT) as lat:
        for i in range(6):
            h = lat.sweep_measure(1, reunit_every=4).cpu().numpy()
            assert abs(h[0, 0] - lat.plaquette()) < 1e-6
        # reunitarised after sweep index 3 (the 4th sweep): unit to FP32 precision
        assert lat.sweep == 6
    with su2.Lattice(dims, 2.3, 7, su2.SU2_HOT) as a, su2.Lattice(dims, 2.3, 7, su2.SU2_HOT) as b:
        a.sweep_measure(8, reunit_every=4)
        b.heatbath_sweep(4)
        b.reunitarize()
        b.heatbath_sweep(4)
        b.reunitarize()
        np.testing.assert_array_equal(a.get_links(), b.get_links())


def test_first_pass_from_cold_in_situ_chi2(su2, orc):
    """From cold, V = 6 at every site: each link of pass (0, even) is X with
    a0 ~ sqrt(1-a0^2) exp(6 beta a0) (Sec. 2); chi-square against the exact CDF."""
    announce("in-situ chi2 first pass")
    dims = [16, 16, 16, 16]
    beta = 0.8
    with su2.Lattice(dims, beta, 99) as lat:
        lat.test_pass(0, 0)
        g = lat.get_links()
    par = (np.indices(dims[::-1]).sum(axis=0).ravel() & 1)
    a0 = g[par == 0, 0, 0].astype(np.float64)
    chi2, dof, p = stats.chi2_equiprobable(a0, 6 * beta, nbins=60)
    assert p > 1e-4, (chi2, dof)


@pytest.mark.parametrize("alpha", [0.05, 0.5, 0.999, 1.0, 3.0, 12.0, 30.0])
def test_gpu_sampler_chi2(su2, alpha):
    announce(f"sampler chi2 alpha={alpha}")
    n = 200_000
    V = np.zeros((n, 4), np.float32)
    V[:, 0] = 1.0
    out = su2.su2_test_heatbath_links(V, alpha, 31, 0, 1)
    a0 = out[:, 0].astype(np.float64)  # U~ = 1 so U' = X
    chi2, dof, p = stats.chi2_equiprobable(a0, alpha, nbins=80)
    assert p > 1e-4, (chi2, dof)
    m1, m2 = stats.bessel_moments(alpha)
    assert abs(a0.mean() - m1) < 5 * a0.std() / np.sqrt(n)
    assert abs((a0 ** 2).mean() - m2) < 5 * (a0 ** 2).std() / np.sqrt(n)


def test_resume_and_determinism(su2):
    announce("resume / run-twice determinism")
    dims = [8, 4, 6, 8]
    with su2.Lattice(dims, 2.2, 5, su2.SU2_HOT) as a:
        a.heatbath_sweep(6)
        full = a.get_links()
    with su2.Lattice(dims, 2.2, 5, su2.SU2_HOT) as b:
        b.heatbath_sweep(3)
        mid, sw = b.get_links(), b.sweep
    with su2.Lattice(dims, 2.2, 5, su2.SU2_COLD) as c:
        c.set_links(mid)
        c.set_sweep(sw)
        c.heatbath_sweep(3)
        np.testing.assert_array_equal(c.get_links(), full)
    with su2.Lattice(dims, 2.2, 5, su2.SU2_HOT) as d:
        d.heatbath_sweep(6)
        np.testing.assert_array_equal(d.get_links(), full)
    # measured histories (fixed-point global sums) are bit-reproducible
    hs = []
    for _ in range(2):
        with su2.Lattice(dims, 2.2, 5, su2.SU2_HOT) as e:
            hs.append(e.sweep_measure(5, reunit_every=2, meas=3).cpu().numpy())
    np.testing.assert_array_equal(hs[0], hs[1])


def test_set_beta_applies_to_later_sweeps(su2):
    """Sweeps after su2_set_beta equal those of a lattice created at the new
    coupling from the same links and sweep index, bit for bit."""
    announce("set_beta")
    dims = [6, 4, 4, 8]
    with su2.Lattice(dims, 1.7, 9, su2.SU2_HOT) as a:
        a.heatbath_sweep(2)
        mid = a.get_links()
        a.set_beta(2.6)
        a.heatbath_sweep(3)
        got = a.get_links()
    with su2.Lattice(dims, 2.6, 9, su2.SU2_COLD) as b:
        b.set_links(mid)
        b.set_sweep(2)
        b.heatbath_sweep(3)
        np.testing.assert_array_equal(b.get_links(), got)


def test_replica_changes_stream(su2):
    dims = [4, 4, 4, 4]
    with su2.Lattice(dims, 2.2, 5, su2.SU2_HOT) as a, su2.Lattice(dims, 2.2, 5, su2.SU2_HOT) as b:
        b.set_replica(3)
        a.heatbath_sweep(1)
        b.heatbath_sweep(1)
        assert np.mean(a.get_links() != b.get_links()) > 0.4


def test_zero_sweeps_and_errors(su2):
    with su2.Lattice([4, 4, 4, 4], 2.0, 1) as lat:
        lat.heatbath_sweep(0)
        assert lat.sweep == 0
        with pytest.raises(su2.SU2Error) as e:
            lat.heatbath_sweep(-1)
        assert e.value.code == su2.SU2_EINVAL
        with pytest.raises(su2.SU2Error) as e:
            lat.heatbath_sweep(1, su2.SU2_LEARNED)
        assert e.value.code == su2.SU2_ESTATE


def test_batch_plaquettes_with_different_planes(su2, orc):
    """The standalone plaquette of a batch whose replicas have different (x, y)
    planes (one workgroup size for all, ragged tiles) and Nt (t-chunks of a
    common divisor), against the oracle per replica."""
    dims = [[6, 4, 8, 2], [10, 8, 6, 4], [32, 32, 4, 4], [2, 2, 2, 2], [24, 16, 2, 6]]
    announce(f"batch plaquettes dims={dims}")
    with su2.Batch(dims, [2.0] * len(dims), [0] * len(dims), 3) as b:
        want = []
        for r, d in enumerate(dims):
            links = inputs.random_links(d, 10 + r, spread=0.5)
            b.set_links(r, links)
            want.append(orc.plaquette(d, links.astype(np.float64)))
        p, _, _ = b.observables()
        np.testing.assert_allclose(p, want, atol=1e-6, rtol=0)
