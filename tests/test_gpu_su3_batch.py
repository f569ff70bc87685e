"""SU(3) batches (su3_batch_*): n replicas of one lattice size, every pass one
launch for all of them.  Replica r uses coupling betas[r] and Philox replica id
r, so it must follow a single lattice with su3_set_replica(r) bit for bit
(links, plaquette history, observables), and its hot start and sweeps must
match the FP64 oracle's for replica r."""
import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

TOL3 = 1e-5


@pytest.fixture(scope="module")
def o3():
    from oracle import su3_oracle
    su3_oracle._load()
    return su3_oracle


def test_su3_batch_hot_starts_match_oracle(su2, o3):
    dims, seed = [4, 4, 4, 6], 9
    announce(f"su3 batch hot starts dims={dims}")
    with su2.Batch3(dims, [5.7, 6.0, 6.3], seed, su2.SU2_HOT) as b:
        assert b.n == 3
        for r in range(3):
            want = o3.init(dims, 1, seed, replica=r)
            assert np.abs(b.get_links(r) - want).max() < 2e-5, r
        p = b.plaquette()
        for r in range(3):
            assert p[r] == pytest.approx(o3.plaquette(dims, o3.init(dims, 1, seed, replica=r)),
                                         abs=2e-6)


@pytest.mark.parametrize("dims", [[6, 4, 4, 8], [8, 8, 8, 4]], ids=lambda d: "x".join(map(str, d)))
def test_su3_batch_replicas_match_single_lattices(su2, dims):
    """Four sweeps (reunitarisation every 2) with the plaquette history, one
    over-relaxation sweep, then the standalone plaquette and Polyakov loop:
    replica r of the batch against a single lattice with replica id r and the
    batch's starting links, bit for bit."""
    announce(f"su3 batch == single lattices dims={dims}")
    betas, seed = [5.5, 5.9, 6.3, 0.0], 17
    with su2.Batch3(dims, betas, seed, su2.SU2_HOT) as b:
        inits = [b.get_links(r) for r in range(len(betas))]
        h = b.heatbath_sweep(4, reunit_every=2, history=True)
        b.overrelax(1)
        links = [b.get_links(r) for r in range(len(betas))]
        plaq, poly = b.plaquette(), b.polyakov()
        assert b.sweep == 4
    assert h.shape == (4, len(betas))
    for r, beta in enumerate(betas):
        with su2.Lattice3(dims, beta, seed, su2.SU2_COLD) as lat:
            lat.set_replica(r)
            lat.set_links(inits[r])
            hs = lat.heatbath_sweep(4, reunit_every=2, history=True)
            lat.overrelax(1)
            np.testing.assert_array_equal(lat.get_links(), links[r])
            np.testing.assert_array_equal(hs, h[:, r])
            assert lat.plaquette() == plaq[r]
            assert lat.polyakov() == tuple(poly[r])
    # the replicas differ (own couplings and randoms)
    assert len({float(x) for x in h[-1]}) == len(betas)


def test_su3_batch_sweep_matches_oracle_for_its_replica(su2, o3):
    """One sweep of every replica from seeded links given to both sides:
    replica r against the oracle's sweep with replica id r and coupling
    betas[r] (links within 1e-5 but for the cones of decisions taken near
    their thresholds, as for a single lattice; plaquettes within 2e-6)."""
    dims, seed = [6, 4, 6, 8], 31
    betas = [5.9, 6.2]
    announce(f"su3 batch sweep vs oracle dims={dims}")
    starts = [inputs.random_su3_links(dims, 140 + r, spread=0.5) for r in range(len(betas))]
    with su2.Batch3(dims, betas, seed) as b:
        for r in range(len(betas)):
            b.set_links(r, starts[r])
        b.set_sweep(3)
        h = b.heatbath_sweep(1, history=True)
        got = [b.get_links(r) for r in range(len(betas))]
    for r, beta in enumerate(betas):
        U = starts[r].copy()
        ph, _ = o3.sweeps(dims, U, 1, 3, beta, seed, replica=r, history=True)
        diff = np.abs(got[r] - U).reshape(-1, 9).max(axis=1)
        announce(f"  replica {r}: max |gpu - oracle| {diff.max():.2e}, "
                 f"fraction > {TOL3}: {np.mean(diff > TOL3):.4f}")
        assert np.mean(diff > TOL3) < 0.02
        assert abs(h[0, r] - ph[0]) < 2e-6


def test_su3_batch_history_longer_than_one_chunk(su2):
    """A history of 1100 sweeps crosses the device history chunk (1024 rows per
    replica); the rows of every replica must still be those of its single
    lattice, in order."""
    dims, betas, seed = [4, 4, 4, 4], [5.8, 6.4], 23
    announce("su3 batch history across the device chunk")
    with su2.Batch3(dims, betas, seed, su2.SU2_HOT) as b:
        inits = [b.get_links(r) for r in range(2)]
        h = b.heatbath_sweep(1100, reunit_every=10, history=True)
    assert h.shape == (1100, 2)
    for r, beta in enumerate(betas):
        with su2.Lattice3(dims, beta, seed) as lat:
            lat.set_replica(r)
            lat.set_links(inits[r])
            np.testing.assert_array_equal(lat.heatbath_sweep(1100, reunit_every=10, history=True),
                                          h[:, r])


def test_su3_batch_arguments(su2):
    with su2.Batch3([4, 4, 4, 4], [5.7, 6.0], 1) as b:
        for r in (-1, 2):
            with pytest.raises(su2.SU2Error) as e:
                b.get_links(r)
            assert e.value.code == su2.SU2_EINVAL
            with pytest.raises(su2.SU2Error) as e:
                b.set_links(r, np.zeros((256, 4, 3, 3), np.complex128))
            assert e.value.code == su2.SU2_EINVAL
        with pytest.raises(su2.SU2Error) as e:
            b.heatbath_sweep(-1)
        assert e.value.code == su2.SU2_EINVAL
        # a cold batch: every replica's plaquette and Polyakov loop are 1
        assert list(b.plaquette()) == [1.0, 1.0]
        assert b.polyakov().tolist() == [[1.0, 0.0, 1.0], [1.0, 0.0, 1.0]]
    with su2.Lattice3([4, 4, 4, 4], 6.0, 1) as lat:
        with pytest.raises(su2.SU2Error) as e:
            lat.set_replica(1 << 26)
        assert e.value.code == su2.SU2_EINVAL
