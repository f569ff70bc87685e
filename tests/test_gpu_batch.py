"""Batched replicas, hipGraph replay, persistent grids and the autotuner.

A batch launches every kernel over all replicas at once; replica r uses
Philox replica id r, so it must follow bit for bit the chain of a single
lattice with the same extents, beta and seed and replica id r.  Launch
configuration (block size, order, tiles, persistent grid) and graph replay
must not change any link."""
import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

DIMS = [[4, 4, 4, 4], [6, 4, 8, 2], [8, 8, 8, 8], [4, 6, 2, 8], [10, 8, 6, 4], [2, 2, 2, 2]]
BETAS = [2.3, 1.9, 2.6, 0.7, 3.0, 2.1]
STARTS = [1, 0, 1, 1, 0, 1]


def test_batch_replicas_match_single_lattices(su2):
    announce("batch == single lattices")
    seed = 41
    with su2.Batch(DIMS, BETAS, STARTS, seed) as b:
        h = b.sweep_measure(5, meas=3, reunit_every=2).cpu().numpy()
        bl = [b.get_links(r) for r in range(len(DIMS))]
    # the hot start is keyed by the replica id: start the single lattice from
    # the batch's initial links of replica r, then run it as replica r
    with su2.Batch(DIMS, BETAS, STARTS, seed) as b0:
        inits = [b0.get_links(r) for r in range(len(DIMS))]
    for r, (d, beta, st) in enumerate(zip(DIMS, BETAS, STARTS)):
        init = inits[r]
        with su2.Lattice(d, beta, seed, su2.SU2_COLD) as lat:
            lat.set_replica(r)
            lat.set_links(init)
            hs = lat.sweep_measure(5, meas=3, reunit_every=2).cpu().numpy()
            np.testing.assert_array_equal(lat.get_links(), bl[r])
        # plaquettes are summed in fixed point per site (whole-sweep kernel)
        # or per workgroup of the same partition: identical; the Polyakov
        # product order may differ between a batch and a lone lattice
        np.testing.assert_array_equal(h[:, r, 0], hs[:, 0])
        np.testing.assert_allclose(h[:, r, 1:], hs[:, 1:], atol=1e-6, rtol=0)


def test_graph_replay_equals_direct(su2):
    announce("graph replay == direct")
    import torch
    seed = 42
    side = torch.cuda.Stream()  # capture needs a non-null stream
    with torch.cuda.stream(side):
        with su2.Batch(DIMS, BETAS, STARTS, seed) as a, su2.Batch(DIMS, BETAS, STARTS, seed) as g:
            ha = a.sweep_measure(12, meas=3, reunit_every=4).cpu().numpy()
            hg = torch.zeros((16, len(DIMS), 3), dtype=torch.float64, device="cuda")
            g.capture(4, meas=3, reunit_every=4, hist=hg)
            g.replay(3)
            g.synchronize()
            np.testing.assert_array_equal(hg[:12].cpu().numpy(), ha)
            for r in range(len(DIMS)):
                np.testing.assert_array_equal(g.get_links(r), a.get_links(r))
            # off the reunitarisation period the recorded schedule would drift
            g.sweep(1)
            with pytest.raises(su2.SU2Error) as e:
                g.replay(1)
            assert e.value.code == su2.SU2_ESTATE
            g.sweep(3)
            g.replay(1)  # the fourth replay since the capture: rows 12..15
            g.synchronize()
            assert np.all(hg[12:, :, 0].cpu().numpy() != 0)
            # a fifth replay would write past the 16 rows: refused, nothing enqueued
            g.sweep(4)
            with pytest.raises(su2.SU2Error) as e:
                g.replay(1)
            assert e.value.code == su2.SU2_EINVAL
        with su2.Lattice([8, 8, 8, 8], 2.2, 3, su2.SU2_HOT) as x, \
                su2.Lattice([8, 8, 8, 8], 2.2, 3, su2.SU2_HOT) as y:
            x.heatbath_sweep(6)
            y.capture(2)
            y.replay(3)
            assert y.sweep == 6
            np.testing.assert_array_equal(x.get_links(), y.get_links())
        # every replay against the eager sweeps, with eager work and a
        # synchronisation between the replays
        with su2.Lattice([8, 6, 8, 4], 2.5, 4, su2.SU2_HOT) as x, \
                su2.Lattice([8, 6, 8, 4], 2.5, 4, su2.SU2_HOT) as y:
            hx = x.sweep_measure(9, reunit_every=3, meas=3).cpu().numpy()
            hy = torch.zeros((9, 3), dtype=torch.float64, device="cuda")
            y.capture(3, reunit_every=3, meas=3, hist=hy)
            for k in range(3):
                y.replay(1)
                y.synchronize()
                np.testing.assert_array_equal(hy[3 * k:3 * k + 3].cpu().numpy(),
                                              hx[3 * k:3 * k + 3])
                _ = y.plaquette(), y.polyakov()
            np.testing.assert_array_equal(x.get_links(), y.get_links())
    torch.cuda.synchronize()


@pytest.mark.parametrize("cfg", [(256, 1, 8, 8, 0), (128, 3, 1, 1, 0), (64, 0, 2, 16, 0),
                                 (256, 1, 4, 4, 64), (192, 1, 16, 2, 8), (256, 5, 8, 8, 0),
                                 (128, 7, 2, 4, 16), (256, 68, 8, 8, 0), (128, 70, 1, 1, 0),
                                 (64, 68, 4, 4, 16)], ids=str)
def test_launch_configuration_does_not_change_links(su2, cfg):
    announce(f"launch config {cfg}")
    dims = [8, 6, 8, 16]
    with su2.Lattice(dims, 2.4, 5, su2.SU2_HOT) as a, su2.Lattice(dims, 2.4, 5, su2.SU2_HOT) as b:
        b.set_launch(*cfg)
        a.heatbath_sweep(3)
        b.heatbath_sweep(3)
        np.testing.assert_array_equal(a.get_links(), b.get_links())
        assert abs(a.plaquette() - b.plaquette()) < 1e-12
    with su2.Batch(DIMS, BETAS, STARTS, 6) as a, su2.Batch(DIMS, BETAS, STARTS, 6) as b:
        b.set_launch(*cfg)
        a.sweep(2)
        b.sweep(2)
        for r in range(len(DIMS)):
            np.testing.assert_array_equal(a.get_links(r), b.get_links(r))


def test_autotune_preserves_state_and_caches(su2, tmp_path):
    announce("autotune")
    cache = str(tmp_path / "tune.jsonl")
    with su2.Batch(DIMS, BETAS, STARTS, 7) as a, su2.Batch(DIMS, BETAS, STARTS, 7) as b:
        a.sweep(2)
        b.sweep(2)
        us = b.autotune(cache)
        assert us > 0
        for r in range(len(DIMS)):
            np.testing.assert_array_equal(a.get_links(r), b.get_links(r))
        a.sweep(2)
        b.sweep(2)
        for r in range(len(DIMS)):
            np.testing.assert_array_equal(a.get_links(r), b.get_links(r))
        assert b.autotune(cache) == pytest.approx(us, abs=1e-3)  # cached (3 decimals)
    text = open(cache).read()
    assert text.count("\n") == 1 and '"block"' in text


def test_batch_observables_match_oracle(su2, orc):
    """Per-replica plaquette and Polyakov loop of seeded configurations (one
    per replica, given to both sides) against the oracle."""
    announce("batch observables vs oracle")
    links = [inputs.random_links(d, 300 + r, spread=0.6) for r, d in enumerate(DIMS)]
    with su2.Batch(DIMS, BETAS, STARTS, 8) as b:
        b.sweep(3)
        for r in range(len(DIMS)):
            b.set_links(r, links[r])
        p, ls, la = b.observables()
    for r, d in enumerate(DIMS):
        U = links[r].astype(np.float64)
        assert abs(p[r] - orc.plaquette(d, U)) < 1e-6
        wl, wa = orc.polyakov(d, U)
        assert abs(ls[r] - wl) < 1e-6 and abs(la[r] - wa) < 1e-6


def test_batch_learned_matches_single(su2):
    announce("batch learned == single")
    with su2.NN(seed=2) as net:
        net.sample_data(100_000, 0.5, 30.0, seed=3)
        net.train(200, 4096, 3e-3)
        net.build_table()
        with su2.Batch(DIMS, BETAS, STARTS, 9) as b:
            init = [b.get_links(r) for r in range(len(DIMS))]
            b.set_proposal(net)
            b.sweep(3, su2.SU2_LEARNED)
            prop, acc = b.accept_stats()
            assert np.all(prop > 0) and np.all(acc <= prop)
            for r, (d, beta) in enumerate(zip(DIMS, BETAS)):
                with su2.Lattice(d, beta, 9) as lat:
                    lat.set_replica(r)
                    lat.set_links(init[r])
                    lat.set_proposal(net)
                    lat.heatbath_sweep(3, su2.SU2_LEARNED)
                    np.testing.assert_array_equal(lat.get_links(), b.get_links(r))
                    p1, a1 = lat.accept_stats()
                    assert (p1, a1) == (int(prop[r]), int(acc[r]))


def test_batch_errors(su2):
    with pytest.raises(su2.SU2Error) as e:
        su2.Batch([[4, 4, 4, 3]], [2.0], [0], 1)
    assert e.value.code == su2.SU2_EODD
    with su2.Batch([[4, 4, 4, 4]], [2.0], [0], 1) as b:
        with pytest.raises(su2.SU2Error) as e:
            b.sweep(1, su2.SU2_LEARNED)
        assert e.value.code == su2.SU2_ESTATE
        with pytest.raises(su2.SU2Error):
            b.replay(1)
        with pytest.raises(su2.SU2Error):
            b.capture(3)  # null stream


def test_autotune_keeps_accept_statistics(su2):
    """The trial sweeps of the autotuner leave the learned accept counts (and
    every other accumulator) as they were."""
    announce("autotune keeps accept statistics")
    with su2.NN(seed=2) as net, su2.Batch(DIMS, BETAS, STARTS, 9) as b:
        net.build_table()
        b.set_proposal(net)
        b.sweep(3, su2.SU2_LEARNED)
        p0, a0 = b.accept_stats()
        assert p0.sum() > 0
        b.autotune(None, su2.SU2_LEARNED)
        p1, a1 = b.accept_stats()
        np.testing.assert_array_equal(p0, p1)
        np.testing.assert_array_equal(a0, a1)


def test_small_lattice_kernel_matches_pass_kernels(su2):
    """The whole-sweep kernel of small lattices (one workgroup per replica)
    gives the pass kernels' links bit for bit, in heat-bath and learned mode,
    with measurements and reunitarisation inside the launch."""
    announce("whole-sweep kernel == pass kernels")
    p = (np.random.default_rng(21).standard_normal(2671) * 0.2).astype(np.float32)
    runs = []
    with su2.NN(params=p) as net:
        net.build_table()
        for flags in (1, 5):  # bit 2 disables the whole-sweep kernel
            with su2.Batch(DIMS, BETAS, STARTS, 17) as b:
                b.set_proposal(net)
                b.set_launch(256, flags, 8, 8, 0)
                assert b.launch()["flags"] == flags
                h1 = b.sweep_measure(6, meas=3, reunit_every=4).cpu().numpy()
                b.sweep(2, su2.SU2_LEARNED)
                h2 = b.sweep_measure(3, su2.SU2_LEARNED, reunit_every=3, meas=3).cpu().numpy()
                runs.append((h1, h2, [b.get_links(r) for r in range(len(DIMS))],
                             b.accept_stats()))
    (a1, a2, al, ac), (b1, b2, bl, bc) = runs
    for r in range(len(DIMS)):
        np.testing.assert_array_equal(al[r], bl[r])
    for x, y in ((a1, b1), (a2, b2)):
        np.testing.assert_allclose(x[..., 0], y[..., 0], atol=1e-8, rtol=0)
        np.testing.assert_allclose(x[..., 1:], y[..., 1:], atol=1e-6, rtol=0)
    np.testing.assert_array_equal(ac[0], bc[0])
    np.testing.assert_array_equal(ac[1], bc[1])
    assert ac[1].sum() > 0 and ac[1].sum() < ac[0].sum()


def test_xcd_affine_launch_measurements_identical(su2):
    """The XCD-affine pass launch (every replica's workgroups on one XCD)
    partitions the sites into the same workgroups, so the fused plaquette is
    identical and the Polyakov loop agrees; links bit for bit, both modes."""
    announce("xcd-affine launch: measurements")
    p = (np.random.default_rng(31).standard_normal(2671) * 0.2).astype(np.float32)
    runs = []
    with su2.NN(params=p) as net:
        net.build_table()
        for flags in (1 | 4, 64 | 4):
            with su2.Batch(DIMS, BETAS, STARTS, 19) as b:
                b.set_proposal(net)
                b.set_launch(256, flags, 8, 8, 0)
                h1 = b.sweep_measure(5, meas=3, reunit_every=0).cpu().numpy()
                h2 = b.sweep_measure(3, su2.SU2_LEARNED, meas=3).cpu().numpy()
                runs.append((h1, h2, [b.get_links(r) for r in range(len(DIMS))],
                             b.accept_stats()))
    (a1, a2, al, ac), (b1, b2, bl, bc) = runs
    for r in range(len(DIMS)):
        np.testing.assert_array_equal(al[r], bl[r])
    for x, y in ((a1, b1), (a2, b2)):
        np.testing.assert_array_equal(x[..., 0], y[..., 0])
        np.testing.assert_allclose(x[..., 1:], y[..., 1:], atol=1e-6, rtol=0)
    np.testing.assert_array_equal(ac[1], bc[1])


def test_graph_rows_with_direct_measurements_between_replays(su2):
    """The k-th replay since a capture writes rows k*ns.. of the capture's
    history buffer even when direct measured sweeps run between the replays
    (they count their rows from the start of each call), for a lattice and a
    batch; a replay past the buffer's rows is refused."""
    announce("graph rows with direct measurements between replays")
    import torch
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        with su2.Lattice([8, 6, 8, 4], 2.5, 4, su2.SU2_HOT) as x, \
                su2.Lattice([8, 6, 8, 4], 2.5, 4, su2.SU2_HOT) as y:
            hy = torch.zeros((6, 3), dtype=torch.float64, device="cuda")
            y.capture(3, meas=3, hist=hy)
            want = []
            for k in range(2):
                y.replay(1)
                want.append(x.sweep_measure(3, meas=3).cpu().numpy())
                # direct measured sweeps on both lattices between the replays
                ey = y.sweep_measure(2 + k, meas=3).cpu().numpy()
                ex = x.sweep_measure(2 + k, meas=3).cpu().numpy()
                np.testing.assert_array_equal(ey, ex)
            y.synchronize()
            np.testing.assert_array_equal(hy.cpu().numpy(), np.concatenate(want))
            np.testing.assert_array_equal(x.get_links(), y.get_links())
            with pytest.raises(su2.SU2Error) as e:
                y.replay(1)
            assert e.value.code == su2.SU2_EINVAL
        with su2.Batch(DIMS, BETAS, STARTS, 7) as a, su2.Batch(DIMS, BETAS, STARTS, 7) as g:
            hg = torch.zeros((4, len(DIMS), 3), dtype=torch.float64, device="cuda")
            g.capture(2, meas=3, hist=hg)
            want = []
            for k in range(2):
                g.replay(1)
                want.append(a.sweep_measure(2, meas=3).cpu().numpy())
                np.testing.assert_array_equal(g.sweep_measure(1, meas=3).cpu().numpy(),
                                              a.sweep_measure(1, meas=3).cpu().numpy())
            g.synchronize()
            np.testing.assert_array_equal(hg.cpu().numpy(), np.concatenate(want))
            with pytest.raises(su2.SU2Error) as e:
                g.replay(1)
            assert e.value.code == su2.SU2_EINVAL
    torch.cuda.synchronize()
