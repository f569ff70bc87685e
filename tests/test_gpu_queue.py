"""The persistent work-queue launch (one launch per call runs every pass, the
reunitarisation and the measurements of all replicas, ordered per replica by
completion counters).  Links must equal the per-pass launches bit for bit in
every launch shape (block size, grain, grid down to one workgroup), in
heat-bath and learned mode, directly and replayed from a graph; plaquette and
Polyakov sums may differ only by the FP64 rounding of their partial sums.  A
bounded wait that runs out must be reported, not hang."""
import numpy as np
import pytest

from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

DIMS = [[4, 4, 4, 4], [6, 4, 8, 2], [8, 8, 8, 8], [4, 6, 2, 8], [10, 8, 6, 4], [2, 2, 2, 2],
        [12, 12, 12, 12]]
BETAS = [2.3, 1.9, 2.6, 0.7, 3.0, 2.1, 2.4]
STARTS = [1, 0, 1, 1, 0, 1, 1]
PASS_FLAGS = 1 | 4  # XCD remap, per-pass launches even for small lattices
QUEUE = 8


def run(su2, net, block, flags, grid):
    with su2.Batch(DIMS, BETAS, STARTS, 23) as b:
        b.set_proposal(net)
        b.set_launch(block, flags, 8, 8, grid)
        assert b.launch()["flags"] == flags
        h1 = b.sweep_measure(7, meas=3, reunit_every=3).cpu().numpy()
        b.sweep(2, su2.SU2_LEARNED)
        h2 = b.sweep_measure(4, su2.SU2_LEARNED, reunit_every=2, meas=3).cpu().numpy()
        b.sweep(1)
        links = [b.get_links(r) for r in range(len(DIMS))]
        return h1, h2, links, b.accept_stats()


@pytest.mark.parametrize("block,flags,grid", [
    (256, QUEUE | 1, 0), (128, QUEUE | 1 | (2 << 4), 16), (64, QUEUE | (1 << 4), 24),
    (192, QUEUE | 3, 1)], ids=["256-auto", "128-grain4-grid16", "64-grain2-grid24",
                               "192-one-workgroup-per-xcd"])
def test_queue_matches_pass_launches(su2, block, flags, grid):
    announce(f"queue launch {block} {flags} {grid} == pass launches")
    p = (np.random.default_rng(5).standard_normal(2671) * 0.2).astype(np.float32)
    with su2.NN(params=p) as net:
        net.build_table()
        a1, a2, al, ac = run(su2, net, block, PASS_FLAGS, 0)
        b1, b2, bl, bc = run(su2, net, block, flags, grid)
    for r in range(len(DIMS)):
        np.testing.assert_array_equal(al[r], bl[r])
    for x, y in ((a1, b1), (a2, b2)):
        np.testing.assert_allclose(x[..., 0], y[..., 0], atol=1e-9, rtol=0)
        np.testing.assert_allclose(x[..., 1:], y[..., 1:], atol=1e-6, rtol=0)
    # sweeps without reunitarisation fuse the plaquette into the same
    # workgroup partition: identical sums
    for j in (0, 1, 3, 4, 6):
        np.testing.assert_array_equal(a1[j, :, 0], b1[j, :, 0])
    np.testing.assert_array_equal(ac[0], bc[0])
    np.testing.assert_array_equal(ac[1], bc[1])
    assert bc[1].sum() > 0


def test_queue_single_lattice_and_graph(su2):
    announce("queue: single lattice, graph replay")
    import torch
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        with su2.Lattice([16, 16, 16, 16], 2.4, 9, su2.SU2_HOT) as x, \
                su2.Lattice([16, 16, 16, 16], 2.4, 9, su2.SU2_HOT) as y:
            y.set_launch(256, QUEUE | 1)
            hx = x.sweep_measure(10, meas=3, reunit_every=5).cpu().numpy()
            hy = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
            y.capture(5, meas=3, reunit_every=5, hist=hy)
            y.replay(2)
            y.synchronize()
            np.testing.assert_array_equal(x.get_links(), y.get_links())
            hy = hy.cpu().numpy()
            np.testing.assert_allclose(hy[:, 0], hx[:, 0], atol=1e-9, rtol=0)
            np.testing.assert_allclose(hy[:, 1:], hx[:, 1:], atol=1e-6, rtol=0)
            assert y.sweep == 10
    torch.cuda.synchronize()


def test_queue_wait_limit_is_reported(su2):
    """With a bounded wait of zero polls the first unmet dependency raises the
    error flag; the launch still drains and the next synchronising call
    reports it; with the normal limit the batch runs on."""
    announce("queue: bounded wait runs out")
    with su2.Batch(DIMS, BETAS, STARTS, 29) as b:
        b.set_launch(256, QUEUE | 1)
        b.test_spin_limit(0)
        b.sweep(20)
        with pytest.raises(su2.SU2Error) as e:
            b.synchronize()
        assert e.value.code == su2.SU2_EHIP
        b.test_spin_limit(1 << 22)
        b.sweep(2)
        b.synchronize()
