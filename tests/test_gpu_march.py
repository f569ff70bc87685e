"""The pass with LDS-staged neighbour links (launch flag 128) against the
plain pass kernel and the FP64 oracle: the same links from the same inputs,
bit for bit, for every (mu, parity) pass, heat bath and over-relaxation, on
lattices with one and several row tiles and t-chunks (a ragged last wave of
64 lanes included), and whole sweeps with the fused plaquette, the
reunitarisation and the Polyakov loop."""
import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import announce, compare_pass, parities

pytestmark = pytest.mark.gpu

# (dims, rows R, planes T)
SHAPES = [([8, 8, 8, 8], 4, 4), ([8, 8, 8, 8], 2, 8), ([12, 10, 8, 6], 5, 3),
          ([6, 4, 2, 2], 2, 1), ([16, 16, 16, 16], 8, 4), ([48, 48, 48, 48], 8, 8)]
MARCH = 1 | 4 | 128


@pytest.mark.parametrize("dims,R,T", SHAPES, ids=lambda v: "x".join(map(str, v)) if isinstance(v, list) else str(v))
def test_march_passes_equal_plain_passes(su2, orc, dims, R, T):
    announce(f"march passes dims={dims} R={R} T={T}")
    links = inputs.random_links(dims, 300 + dims[0] + R, spread=0.7)
    big = np.prod(dims) > 10 ** 6
    with su2.Lattice(dims, 2.3, 9) as plain, su2.Lattice(dims, 2.3, 9) as lat:
        lat.set_launch(256, MARCH, R, T, 0)
        assert lat.launch()["flags"] & 128 and lat.launch()["tile_z"] == R
        for mode in (su2.SU2_KP, su2.SU2_KP_OR):
            for mu in range(4):
                for p in range(2):
                    for x in (plain, lat):
                        x.set_links(links)
                        x.set_sweep(3)
                        x.test_pass(mu, p, mode)
                    a, b = plain.get_links(), lat.get_links()
                    if not np.array_equal(a, b):
                        d = np.abs(a - b).max(axis=2)
                        print(f"[gpu-test] mode {mode} pass ({mu},{p}): {int((d > 0).sum())} links "
                              f"differ, max {d.max():.3e}", flush=True)
                    assert np.array_equal(a, b), (mode, mu, p, int((a != b).sum()))
        if not big:  # and the oracle on one pass of each kind
            par_of = parities(orc, dims)
            U = links.astype(np.float64)
            m = orc.do_pass(dims, U, 3, 1, 3, 2.3, 9, want_margin=True)
            lat.set_links(links)
            lat.test_pass(3, 1)
            err, nflag = compare_pass(lat.get_links(), U, m, 1, 3, par_of)
            assert err < 1e-5


@pytest.mark.parametrize("dims,R,T", SHAPES[:5], ids=lambda v: "x".join(map(str, v)) if isinstance(v, list) else str(v))
def test_march_sweeps_equal_plain_sweeps(su2, dims, R, T):
    announce(f"march sweeps dims={dims} R={R} T={T}")
    with su2.Lattice(dims, 2.4, 5, su2.SU2_HOT) as plain, \
            su2.Lattice(dims, 2.4, 5, su2.SU2_HOT) as lat:
        plain.set_launch(256, 1 | 4, 8, 8, 0)  # per-pass plain kernels
        lat.set_launch(256, MARCH, R, T, 0)
        for mode in (su2.SU2_KP, su2.SU2_KP_OR):
            ha = plain.sweep_measure(4, mode, reunit_every=2, meas=3).cpu().numpy()
            hb = lat.sweep_measure(4, mode, reunit_every=2, meas=3).cpu().numpy()
            np.testing.assert_array_equal(plain.get_links(), lat.get_links())
            np.testing.assert_allclose(ha, hb, atol=1e-9, rtol=0)


def test_march_launch_arguments(su2):
    with su2.Lattice([8, 8, 8, 8], 2.0, 1) as lat:
        for R, T in ((3, 4), (4, 3), (0, 4), (1, 4)):
            with pytest.raises(su2.SU2Error) as e:
                lat.set_launch(256, MARCH, R, T, 0)
            assert e.value.code == su2.SU2_EINVAL
        with pytest.raises(su2.SU2Error):
            lat.set_launch(256, MARCH | 8, 4, 4, 0)
    with su2.Lattice([48, 48, 48, 48], 2.0, 1) as lat:
        with pytest.raises(su2.SU2Error):  # 16 rows of 24 half-sites: 384 threads
            lat.set_launch(256, MARCH, 16, 8, 0)
    with su2.Batch([[8, 8, 8, 8]] * 2, [2.0, 2.1], [0, 0], 1) as b:
        with pytest.raises(su2.SU2Error):
            b.set_launch(256, MARCH, 4, 4, 0)
