"""Rectangular Wilson loops on the GPU (su2_wilson_loops) against the FP64
oracle on identical links: per-site FP32 products of up to 16 links, FP64
sums, so the averages agree to ~1e-7; the cold start gives exactly 1 and
W(1,1) is the plaquette."""
import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,rt", [([8, 6, 8, 10], (4, 4)), ([4, 4, 4, 6], (3, 2)),
                                     ([16, 16, 16, 16], (4, 4)), ([2, 4, 6, 8], (1, 1)),
                                     ([6, 10, 8, 6], (4, 2)), ([10, 6, 6, 8], (2, 4))],
                         ids=["8x6x8x10", "4x4x4x6", "16^4", "2x4x6x8", "6x10x8x6-r4t2",
                              "10x6x6x8-r2t4"])
def test_wilson_loops_match_oracle(su2, orc, dims, rt):
    announce(f"wilson loops dims={dims} rt={rt}")
    links = inputs.random_links(dims, 40 + sum(dims), spread=0.6)
    with su2.Lattice(dims, 2.3, 1) as lat:
        lat.set_links(links)
        got = lat.wilson_loops(*rt)
        p = lat.plaquette()
    want = orc.wilson_loops(dims, inputs.as_f64(links), *rt)
    assert np.abs(got - want).max() < 1e-6, np.abs(got - want).max()
    assert abs(got[0, 0] - p) < 1e-7
    assert np.all(np.abs(want) > 1e-4)  # loops of every size are resolved


def test_wilson_loops_cold_and_errors(su2):
    announce("wilson loops cold start, bad arguments")
    with su2.Lattice([6, 6, 6, 6], 2.3, 1, su2.SU2_COLD) as lat:
        np.testing.assert_array_equal(lat.wilson_loops(4, 4), np.ones((4, 4)))
        for bad in ((0, 2), (2, 5), (6, 2)):
            with pytest.raises(su2.SU2Error) as e:
                lat.wilson_loops(*bad)
            assert e.value.code == su2.SU2_EINVAL
    with su2.Lattice([4, 4, 4, 4], 2.3, 1) as lat:
        with pytest.raises(su2.SU2Error):
            lat.wilson_loops(4, 1)  # R must stay below every extent
    with su2.Lattice64([4, 4, 4, 4], 2.3, 1) as lat:
        with pytest.raises(su2.SU2Error) as e:
            lat.wilson_loops(2, 2)
        assert e.value.code == su2.SU2_ESTATE
