"""The allocation-free entry point su2_sweep_measure_static against
su2_sweep_measure on a context (su2_init_ext, default launch): the same links,
beta, seed and sweep index give bit-identical links and history, for two calls
in a row on one GPU, the second on a smaller lattice (the static scratch keeps
the first call's counters and sums, which the second must clear); and the
entry point recorded into a graph and replayed equals direct calls."""
import numpy as np
import pytest

from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def run_pair(su2, torch, dims, beta, seed, sweep0, ns, reunit, meas):
    with su2.Lattice(dims, beta, seed, su2.SU2_HOT) as ref:
        ref.heatbath_sweep(2)  # a thermalising start, as the caller would hold it
        ref.set_sweep(sweep0)
        links = ref.links_t.clone()  # the same device layout, the caller's buffer
        torch.cuda.synchronize()
        want = ref.sweep_measure(ns, reunit_every=reunit, meas=meas).cpu().numpy()
        want_links = ref.links_t.cpu().numpy()
    hist = torch.full((ns, 3), -7.0, dtype=torch.float64, device=links.device)
    got = su2.su2_sweep_measure_static(links, dims, beta, seed, sweep0, ns, reunit, meas, hist)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), want)
    np.testing.assert_array_equal(links.cpu().numpy(), want_links)
    return want


def test_static_sweeps_equal_context_sweeps(su2):
    import torch
    announce("allocation-free sweeps: 16^4 (per-pass launches), then 8x6x8x4 (one launch)")
    h1 = run_pair(su2, torch, [16, 16, 16, 16], 2.4, 21, 10, 12, 10, 3)
    assert np.all(h1[:, 0] > 0)
    h2 = run_pair(su2, torch, [8, 6, 8, 4], 2.1, 22, 3, 7, 4, 1)
    assert np.all(h2[:, 1] == 0)  # no Polyakov loop asked for
    # argument errors come back before any device work
    links = torch.zeros(su2.su2_links_bytes([4, 4, 4, 4]), dtype=torch.uint8, device="cuda")
    with pytest.raises(su2.SU2Error) as e:
        su2.su2_sweep_measure_static(links, [4, 4, 4, 5], 2.0, 1, 0, 1)
    assert e.value.code == su2.SU2_EODD
    with pytest.raises(su2.SU2Error) as e:
        su2.su2_sweep_measure_static(links, [4, 4, 4, 4], -1.0, 1, 0, 1)
    assert e.value.code == su2.SU2_EINVAL


def test_static_sweeps_under_graph_capture(su2):
    """The use the entry point is for: recorded into a graph (torch.cuda.graph;
    nothing is allocated inside the capture) and replayed three times with eager
    work in between, it gives the links and history of three direct calls with
    the same arguments, bit for bit."""
    import torch
    announce("allocation-free sweeps under graph capture")
    dims, beta, seed = [8, 8, 8, 8], 2.3, 24
    with su2.Lattice(dims, beta, seed, su2.SU2_HOT) as ref:
        a = ref.links_t.clone()
        b = ref.links_t.clone()
    ha = torch.zeros((4, 3), dtype=torch.float64, device="cuda")
    hb = torch.zeros((4, 3), dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    # a first call outside the capture looks up the device array's address
    warm = a.clone()
    su2.su2_sweep_measure_static(warm, dims, beta, seed, 0, 1, 0, 1,
                                 torch.zeros((1, 3), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        su2.su2_sweep_measure_static(b, dims, beta, seed, 5, 4, 2, 3, hb)
    for _ in range(3):
        su2.su2_sweep_measure_static(a, dims, beta, seed, 5, 4, 2, 3, ha)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(hb.cpu().numpy(), ha.cpu().numpy())
        np.testing.assert_array_equal(b.cpu().numpy(), a.cpu().numpy())
    assert np.all(ha.cpu().numpy()[:, 0] > 0)
