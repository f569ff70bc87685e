"""Combinations of entry points that the per-feature tests do not reach on
their own: the float link exchange of an FP64 context, the heat bath with
over-relaxation (SU2_KP_OR) under graph capture, the autotuner and the
batched launch shapes, and learned batches under graph capture.  Each compares
two routes that must agree bit for bit."""
import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def test_f64_context_exchanges_float_links(su2):
    """On an FP64 context, su2_get_links (float host array) returns the FP64
    links rounded to FP32, and su2_set_links (float host array) stores them
    widened exactly."""
    announce("fp64 context, float link exchange")
    dims = [6, 4, 8, 2]
    V = int(np.prod(dims))
    with su2.Lattice64(dims, 2.0, 17, su2.SU2_HOT) as lat:
        d = lat.get_links()
        f = su2.su2_get_links(lat.h, V)
        np.testing.assert_array_equal(f, d.astype(np.float32))
        g = inputs.random_links(dims, 18)
        su2.su2_set_links(lat.h, g)
        np.testing.assert_array_equal(lat.get_links(), g.astype(np.float64))


def test_overrelaxed_sweeps_replayed_from_a_graph_equal_direct(su2):
    """Heat bath plus two over-relaxation sweeps per sweep, reunitarised every
    third sweep and measured every sweep: a captured graph of three sweeps
    replayed twice (with eager work between the replays) gives the links and
    history rows of six direct sweeps bit for bit."""
    import torch
    announce("KP_OR capture/replay == direct")
    dims = [8, 6, 4, 8]
    side = torch.cuda.Stream()  # capture needs a non-null stream
    with torch.cuda.stream(side):
        with su2.Lattice(dims, 2.3, 21, su2.SU2_HOT) as a, \
                su2.Lattice(dims, 2.3, 21, su2.SU2_HOT) as g:
            for lat in (a, g):
                lat.set_hb_overrelax(2)
            ha = a.sweep_measure(6, su2.SU2_KP_OR, reunit_every=3, meas=3).cpu().numpy()
            hg = torch.zeros((6, 3), dtype=torch.float64, device="cuda")
            g.capture(3, su2.SU2_KP_OR, reunit_every=3, meas=3, hist=hg)
            for k in range(2):
                g.replay(1)
                g.synchronize()
                assert g.sweep == 3 * (k + 1)
                _ = g.plaquette()
            np.testing.assert_array_equal(hg.cpu().numpy(), ha)
            np.testing.assert_array_equal(g.get_links(), a.get_links())
    torch.cuda.synchronize()


def test_overrelaxed_autotune_keeps_state_and_links(su2):
    """Autotuning for SU2_KP_OR restores the links and the sweep index, and the
    launch it picks sweeps the links of the default launch bit for bit."""
    announce("KP_OR autotune")
    dims = [16, 16, 16, 16]
    with su2.Lattice(dims, 2.4, 23, su2.SU2_HOT) as t, \
            su2.Lattice(dims, 2.4, 23, su2.SU2_HOT) as d:
        for lat in (t, d):
            lat.set_hb_overrelax(1)
        before = t.get_links()
        assert t.autotune(None, su2.SU2_KP_OR) > 0
        np.testing.assert_array_equal(t.get_links(), before)
        assert t.sweep == 0
        t.heatbath_sweep(2, su2.SU2_KP_OR)
        d.heatbath_sweep(2, su2.SU2_KP_OR)
        np.testing.assert_array_equal(t.get_links(), d.get_links())


@pytest.mark.parametrize("flags", [1 | 4, 64 | 1, 64 | 2, 3 | 4], ids=["per-pass", "xcd-affine",
                                                                       "xcd-affine-no-snake",
                                                                       "remap-no-snake"])
def test_overrelaxed_batch_launch_shapes_are_bitwise_neutral(su2, flags):
    """A batch of unequal replicas swept in SU2_KP_OR mode gives the same links
    bit for bit in every launch shape (per-pass, XCD-affine, pass order)."""
    announce(f"KP_OR batch launch flags={flags}")
    dims = [[8, 8, 8, 8], [6, 4, 8, 2], [10, 8, 6, 4]]
    betas, starts = [2.2, 1.9, 2.6], [1, 0, 1]
    out = []
    for fl in (None, flags):
        with su2.Batch(dims, betas, starts, 29) as b:
            b.set_hb_overrelax(1)
            if fl is not None:
                b.set_launch(256, fl, 4, 4, 0)
            b.sweep(3, su2.SU2_KP_OR)
            out.append([b.get_links(r) for r in range(len(dims))])
    for r in range(len(dims)):
        np.testing.assert_array_equal(out[0][r], out[1][r])


@pytest.mark.parametrize("small", [False, True], ids=["per-pass", "whole-sweep-kernel"])
@pytest.mark.parametrize("width", [-1.0, 0.02], ids=["independence", "overrelaxed"])
def test_learned_sweeps_replayed_from_a_graph_equal_direct(su2, width, small):
    """Learned Metropolis sweeps of a batch (independence or over-relaxed
    proposal; replicas large enough for per-pass launches, or all small enough
    for the whole-sweep kernel) captured once and replayed twice give the links,
    history rows and accept counts of the same sweeps run directly, bit for
    bit."""
    import torch
    announce(f"learned capture/replay == direct width={width} small={small}")
    p = (np.random.default_rng(31).standard_normal(2671) * 0.2).astype(np.float32)
    dims = ([[8, 8, 8, 8], [6, 4, 8, 2], [4, 6, 2, 8]] if small else
            [[8, 8, 8, 8], [6, 4, 8, 2], [12, 10, 8, 6]])
    betas, starts = [2.2, 1.9, 2.6], [1, 0, 1]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side), su2.NN(params=p) as net:
        net.build_table()
        res = []
        for graph in (False, True):
            with su2.Batch(dims, betas, starts, 33) as b:
                b.set_proposal(net)
                b.set_overrelax(width)
                b.sweep(3)  # heat-bath start (the capture starts at a reunitarisation boundary)
                b.accept_stats(reset=True)
                if graph:
                    h = torch.zeros((6, len(dims), 3), dtype=torch.float64, device="cuda")
                    b.capture(3, su2.SU2_LEARNED, reunit_every=3, meas=3, hist=h)
                    for _ in range(2):
                        b.replay(1)
                        b.synchronize()
                        _ = b.observables()  # eager work between the replays
                else:
                    h = b.sweep_measure(6, su2.SU2_LEARNED, reunit_every=3, meas=3)
                b.synchronize()
                res.append((h.cpu().numpy(), [b.get_links(r) for r in range(len(dims))],
                            b.accept_stats()))
    (ha, la, aa), (hg, lg, ag) = res
    np.testing.assert_array_equal(hg, ha)
    for r in range(len(dims)):
        np.testing.assert_array_equal(lg[r], la[r])
    np.testing.assert_array_equal(ag[0], aa[0])
    np.testing.assert_array_equal(ag[1], aa[1])
    assert aa[1].sum() > 0


@pytest.mark.parametrize("change", ["beta", "replica", "overrelax", "launch"])
def test_settings_changed_after_capture_drop_the_recording(su2, change):
    """A captured graph holds the settings of its capture: changing beta, the
    replica id, an over-relaxation setting or the launch drops it, and a
    replay is refused (SU2_ESTATE) with nothing enqueued."""
    import torch
    announce(f"capture dropped by a {change} change")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side), su2.Lattice([8, 8, 8, 8], 2.3, 41, su2.SU2_HOT) as g:
        g.capture(2)
        g.replay(1)
        g.synchronize()
        {"beta": lambda: g.set_beta(2.5), "replica": lambda: g.set_replica(3), "overrelax": lambda: g.set_hb_overrelax(1),
         "launch": lambda: g.set_launch(128, 1 | 4, 4, 4)}[change]()
        before = g.get_links()
        s0 = g.sweep
        with pytest.raises(su2.SU2Error) as ei:
            g.replay(1)
        assert ei.value.code == su2.SU2_ESTATE
        g.synchronize()
        np.testing.assert_array_equal(g.get_links(), before)
        assert g.sweep == s0
    torch.cuda.synchronize()


def test_replays_continue_from_a_set_sweep_index(su2):
    """su2_set_sweep keeps the recording: replays read the sweep index on the
    device, so after set_sweep(10) the next replay runs sweeps 10 and 11, as a
    context that runs them directly."""
    import torch
    announce("replay after set_sweep")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side), su2.Lattice([8, 8, 8, 8], 2.3, 43, su2.SU2_HOT) as g, \
            su2.Lattice([8, 8, 8, 8], 2.3, 43, su2.SU2_HOT) as d:
        g.capture(2)
        g.replay(1)
        g.set_sweep(10)
        g.replay(1)
        g.synchronize()
        d.heatbath_sweep(2)
        d.set_sweep(10)
        d.heatbath_sweep(2)
        assert g.sweep == d.sweep == 12
        np.testing.assert_array_equal(g.get_links(), d.get_links())
    torch.cuda.synchronize()


@pytest.mark.parametrize("flags", [64 | 1, 1 | 4], ids=["xcd-affine", "per-pass"])
def test_batch_graph_in_each_launch_shape_equals_direct(su2, flags):
    """Batched heat-bath sweeps captured in the XCD-affine or the per-pass launch
    and replayed twice give the links of direct sweeps in the default launch bit
    for bit, and their history within the rounding of the FP64 partial sums."""
    import torch
    announce(f"batch graph in launch flags={flags}")
    dims = [[16, 16, 16, 16], [12, 12, 12, 12], [8, 8, 8, 8]]
    betas, starts = [2.4, 2.1, 2.7], [1, 1, 0]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        with su2.Batch(dims, betas, starts, 37) as a, su2.Batch(dims, betas, starts, 37) as g:
            ha = a.sweep_measure(8, reunit_every=4, meas=3).cpu().numpy()
            g.set_launch(256, flags, 8, 8, 0)
            hg = torch.zeros((8, len(dims), 3), dtype=torch.float64, device="cuda")
            g.capture(4, reunit_every=4, meas=3, hist=hg)
            for _ in range(2):
                g.replay(1)
                g.synchronize()
            for r in range(len(dims)):
                np.testing.assert_array_equal(g.get_links(r), a.get_links(r))
            hg = hg.cpu().numpy()
            np.testing.assert_allclose(hg[..., 0], ha[..., 0], atol=1e-9, rtol=0)
            np.testing.assert_allclose(hg[..., 1:], ha[..., 1:], atol=1e-6, rtol=0)
    torch.cuda.synchronize()


def test_autotune_cache_keeps_precisions_and_modes_apart(su2, tmp_path):
    """The autotuner's cache distinguishes an FP64 context from an FP32 one of
    the same extents, and over-relaxation settings: each tunes and records its
    own entry, and a second FP64 context reuses the FP64 entry."""
    announce("autotune cache keys")
    cache = str(tmp_path / "tune.jsonl")
    dims = [12, 8, 10, 6]
    with su2.Lattice(dims, 2.2, 71, su2.SU2_HOT) as a:
        a.autotune(cache)
    with su2.Lattice64(dims, 2.2, 71, su2.SU2_HOT) as b:
        us64 = b.autotune(cache)
        cfg = b.launch()
        assert cfg["grid_cap"] == 0 and not cfg["flags"] & (4 | 8 | 64 | 128), cfg
    with su2.Lattice(dims, 2.2, 71, su2.SU2_HOT) as c:
        c.set_hb_overrelax(1)
        c.autotune(cache, su2.SU2_KP_OR)
        c.set_hb_overrelax(2)
        c.autotune(cache, su2.SU2_KP_OR)
    with open(cache) as f:
        lines = [l for l in f if l.strip()]
    assert len(lines) == 4, lines
    with su2.Lattice64(dims, 2.2, 72, su2.SU2_HOT) as d:
        assert d.autotune(cache) == pytest.approx(us64, abs=1e-3)  # cached
        assert d.launch() == cfg
    with open(cache) as f:
        assert len([l for l in f if l.strip()]) == 4
