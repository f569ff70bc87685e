"""FP64 links (su2_init_f64) against the FP64 oracle, and FP32 against FP64
at equal seeds.

Both FP64 sides draw the same Philox streams and follow the same sampler, so
they agree to FP64 rounding (1e-12 per link component here); a decision flips
only when its margin is below ~1e-13, and links whose oracle margin is below
1e-10 are excluded and counted (none are expected).  The FP32 path from the
same inputs differs by its own rounding (~1e-6), which this file states for a
24^4 lattice."""
import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import MARGIN_FLAG, announce, parities

pytestmark = pytest.mark.gpu

FLAG64 = 1e-10


@pytest.mark.parametrize("dims", [[4, 4, 4, 6], [8, 6, 8, 10]], ids=lambda d: "x".join(map(str, d)))
def test_f64_hot_start_matches_oracle(su2, orc, dims):
    announce(f"fp64 hot start dims={dims}")
    with su2.Lattice64(dims, 2.3, 7, su2.SU2_HOT) as lat:
        got = lat.get_links()
    want = orc.init(dims, 1, 7)
    assert np.abs(got - want).max() < 1e-14
    with su2.Lattice64(dims, 2.3, 7, su2.SU2_COLD) as lat:
        assert lat.plaquette() == 1.0
        assert lat.polyakov() == (1.0, 1.0)


@pytest.mark.parametrize("dims", [[4, 4, 4, 4], [8, 6, 8, 10], [12, 10, 8, 6]],
                         ids=lambda d: "x".join(map(str, d)))
def test_f64_every_pass_matches_oracle(su2, orc, dims):
    announce(f"fp64 per-pass parity dims={dims}")
    links = inputs.as_f64(inputs.random_links(dims, 20 + sum(dims), spread=0.6))
    beta, seed = 2.4, 777
    par_of = parities(orc, dims)
    with su2.Lattice64(dims, beta, seed) as lat:
        lat.set_sweep(4)
        flagged = 0
        for mu in range(4):
            for p in range(2):
                lat.set_links(links)
                before = links
                U = links.copy()
                margin = orc.do_pass(dims, U, mu, p, 4, beta, seed, want_margin=True)
                lat.test_pass(mu, p)
                got = lat.get_links()
                upd = par_of == p
                ok = upd & (margin >= FLAG64)
                flagged += int((upd & (margin < FLAG64)).sum())
                assert np.abs(got[ok, mu] - U[ok, mu]).max() < 1e-12, (mu, p)
                mask = np.ones(got.shape[:2], bool)
                mask[upd, mu] = False
                np.testing.assert_array_equal(got[mask], before[mask])
        assert flagged == 0


def test_f64_sweeps_and_measurements_match_oracle(su2, orc):
    """Hot start, five sweeps with reunitarisation every 2 and the plaquette and
    Polyakov loop every sweep, against the oracle's chain (no resynchronisation)."""
    announce("fp64 sweeps + measurements")
    dims, beta, seed = [8, 8, 8, 8], 2.4, 5
    with su2.Lattice64(dims, beta, seed, su2.SU2_HOT) as lat:
        h = lat.sweep_measure(5, reunit_every=2,
                              meas=su2.SU2_MEAS_PLAQ | su2.SU2_MEAS_POLY).cpu().numpy()
        got = lat.get_links()
        p_s = lat.plaquette()
        l_s, la_s = lat.polyakov()
    U = orc.init(dims, 1, seed)
    ph, lh = orc.sweeps(dims, U, 5, 0, beta, seed, reunit_every=2, measure=True)
    assert np.abs(got - U).max() < 1e-11
    # the sums round each workgroup's FP64 total to a multiple of 2^-28 (fixed
    # point across workgroups): at most 2^-29 per workgroup, divided by the
    # 6 V plaquettes or the Ns^3 Polyakov loops
    tol_p, tol_l = 1e-11, 1e-10
    np.testing.assert_allclose(h[:, 0], ph, atol=tol_p, rtol=0)
    np.testing.assert_allclose(h[:, 1], lh, atol=tol_l, rtol=0)
    np.testing.assert_allclose(h[:, 2], np.abs(lh), atol=tol_l, rtol=0)
    assert abs(p_s - orc.plaquette(dims, U)) < tol_p
    ls, la = orc.polyakov(dims, U)
    assert abs(l_s - ls) < tol_l and abs(la_s - la) < tol_l


def test_f32_against_f64_at_equal_seeds(su2, orc):
    """24^4, beta 2.0, the same FP64 hot start in both precisions.  Pass by
    pass from a seeded configuration (the FP32 lattice gets it rounded)
    the FP32 links differ from the FP64 ones by FP32 rounding, decisions the
    oracle places within 2e-5 of their threshold excluded.  Over one whole
    sweep without resynchronisation a flipped decision also changes the
    neighbours it feeds, so only a small fraction of links may differ by more
    than FP32 rounding; the plaquette and Polyakov loop of the two results
    agree to FP32 precision."""
    announce("fp32 vs fp64 at equal seeds")
    dims, beta, seed = [24, 24, 24, 24], 2.0, 9
    par_of = parities(orc, dims)
    with su2.Lattice64(dims, beta, seed, su2.SU2_HOT) as l64, \
            su2.Lattice(dims, beta, seed, su2.SU2_COLD) as l32:
        start = l64.get_links()
        # one sweep in each precision from the same start
        l32.set_links(start.astype(np.float32))
        l64.heatbath_sweep(1)
        l32.heatbath_sweep(1)
        g64, g32 = l64.get_links(), l32.get_links().astype(np.float64)
        p64, p32 = l64.plaquette(), l32.plaquette()
        (s64, a64), (s32, a32) = l64.polyakov(), l32.polyakov()
        dl = np.abs(g32 - g64).max(axis=-1)
        big = float(np.mean(dl > 1e-4))
        # pass by pass from a seeded configuration given to both precisions and the oracle
        links = inputs.as_f64(inputs.random_links(dims, 91, spread=0.8))
        l64.set_sweep(0)
        l32.set_sweep(0)
        worst, nflag = 0.0, 0
        for mu in range(4):
            for p in range(2):
                l64.set_links(links)
                l32.set_links(links.astype(np.float32))
                W = links.copy()
                margin = orc.do_pass(dims, W, mu, p, 0, beta, seed, want_margin=True)
                l64.test_pass(mu, p)
                l32.test_pass(mu, p)
                a, b32 = l64.get_links(), l32.get_links().astype(np.float64)
                upd = par_of == p
                ok = upd & (margin >= MARGIN_FLAG)
                nflag += int((upd & (margin < MARGIN_FLAG)).sum())
                assert np.abs(a[upd, mu] - W[upd, mu]).max() < 1e-11
                worst = max(worst, float(np.abs(b32[ok, mu] - a[ok, mu]).max()))
    print(f"\n[fp32-vs-fp64] 24^4 beta 2.0: per pass from identical links max|dU| {worst:.2e} "
          f"({nflag} flagged decisions of {4 * int(np.prod(dims))}); after one sweep "
          f"{big:.1e} of the links differ by more than 1e-4, plaquette {abs(p32 - p64):.1e}, "
          f"Polyakov signed {abs(s32 - s64):.1e} abs {abs(a32 - a64):.1e}", flush=True)
    assert 1e-9 < worst < 1e-5
    assert big < 1e-3
    assert abs(p32 - p64) < 1e-5 and abs(s32 - s64) < 1e-4


def test_f64_graph_replay_equals_direct_sweeps(su2):
    """FP64 sweeps with reunitarisation and the fused plaquette, captured once
    and replayed several times with eager work and synchronisation between the
    replays, end bit for bit where the same sweeps run directly, and so do
    their measurement histories."""
    import torch
    announce("fp64 graph replay == direct")
    dims = [8, 6, 4, 8]
    side = torch.cuda.Stream()  # capture needs a non-null stream
    with torch.cuda.stream(side):
        with su2.Lattice64(dims, 2.4, 51, su2.SU2_HOT) as a, \
                su2.Lattice64(dims, 2.4, 51, su2.SU2_HOT) as g:
            ha = a.sweep_measure(12, reunit_every=4, meas=3).cpu().numpy()
            hg = torch.zeros((12, 3), dtype=torch.float64, device="cuda")
            g.capture(4, reunit_every=4, meas=3, hist=hg)
            for k in range(3):
                g.replay(1)
                g.synchronize()
                assert g.sweep == 4 * (k + 1)
                _ = g.plaquette()  # eager work between the replays
            np.testing.assert_array_equal(hg.cpu().numpy(), ha)
            np.testing.assert_array_equal(g.get_links(), a.get_links())
    torch.cuda.synchronize()


def test_f64_autotune_keeps_state_and_links(su2):
    """The FP64 autotuner restores links, sweep index and measurements after its
    trial sweeps, picks a launch the FP64 pass supports (no grid cap, no
    whole-sweep or work-queue launch), and sweeps in that launch give the links
    of the default launch bit for bit (every update depends only on its
    neighbours and its Philox stream, not on the workgroup partition)."""
    announce("fp64 autotune")
    dims = [12, 8, 10, 6]
    with su2.Lattice64(dims, 2.2, 61, su2.SU2_HOT) as t, \
            su2.Lattice64(dims, 2.2, 61, su2.SU2_HOT) as d:
        before = t.get_links()
        us = t.autotune(None, su2.SU2_KP)
        assert us > 0
        np.testing.assert_array_equal(t.get_links(), before)
        assert t.sweep == 0
        cfg = t.launch()
        assert cfg["grid_cap"] == 0 and not cfg["flags"] & (4 | 8 | 64 | 128), cfg
        t.heatbath_sweep(3)
        d.heatbath_sweep(3)
        np.testing.assert_array_equal(t.get_links(), d.get_links())
        assert abs(t.plaquette() - d.plaquette()) < 1e-12
