"""SU(3) heat bath (Cabibbo-Marinari subgroups on the SU(2) step of Sec. 2) on
the GPU against the FP64 SU(3) oracle.  Inputs reach the oracle only from the
seeded generator or the oracle's own starts.

Both sides draw the same Philox streams, so each link agrees to FP32 rounding.
The FP32 error of an a0 decision is larger than for SU(2) (six staples of three
SU(3) factors, then W = U A and two earlier subgroup rotations feed each
subgroup's k), so links whose smallest oracle decision margin is below
FLAG3 = 2e-4 are excluded and counted against a bound; every flagged link must
still be in SU(3).  Every other link agrees within TOL3 = 1e-5 per component.
"""
import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

FLAG3 = 2e-4
TOL3 = 1e-5


@pytest.fixture(scope="module")
def o3():
    from oracle import su3_oracle
    su3_oracle._load()
    return su3_oracle


def parities(dims):
    V = int(np.prod(dims))
    s = np.arange(V)
    x = s % dims[0]
    y = (s // dims[0]) % dims[1]
    z = (s // (dims[0] * dims[1])) % dims[2]
    t = s // (dims[0] * dims[1] * dims[2])
    return (x + y + z + t) & 1


def su3_defect(U):
    M = U.reshape(-1, 3, 3)
    return max(np.abs(M @ np.conj(np.swapaxes(M, 1, 2)) - np.eye(3)).max(),
               np.abs(np.linalg.det(M) - 1.0).max())


def max_flags3(n_links):
    return int(10 * 3 * 2 * FLAG3 * n_links) + 3


@pytest.mark.parametrize("dims", [[4, 4, 4, 6], [6, 6, 6, 10]], ids=lambda d: "x".join(map(str, d)))
def test_su3_starts_match_oracle(su2, o3, dims):
    announce(f"su3 hot/cold start dims={dims}")
    with su2.Lattice3(dims, 6.0, 9, su2.SU2_HOT) as lat:
        got = lat.get_links()
        plaq = lat.plaquette()
    want = o3.init(dims, 1, 9)
    assert np.abs(got - want).max() < 2e-5
    assert su3_defect(got) < 2e-6
    assert plaq == pytest.approx(o3.plaquette(dims, want), abs=2e-6)
    with su2.Lattice3(dims, 6.0, 9, su2.SU2_COLD) as lat:
        assert lat.plaquette() == 1.0
        assert lat.polyakov() == (1.0, 0.0, 1.0)
        assert np.array_equal(lat.get_links(), o3.init(dims, 0, 9))


@pytest.mark.parametrize("dims,spread,beta", [([2, 2, 2, 2], None, 5.7), ([2, 4, 2, 6], 0.4, 6.0),
                                              ([4, 4, 4, 4], None, 5.7), ([6, 6, 6, 10], 0.3, 6.0),
                                              ([8, 4, 6, 4], 0.15, 8.0), ([4, 4, 4, 4], None, 0.0),
                                              ([4, 6, 2, 8], 0.15, 40.0)],
                         ids=["2^4-haar", "2x4x2x6", "4^4-haar", "6^3x10-ordered", "8x4x6x4-cold",
                              "4^4-beta0", "4x6x2x8-beta40"])
def test_su3_every_pass_matches_oracle(su2, o3, dims, spread, beta):
    """All eight (mu, parity) passes from the same links; V/2 = 1080 for
    6^3 x 10 spans four full workgroups and a ragged tail."""
    announce(f"su3 per-pass parity dims={dims} spread={spread} beta={beta}")
    links = inputs.random_su3_links(dims, 40 + sum(dims), spread=spread)
    seed, sweep = 4242, 5
    par_of = parities(dims)
    V = int(np.prod(dims))
    flagged, worst = 0, 0.0
    with su2.Lattice3(dims, beta, seed) as lat:
        lat.set_sweep(sweep)
        lat.set_links(links)
        stored = lat.get_links()  # the seeded links as the GPU holds them (rows 0, 1 in FP32)
        for mu in range(4):
            for p in range(2):
                lat.set_links(links)
                before = stored
                U = links.copy()
                margin = np.zeros(V)
                o3.pass_(dims, U, mu, p, sweep, beta, seed, margin=margin)
                lat.test_pass(mu, p)
                got = lat.get_links()
                upd = par_of == p
                ok = upd & (margin >= FLAG3)
                flagged += int((upd & (margin < FLAG3)).sum())
                err = np.abs(got[ok, mu] - U[ok, mu]).max()
                worst = max(worst, err)
                assert err < TOL3, (mu, p, err)
                assert su3_defect(got[upd, mu]) < 5e-6
                mask = np.ones(got.shape[:2], bool)
                mask[upd, mu] = False
                np.testing.assert_array_equal(got[mask], before[mask])
    announce(f"  max |gpu - oracle| = {worst:.2e}, flagged {flagged} of {4 * V}")
    assert flagged <= max_flags3(4 * V)


def test_su3_sweeps_match_oracle_with_measurements(su2, o3):
    """Three sweeps (reunitarisation after sweep 2) from a seeded configuration
    given to both sides: per-sweep plaquette history (fused into the odd
    passes) and final links against the oracle's sweeps, the standalone
    plaquette and Polyakov loop against the oracle's of its final links, and
    the standalone plaquette against the fused one."""
    dims, beta, seed = [6, 4, 6, 8], 5.9, 31
    announce(f"su3 sweeps dims={dims}")
    links = inputs.random_su3_links(dims, 131, spread=0.5)
    with su2.Lattice3(dims, beta, seed) as lat:
        lat.set_links(links)
        hist = lat.heatbath_sweep(3, reunit_every=2, history=True)
        got = lat.get_links()
        plaq = lat.plaquette()
        poly = lat.polyakov()
        assert lat.sweep == 3
    U = links.copy()
    ph, _ = o3.sweeps(dims, U, 3, 0, beta, seed, reunit_every=2, history=True)
    assert np.allclose(hist, ph, atol=2e-6), (hist, ph)
    diff = np.abs(got - U).reshape(-1, 9).max(axis=1)
    assert np.mean(diff > TOL3) < 0.02, np.mean(diff > TOL3)
    assert plaq == pytest.approx(o3.plaquette(dims, U), abs=2e-6)
    assert plaq == pytest.approx(hist[-1], abs=1e-6)  # no reunitarisation after sweep 3
    want = o3.polyakov(dims, U)
    assert np.allclose(poly, want, atol=5e-6), (poly, want)


def test_su3_fused_plaquette_equals_standalone(su2):
    dims = [8, 8, 8, 8]
    announce("su3 fused vs standalone plaquette")
    with su2.Lattice3(dims, 6.0, 5, su2.SU2_HOT) as lat:
        h = lat.heatbath_sweep(4, history=True)
        assert h[-1] == pytest.approx(lat.plaquette(), abs=1e-6)
        assert np.all(np.diff(h) > 0)  # ordering from a hot start at beta = 6


def test_su3_links_stay_unitary_without_reunitarisation(su2):
    """Only rows 0 and 1 are stored and the subgroup rotations mix the rebuilt
    row 2 back into them, so an unnormalised FP32 update would let deviations
    from unitarity grow from sweep to sweep.  The pass re-orthonormalises every
    link it stores: after 120 sweeps with no reunitarisation call the links are
    unitary to FP32 rounding, and the thermalised plaquette agrees with that of
    a run reunitarised after every sweep (the two chains separate after a few
    sweeps, since reunitarisation moves links by FP32 rounding, so only their
    means are compared)."""
    dims = [8, 8, 8, 8]
    announce("su3 stability without reunitarisation")
    with su2.Lattice3(dims, 6.0, 3, su2.SU2_HOT) as lat:
        h = lat.heatbath_sweep(120, reunit_every=0, history=True)
        links = lat.get_links()
    with su2.Lattice3(dims, 6.0, 3, su2.SU2_HOT) as lat:
        r = lat.heatbath_sweep(120, reunit_every=1, history=True)
    assert su3_defect(links) < 2e-6
    assert abs(h[60:].mean() - r[60:].mean()) < 3e-3, (h[60:].mean(), r[60:].mean())
    assert min(h[60:].mean(), r[60:].mean()) > 0.585


def test_su3_reunitarize_matches_oracle(su2, o3):
    dims = [4, 6, 4, 4]
    announce("su3 reunitarisation")
    rng = np.random.default_rng(12)
    links = inputs.random_su3_links(dims, 12, spread=0.4)
    links += 3e-3 * (rng.standard_normal(links.shape) + 1j * rng.standard_normal(links.shape))
    with su2.Lattice3(dims, 6.0, 1) as lat:
        lat.set_links(links)  # rows 0, 1 rounded to FP32; row 2 is not stored
        lat.reunitarize()
        got = lat.get_links()
    want = links.copy()
    o3.reunitarize(dims, want)  # Gram-Schmidt reads rows 0 and 1 only
    assert np.abs(got - want).max() < 2e-6
    assert su3_defect(got) < 2e-6


def test_su3_history_longer_than_one_chunk(su2):
    """The plaquette history of one call crosses the 1024-entry device
    history (the call copies it out in chunks) and equals that of two
    shorter calls over the same sweeps, entry for entry."""
    dims = [2, 2, 2, 2]
    announce("su3 history across the 1024-sweep chunk")
    with su2.Lattice3(dims, 5.5, 31, su2.SU2_HOT) as a:
        ha = a.heatbath_sweep(1030, reunit_every=10, history=True)
        la = a.get_links()
    with su2.Lattice3(dims, 5.5, 31, su2.SU2_HOT) as b:
        hb = np.concatenate([b.heatbath_sweep(1000, reunit_every=10, history=True),
                             b.heatbath_sweep(30, reunit_every=10, history=True)])
        assert np.array_equal(b.get_links(), la)
    assert ha.shape == (1030,) and np.array_equal(ha, hb)
    assert np.all(np.abs(ha) <= 1.0) and len(np.unique(ha[1000:])) > 20


def test_su3_set_beta_applies_to_later_sweeps(su2):
    """Sweeps after su3_set_beta are those of a lattice created at the new
    coupling from the same links and sweep index, bit for bit; sweeps before
    it are untouched by it."""
    dims = [4, 6, 4, 4]
    announce("su3 set_beta")
    with su2.Lattice3(dims, 5.0, 41, su2.SU2_HOT) as a:
        a.heatbath_sweep(2)
        mid = a.get_links()
        a.set_beta(6.2)
        a.heatbath_sweep(2)
        got = a.get_links()
    with su2.Lattice3(dims, 6.2, 41, su2.SU2_COLD) as b:
        b.set_links(mid)
        b.set_sweep(2)
        b.heatbath_sweep(2)
        assert np.array_equal(b.get_links(), got)
    with su2.Lattice3(dims, 5.0, 41, su2.SU2_HOT) as c:
        c.heatbath_sweep(2)
        assert np.array_equal(c.get_links(), mid)


def test_su3_checkpoint_and_resume_is_bitwise(su2):
    """A run stopped after a heat-bath sweep, two over-relaxation sweeps and a
    reunitarisation, saved through the host exchange (FP32 rows widened to FP64
    and rounded back exactly) and the sweep index, and resumed in a new
    context, ends bit for bit where the uninterrupted run does."""
    dims = [6, 4, 8, 6]
    announce("su3 checkpoint / resume")

    def tail(lat):
        lat.heatbath_sweep(3, reunit_every=2)
        lat.overrelax(1)
        lat.heatbath_sweep(1)

    with su2.Lattice3(dims, 5.9, 23, su2.SU2_HOT) as ref:
        ref.heatbath_sweep(1)
        ref.overrelax(2)
        ref.reunitarize()
        saved, sweep = ref.get_links(), ref.sweep
        tail(ref)
        want, want_sweep = ref.get_links(), ref.sweep
        want_p = ref.plaquette()
    assert sweep == 1 and want_sweep == 5
    with su2.Lattice3(dims, 5.9, 23, su2.SU2_COLD) as lat:
        lat.set_links(saved)
        lat.set_sweep(sweep)
        tail(lat)
        assert lat.sweep == want_sweep
        assert np.array_equal(lat.get_links(), want)
        assert lat.plaquette() == want_p


@pytest.mark.parametrize("launch", [(64, 0, 0, 1, 1), (128, 1, 1, 2, 4), (192, 1, 0, 0, 0),
                                    (256, 0, 1, 8, 8)])
def test_su3_launch_shape_does_not_change_results(su2, launch):
    """Every site's update reads only links the pass does not write, so the
    traversal (block, remap, snake, tiles) cannot change any bit."""
    dims = [8, 6, 8, 8]
    announce(f"su3 launch {launch}")
    with su2.Lattice3(dims, 5.8, 17, su2.SU2_HOT) as ref:
        ref.heatbath_sweep(2)
        want = ref.get_links()
    with su2.Lattice3(dims, 5.8, 17, su2.SU2_HOT) as lat:
        lat.set_launch(*launch)
        lat.heatbath_sweep(2)
        assert np.array_equal(lat.get_links(), want)


def test_su3_ensemble_matches_oracle_chains(su2, o3):
    """Mean plaquette at beta = 6.0 on 6^4 from 8 GPU chains against 4 oracle
    chains (independent seeds, 100 thermalisation sweeps from cold, 200
    measured sweeps, reunitarisation every 10); each side's error is the spread
    of its chain means, which also covers slow modes a batch-means error
    within one chain would miss."""
    dims, beta, therm, nmeas = [6, 6, 6, 6], 6.0, 100, 200
    announce("su3 ensemble vs oracle")
    g = []
    for r in range(8):
        with su2.Lattice3(dims, beta, 600 + r, su2.SU2_COLD) as lat:
            h = lat.heatbath_sweep(therm + nmeas, reunit_every=10, history=True)
            g.append(h[therm:].mean())
    o = []
    for r in range(4):
        U = o3.init(dims, 0, 0)
        ph, _ = o3.sweeps(dims, U, therm + nmeas, 0, beta, 700 + r, reunit_every=10,
                          nthreads=8, history=True)
        o.append(ph[therm:].mean())
    g, o = np.array(g), np.array(o)
    dg, do = g.std(ddof=1) / np.sqrt(len(g)), o.std(ddof=1) / np.sqrt(len(o))
    pull = (g.mean() - o.mean()) / np.hypot(dg, do)
    announce(f"  gpu {g.mean():.5f}({dg:.5f}) oracle {o.mean():.5f}({do:.5f}) pull {pull:.2f}")
    assert abs(pull) < 4


def test_su3_full_size_pass_sampled_against_oracle(su2, o3):
    """48^4 at beta = 6.0 (the benchmarked workload, default launch) from the
    oracle's own Haar configuration, given to the GPU: its plaquette and
    Polyakov loop against the oracle's, then one odd pass of mu = 2 and 3000
    sampled updated sites recomputed by the oracle from that configuration."""
    dims, beta, seed = [48, 48, 48, 48], 6.0, 2010
    announce("su3 full-size 48^4 sampled pass")
    pre = o3.init(dims, 1, 77)
    sweep = 3
    with su2.Lattice3(dims, beta, seed) as lat:
        lat.set_links(pre)
        lat.set_sweep(sweep)
        plaq, poly = lat.plaquette(), lat.polyakov()
        lat.test_pass(2, 1)
        post = lat.get_links()
    # observables of the 48^4 field against the oracle's on the same links
    assert plaq == pytest.approx(o3.plaquette(dims, pre), abs=1e-7)
    assert np.allclose(poly, o3.polyakov(dims, pre), atol=1e-7)
    par_of = parities(dims)
    odd = np.nonzero(par_of == 1)[0]
    rng = np.random.default_rng(1)
    sites = rng.choice(odd, 3000, replace=False)
    flagged, worst = 0, 0.0
    for s in sites:
        A = o3.staple(dims, pre, s, 2)
        want, m = o3.heatbath_link(pre[s, 2], A, beta, seed, int(s), sweep, 2)
        if m < FLAG3:
            flagged += 1
            continue
        worst = max(worst, np.abs(post[s, 2] - want).max())
    announce(f"  max |gpu - oracle| = {worst:.2e}, flagged {flagged}")
    assert worst < TOL3
    assert flagged <= max_flags3(3000)
    assert np.abs(post[par_of == 0] - pre[par_of == 0]).max() < 1e-6  # FP32 storage only


def test_su3_argument_errors(su2):
    """Bad arguments on a live context are refused with SU2_EINVAL before any
    device work, and the context stays usable."""
    announce("su3 argument errors")
    with su2.Lattice3([4, 4, 4, 4], 6.0, 1, su2.SU2_COLD) as lat:
        for call in (lambda: lat.set_launch(96), lambda: lat.set_launch(256, 1, 1, 3, 0),
                     lambda: lat.test_pass(4, 0), lambda: lat.test_pass(0, 2),
                     lambda: lat.heatbath_sweep(-1), lambda: lat.heatbath_sweep(1, -2),
                     lambda: lat.set_beta(float("nan")), lambda: lat.overrelax(-2),
                     lambda: lat.test_read_links([256], 0), lambda: lat.test_read_links([0], 4)):
            with pytest.raises(su2.SU2Error) as e:
                call()
            assert e.value.code == su2.SU2_EINVAL
        # empty work: nothing changes, the sweep index stays
        before = lat.get_links()
        assert lat.heatbath_sweep(0, history=True).size == 0
        lat.heatbath_sweep(0)
        lat.overrelax(0)
        assert lat.sweep == 0 and np.array_equal(lat.get_links(), before)
        lat.heatbath_sweep(1)
        assert 0.0 < lat.plaquette() < 1.0


def test_su3_deconfinement_at_nt4(su2):
    """Physics beyond the oracle comparison: on 12^3 x 4 the centre symmetry is
    restored below the deconfinement coupling (beta_c = 5.69 for N_t = 4) and
    broken above it, so <|mean Polyakov loop|> is several times larger at
    beta = 5.9 than at beta = 5.5 (it falls like 1/sqrt(N_s^3) in the confined
    phase)."""
    announce("su3 deconfinement 12^3 x 4")
    absL = {}
    for b in (5.5, 5.9):
        with su2.Lattice3([12, 12, 12, 4], b, 77, su2.SU2_COLD) as lat:
            lat.heatbath_sweep(200, reunit_every=10)
            v = []
            for _ in range(100):
                lat.heatbath_sweep(2, reunit_every=10)
                re, im, _ = lat.polyakov()
                v.append(abs(complex(re, im)))
            absL[b] = float(np.mean(v))
    announce(f"  <|L|> beta 5.5: {absL[5.5]:.4f}, beta 5.9: {absL[5.9]:.4f}")
    assert absL[5.9] > 4 * absL[5.5]
    assert absL[5.5] < 0.1


@pytest.mark.parametrize("dims,spread", [([2, 2, 2, 2], None), ([4, 4, 4, 4], None),
                                         ([6, 6, 6, 10], 0.3)],
                         ids=["2^4-haar", "4^4-haar", "6^3x10-ordered"])
def test_su3_overrelaxation_pass_matches_oracle(su2, o3, dims, spread):
    """Every (mu, parity) over-relaxation pass from the same seeded links on
    both sides (deterministic: no decisions to flag)."""
    announce(f"su3 over-relaxation pass parity dims={dims}")
    links = inputs.random_su3_links(dims, 60 + sum(dims), spread=spread)
    par_of = parities(dims)
    worst = 0.0
    with su2.Lattice3(dims, 6.0, 1) as lat:
        for mu in range(4):
            for p in range(2):
                lat.set_links(links)
                lat.test_or_pass(mu, p)
                got = lat.get_links()
                U = links.copy()
                o3.or_pass(dims, U, mu, p)
                upd = par_of == p
                worst = max(worst, float(np.abs(got[upd, mu] - U[upd, mu]).max()))
                assert np.abs(got[upd, mu] - links[upd, mu]).max() > 0.05
    announce(f"  max |gpu - oracle| = {worst:.2e}")
    assert worst < 1e-5


def test_su3_overrelaxation_keeps_the_action(su2):
    """Over-relaxation sweeps leave every link's Re Tr(U A), hence the
    plaquette, unchanged (to FP32 rounding) while moving the links by O(1); the
    sweep index does not advance."""
    announce("su3 over-relaxation keeps the action")
    dims = [8, 8, 8, 8]
    with su2.Lattice3(dims, 6.0, 4, su2.SU2_HOT) as lat:
        lat.heatbath_sweep(20, reunit_every=10)
        p0, before, sw = lat.plaquette(), lat.get_links(), lat.sweep
        lat.overrelax(3)
        assert abs(lat.plaquette() - p0) < 1e-6
        assert np.abs(lat.get_links() - before).max() > 0.5
        assert lat.sweep == sw
        with pytest.raises(su2.SU2Error):
            lat.overrelax(-1)


def test_su3_heatbath_with_overrelaxation_matches_oracle_chains(su2, o3):
    """Chains of one heat-bath and three over-relaxation sweeps (8 on the GPU)
    against the oracle's heat-bath chains (4): the same equilibrium plaquette at
    beta = 6.0 on 6^4 (100 + 200 groups, reunitarisation every 10)."""
    dims, beta, therm, nmeas = [6, 6, 6, 6], 6.0, 100, 200
    announce("su3 heat bath + over-relaxation vs oracle")
    g = []
    for r in range(8):
        with su2.Lattice3(dims, beta, 800 + r, su2.SU2_COLD) as lat:
            h = []
            for i in range(therm + nmeas):
                h.append(lat.heatbath_sweep(1, reunit_every=10, history=True)[0])
                lat.overrelax(3)
            g.append(np.mean(h[therm:]))
    o = []
    for r in range(4):
        U = o3.init(dims, 0, 0)
        ph, _ = o3.sweeps(dims, U, therm + nmeas, 0, beta, 900 + r, reunit_every=10,
                          nthreads=8, history=True)
        o.append(ph[therm:].mean())
    g, o = np.array(g), np.array(o)
    dg, do = g.std(ddof=1) / np.sqrt(len(g)), o.std(ddof=1) / np.sqrt(len(o))
    pull = (g.mean() - o.mean()) / np.hypot(dg, do)
    announce(f"  gpu HB+3OR {g.mean():.5f}({dg:.5f}) oracle HB {o.mean():.5f}({do:.5f}) "
             f"pull {pull:.2f}")
    assert abs(pull) < 4


def test_su3_graph_replay_equals_direct_sweeps(su2):
    """Heat-bath sweeps recorded as a graph (su3_capture_sweeps, fused plaquette
    into a device history, reunitarisation every second sweep) and replayed
    three times with eager work between the replays give the links and
    plaquettes of the same sweeps run directly, bit for bit; replays past the
    history rows or off a reunitarisation boundary are refused, a coupling
    change drops the recording, and a recording without measurements replays
    like direct sweeps too."""
    import torch
    announce("su3 graph replay == direct")
    dims = [8, 6, 4, 8]
    side = torch.cuda.Stream()  # capture needs a non-null stream
    with torch.cuda.stream(side):
        with su2.Lattice3(dims, 5.8, 61, su2.SU2_HOT) as a, \
                su2.Lattice3(dims, 5.8, 61, su2.SU2_HOT) as g:
            ha = a.heatbath_sweep(12, reunit_every=2, history=True)
            hg = torch.full((12,), -1.0, dtype=torch.float64, device="cuda")
            with pytest.raises(su2.SU2Error) as e:
                g.capture(3, reunit_every=2, hist=hg)  # not whole periods
            assert e.value.code == su2.SU2_EINVAL
            g.capture(4, reunit_every=2, hist=hg)
            for k in range(3):
                g.replay(1)
                g.synchronize()
                assert g.sweep == 4 * (k + 1)
                _ = g.plaquette()  # eager work between the replays
            np.testing.assert_array_equal(hg.cpu().numpy(), ha)
            np.testing.assert_array_equal(g.get_links(), a.get_links())
            with pytest.raises(su2.SU2Error) as e:
                g.replay(1)  # would write rows 12..15 of 12
            assert e.value.code == su2.SU2_EINVAL
            g.set_sweep(13)
            with pytest.raises(su2.SU2Error) as e:
                g.replay(1)  # sweep 13 is not a period boundary
            assert e.value.code == su2.SU2_ESTATE
            g.set_beta(5.9)
            g.set_sweep(14)
            with pytest.raises(su2.SU2Error) as e:
                g.replay(1)  # dropped by the coupling change
            assert e.value.code == su2.SU2_ESTATE
            before = g.get_links()
            np.testing.assert_array_equal(before, a.get_links())  # nothing ran
        with su2.Lattice3(dims, 6.1, 62, su2.SU2_HOT) as a, \
                su2.Lattice3(dims, 6.1, 62, su2.SU2_HOT) as g:
            a.heatbath_sweep(6)
            g.capture(2)
            g.replay(3)
            g.synchronize()
            assert g.sweep == 6
            np.testing.assert_array_equal(g.get_links(), a.get_links())
    torch.cuda.synchronize()
