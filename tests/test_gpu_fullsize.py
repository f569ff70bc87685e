"""Parity at the full 48^4 size (beta 6.0), in the launch configuration the
autotuner picks, which is the one the throughput benchmark times; also a
persistent (grid-stride) launch.

The oracle cannot redo many 48^4 sweeps in seconds, so single passes are
checked on sampled links, each recomputed by the oracle (staple, k, exact
sampler, direction, U' = X U~^+; Sec. 2) from the same seeded configuration the
GPU pass started from; the fused sweep measurements are checked against the
standalone kernels after the sweep, the standalone kernels against the oracle
on the seeded configuration, and the whole sweep against the oracle's sweep of
that configuration.  Inputs reach the oracle only from the seeded generator."""
import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import MARGIN_FLAG, announce, max_flags

pytestmark = pytest.mark.gpu

DIMS, BETA, SEED = [48, 48, 48, 48], 6.0, 3
NSAMPLE = 6000


def sample_sites(orc, par, n, seed):
    """n distinct sites of parity `par` (half the sites of each parity lie on
    even x + y + z + t), including the first and last of that parity."""
    V = int(np.prod(DIMS))
    rng = np.random.default_rng(seed)
    s = rng.choice(V, size=3 * n, replace=False)
    s = s[[orc.parity(DIMS, int(x)) == par for x in s]][:n]
    ends = [x for x in (0, 1, V - 2, V - 1) if orc.parity(DIMS, x) == par]
    return np.unique(np.concatenate([s, ends]))


def staple_norms_at_update(orc, links, sweep, mask):
    """k = |V| of each link in mask ((V, 4) booleans, row-major order) when the
    oracle's sweep from `links` updates it: the passes are replayed in sweep
    order and each link's staple is taken just before its pass."""
    U = links.astype(np.float64)
    idx = [(int(s), int(m)) for s, m in np.argwhere(mask)]
    k = {}
    for mu in range(4):
        for p in range(2):
            for s, m in idx:
                if m == mu and orc.parity(DIMS, s) == p:
                    k[(s, m)] = float(np.linalg.norm(orc.staple(DIMS, U, s, mu)))
            orc.do_pass(DIMS, U, mu, p, sweep, BETA, SEED, order=3)
    return np.array([k[i] for i in idx])


def check_pass(lat, orc, links, U, mu, par, seed):
    """One pass from the seeded configuration `links` (U: the same in FP64)."""
    lat.set_links(links)
    sweep = lat.sweep
    lat.test_pass(mu, par)
    got = lat.get_links()
    # links outside the pass are untouched, bit for bit
    changed = np.any(got != links, axis=2)
    assert not changed[:, [m for m in range(4) if m != mu]].any()
    sites = sample_sites(orc, par, NSAMPLE, seed)
    nflag, worst = 0, 0.0
    for s in sites:
        s = int(s)
        V = orc.staple(DIMS, U, s, mu)
        want, m = orc.heatbath_link(V, BETA, SEED, s, sweep, mu)
        if m < MARGIN_FLAG:
            nflag += 1
            continue
        worst = max(worst, float(np.abs(got[s, mu] - want).max()))
    assert worst < 1e-5, (mu, par, worst)
    assert nflag <= max_flags(len(sites))
    # every link of the pass's parity and direction changed (p(unchanged) ~ 0)
    par_of = (np.indices(DIMS[::-1]).sum(axis=0).ravel() & 1)
    assert changed[par_of == par, mu].mean() > 0.999
    return worst


def test_full_size_passes_autotuned_and_persistent(su2, orc):
    announce("48^4 sampled pass parity (autotuned launch)")
    links = inputs.random_links(DIMS, 31, spread=0.6)
    U = links.astype(np.float64)
    with su2.Lattice(DIMS, BETA, SEED, su2.SU2_HOT) as lat:
        lat.autotune()
        print(f"[gpu-test] launch {lat.launch()}", flush=True)
        lat.set_sweep(2)
        for mu in range(4):
            for par in range(2):
                w = check_pass(lat, orc, links, U, mu, par, 100 + 2 * mu + par)
                print(f"[gpu-test] pass ({mu},{par}) max err {w:.2e}", flush=True)
        announce("48^4 sampled pass parity (persistent grid)")
        lat.set_launch(256, 1, 8, 8, 2048)
        for mu, par in ((1, 1), (2, 0)):
            w = check_pass(lat, orc, links, U, mu, par, 200 + mu)
            print(f"[gpu-test] pass ({mu},{par}) max err {w:.2e}", flush=True)


@pytest.mark.parametrize("fused", [False, True], ids=["sweep0", "reunit-sweep-fused"])
def test_full_size_sweep_measurements(su2, orc, fused):
    """sweep0: sweep 0 (no reunitarisation).  reunit-sweep-fused: sweep 9 with
    reunit_every 10 and the reunitarisation fused into the passes, as the
    benchmark runs it; the oracle reunitarises after its sweep, and every link
    must come out unit to FP32 rounding."""
    announce(f"48^4 fused sweep measurements fused_reunit={fused}")
    sweep0 = 9 if fused else 0
    links = inputs.random_links(DIMS, 32, spread=0.6)
    U = links.astype(np.float64)
    p0 = orc.plaquette(DIMS, U)
    ls0, la0 = orc.polyakov(DIMS, U)
    with su2.Lattice(DIMS, BETA, SEED, su2.SU2_HOT) as lat:
        lat.autotune()
        lat.set_reunit_fused(fused)
        lat.set_links(links)
        lat.set_sweep(sweep0)
        # standalone kernels on the seeded configuration
        assert abs(lat.plaquette() - p0) < 1e-6
        s, a = lat.polyakov()
        assert abs(s - ls0) < 1e-6 and abs(a - la0) < 1e-6
        hist = lat.sweep_measure(1, reunit_every=10,
                                 meas=su2.SU2_MEAS_PLAQ | su2.SU2_MEAS_POLY).cpu().numpy()
        got = lat.get_links()
        # the fused measurements equal the standalone kernels on the swept links
        assert abs(hist[0, 0] - lat.plaquette()) < 1e-6
        s, a = lat.polyakov()
        assert abs(hist[0, 1] - s) < 1e-6 and abs(hist[0, 2] - a) < 1e-6
    n2 = np.einsum("vmc,vmc->vm", got.astype(np.float64), got.astype(np.float64))
    assert np.abs(n2 - 1).max() < (3e-7 if fused else 1e-5)
    # the oracle's sweep of the same configuration (all host threads), with the
    # margin of every accept decision it took
    ph, lh, margin = orc.sweeps(DIMS, U, 1, sweep0, BETA, SEED, reunit_every=10, nthreads=16,
                                measure=True, want_margin=True)
    off = np.abs(got - U).max(axis=2) > 1e-5
    nbad = int(off.sum())
    nflag = int((margin < MARGIN_FLAG).sum())
    V = int(np.prod(DIMS))
    print(f"[gpu-test] links off by > 1e-5 after the sweep: {nbad} of {4 * V}; decisions "
          f"within {MARGIN_FLAG} of their threshold: {nflag}; plaquette {hist[0, 0]:.9f} vs "
          f"oracle {ph[0]:.9f}, Polyakov {hist[0, 1]:.3e} vs {lh[0]:.3e}", flush=True)
    # Only a decision the oracle takes within MARGIN_FLAG of its threshold may
    # flip in FP32.  A flipped decision changes its link by O(1) and, through
    # the staples, links updated after it in the same sweep (fewer than 500
    # within the seven passes that follow).  With no flagged decision every
    # link matches.
    assert nflag <= max_flags(4 * V)
    dev = np.abs(got - U).max(axis=2)
    moved = dev > 1e-3  # flipped decisions and the links updated after them
    assert int(moved.sum()) <= 500 * nflag, (int(moved.sum()), nflag)
    if moved.any():
        # every mismatched cone starts at a flagged decision of its own sweep
        assert (moved & (margin < MARGIN_FLAG)).any()
    lone = off & ~moved
    if lone.any():
        # U~ = V/k carries the FP32 error of the staple sum V (a few 1e-6
        # absolute over six products of unit quaternions) divided by k, so a
        # link whose staple nearly cancels can miss 1e-5 without any decision
        # moving: each such link's k at its update (the oracle's staple, pass
        # by pass from the seeded links) must explain its deviation
        ks = staple_norms_at_update(orc, links, sweep0, lone)
        d = dev[lone]
        print(f"[gpu-test] links off by 1e-5..1e-3: deviation {d.tolist()}, k at the update "
              f"{ks.tolist()}, margins {margin[lone].tolist()}", flush=True)
        assert int(lone.sum()) <= 20
        assert np.all(d * ks < 5e-6), (d, ks)
    # each changed link moves its six plaquettes and one Polyakov line by O(1)
    assert abs(hist[0, 0] - ph[0]) < 1e-6 + 6.0 * nbad / (6 * V)
    assert abs(hist[0, 1] - lh[0]) < 1e-6 + 2.0 * nbad / (V // DIMS[3])


def test_full_size_learned_pass(su2, orc):
    """The learned Metropolis pass at 48^4 in its autotuned launch, on sampled
    links of a seeded configuration (a random network, so proposals are
    accepted, rejected and, for alpha outside the table range, replaced by the
    exact sampler)."""
    from tests.gpu_util import learned_flagged, max_learned_flags
    announce("48^4 sampled learned pass parity")
    p = (np.random.default_rng(12).standard_normal(orc.NN_NPARAM) * 0.2).astype(np.float32)
    table = orc.nn_table(p)
    links = inputs.random_links(DIMS, 33, spread=0.6)
    U = links.astype(np.float64)
    with su2.NN(params=p) as net, su2.Lattice(DIMS, BETA, SEED, su2.SU2_HOT) as lat:
        net.build_table()
        lat.set_proposal(net)
        lat.autotune(None, su2.SU2_LEARNED)
        lat.set_links(links)
        lat.set_sweep(2)
        lat.test_pass(1, 0, su2.SU2_LEARNED)
        got = lat.get_links()
        sites = sample_sites(orc, 0, NSAMPLE, 300)
        nflag, kinds, worst = 0, {-1: 0, 0: 0, 1: 0}, 0.0
        for s in sites:
            s = int(s)
            V = orc.staple(DIMS, U, s, 1)
            want, m, a = orc.learned_link(V, U[s, 1], table, BETA, SEED, s, 2, 1)
            if learned_flagged(m)[0]:
                nflag += 1
                continue
            kinds[a] += 1
            worst = max(worst, float(np.abs(got[s, 1] - want).max()))
        print(f"[gpu-test] learned pass max err {worst:.2e}, outcomes {kinds}", flush=True)
        assert worst < 1e-5
        assert nflag <= max_learned_flags(len(sites))
        assert kinds[0] > 0 and kinds[1] > 0


@pytest.mark.parametrize("workload", ["beta_scan_16", "beta_scan_24", "polyakov", "replicas64"])
def test_batched_workload_in_autotuned_launch(su2, orc, workload):
    """Each batched benchmark workload at its full size, in the launch the
    autotuner picks for it (per-pass, XCD-affine, work queue or persistent, as
    the benchmark times it): after one sweep from the batch's hot start, sampled
    replicas equal the oracle's sweep of the same replica (replica id, beta,
    seed) within 1e-5 per link component.  A decision the oracle takes within
    2e-5 of its threshold may flip in FP32 and then also changes the links it
    feeds later in the sweep, so each flagged decision may account for a few
    hundred mismatched links; without flagged decisions every link matches."""
    import bench
    announce(f"full-size batch {workload}, autotuned launch")
    dims, betas, starts, seed, pick = {
        "beta_scan_16": (*bench._beta_scan(16), 1000, [0, 9, 20, 31]),
        "beta_scan_24": (*bench._beta_scan(24), 1000, [3, 30]),
        "polyakov": (*bench._polyakov_grid(), 4000, [0, 14, 38]),
        "replicas64": (*bench._replicas64(), 5, [0, 1, 2, 7, 8, 9, 16, 6]),
    }[workload]
    n = len(dims)
    starts = np.broadcast_to(np.asarray(starts), (n,))
    with su2.Batch(dims, betas, starts, seed) as b:
        b.autotune(None, su2.SU2_KP)
        launch = b.launch()
        b.sweep(1)
        got = {r: b.get_links(r) for r in pick}
    for r in pick:
        d = dims[r]
        U = orc.init(d, int(starts[r]), seed, replica=r)
        nflag = 0
        for mu in range(4):
            for p in range(2):
                m = orc.do_pass(d, U, mu, p, 0, float(betas[r]), seed, replica=r,
                                want_margin=True)
                nflag += int((m < MARGIN_FLAG).sum())
        bad = int((np.abs(got[r] - U).max(axis=2) > 1e-5).sum())
        assert bad <= 500 * nflag, (workload, r, launch, bad, nflag)
        assert bad < 0.01 * U.shape[0] * 4, (workload, r, launch, bad)
