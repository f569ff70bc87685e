"""GPU heat bath vs the FP64 CPU oracle from identical inputs (through the C ABI).

Inputs reach the oracle only from the seeded generators (tests/inputs.py) or the
oracle's own hot start; the GPU's links are only ever compared, never fed to
the oracle.

Link-level parity holds because both sides draw the same Philox streams and
follow the same sampler; FP32-vs-FP64 can flip only decisions whose margin is
below the flag threshold, which are excluded and counted (expected ~1e-6 per
decision).  Tolerance: 1e-5 absolute per link component.
"""
import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import MARGIN_FLAG, announce, compare_pass, max_flags, parities

pytestmark = pytest.mark.gpu

DIMS = [[2, 2, 2, 2], [4, 4, 4, 4], [4, 6, 2, 8], [8, 6, 8, 10], [12, 10, 8, 6]]


def test_philox_bitwise(su2, orc):
    announce("philox bitwise")
    rng = np.random.default_rng(1)
    ctr = rng.integers(0, 2 ** 32, (5000, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:3] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [5308415, 1999, 0x1C3, 7]]
    for seed in (0, 1, 2 ** 64 - 1, 0xDEADBEEF12345678):
        np.testing.assert_array_equal(su2.su2_test_philox(ctr, seed), orc.philox(ctr, seed))


def test_single_link_updates(su2, orc):
    announce("single-link heat bath vs oracle")
    V = inputs.random_staples(20000, 3, kmin=0.01, kmax=6.0)
    V[:3] = 0.0  # k = 0: Haar
    beta = 2.3
    got, ntr = su2.su2_test_heatbath_links(V, beta, 17, 9, 2, replica=5, want_trials=True)
    nflag = 0
    for i in range(V.shape[0]):
        want, m = orc.heatbath_link(V[i].astype(np.float64), beta, 17, i, 9, 2, 5)
        if m < MARGIN_FLAG:
            nflag += 1
            continue
        assert np.abs(got[i] - want).max() < 1e-5, (i, got[i], want, m)
    _, otr, om = orc.sample_delta(beta * np.linalg.norm(V.astype(np.float64), axis=1), 17,
                                  np.arange(V.shape[0], dtype=np.uint32), 9, 2, 5)
    keep = om >= MARGIN_FLAG
    np.testing.assert_array_equal(ntr[keep], otr[keep])
    assert nflag <= max_flags(V.shape[0])


@pytest.mark.parametrize("dims", DIMS, ids=lambda d: "x".join(map(str, d)))
def test_every_pass_matches_oracle(su2, orc, dims):
    """Each of the eight (mu, parity) passes from the same seeded links on
    both sides."""
    announce(f"per-pass parity dims={dims}")
    links = inputs.random_links(dims, 10 + sum(dims), spread=0.6)
    beta, seed = 2.4, 12345
    par_of = parities(orc, dims)
    with su2.Lattice(dims, beta, seed) as lat:
        lat.set_sweep(3)
        total_flag = 0
        for mu in range(4):
            for p in range(2):
                lat.set_links(links)
                U = links.astype(np.float64)
                margin = orc.do_pass(dims, U, mu, p, 3, beta, seed, want_margin=True)
                lat.test_pass(mu, p)
                got = lat.get_links()
                err, nflag = compare_pass(got, U, margin, p, mu, par_of)
                total_flag += nflag
                assert err < 1e-5, (mu, p, err)
                # everything else untouched, bit for bit
                mask = np.ones(got.shape[:2], bool)
                mask[par_of == p, mu] = False
                np.testing.assert_array_equal(got[mask], links[mask])
        assert total_flag <= max_flags(4 * int(np.prod(dims)))


@pytest.mark.parametrize("beta", [0.0, 60.0], ids=["beta0-haar", "beta60"])
def test_pass_at_extreme_couplings(su2, orc, beta):
    """The degenerate couplings: beta = 0 (alpha = 0 at every site, so every
    updated link is Haar-random: only the alpha < 1 branch, which then accepts
    every trial) and beta = 60 (alpha up to ~400: Kennedy-Pendleton with
    1 - a0 ~ 1e-3), every pass from the same seeded links on both sides."""
    dims = [4, 6, 2, 8]
    announce(f"per-pass parity at beta={beta}")
    links = inputs.random_links(dims, 77, spread=0.6)
    seed = 4711
    par_of = parities(orc, dims)
    with su2.Lattice(dims, beta, seed) as lat:
        lat.set_sweep(11)
        total_flag = 0
        for mu in range(4):
            for p in range(2):
                lat.set_links(links)
                U = links.astype(np.float64)
                margin = orc.do_pass(dims, U, mu, p, 11, beta, seed, want_margin=True)
                lat.test_pass(mu, p)
                got = lat.get_links()
                err, nflag = compare_pass(got, U, margin, p, mu, par_of)
                total_flag += nflag
                assert err < 1e-5, (mu, p, err)
                upd = got[par_of == p, mu].astype(np.float64)
                assert np.abs((upd ** 2).sum(axis=1) - 1.0).max() < 2e-6
        assert total_flag <= max_flags(4 * int(np.prod(dims)))


@pytest.mark.parametrize("dims", [[4, 4, 4, 4], [4, 6, 2, 8]], ids=lambda d: "x".join(map(str, d)))
def test_hot_start_and_sweeps_match_oracle(su2, orc, dims):
    """Config-1 style: the hot start (Philox seed 1) against the oracle's; then
    twelve whole sweeps at beta 2.3, sweep index sw, each from a fresh seeded
    configuration given to both sides (the eight passes of a sweep chain on
    each side independently)."""
    announce(f"hot start + sweeps dims={dims}")
    beta, seed = 2.3, 1
    with su2.Lattice(dims, beta, seed, su2.SU2_HOT) as lat:
        np.testing.assert_allclose(lat.get_links(), orc.init(dims, 1, seed), atol=2e-6, rtol=0)
        skipped = 0
        for sw in range(12):
            links = inputs.random_links(dims, 500 + sw)
            U = links.astype(np.float64)
            margins = [orc.do_pass(dims, U, mu, p, sw, beta, seed, want_margin=True)
                       for mu in range(4) for p in range(2)]
            lat.set_links(links)
            lat.set_sweep(sw)
            lat.heatbath_sweep(1)
            got = lat.get_links()
            if min(np.min(m) for m in margins) < MARGIN_FLAG:
                skipped += 1
                continue
            assert np.abs(got - U).max() < 1e-5, sw
        assert skipped <= 3
        assert lat.sweep == 12


def test_plaquette_history_config1(su2, orc):
    """4^4, hot start seed 1, beta 2.3: the GPU's and the oracle's trajectories
    from their own hot starts (the same Philox recipe), run side by side for 20
    sweeps with the plaquette and Polyakov loop measured every sweep (fused into
    the GPU's passes).  The two starts differ by FP32 rounding (~1e-6) and the
    dynamics amplifies a difference by about 1.5x per sweep, so the chains are
    compared while their links agree within 1e-3 and until the oracle meets a
    decision within the flag margin: links, plaquette and Polyakov loop
    sweep by sweep (the observables within 1e-6 plus a tenth of the link
    difference); at least the first 10 sweeps must be compared."""
    announce("config-1 plaquette history")
    dims, beta, seed = [4, 4, 4, 4], 2.3, 1
    U = orc.init(dims, 1, seed)
    compared = 0
    with su2.Lattice(dims, beta, seed, su2.SU2_HOT) as lat:
        for sw in range(20):
            m = min(float(np.min(orc.do_pass(dims, U, mu, p, sw, beta, seed, want_margin=True)))
                    for mu in range(4) for p in range(2))
            hist = lat.sweep_measure(1, meas=su2.SU2_MEAS_PLAQ | su2.SU2_MEAS_POLY).cpu().numpy()
            if m < MARGIN_FLAG:
                break
            got = lat.get_links().astype(np.float64)
            du = float(np.abs(got - U).max())
            dp = abs(hist[0, 0] - orc.plaquette(dims, U))
            dl = abs(hist[0, 1] - orc.polyakov(dims, U)[0])
            announce(f"  sweep {sw}: max |dU| {du:.2e}, |dP| {dp:.2e}, |dL| {dl:.2e}")
            if du > 1e-3:
                break
            assert dp < 1e-6 + 0.1 * du and dl < 1e-6 + 0.1 * du, sw
            compared += 1
    assert compared >= 10, compared


def test_stream_floor_kernel_moves_the_pass_bytes(su2, orc):
    """The streaming reference of a pass writes, per half-site, the sum of the
    seven plane groups the pass reads and leaves the lattice untouched."""
    import torch
    announce("stream floor kernel")
    dims = [4, 6, 2, 8]
    V = int(np.prod(dims))
    par_of = parities(orc, dims)
    links = inputs.random_links(dims, 77)
    with su2.Lattice(dims, 2.0, 5) as lat:
        lat.set_links(links)
        before = links.astype(np.float64)
        out = torch.zeros(2 * V, dtype=torch.float32, device="cuda:0")
        for mu, p in ((0, 0), (3, 1)):
            lat.test_stream_pass(mu, p, out)
            lat.synchronize()
            got = out.cpu().numpy().reshape(V // 2, 4).sum(axis=0)
            want = before[:, [n for n in range(4) if n != mu]].sum(axis=(0, 1)) + \
                before[par_of != p, mu].sum(axis=0)
            np.testing.assert_allclose(got, want, atol=1e-3)
        np.testing.assert_array_equal(lat.get_links(), links)
    with su2.Lattice(dims, 2.0, 5, su2.SU2_COLD) as lat:
        lat.test_stream_pass(1, 0, out)
        lat.synchronize()
        o = out.cpu().numpy().reshape(V // 2, 4)
        assert np.all(o[:, 0] == 7.0) and np.all(o[:, 1:] == 0.0)
