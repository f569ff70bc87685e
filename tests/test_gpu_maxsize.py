"""The largest lattice the library accepts: V/2 just below 2^28, where the
kernels' 32-bit byte offsets (half-site index x 16 B) are at their limit.

The oracle cannot hold this lattice in FP64 on the host, so it computes what it
needs link by link: the hot start (the same Philox recipe) and, for sampled
sites, the staple sum of the hot-start configuration and the heat-bath update
from it.  The GPU's links at the sampled sites are read from device memory.
"""
import numpy as np
import pytest

from tests.gpu_util import MARGIN_FLAG, announce, max_flags

pytestmark = pytest.mark.gpu

DIMS = [512, 512, 510, 4]  # V/2 = 267,386,880 < 2^28
BETA, SEED = 2.3, 41


def coords(s):
    s = np.asarray(s, dtype=np.int64)
    x = s % DIMS[0]
    y = (s // DIMS[0]) % DIMS[1]
    z = (s // (DIMS[0] * DIMS[1])) % DIMS[2]
    t = s // (DIMS[0] * DIMS[1] * DIMS[2])
    return x, y, z, t


def parity(s):
    x, y, z, t = coords(s)
    return (x + y + z + t) & 1


def sample_sites(n, seed):
    """Random sites plus the lattice's first and last sites and sites on every
    wrap-around face (the largest half-site offsets are at the end)."""
    V = int(np.prod(DIMS))
    rng = np.random.default_rng(seed)
    s = list(rng.integers(0, V, n))
    s += list(range(8)) + list(range(V - 8, V))
    nx, ny, nz = DIMS[0], DIMS[1], DIMS[2]
    for t in (0, DIMS[3] - 1):
        for z in (0, nz - 1):
            for y in (0, ny - 1):
                for x in (0, 1, nx - 2, nx - 1):
                    s.append(x + nx * (y + ny * (z + nz * t)))
    return np.unique(np.asarray(s, dtype=np.int64))


def test_su2_maximum_size_hot_start_pass_and_observables(su2, orc):
    import torch
    announce(f"maximum size {DIMS}: hot start, one pass, observables")
    V = int(np.prod(DIMS))
    vh = V // 2
    assert vh < 2 ** 28 and su2.su2_links_bytes(DIMS) == 64 * V
    sites = sample_sites(1500, 3)
    with su2.Lattice(DIMS, BETA, SEED, su2.SU2_HOT) as lat:
        lf = lat.links_t.view(torch.float32)

        def read(s, mu):
            base = ((mu * 2 + parity(s)) * vh + (s >> 1)) * 4
            idx = torch.as_tensor((base[:, None] + np.arange(4)).ravel(), device=lf.device)
            return lf[idx].cpu().numpy().astype(np.float64).reshape(-1, 4)

        for mu in range(4):
            want = np.array([orc.hot_link(s, mu, SEED) for s in sites])
            assert np.abs(read(sites, mu) - want).max() < 2e-6, mu
        P0 = lat.plaquette()
        lat.test_pass(2, 1)  # direction z, odd sites, sweep 0
        odd, even = sites[parity(sites) == 1], sites[parity(sites) == 0]
        got = read(odd, 2)
        nflag, worst = 0, 0.0
        for i, s in enumerate(odd):
            want, m = orc.heatbath_link(orc.hot_staple(DIMS, s, 2, SEED), BETA, SEED, int(s), 0, 2)
            if m < MARGIN_FLAG:
                nflag += 1
                continue
            worst = max(worst, float(np.abs(got[i] - want).max()))
        untouched = np.array([orc.hot_link(s, 2, SEED) for s in even])
        assert np.abs(read(even, 2) - untouched).max() < 2e-6
        P = lat.plaquette()
        Ls, La = lat.polyakov()
    announce(f"  {len(odd)} updated links: max |gpu - oracle| {worst:.2e}, flagged {nflag}; "
             f"plaquette {P0:.3e} -> {P:.3e}, Polyakov {Ls:.3e} / {La:.3e}")
    assert worst < 1e-5
    assert nflag <= max_flags(len(odd))
    # Haar start: plaquette and Polyakov loop ~ 1/sqrt(volume); the pass aligns the updated
    # links (in half of all plaquettes) with their staples; it leaves U_3 alone
    assert abs(P0) < 0.01 and 0.05 < P < 0.5
    assert abs(Ls) < 0.01 and 0 <= La < 0.01


def test_su3_maximum_size_hot_start_pass_and_observables(su2):
    """The same for SU(3) (192 B per site: 103 GB of links): hot start, one
    heat-bath pass against the SU(3) oracle's link-by-link hot start and
    staples, the untouched links, plaquette and Polyakov loop."""
    import torch
    from oracle import su3_oracle as o3
    torch.cuda.empty_cache()  # the SU(2) test's 34 GB
    announce(f"SU(3) maximum size {DIMS}: hot start, one pass, observables")
    V = int(np.prod(DIMS))
    assert V // 2 < 2 ** 28
    beta, seed = 6.0, 43
    flag3, tol3 = 2e-4, 1e-4
    sites = sample_sites(600, 5)
    with su2.Lattice3(DIMS, beta, seed, su2.SU2_HOT) as lat:
        for mu in range(4):
            want = np.array([o3.hot_link(s, mu, seed) for s in sites])
            assert np.abs(lat.test_read_links(sites, mu) - want).max() < 2e-5, mu
        P0 = lat.plaquette()
        lat.test_pass(2, 1)
        odd, even = sites[parity(sites) == 1], sites[parity(sites) == 0]
        got = lat.test_read_links(odd, 2)
        nflag, worst = 0, 0.0
        for i, s in enumerate(odd):
            want, m = o3.heatbath_link(o3.hot_link(s, 2, seed), o3.hot_staple(DIMS, s, 2, seed),
                                       beta, seed, int(s), 0, 2)
            if m < flag3:
                nflag += 1
                continue
            worst = max(worst, float(np.abs(got[i] - want).max()))
        untouched = np.array([o3.hot_link(s, 2, seed) for s in even])
        assert np.abs(lat.test_read_links(even, 2) - untouched).max() < 2e-5
        P = lat.plaquette()
        re, im, mag = lat.polyakov()
    announce(f"  {len(odd)} updated links: max |gpu - oracle| {worst:.2e}, flagged {nflag}; "
             f"plaquette {P0:.3e} -> {P:.3e}, Polyakov ({re:.2e}, {im:.2e}), mean |L| {mag:.3f}")
    assert worst < tol3
    assert nflag <= int(60 * flag3 * len(odd)) + 3
    assert abs(P0) < 0.01 and 0.01 < P < 0.5
    # U_3 untouched: Haar lines of length 4, <|Tr L / 3|> ~ 0.29 per site, mean ~ 0
    assert abs(re) < 0.01 and abs(im) < 0.01 and 0.2 < mag < 0.4
