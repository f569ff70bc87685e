"""Precision of every observable against the FP64 oracle, for each workload
configuration, on seeded configurations given to both sides: the links after
each (mu, parity) pass (flagged decisions excluded), the plaquette and the
Polyakov loop (signed and absolute) from the standalone kernels, the same
measurements fused into a sweep against the standalone kernels on the swept
links, and the links after reunitarisation.  Links and staples are FP32; every
global sum is FP64 (fixed point across workgroups), the reunitarisation norm
FP64.  One line per configuration reports the measured errors."""
import numpy as np
import pytest

from tests import inputs
from tests.gpu_util import announce, compare_pass, max_flags, parities

pytestmark = pytest.mark.gpu

# (name, dims, beta, seed, spread of the seeded links around the identity)
CONFIGS = [("4^4", [4, 4, 4, 4], 2.3, 1, 0.7), ("16^4", [16] * 4, 2.5, 1000, 0.6),
           ("24^4", [24] * 4, 2.0, 1001, 0.8), ("32^3x4", [32, 32, 32, 4], 2.3, 4000, 0.7),
           ("48^4", [48] * 4, 6.0, 3, 0.3)]


@pytest.mark.parametrize("name,dims,beta,seed,spread", CONFIGS, ids=[c[0] for c in CONFIGS])
def test_observable_errors_against_oracle(su2, orc, name, dims, beta, seed, spread):
    announce(f"precision {name}")
    par_of = parities(orc, dims)
    links = inputs.random_links(dims, 70 + seed, spread=spread)
    U0 = links.astype(np.float64)
    with su2.Lattice(dims, beta, seed) as lat:
        sweep = 2
        lat.set_sweep(sweep)
        worst, nflag = 0.0, 0
        for mu in range(4):
            for p in range(2):
                lat.set_links(links)
                U = U0.copy()
                margin = orc.do_pass(dims, U, mu, p, sweep, beta, seed, want_margin=True)
                lat.test_pass(mu, p)
                err, nf = compare_pass(lat.get_links(), U, margin, p, mu, par_of)
                worst, nflag = max(worst, err), nflag + nf
        assert worst < 1e-5 and nflag <= max_flags(4 * int(np.prod(dims)))
        # standalone measurements on the seeded links
        lat.set_links(links)
        p_ref = orc.plaquette(dims, U0)
        l_ref, la_ref = orc.polyakov(dims, U0)
        ls, la = lat.polyakov()
        d_ps = abs(lat.plaquette() - p_ref)
        d_ls, d_la = abs(ls - l_ref), abs(la - la_ref)
        # measurements fused into a sweep, against the standalone kernels on its result
        h = lat.sweep_measure(1, meas=su2.SU2_MEAS_PLAQ | su2.SU2_MEAS_POLY).cpu().numpy()
        l2, la2 = lat.polyakov()
        d_pf = abs(h[0, 0] - lat.plaquette())
        d_lf = max(abs(h[0, 1] - l2), abs(h[0, 2] - la2))
        # reunitarisation (FP64 norm) against the oracle's on the same (off-unit) links
        off = links * np.float32(1.003)
        lat.set_links(off)
        lat.reunitarize()
        R = lat.get_links().astype(np.float64)
        W = off.astype(np.float64)
        orc.reunitarize(dims, W)
        d_r = np.abs(R - W).max()
        d_n = np.abs(np.einsum("vmc,vmc->vm", R, R) - 1.0).max()
    print(f"\n[precision] {name} beta {beta}: links max|dU| {worst:.2e} "
          f"({nflag} flagged of {4 * int(np.prod(dims))}); plaquette standalone {d_ps:.1e} "
          f"fused {d_pf:.1e}; Polyakov signed {d_ls:.1e} abs {d_la:.1e} fused {d_lf:.1e}; "
          f"reunitarised max|dU| {d_r:.1e}, max||U|^2 - 1| {d_n:.1e}", flush=True)
    assert d_ps < 1e-6 and d_pf < 1e-6
    assert d_ls < 1e-6 and d_la < 1e-6 and d_lf < 1e-6
    assert d_r < 1e-6 and d_n < 1e-6
