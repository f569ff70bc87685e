"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np

# Decisions whose FP64 margin is below this may flip in FP32: the FP32 error of
# a margin is <= ~2e-6 (ln of a uniform >= 2^-24 is <= 16.6 in size, relative
# error ~1 ulp, divided by alpha >= 1), so 2e-5 leaves a 10x safety factor.
MARGIN_FLAG = 2e-5


def max_flags(n_decisions):
    """Generous bound on flagged decisions: margins have O(1) density near 0."""
    return int(10 * 2 * MARGIN_FLAG * n_decisions) + 3


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def parities(orc, dims):
    return np.array([orc.parity(dims, s) for s in range(int(np.prod(dims)))])


def compare_pass(got, want, margin, par, mu, parity_of_site, tol=1e-5):
    """Compare the links of one pass.  Returns (max error over unflagged
    updated links, number flagged).  Flagged links must still be unit."""
    upd = parity_of_site == par
    flagged = upd & (margin < MARGIN_FLAG)
    ok = upd & ~flagged
    err = np.abs(got[ok, mu] - want[ok, mu]).max() if ok.any() else 0.0
    # links not updated by the pass are bit-identical to the input
    if flagged.any():
        n = np.linalg.norm(got[flagged, mu], axis=1)
        assert np.all(np.abs(n - 1) < 1e-5)
    return err, int(flagged.sum())


# Learned-update decisions (per type, each about 10x its FP32 error): the
# Metropolis log-ratio (alpha <= 30 times an a0 error of ~1e-6), the table row
# (the row position has an FP32 error of ~1e-4 rows), the table range ends.
LEARNED_FLAGS = (3e-4, 2e-3, 3e-4)


def learned_flagged(margins):
    m = np.asarray(margins).reshape(-1, 3)
    return (m[:, 0] < LEARNED_FLAGS[0]) | (m[:, 1] < LEARNED_FLAGS[1]) | (m[:, 2] < LEARNED_FLAGS[2])


def max_learned_flags(n_updates):
    """Row rounding dominates: 2 x 2e-3 of the updates, with a 5x margin."""
    return int(5 * (2 * LEARNED_FLAGS[1] + 2 * LEARNED_FLAGS[0]) * n_updates) + 3
