"""Statistical pins of the oracle heat bath against closed forms.

- first pass from a cold start: V = 6 * 1, so each updated link is X with
  a0 ~ sqrt(1-a0^2) exp(6 beta a0) (Sec. 2 with k = 6);
- strong coupling: <P> = u + O(u^5), u = I2(beta)/I1(beta) (the analytic
  strong-coupling curve of the paper's plaquette-vs-beta figure);
- weak coupling: <P> ~ 1 - 3/(4 beta) (loose sanity bound).
"""
import numpy as np
import pytest

from tests import stats


def test_first_pass_from_cold_samples_alpha_6beta(orc):
    dims = [8, 8, 8, 8]
    beta = 0.9
    a0 = []
    for seed in range(4):
        U = orc.init(dims, 0, 0)
        orc.do_pass(dims, U, mu=0, par=0, sweep=0, beta=beta, seed=100 + seed)
        par = np.array([orc.parity(dims, s) for s in range(U.shape[0])])
        a0.append(U[par == 0, 0, 0])
    a0 = np.concatenate(a0)
    chi2, dof, p = stats.chi2_equiprobable(a0, 6 * beta, nbins=40)
    assert p > 1e-4, (chi2, dof)


@pytest.mark.parametrize("beta", [0.25, 0.5])
def test_strong_coupling_plaquette(orc, beta):
    row = [r for r in stats.golden("sampler_moments.json")["strong_coupling"]
           if r["beta"] == beta][0]
    u = row["u"]
    dims = [8, 8, 8, 8]
    U = orc.init(dims, 1, 31)
    orc.sweeps(dims, U, 10, 0, beta, 31, nthreads=4)
    ph, _ = orc.sweeps(dims, U, 120, 10, beta, 31, nthreads=4, measure=True)
    m, e = stats.mean_err(ph)
    assert abs(m - u) < 3 * e + 5 * u ** 5, (m, e, u)
    # a factor-2 error in the coupling would move <P> by ~u: far outside
    assert e < u / 20


def test_weak_coupling_plaquette(orc):
    beta = 6.0
    dims = [4, 4, 4, 4]
    U = orc.init(dims, 0, 32)
    ph, _ = orc.sweeps(dims, U, 200, 0, beta, 32, measure=True)
    m = ph[50:].mean()
    assert abs(m - (1 - 3 / (4 * beta))) < 0.01, m
