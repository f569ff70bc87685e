"""Write tests/golden/sampler_moments.json from closed forms (scipy only).

Sec. 2 of the paper fixes the a0 density p(a0) ~ sqrt(1 - a0^2) exp(alpha a0)
on [-1, 1] (alpha = beta k).  Its normaliser is Z = pi I1(alpha)/alpha, so
  <a0>   = Z'/Z  = I2(alpha)/I1(alpha)
  <a0^2> = Z''/Z = 1 - 3 I2(alpha)/(alpha I1(alpha))
The exact-sampler acceptance rates are integrals of the same density:
  Kennedy-Pendleton  A = E[sqrt(1 - d/2); d < 2], d ~ Gamma(3/2, rate alpha)
  semicircle         A = exp(-alpha) 2 I1(alpha)/alpha
Strong coupling (analytic curve of the paper's plaquette figure): the
leading-order plaquette is u = I2(beta)/I1(beta).
"""
import json
import os

import numpy as np
from scipy import integrate, special

ALPHAS = [0.05, 0.3, 0.7, 0.999, 1.0, 2.0, 4.0, 8.0, 16.0, 30.0]


def main():
    rows = []
    for a in ALPHAS:
        i1, i2 = special.ive(1, a), special.ive(2, a)
        kp = integrate.quad(lambda d: np.sqrt(1 - d / 2) * np.sqrt(d) * np.exp(-a * d)
                            * a ** 1.5 / special.gamma(1.5), 0, 2, epsabs=1e-14)[0]
        sc = np.exp(-a) * 2 * special.i1(a) / a
        rows.append({"alpha": a, "mean_a0": i2 / i1, "mean_a0_sq": 1 - 3 * i2 / (a * i1),
                     "accept_kp": kp, "accept_semicircle": sc})
    strong = [{"beta": b, "u": special.ive(2, b) / special.ive(1, b)} for b in (0.25, 0.5)]
    out = {"citation": "Sec. 2 (a0 density), Fig. 5 caption (analytic plaquette curves)",
           "rows": rows, "strong_coupling": strong}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sampler_moments.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()
