"""Fit the single-precision erfc used by the mixed-precision pair kernels.

erfc(x) = exp(-x^2) * g(x) with g(x) = exp(x^2) erfc(x), and g is approximated as

    g(x) ~= t * P(t),   t = 1 / (1 + p x),   P a polynomial of degree DEG,

the substitution of Abramowitz & Stegun 7.1.26 (Hastings' form), here refitted
with more terms and with p tuned, so that one reciprocal, a Horner chain and the
exp(-x^2) that the force needs anyway give erfc to ~1e-8 relative on x >= 0.

The fit minimises the maximum relative error of g on [0, XMAX] by iteratively
reweighted least squares (Lawson's algorithm) against 40-digit mpmath values.
Run it to regenerate the constants printed into nb_pair.hip:

    python gen_erfc_coeffs.py
"""

import mpmath as mp
import numpy as np

P = 0.47047
DEG = 8
XMAX = 6.0


def fit(p=P, deg=DEG, xmax=XMAX, iters=60):
    mp.mp.dps = 40
    xs = np.linspace(0.0, xmax, 3001)
    g = np.array([float(mp.erfc(mp.mpf(x)) * mp.exp(mp.mpf(x) ** 2)) for x in xs])
    t = 1.0 / (1.0 + p * xs)
    A = (t[:, None] ** np.arange(1, deg + 2)[None, :]) / g[:, None]
    w = np.ones_like(xs)
    for _ in range(iters):
        sw = np.sqrt(w)
        c, *_ = np.linalg.lstsq(A * sw[:, None], sw, rcond=None)
        err = np.abs(A @ c - 1.0)
        w = w * (err + 1e-30)
        w /= w.sum()
    return c, float(np.max(np.abs(A @ c - 1.0)))


if __name__ == "__main__":
    c, e = fit()
    print(f"// p = {P}, degree {DEG}, max relative error of g on [0, {XMAX}]: {e:.2e}")
    for k, v in enumerate(c):
        print(f"constexpr float kErfcC{k} = {v:.9e}f;")
