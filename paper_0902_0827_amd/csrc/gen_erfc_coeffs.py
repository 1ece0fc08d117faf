"""Fit the single-precision erfc used by the mixed-precision pair kernels.

erfc(x) = exp(-x^2) * g(x) with g(x) = exp(x^2) erfc(x), and g is approximated as

    g(x) ~= t * P(t),   t = 1 / (1 + p x),   P a polynomial of degree DEG,

the substitution of Abramowitz & Stegun 7.1.26 (Hastings' form), here refitted
with more terms and with p tuned, so that one reciprocal, a Horner chain and the
exp(-x^2) that the force needs anyway give erfc to ~1e-8 relative on x >= 0.

The fit minimises the maximum relative error of g on [0, XMAX] by iteratively
reweighted least squares (Lawson's algorithm) against 40-digit mpmath values.

The double-precision kernels use the same split, erfc(x) = exp(-x^2) g(x), with g
written as a polynomial of degree DEG64 in

    s = (x - K64) / (x + K64),

which maps [0, inf) onto [-1, 1) and makes g smooth enough in s (it tends to zero
linearly as s -> 1) that a Chebyshev interpolant of g(x(s)) at DEG64 + 1 nodes,
computed in 40-digit arithmetic and converted to monomial coefficients, gives g to
about 2e-16 relative by Horner's rule in double precision over all x >= 0.  A second
table of degree DEG64_SHORT interpolates g on x <= XMAX64_SHORT only (beta R <= 4.2,
the usual Ewald settings) to the same accuracy with six terms fewer.

Run it to regenerate the constants printed into nb_pair_math.h:

    python gen_erfc_coeffs.py          # single precision (t * P(t))
    python gen_erfc_coeffs.py --f64    # double precision (polynomial in s), both tables
"""

import mpmath as mp
import numpy as np

P = 0.47047
DEG = 8
XMAX = 6.0
K64 = 3
DEG64 = 24
DEG64_SHORT = 18
XMAX64_SHORT = 4.2


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


def g_exact(x):
    return mp.exp(x * x) * mp.erfc(x)


def fit_f64(k=K64, deg=DEG64):
    """Monomial coefficients (lowest first) of g(x(s)), x(s) = k (1 + s) / (1 - s)."""
    mp.mp.dps = 40
    k = mp.mpf(k)
    n = deg + 1
    nodes = [mp.cos(mp.pi * (j + mp.mpf(1) / 2) / n) for j in range(n)]
    vals = [g_exact(k * (1 + s) / (1 - s)) for s in nodes]
    cheb = [(2 if m else 1) * mp.fsum(vals[j] * mp.cos(mp.pi * m * (j + mp.mpf(1) / 2) / n) for j in range(n)) / n
            for m in range(n)]
    # Chebyshev -> monomial: T_0 = 1, T_1 = s, T_{m+1} = 2 s T_m - T_{m-1}
    mono = [mp.mpf(0)] * n
    t_prev, t_cur = [mp.mpf(1)], [mp.mpf(0), mp.mpf(1)]
    for m in range(n):
        tm = t_prev if m == 0 else t_cur
        if m >= 2:
            nxt = [mp.mpf(0)] + [2 * v for v in t_cur]
            for i, v in enumerate(t_prev):
                nxt[i] -= v
            t_prev, t_cur = t_cur, nxt
            tm = t_cur
        for i, v in enumerate(tm):
            mono[i] += cheb[m] * v
    return [float(v) for v in mono]


def fit_f64_short(k=K64, deg=DEG64_SHORT, xmax=XMAX64_SHORT):
    """Monomial coefficients (lowest first) of g(x(s)) interpolated at Chebyshev nodes of
    s in [-1, s(xmax)] only: the range x <= xmax that a cutoff with beta R <= xmax uses."""
    mp.mp.dps = 40
    k = mp.mpf(k)
    a, b = mp.mpf(-1), (mp.mpf(xmax) - k) / (mp.mpf(xmax) + k)
    n = deg + 1
    nodes = [(a + b) / 2 + (b - a) / 2 * mp.cos(mp.pi * (j + mp.mpf(1) / 2) / n) for j in range(n)]
    vals = [g_exact(k * (1 + s) / (1 - s)) for s in nodes]
    coef = mp.lu_solve(mp.matrix([[s ** i for i in range(n)] for s in nodes]), mp.matrix(vals))
    return [float(coef[i]) for i in range(n)]


def horner_f64(coef, x, k=K64):
    s = (x - k) / (x + k)
    acc = coef[-1]
    for v in reversed(coef[:-1]):
        acc = acc * s + v
    return acc


def check_f64(coef, xmax=30.0, n=3001):
    mp.mp.dps = 40
    worst = 0.0
    for x in np.linspace(0.0, xmax, n):
        ref = g_exact(mp.mpf(float(x)))
        worst = max(worst, float(abs((horner_f64(coef, float(x)) - ref) / ref)))
    return worst


if __name__ == "__main__":
    import sys
    if "--f64" in sys.argv:
        coef = fit_f64()
        print(f"// s = (x - {K64})/(x + {K64}), degree {DEG64}, "
              f"max relative error of g in double on [0, 30]: {check_f64(coef):.2e}")
        print("constexpr double kErfcxS[] = {")
        for v in coef:
            print(f"    {v:.17e},")
        print("};")
        short = fit_f64_short()
        print(f"// s = (x - {K64})/(x + {K64}), degree {DEG64_SHORT}, "
              f"max relative error of g in double on [0, {XMAX64_SHORT}]: "
              f"{check_f64(short, XMAX64_SHORT, 801):.2e}")
        print("constexpr double kErfcxShort[] = {")
        for v in short:
            print(f"    {v:.17e},")
        print("};")
    else:
        c, e = fit()
        print(f"// p = {P}, degree {DEG}, max relative error of g on [0, {XMAX}]: {e:.2e}")
        for k, v in enumerate(c):
            print(f"constexpr float kErfcC{k} = {v:.9e}f;")
