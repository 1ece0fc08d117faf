"""The erfc approximations compiled into the pair kernels, checked on the CPU against
40-digit mpmath values: the coefficient tables are read from the kernel header itself.

erfc(x) = exp(-x^2) g(x), g(x) = exp(x^2) erfc(x); the real-space Ewald term of
section 3 needs erfc(beta r) for 0 <= beta r <= beta R (about 3 here)."""

import os
import re

import mpmath as mp
import numpy as np
import pytest

HDR = os.path.join(os.path.dirname(__file__), "..", "paper_0902_0827_amd", "csrc", "nb_pair_math.h")


def _text():
    with open(HDR) as f:
        return f.read()


def _g(x):
    mp.mp.dps = 40
    x = mp.mpf(float(x))
    return mp.exp(x * x) * mp.erfc(x)


def test_f64_erfcx_table_relative_error_below_4e_16():
    txt = _text()
    init = txt[txt.index("kErfcxS[25] = {"):]
    init = init[:init.index("};")]
    coef = [float(v) for v in re.findall(r"-?\d\.\d+e[-+]\d+", init)]
    assert len(coef) == 25
    worst = 0.0
    for x in np.concatenate([np.linspace(0.0, 10.0, 401), [1e-300, 0.5, 3.06]]):
        s = (x - 3.0) / (x + 3.0)
        p = coef[24]
        for c in reversed(coef[:24]):
            p = p * s + c  # the kernel uses fma; plain double Horner bounds it from above
        worst = max(worst, abs(float((p - _g(x)) / _g(x))))
    assert worst < 4e-16, worst


def test_f32_erfcx_fit_error_below_1e_8():
    txt = _text()
    p = float(re.search(r"kErfcP = ([0-9.eE+-]+)f;", txt).group(1))
    coef = [float(re.search(rf"kErfcC{k} = ([0-9.eE+-]+)f;", txt).group(1)) for k in range(9)]
    worst = 0.0
    for x in np.linspace(0.0, 6.0, 301):
        t = 1.0 / (1.0 + p * x)
        g = t * sum(c * t ** k for k, c in enumerate(coef))
        worst = max(worst, abs(float((g - _g(x)) / _g(x))))
    assert worst < 1e-8, worst


@pytest.mark.parametrize("x", [0.0, 0.25, 1.0, 2.5, 3.06])
def test_tables_give_erfc(x):
    """Both forms times exp(-x^2) reproduce erfc itself (not only g)."""
    txt = _text()
    init = txt[txt.index("kErfcxS[25] = {"):]
    coef = [float(v) for v in re.findall(r"-?\d\.\d+e[-+]\d+", init[:init.index("};")])]
    s = (x - 3.0) / (x + 3.0)
    g = np.polynomial.polynomial.polyval(s, coef)
    assert abs(g * np.exp(-x * x) - float(mp.erfc(x))) <= 1e-15 * float(mp.erfc(x)) + 1e-300


def test_exp_neg_reduction_and_taylor_table():
    """exp(-y) = 2^-n exp(-r), y = n ln 2 + r, Taylor series of exp(-r) to degree 13,
    with the constants of the kernel header, emulated in double precision."""
    txt = _text()
    init = txt[txt.index("kExpNegTaylor[14] = {"):]
    init = init[init.index("{") + 1:init.index("};")]
    coef = [eval(v.strip(), {}) for v in init.split(",")]  # literals such as 1.0 / 720
    assert len(coef) == 14
    for k, c in enumerate(coef):
        assert c == float(1 / mp.factorial(k))
    hi = float(re.search(r"kLn2Hi = ([0-9.eE+-]+);", txt).group(1))
    lo = float(re.search(r"kLn2Lo = ([0-9.eE+-]+);", txt).group(1))
    inv = float(re.search(r"kInvLn2 = ([0-9.eE+-]+);", txt).group(1))
    mp.mp.dps = 40
    assert abs(mp.mpf(hi) + mp.mpf(lo) - mp.log(2)) < mp.mpf(2) ** -110
    def fma(a, b, c):  # one rounding of the exact a*b + c, as the hardware instruction
        return float(mp.mpf(a) * mp.mpf(b) + mp.mpf(c))

    worst = 0.0
    for y in np.concatenate([np.linspace(0.0, 12.0, 601), [1e-12, 0.3465, 0.3466, 40.0, 700.0]]):
        y = float(y)
        n = float(np.rint(y * inv))
        r = fma(-n, lo, fma(-n, hi, y))
        m = -r
        p = coef[13]
        for c in reversed(coef[:13]):
            p = fma(p, m, c)
        v = np.ldexp(p, -int(n))
        ref = mp.exp(-mp.mpf(float(y)))
        worst = max(worst, abs(float((v - ref) / ref)))
    assert worst < 4e-16, worst


def test_f64_short_erfcx_table_relative_error_below_4e_16_up_to_4_2():
    """The table used when beta R <= 4.2."""
    txt = _text()
    init = txt[txt.index("kErfcxShort[19] = {"):]
    coef = [float(v) for v in re.findall(r"-?\d\.\d+e[-+]\d+", init[:init.index("};")])]
    assert len(coef) == 19
    assert float(re.search(r"kErfcxShortMax = ([0-9.]+);", txt).group(1)) == 4.2
    worst = 0.0
    for x in np.concatenate([np.linspace(0.0, 4.2, 421), [3.06, 4.2 + 1e-9]]):
        s = (x - 3.0) / (x + 3.0)
        p = coef[18]
        for c in reversed(coef[:18]):
            p = p * s + c
        worst = max(worst, abs(float((p - _g(x)) / _g(x))))
    assert worst < 4.5e-16, worst
