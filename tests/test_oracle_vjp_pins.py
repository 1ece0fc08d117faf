"""Pins for the oracle's force vector-Jacobian product (the double backward of force
matching): the derivatives of L = sum_i v_i . F_i with respect to every charge, sigma_t
and eps_t, against central differences of L built from the oracle's forces (themselves
pinned as -dE/dx), with and without the switch and 1-4 pairs; and L's linearity in v."""

import numpy as np
import pytest

from oracle import oracle as O
from paper_0902_0827_amd import systems as S

FF = dict(lj_switch_on=7.5, scale14_lj=0.5, scale14_coul=1 / 1.2)


@pytest.fixture(scope="module")
def chain14():
    return S.with_chain_14(S.solvated_chain(18.6, 30, 190, seed=11, cutoff=9.0, beta=0.34, name="small"))


def _L(s, v, ff, q=None, sig=None, eps=None):
    r = O.evaluate(s.pos, s.charge if q is None else q, s.type, s.sigma if sig is None else sig,
                   s.eps if eps is None else eps, s.excl_offset, s.excl_index, s.box, s.cutoff, s.beta, **ff)
    return float(np.sum(v * r["force"]))


@pytest.mark.parametrize("use_ff", [False, True])
def test_force_vjp_by_finite_differences(chain14, use_ff):
    s = chain14
    ff = dict(FF, pair14_offset=s.pair14_offset, pair14_index=s.pair14_index) if use_ff else {}
    v = np.random.default_rng(8).normal(size=(s.n, 3))
    out = O.evaluate(s.pos, s.charge, s.type, s.sigma, s.eps, s.excl_offset, s.excl_index, s.box, s.cutoff,
                     s.beta, vjp=v, **ff)
    h = 1e-4
    for i in (0, 4, 31, 200, 500):
        qp = s.charge.copy(); qp[i] += h
        qm = s.charge.copy(); qm[i] -= h
        fd = (_L(s, v, ff, q=qp) - _L(s, v, ff, q=qm)) / (2 * h)
        assert fd == pytest.approx(out["vjp_charge"][i], rel=1e-6, abs=1e-6)
    for t in np.unique(s.type):
        sp = s.sigma.copy(); sp[t] += h
        sm = s.sigma.copy(); sm[t] -= h
        fd = (_L(s, v, ff, sig=sp) - _L(s, v, ff, sig=sm)) / (2 * h)
        assert fd == pytest.approx(out["vjp_sigma"][t], rel=1e-6, abs=1e-5)
        if s.eps[t] > 0:
            ep = s.eps.copy(); ep[t] += h * s.eps[t]
            em = s.eps.copy(); em[t] -= h * s.eps[t]
            fd = (_L(s, v, ff, eps=ep) - _L(s, v, ff, eps=em)) / (2 * h * s.eps[t])
            assert fd == pytest.approx(out["vjp_eps"][t], rel=1e-6, abs=1e-6)


def test_force_vjp_is_linear_in_v_and_zero_for_a_uniform_v(chain14):
    s = chain14
    rng = np.random.default_rng(9)
    v1, v2 = rng.normal(size=(s.n, 3)), rng.normal(size=(s.n, 3))
    ev = lambda v: O.evaluate_system(s, vjp=v)
    a, b, c = ev(v1), ev(v2), ev(2 * v1 - 3 * v2)
    for k in ("vjp_charge", "vjp_sigma", "vjp_eps"):
        np.testing.assert_allclose(c[k], 2 * a[k] - 3 * b[k], rtol=1e-10, atol=1e-10)
    # a translation-like v (the same vector on every atom) sees sum_i F_i = 0: every
    # derivative of L vanishes (each pair term carries v_i - v_j)
    u = ev(np.tile([0.3, -1.2, 0.7], (s.n, 1)))
    for k in ("vjp_charge", "vjp_sigma", "vjp_eps"):
        assert np.abs(u[k]).max() < 1e-10
