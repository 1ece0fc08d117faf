"""Pins for the oracle's force-field options: the CHARMM switch of the Lennard-Jones term
between r_on and the cutoff, and scaled 1-4 pairs (LJ by s14_lj, real-space Coulomb by
s14_coul, the Ewald corrections completing the Coulomb term to s14_coul k_e q q / r).

Pinned by: the switch's special values in x = (r^2 - r_on^2)/(R^2 - r_on^2) (S = 1, 27/32,
1/2, 0 at x = 0, 1/4, 1/2, 1), the unchanged energy inside r_on, forces continuous at r_on
and vanishing at R, finite differences of the energy (forces, charge / sigma / eps
gradients, virial by strain); the 1-4 scaling reducing to the plain pair (scales 1) and to
an excluded pair (scales 0), a two-body 1-4 pair equal to the scaled terms of the plain
pair, the union of one-sided rows, exclusion taking precedence, and the whole Coulomb
interaction of a 1-4 pair (real space + corrections + the reciprocal part's erf term at
30 digits) equal to s14_coul k_e q q / r.
"""

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O
from paper_0902_0827_amd import systems as S

KE = O.COULOMB_K
mp.mp.dps = 30
R, R_ON = 9.0, 7.5


def two_body(r, q1=0.0, q2=0.0, sig=3.15061, eps=0.6364, beta=0.34, axis=(1.0, 2.0, -0.5), **ff):
    u = np.asarray(axis, float) / np.linalg.norm(axis)
    pos = np.array([[10.0, 11.0, 12.0], [10.0, 11.0, 12.0]]) + np.outer([0.0, 1.0], u * r)
    res = O.evaluate(pos, [q1, q2], [0, 0], [sig], [eps], [0, 0, 0], [], [40.0] * 3, R, beta, **ff)
    return res, -float(res["force"][0] @ u)  # radial force, repulsion positive


def r_at_x(x):
    return float(np.sqrt(R_ON ** 2 + x * (R ** 2 - R_ON ** 2)))


@pytest.mark.parametrize("x,s_ref", [(0.0, 1.0), (0.25, 27.0 / 32.0), (0.5, 0.5), (0.75, 5.0 / 32.0)])
def test_switch_special_values(x, s_ref):
    r = r_at_x(x)
    plain, _ = two_body(r)
    sw, _ = two_body(r, lj_switch_on=R_ON)
    assert sw["e_lj"] == pytest.approx(s_ref * plain["e_lj"], rel=1e-13)


def test_switch_leaves_the_inside_alone_and_coulomb_unswitched():
    for r in (3.0, 5.0, 7.49):
        plain, fp = two_body(r, 0.4, -0.6)
        sw, fs = two_body(r, 0.4, -0.6, lj_switch_on=R_ON)
        assert sw["energy_total"] == plain["energy_total"] and fs == fp
    plain, _ = two_body(8.2, 0.4, -0.6)
    sw, _ = two_body(8.2, 0.4, -0.6, lj_switch_on=R_ON)
    assert sw["e_c"] == plain["e_c"] and sw["e_lj"] != plain["e_lj"]


def test_switched_force_is_continuous_and_vanishes_at_the_cutoff():
    h = 1e-7
    _, f_in = two_body(R_ON - h, lj_switch_on=R_ON)
    _, f_out = two_body(R_ON + h, lj_switch_on=R_ON)
    assert abs(f_in - f_out) < 1e-8
    # S and dS/dr vanish at R, so the force goes to zero linearly in R - r
    _, f6 = two_body(R - 1e-6, lj_switch_on=R_ON)
    _, f5 = two_body(R - 1e-5, lj_switch_on=R_ON)
    _, f_mid = two_body(8.0, lj_switch_on=R_ON)
    assert abs(f5) < 1e-4 * abs(f_mid)
    assert f6 / f5 == pytest.approx(0.1, rel=1e-3)
    # and between: the radial force is -dE/dr by central differences (30-digit-free check)
    for r in (7.6, 8.0, 8.5, 8.9):
        e_p, _ = two_body(r + 1e-5, lj_switch_on=R_ON)
        e_m, _ = two_body(r - 1e-5, lj_switch_on=R_ON)
        _, f = two_body(r, lj_switch_on=R_ON)
        assert f == pytest.approx(-(e_p["e_lj"] - e_m["e_lj"]) / 2e-5, rel=1e-6, abs=1e-10)


# --- 1-4 scaling ----------------------------------------------------------------------------

def test_two_body_14_pair_scales_each_term():
    for r in (2.9, 3.6, 6.0):
        p14 = dict(pair14_offset=[0, 1, 1], pair14_index=[1])
        plain, fp = two_body(r, 0.5, -0.3)
        sc, fs = two_body(r, 0.5, -0.3, scale14_lj=0.5, scale14_coul=1 / 1.2, **p14)
        assert sc["e_lj"] == pytest.approx(0.5 * plain["e_lj"], rel=1e-12)
        assert sc["e_c"] == pytest.approx(plain["e_c"] / 1.2, rel=1e-12)
        lj_only, f_lj = two_body(r, 0.0, 0.0)
        c_only, f_c = two_body(r, 0.5, -0.3, eps=0.0)
        assert fs == pytest.approx(0.5 * f_lj + f_c / 1.2, rel=1e-12)


@pytest.fixture(scope="module")
def chain14():
    return S.with_chain_14(S.solvated_chain(18.6, 30, 190, seed=11, cutoff=9.0, beta=0.34, name="small"))


def test_scales_one_is_the_plain_pair_and_scales_zero_an_excluded_pair(chain14):
    s = chain14
    plain = O.evaluate_system(s, pair14_offset=None)
    ones = O.evaluate_system(s, scale14_lj=1.0, scale14_coul=1.0)
    # equal pair by pair (the threads' partial sums of the total may meet in any order)
    assert ones["energy_total"] == pytest.approx(plain["energy_total"], rel=1e-12)
    np.testing.assert_array_equal(ones["force"], plain["force"])
    zeros = O.evaluate_system(s, scale14_lj=0.0, scale14_coul=0.0)
    # the 1-4 pairs added to the exclusion lists
    rows = [list(s.excl_index[s.excl_offset[i]:s.excl_offset[i + 1]]) +
            list(s.pair14_index[s.pair14_offset[i]:s.pair14_offset[i + 1]]) for i in range(s.n)]
    off = np.zeros(s.n + 1, np.int32)
    off[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([j for r in rows for j in sorted(r)], np.int32)
    excl = O.evaluate(s.pos, s.charge, s.type, s.sigma, s.eps, off, idx, s.box, s.cutoff, s.beta)
    assert zeros["energy_total"] == pytest.approx(excl["energy_total"], rel=1e-13)
    np.testing.assert_allclose(zeros["force"], excl["force"], rtol=0, atol=1e-11 * np.abs(excl["force"]).max())


def test_one_sided_14_rows_and_exclusion_precedence(chain14):
    s = chain14
    both = O.evaluate_system(s, scale14_lj=0.5, scale14_coul=0.8)
    # each 1-4 pair named in its lower atom's row only
    rows = [[j for j in s.pair14_index[s.pair14_offset[i]:s.pair14_offset[i + 1]] if j > i] for i in range(s.n)]
    off = np.zeros(s.n + 1, np.int32)
    off[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([j for r in rows for j in r], np.int32)
    one = O.evaluate_system(s, pair14_offset=off, pair14_index=idx, scale14_lj=0.5, scale14_coul=0.8)
    assert one["energy_total"] == pytest.approx(both["energy_total"], rel=1e-12)
    np.testing.assert_array_equal(one["force"], both["force"])
    # a 1-2 pair (already excluded) also listed as 1-4 stays excluded
    rows2 = [list(s.pair14_index[s.pair14_offset[i]:s.pair14_offset[i + 1]]) for i in range(s.n)]
    rows2[0].append(1)
    off2 = np.zeros(s.n + 1, np.int32)
    off2[1:] = np.cumsum([len(r) for r in rows2])
    idx2 = np.array([j for r in rows2 for j in r], np.int32)
    extra = O.evaluate_system(s, pair14_offset=off2, pair14_index=idx2, scale14_lj=0.5, scale14_coul=0.8)
    assert extra["energy_total"] == pytest.approx(both["energy_total"], rel=1e-12)
    np.testing.assert_array_equal(extra["force"], both["force"])


@pytest.mark.parametrize("r,beta", [(3.1, 0.34), (3.9, 0.26), (2.6, 0.5)])
def test_whole_coulomb_of_a_14_pair_is_the_scaled_bare_term(r, beta):
    """real space (s erfc/r) + correction (-(1 - s) erf/r) + the reciprocal part's erf/r
    = s k_e q q / r."""
    q1, q2, s_c = 0.31, -0.52, 1 / 1.2
    u = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    pos = np.array([[10.0, 11.0, 12.0], [10.0, 11.0, 12.0]]) + np.outer([0.0, 1.0], u * r)
    p14 = dict(pair14_offset=[0, 1, 1], pair14_index=[1])
    real = O.evaluate(pos, [q1, q2], [0, 0], [3.0], [0.0], [0, 0, 0], [], [40.0] * 3, 12.0, beta,
                      scale14_coul=s_c, **p14)
    corr = O.ewald_corrections(pos, [q1, q2], [0, 0, 0], [], [40.0] * 3, beta, scale14_coul=s_c, **p14)
    recip = float(KE * q1 * q2 * mp.erf(beta * mp.mpf(r)) / r)
    assert real["e_c"] + corr["e_excl"] + recip == pytest.approx(s_c * KE * q1 * q2 / r, rel=1e-13)


# --- finite differences on a switched system with 1-4 pairs ------------------------------------

def _e(s, **kw):
    return O.evaluate(kw.get("pos", s.pos), kw.get("q", s.charge), s.type, kw.get("sig", s.sigma),
                      kw.get("eps", s.eps), s.excl_offset, s.excl_index, kw.get("box", s.box), s.cutoff,
                      s.beta, pair14_offset=s.pair14_offset, pair14_index=s.pair14_index, scale14_lj=0.5,
                      scale14_coul=1 / 1.2, lj_switch_on=R_ON)


def test_forces_and_parameter_gradients_by_finite_differences(chain14):
    s = chain14
    r = _e(s)
    rng = np.random.default_rng(4)
    h = 1e-5
    checked = 0
    for i in list(range(8)) + list(rng.choice(s.n, 30, replace=False)):
        d = s.pos - s.pos[i]
        d -= s.box * np.rint(d / s.box)
        if np.any(np.abs(np.sqrt((d * d).sum(1)) - s.cutoff) <= 2 * h):
            continue
        for a in range(3):
            p = s.pos.copy(); p[i, a] += h
            m = s.pos.copy(); m[i, a] -= h
            fd = -(_e(s, pos=p)["energy_total"] - _e(s, pos=m)["energy_total"]) / (2 * h)
            assert fd == pytest.approx(r["force"][i, a], rel=2e-6, abs=2e-6 * (1 + abs(r["force"][i]).max()))
        checked += 1
    assert checked >= 20
    full = O.evaluate(s.pos, s.charge, s.type, s.sigma, s.eps, s.excl_offset, s.excl_index, s.box, s.cutoff,
                      s.beta, pair14_offset=s.pair14_offset, pair14_index=s.pair14_index, scale14_lj=0.5,
                      scale14_coul=1 / 1.2, lj_switch_on=R_ON)
    h = 1e-4
    for i in (0, 3, 5, 100):
        qp = s.charge.copy(); qp[i] += h
        qm = s.charge.copy(); qm[i] -= h
        fd = (_e(s, q=qp)["energy_total"] - _e(s, q=qm)["energy_total"]) / (2 * h)
        assert fd == pytest.approx(full["phi"][i], rel=1e-6, abs=1e-6)
    for t in np.unique(s.type):
        sp = s.sigma.copy(); sp[t] += h
        sm = s.sigma.copy(); sm[t] -= h
        fd = (_e(s, sig=sp)["energy_total"] - _e(s, sig=sm)["energy_total"]) / (2 * h)
        assert fd == pytest.approx(full["dsigma"][t], rel=1e-6, abs=1e-6)
        if s.eps[t] > 0:
            ep = s.eps.copy(); ep[t] += h
            em = s.eps.copy(); em[t] -= h
            fd = (_e(s, eps=ep)["energy_total"] - _e(s, eps=em)["energy_total"]) / (2 * h)
            assert fd == pytest.approx(full["deps"][t], rel=1e-6, abs=1e-6)
    # homogeneity still holds: E_C bilinear in the charges, E_LJ linear in sqrt(eps eps)
    assert float(s.charge @ full["phi"]) == pytest.approx(2 * full["e_c"], rel=1e-12)
    assert float(s.eps @ full["deps"]) == pytest.approx(full["e_lj"], rel=1e-12)


def test_switched_virial_diagonal_by_axis_scaling(chain14):
    s = chain14
    r = _e(s)
    h = 1e-6
    for a in range(3):
        sc = np.ones(3); sc[a] = 1 + h
        ep = _e(s, pos=s.pos * sc, box=s.box * sc)["energy_total"]
        sc[a] = 1 - h
        em = _e(s, pos=s.pos * sc, box=s.box * sc)["energy_total"]
        assert -(ep - em) / (2 * h) == pytest.approx(r["virial"][a, a], rel=1e-5), a
