"""Pins for the oracle's Ewald corrections (the excluded-pair erf term and the self
term that complete the real-space sum): 30-digit erf values and their derivative,
the identity "correction = real-space term - bare Coulomb term" through the oracle's
separate erfc path, the r -> 0 limit that equals the self term, finite differences,
invariants and the union semantics of the exclusion lists."""

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O
from paper_0902_0827_amd import systems as S

KE = O.COULOMB_K
mp.mp.dps = 30
BOX = [40.0, 41.0, 42.0]


def pair(r, q1, q2, beta, axis=(1.0, 0.0, 0.0)):
    u = np.asarray(axis, float) / np.linalg.norm(axis)
    pos = np.array([[10.0, 11.0, 12.0], [10.0, 11.0, 12.0]]) + np.outer([0.0, 1.0], u * r)
    return pos, u


@pytest.mark.parametrize("q1,q2,r,beta", [(-0.834, 0.417, 0.9572, 0.34), (0.417, 0.417, 1.5139, 0.34),
                                          (-0.5, 0.3, 2.5, 0.26), (0.3, 0.7, 17.0, 0.5),
                                          (1.0, -1.0, 0.05, 0.34)])
def test_excluded_pair_matches_30_digit_erf_and_its_derivative(q1, q2, r, beta):
    pos, u = pair(r, q1, q2, beta)
    res = O.ewald_corrections(pos, [q1, q2], [0, 1, 1], [1], BOX, beta)
    e_ref = -KE * q1 * q2 * mp.erf(beta * mp.mpf(r)) / r
    f_ref = -mp.diff(lambda x: -KE * q1 * q2 * mp.erf(beta * x) / x, mp.mpf(r))  # along 0 -> 1, repulsion > 0
    assert res["e_excl"] == pytest.approx(float(e_ref), rel=1e-13)
    assert -float(res["force"][0] @ u) == pytest.approx(float(f_ref), rel=1e-11, abs=1e-12)
    assert res["e_self"] == pytest.approx(float(-KE * beta / mp.sqrt(mp.pi) * (q1 * q1 + q2 * q2)), rel=1e-14)


@pytest.mark.parametrize("r,beta", [(0.9572, 0.34), (3.3, 0.34), (7.5, 0.26), (2.0, 0.5)])
def test_correction_is_the_real_space_term_minus_the_bare_coulomb_term(r, beta):
    # erf = 1 - erfc: the reciprocal part holds k q q erf(beta r)/r for every pair, so for
    # an excluded pair the correction equals the pair's real-space term (the oracle's erfc
    # path, pair not excluded) minus the bare Coulomb term k q q / r, energy and force.
    q1, q2 = -0.834, 0.417
    pos, u = pair(r, q1, q2, beta, axis=(0.3, -0.5, 0.8))
    corr = O.ewald_corrections(pos, [q1, q2], [0, 1, 1], [1], BOX, beta)
    real = O.evaluate(pos, [q1, q2], [0, 0], [1.0], [0.0], [0, 0, 0], [], BOX, 12.0, beta)
    bare_e = KE * q1 * q2 / r
    bare_f0 = -KE * q1 * q2 / r ** 2 * u  # force on atom 0 (atom 1 along +u)
    assert corr["e_excl"] == pytest.approx(real["e_c"] - bare_e, rel=1e-13)
    np.testing.assert_allclose(corr["force"][0], real["force"][0] - bare_f0, rtol=1e-12, atol=1e-12)


def test_zero_distance_limit_equals_the_self_term():
    # erf(beta r)/r -> 2 beta/sqrt(pi): two equal charges excluded at r -> 0 carry the same
    # energy as their two self terms.
    q, beta = 0.417, 0.34
    pos, _ = pair(1e-7, q, q, beta)
    res = O.ewald_corrections(pos, [q, q], [0, 1, 1], [1], BOX, beta)
    assert res["e_excl"] == pytest.approx(res["e_self"], rel=1e-12)
    pos0, _ = pair(0.0, q, q, beta)
    res0 = O.ewald_corrections(pos0, [q, q], [0, 1, 1], [1], BOX, beta)
    assert res0["e_excl"] == pytest.approx(res0["e_self"], rel=1e-15)
    assert np.all(res0["force"] == 0.0)


@pytest.fixture(scope="module")
def small():
    s = S.solvated_chain(18.6, 30, 190, seed=11, cutoff=9.0, beta=0.34, name="small")
    # add far exclusions (beyond the 64-index window), listed in one row only
    rows = [list(s.excl_index[s.excl_offset[i]:s.excl_offset[i + 1]]) for i in range(s.n)]
    for a, b in [(2, 300), (5, 500), (17, 410)]:
        rows[a].append(b)
    off = np.zeros(s.n + 1, np.int32)
    off[1:] = np.cumsum([len(r) for r in rows])
    s.excl_offset, s.excl_index = off, np.array([j for r in rows for j in r], np.int32)
    return s


def test_forces_are_minus_the_energy_gradient(small):
    res = O.ewald_corrections_system(small)
    h = 1e-5
    for i in (0, 2, 300, 17, 100):
        for a in range(3):
            pp = small.pos.copy(); pp[i, a] += h
            pm = small.pos.copy(); pm[i, a] -= h
            ep = O.ewald_corrections(pp, small.charge, small.excl_offset, small.excl_index, small.box, small.beta)
            em = O.ewald_corrections(pm, small.charge, small.excl_offset, small.excl_index, small.box, small.beta)
            fd = -(ep["e_excl"] - em["e_excl"]) / (2 * h)
            assert res["force"][i, a] == pytest.approx(fd, rel=1e-6, abs=1e-6)


def test_newton_third_law_translation_and_per_atom_split(small):
    res = O.ewald_corrections_system(small)
    np.testing.assert_allclose(res["force"].sum(0), 0.0, atol=1e-9)
    moved = O.ewald_corrections(small.pos + np.array([3.7, -11.2, 25.0]), small.charge, small.excl_offset,
                                small.excl_index, small.box, small.beta)
    np.testing.assert_allclose(moved["force"], res["force"], rtol=1e-9, atol=1e-9)
    assert moved["energy_total"] == pytest.approx(res["energy_total"], rel=1e-12)
    assert res["energy"].sum() == pytest.approx(res["energy_total"], rel=1e-12)


def test_union_semantics_one_sided_and_repeated_entries(small):
    res = O.ewald_corrections_system(small)
    # every pair listed in both rows, and some twice: the same result
    rows = [set() for _ in range(small.n)]
    for i in range(small.n):
        for j in small.excl_index[small.excl_offset[i]:small.excl_offset[i + 1]]:
            rows[i].add(int(j)); rows[int(j)].add(i)
    lists = [sorted(r) + (sorted(r)[:1] if i % 3 == 0 else []) for i, r in enumerate(rows)]
    off = np.zeros(small.n + 1, np.int32)
    off[1:] = np.cumsum([len(r) for r in lists])
    idx = np.array([j for r in lists for j in r], np.int32)
    sym = O.ewald_corrections(small.pos, small.charge, off, idx, small.box, small.beta)
    np.testing.assert_allclose(sym["force"], res["force"], rtol=1e-13, atol=1e-13)
    assert sym["energy_total"] == pytest.approx(res["energy_total"], rel=1e-14)


def test_beta_zero_removes_nothing(small):
    res = O.ewald_corrections(small.pos, small.charge, small.excl_offset, small.excl_index, small.box, 0.0)
    assert res["energy_total"] == 0.0 and np.all(res["force"] == 0.0)
