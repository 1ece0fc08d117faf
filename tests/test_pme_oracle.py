"""Pins of the reciprocal-space oracle (oracle/pme.py) against things other than itself:
known B-spline values, the Madelung constant of rock salt, the independence of the full
Ewald energy from the splitting parameter, convergence of SPME to the plain k-space sum
at the rate of its interpolation order, and forces and virial by finite differences."""

import numpy as np
import pytest

from oracle import oracle as O
from oracle import pme as P

pytestmark = pytest.mark.timeout(600)

# Madelung constant of the rock-salt (NaCl) structure referred to the nearest-neighbour
# distance (e.g. Kittel, Introduction to Solid State Physics, ch. 3).
MADELUNG_NACL = 1.747564594633


def _random_neutral(n, box, seed):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3)) * np.asarray(box)
    q = rng.normal(size=n)
    return pos, q - q.mean()


def _rock_salt(cells, a):
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    pos, q = [], []
    for o in np.ndindex(cells, cells, cells):
        for b in fcc:
            pos.append((np.array(o) + b) * a)
            q.append(1.0)
            pos.append(((np.array(o) + b + [0.5, 0, 0]) % cells) * a)
            q.append(-1.0)
    return np.array(pos), np.array(q), np.full(3, cells * a)


def _real_space(pos, q, box, cutoff, beta):
    n = len(q)
    r = O.evaluate(pos, q, np.zeros(n, np.int32), np.ones(1), np.zeros(1), np.zeros(n + 1, np.int32),
                   np.zeros(0, np.int32), box, cutoff, beta)
    return r["energy_total"], r["force"]


def test_bspline_known_values():
    # M_4 at the integers 1, 2, 3 is 1/6, 2/3, 1/6; at the half-integers 1/48, 23/48, 23/48, 1/48
    np.testing.assert_allclose(P.cardinal_bspline([1.0, 2.0, 3.0], 4), [1 / 6, 2 / 3, 1 / 6], rtol=1e-15)
    np.testing.assert_allclose(P.cardinal_bspline([0.5, 1.5, 2.5, 3.5], 4), np.array([1, 23, 23, 1]) / 48,
                               rtol=1e-15)
    # support [0, n]: zero outside
    assert np.all(P.cardinal_bspline([-0.5, 0.0, 4.0, 4.5], 4) == 0.0)


@pytest.mark.parametrize("n", [3, 4, 5, 6, 8])
def test_bspline_partition_of_unity_and_derivative(n):
    w = np.random.default_rng(n).random(50)
    s = sum(P.cardinal_bspline(w + j, n) for j in range(n))
    np.testing.assert_allclose(s, 1.0, rtol=0, atol=1e-14)
    ds = sum(P.cardinal_bspline_deriv(w + j, n) for j in range(n))
    np.testing.assert_allclose(ds, 0.0, rtol=0, atol=1e-13)
    h = 1e-6
    x = w + 1.0
    fd = (P.cardinal_bspline(x + h, n) - P.cardinal_bspline(x - h, n)) / (2 * h)
    np.testing.assert_allclose(P.cardinal_bspline_deriv(x, n), fd, rtol=0, atol=1e-8)


def test_bmod_order4_closed_form():
    # for n = 4 the denominator 1/6 + (2/3) e^{i t} + (1/6) e^{2 i t} has modulus (2 + cos t)/3
    K = 20
    t = 2 * np.pi * np.arange(K) / K
    np.testing.assert_allclose(P._bmod2(K, 4), 9.0 / (2.0 + np.cos(t)) ** 2, rtol=1e-14)


def test_madelung_constant_of_rock_salt():
    a = 5.64
    pos, q, box = _rock_salt(4, a)                       # 512 ions, 22.56 A box
    beta, cutoff = 0.45, 11.0                            # erfc(beta R) ~ 3e-12
    e_real, _ = _real_space(pos, q, box, cutoff, beta)
    e_self = -O.COULOMB_K * beta / np.sqrt(np.pi) * np.sum(q * q)
    e_rec = P.ewald_reciprocal_direct(pos, q, box, beta, nmax=(20, 20, 20))["energy"]
    madelung = -(e_real + e_self + e_rec) / (len(q) / 2) * (a / 2) / O.COULOMB_K
    assert abs(madelung - MADELUNG_NACL) < 1e-10
    # SPME on a grid the lattice sits on: the same reciprocal energy
    e_spme = P.spme_reciprocal(pos, q, box, beta, (48, 48, 48))["energy"]
    assert abs(e_spme - e_rec) <= 1e-9 * abs(e_rec)


def test_full_ewald_energy_independent_of_beta():
    box = np.array([24.0, 24.0, 24.0])
    pos, q = _random_neutral(64, box, seed=3)
    totals, forces = [], []
    for beta in (0.45, 0.52):
        e_real, f_real = _real_space(pos, q, box, 11.9, beta)
        rec = P.ewald_reciprocal_direct(pos, q, box, beta, nmax=(26, 26, 26))
        totals.append(e_real + rec["energy"] - O.COULOMB_K * beta / np.sqrt(np.pi) * np.sum(q * q))
        forces.append(f_real + rec["force"])
    assert abs(totals[0] - totals[1]) <= 1e-9 * np.sum(np.abs(q)) ** 2
    np.testing.assert_allclose(forces[0], forces[1], rtol=0, atol=1e-8 * np.abs(forces[0]).max())


def test_spme_converges_to_the_plain_sum_at_fourth_order():
    box = np.array([12.0, 13.0, 14.0])
    pos, q = _random_neutral(40, box, seed=1)
    beta = 0.34
    d = P.ewald_reciprocal_direct(pos, q, box, beta, nmax=(10, 10, 10))
    err = {}
    for K in (16, 32, 48):
        s = P.spme_reciprocal(pos, q, box, beta, (K, K, K))
        err[K] = (abs(s["energy"] - d["energy"]) / abs(d["energy"]),
                  np.linalg.norm(s["force"] - d["force"]) / np.linalg.norm(d["force"]),
                  np.abs(s["virial"] - d["virial"]).max() / np.abs(d["virial"]).max())
    assert err[16][0] / err[32][0] > 8.0                 # about 2^4 for order-4 splines
    assert err[48][0] < 1e-5 and err[48][1] < 1e-4 and err[48][2] < 2e-5
    # a higher order is more accurate on the same grid
    s6 = P.spme_reciprocal(pos, q, box, beta, (32, 32, 32), order=6)
    assert abs(s6["energy"] - d["energy"]) / abs(d["energy"]) < err[32][0] / 4


def test_plain_sum_forces_and_virial_by_finite_differences():
    box = np.array([10.0, 11.0, 12.0])
    pos, q = _random_neutral(12, box, seed=5)
    beta, nmax = 0.4, (8, 8, 8)
    ref = P.ewald_reciprocal_direct(pos, q, box, beta, nmax=nmax)
    h = 1e-5
    for i, a in [(0, 0), (3, 1), (7, 2), (11, 0)]:
        p1, p2 = pos.copy(), pos.copy()
        p1[i, a] += h
        p2[i, a] -= h
        fd = -(P.ewald_reciprocal_direct(p1, q, box, beta, nmax=nmax)["energy"] -
               P.ewald_reciprocal_direct(p2, q, box, beta, nmax=nmax)["energy"]) / (2 * h)
        assert abs(fd - ref["force"][i, a]) <= 1e-6 * np.abs(ref["force"]).max()
    for a in range(3):   # W_aa = -dE/d(strain_aa): positions and box scaled along a (same n-vectors)
        e = []
        for eps in (h, -h):
            s = np.ones(3)
            s[a] += eps
            e.append(P.ewald_reciprocal_direct(pos * s, q, box * s, beta, nmax=nmax)["energy"])
        assert abs(-(e[0] - e[1]) / (2 * h) - ref["virial"][a, a]) <= 1e-6 * np.abs(ref["virial"]).max()
    np.testing.assert_allclose(ref["virial"], ref["virial"].T, rtol=0, atol=1e-12 * np.abs(ref["virial"]).max())


def test_spme_forces_and_virial_by_finite_differences():
    box = np.array([12.0, 12.5, 13.0])
    pos, q = _random_neutral(30, box, seed=7)
    beta, grid = 0.34, (20, 24, 28)
    ref = P.spme_reciprocal(pos, q, box, beta, grid)
    h = 1e-5
    for i, a in [(0, 0), (4, 1), (9, 2), (29, 1)]:
        p1, p2 = pos.copy(), pos.copy()
        p1[i, a] += h
        p2[i, a] -= h
        fd = -(P.spme_reciprocal(p1, q, box, beta, grid)["energy"] -
               P.spme_reciprocal(p2, q, box, beta, grid)["energy"]) / (2 * h)
        assert abs(fd - ref["force"][i, a]) <= 1e-6 * np.abs(ref["force"]).max()
    for a in range(3):   # the grid is fixed, so fractional coordinates and the charge grid do not change
        e = []
        for eps in (h, -h):
            s = np.ones(3)
            s[a] += eps
            e.append(P.spme_reciprocal(pos * s, q, box * s, beta, grid)["energy"])
        assert abs(-(e[0] - e[1]) / (2 * h) - ref["virial"][a, a]) <= 1e-6 * np.abs(ref["virial"]).max()
    # E = (1/2) sum_k Q(k) phi(k)
    assert abs(0.5 * np.sum(ref["Q"] * ref["phi"]) - ref["energy"]) <= 1e-12 * abs(ref["energy"])


def test_spme_translation_and_wrap():
    box = np.array([12.0, 12.0, 12.0])
    pos, q = _random_neutral(20, box, seed=11)
    grid = (24, 24, 24)
    a = P.spme_reciprocal(pos, q, box, 0.34, grid)
    # a shift by whole grid spacings leaves SPME exactly invariant (the grid is relabelled)
    shift = np.array([3, -5, 7]) * box / np.array(grid)
    b = P.spme_reciprocal(pos + shift, q, box, 0.34, grid)
    assert abs(a["energy"] - b["energy"]) <= 1e-12 * abs(a["energy"])
    np.testing.assert_allclose(a["force"], b["force"], rtol=0, atol=1e-10 * np.abs(a["force"]).max())
    # positions outside the box are wrapped
    c = P.spme_reciprocal(pos + box * np.array([2, -1, 3]), q, box, 0.34, grid)
    assert abs(a["energy"] - c["energy"]) <= 1e-12 * abs(a["energy"])
