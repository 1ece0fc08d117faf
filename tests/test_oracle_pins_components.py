"""Pins for the oracle outputs that the invariant tests reach only through sums: the
per-atom energy split, every component of the virial tensors (pair term, Ewald
corrections, reciprocal sum).

Each output is checked against something that does not reuse its own formula:
  * the per-atom split E_i = (1/2) sum_j u_ij against derivatives of the TOTAL energy:
    E is bilinear in the charges, so (1/2) q_i dE/dq_i is atom i's Coulomb share, and
    with atom i given a private LJ type t', eps_t' dE/deps_t' is its LJ share (u^LJ is
    linear in sqrt(eps_ti eps_tj)); both derivatives by central differences;
  * virial components against two-body closed forms along a skew axis, against the
    identity W = sum_i x_i (x) F_i of an isolated cluster (Newton's third law, no
    periodic images), and against derivatives of the energy under a strain
    x'_a = x_a + h x_b: dE/dh = -sum_pairs F_a d_b = -W_ba.  Diagonal entries come from
    scaling one box axis (periodic systems), off-diagonal ones from shearing an
    isolated cluster;
  * the reciprocal sum's off-diagonal virial against a shear of the cell: positions
    x' = (I + e) x, reciprocal vectors m' = (I + e)^-T m and volume V det(I + e), the
    energy evaluated by a triclinic form of the plain sum written here.
"""

import math

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O
from oracle import pme as PO
from paper_0902_0827_amd import systems as S

KE = O.COULOMB_K
mp.mp.dps = 30


@pytest.fixture(scope="module")
def small_chain():
    return S.solvated_chain(18.6, 30, 190, seed=11, cutoff=9.0, beta=0.34, name="small")


def _evaluate(s, pos=None, q=None, types=None, sig=None, eps=None, box=None, rows=None):
    return O.evaluate(s.pos if pos is None else pos, s.charge if q is None else q,
                      s.type if types is None else types, s.sigma if sig is None else sig,
                      s.eps if eps is None else eps, s.excl_offset, s.excl_index,
                      s.box if box is None else box, s.cutoff, s.beta, rows=rows)


# --- per-atom energy split ------------------------------------------------------------------

def test_per_atom_energies_sum_to_the_total(small_chain):
    for s in (small_chain, S.config1()):
        r = O.evaluate_system(s)
        assert r["energy"].sum() == pytest.approx(r["energy_total"], rel=1e-12, abs=1e-10)


def test_per_atom_energy_equals_its_charge_and_private_eps_derivatives(small_chain):
    s = small_chain
    full = O.evaluate_system(s)
    T = s.sigma.shape[0]
    rng = np.random.default_rng(3)
    beads = np.flatnonzero(s.type >= 2)
    oxygens = np.flatnonzero(s.type == 0)
    hydrogens = np.flatnonzero(s.type == 1)
    atoms = np.concatenate([rng.choice(beads, 3, replace=False), rng.choice(oxygens, 3, replace=False),
                            rng.choice(hydrogens, 2, replace=False)])
    for i in atoms:
        # Coulomb share: E_C is bilinear in the charges, so q_i dE/dq_i = sum_j u^C_ij
        hq = 1e-4
        qp = s.charge.copy(); qp[i] += hq
        qm = s.charge.copy(); qm[i] -= hq
        dEdq = (_evaluate(s, q=qp)["energy_total"] - _evaluate(s, q=qm)["energy_total"]) / (2 * hq)
        e_coul = 0.5 * s.charge[i] * dEdq
        # LJ share: atom i alone gets a copy of its type, t' = T; eps_ij = sqrt(eps_t' eps_tj),
        # so eps_t' dE/deps_t' = (1/2) sum_j u^LJ_ij
        e_lj = 0.0
        t = int(s.type[i])
        if s.eps[t] > 0:
            types = s.type.copy(); types[i] = T
            sig = np.append(s.sigma, s.sigma[t])
            he = 1e-4 * s.eps[t]
            ep = np.append(s.eps, s.eps[t] + he)
            em = np.append(s.eps, s.eps[t] - he)
            dEde = (_evaluate(s, types=types, sig=sig, eps=ep)["energy_total"] -
                    _evaluate(s, types=types, sig=sig, eps=em)["energy_total"]) / (2 * he)
            e_lj = s.eps[t] * dEde
        assert full["energy"][i] == pytest.approx(e_coul + e_lj, rel=1e-7, abs=1e-8), i


# --- virial of the pair term ----------------------------------------------------------------

def _two_body(r, q1, q2, s1, e1, beta, axis, L=40.0, cutoff=12.0):
    u = np.asarray(axis, float) / np.linalg.norm(axis)
    pos = np.array([[10.0, 11.0, 12.0], [10.0, 11.0, 12.0]]) + np.outer([0.0, 1.0], u * r)
    return O.evaluate(pos, [q1, q2], [0, 0], [s1], [e1], [0, 0, 0], [], [L, L, L], cutoff, beta), u


@pytest.mark.parametrize("axis", [(1.0, 2.0, -0.5), (-0.3, 0.7, 0.9)])
def test_pair_virial_tensor_two_body_closed_forms(axis):
    # LJ at r = sigma: radial force 24 eps / sigma (repulsive), so with d = x_0 - x_1 = -r u
    # and F_0 = (24 eps/sigma) d / r the tensor is W = d (x) F_0 = 24 eps u (x) u.
    sig, eps = 3.15061, 0.6364
    res, u = _two_body(sig, 0.0, 0.0, sig, eps, 0.34, axis)
    np.testing.assert_allclose(res["virial"], 24 * eps * np.outer(u, u), rtol=0, atol=1e-12)
    # bare Coulomb (beta = 0) of two unit charges at r = 5: radial force k_e/r^2, W = (k_e/r) u (x) u
    res, u = _two_body(5.0, 1.0, 1.0, 3.0, 0.0, 0.0, axis)
    np.testing.assert_allclose(res["virial"], KE / 5.0 * np.outer(u, u), rtol=0, atol=1e-11)
    # Ewald real space at 30 digits: W = -r du/dr u (x) u with u(r) = k q q erfc(beta r)/r
    q1, q2, r, beta = -0.834, 0.417, 2.7, 0.34
    res, u = _two_body(r, q1, q2, 3.0, 0.0, beta, axis)
    dudr = mp.diff(lambda x: KE * q1 * q2 * mp.erfc(beta * x) / x, mp.mpf(r))
    np.testing.assert_allclose(res["virial"], float(-r * dudr) * np.outer(u, u), rtol=0, atol=1e-11)


def _isolated_cluster(seed=5):
    """A 12-molecule water cluster plus a 6-bead chain, in the middle of a 40 A box with a
    9 A cutoff: no pair crosses the boundary (extent < 15 A, 40 - 15 > 9)."""
    w = S.water_lattice(3, 3.1, seed=seed, cutoff=4.0, beta=0.34)
    keep = 12 * 3
    pos = w.pos[:keep] + 14.0
    rng = np.random.default_rng(seed)
    beads = 14.0 + np.array([[-2.5, 1.0 + 1.5 * k, -2.0 + 0.4 * k] for k in range(6)]) + rng.normal(0, 0.05, (6, 3))
    pos = np.concatenate([pos, beads])
    q = np.concatenate([w.charge[:keep], rng.uniform(-0.4, 0.4, 6)])
    q[keep:] -= q[keep:].mean()
    types = np.concatenate([w.type[:keep], np.full(6, 2, np.int32)]).astype(np.int32)
    sig = np.array([w.sigma[0], w.sigma[1], 3.4])
    eps = np.array([w.eps[0], w.eps[1], 0.45])
    rows = [[] for _ in range(keep + 6)]
    for i in range(keep):
        for k in range(w.excl_offset[i], w.excl_offset[i + 1]):
            rows[i].append(int(w.excl_index[k]))
    for k in range(5):
        rows[keep + k].append(keep + k + 1)
    off = np.zeros(len(rows) + 1, np.int32)
    off[1:] = np.cumsum([len(x) for x in rows])
    idx = np.array([j for x in rows for j in x], np.int32)
    ext = pos.max(0) - pos.min(0)
    assert ext.max() < 15.0
    return dict(pos=pos, q=q, types=types, sig=sig, eps=eps, off=off, idx=idx, box=np.array([40.0, 40.0, 40.0]))


def _cluster_eval(c, pos=None):
    return O.evaluate(c["pos"] if pos is None else pos, c["q"], c["types"], c["sig"], c["eps"], c["off"],
                      c["idx"], c["box"], 9.0, 0.34)


def test_pair_virial_of_an_isolated_cluster_is_sum_of_x_outer_f():
    c = _isolated_cluster()
    r = _cluster_eval(c)
    assert r["pairs"] > 400
    w = c["pos"].T @ r["force"]  # sum_i x_i (x) F_i
    np.testing.assert_allclose(r["virial"], w, rtol=0, atol=1e-10 * np.abs(w).max())


def test_pair_virial_off_diagonal_by_shear_of_an_isolated_cluster():
    c = _isolated_cluster()
    r = _cluster_eval(c)
    x0 = c["pos"] - c["pos"].mean(0)
    h = 1e-6
    for a in range(3):
        for b in range(3):
            if a == b:
                continue
            pp = c["pos"].copy(); pp[:, a] += h * x0[:, b]
            pm = c["pos"].copy(); pm[:, a] -= h * x0[:, b]
            dEdh = (_cluster_eval(c, pp)["energy_total"] - _cluster_eval(c, pm)["energy_total"]) / (2 * h)
            assert -dEdh == pytest.approx(r["virial"][b, a], rel=1e-6, abs=1e-6), (a, b)


def test_pair_virial_diagonal_by_scaling_one_box_axis(small_chain):
    s = small_chain
    r = O.evaluate_system(s)
    h = 1e-6
    for a in range(3):
        sc = np.ones(3); sc[a] = 1 + h
        ep = _evaluate(s, pos=s.pos * sc, box=s.box * sc)["energy_total"]
        sc[a] = 1 - h
        em = _evaluate(s, pos=s.pos * sc, box=s.box * sc)["energy_total"]
        assert -(ep - em) / (2 * h) == pytest.approx(r["virial"][a, a], rel=1e-5), a


# --- virial of the Ewald corrections ---------------------------------------------------------

@pytest.mark.parametrize("r,beta,axis", [(0.9572, 0.34, (1.0, 2.0, -0.5)), (2.5, 0.26, (-0.3, 0.7, 0.9)),
                                         (6.0, 0.5, (0.2, -1.0, 0.4))])
def test_ewald_correction_virial_two_body_closed_form(r, beta, axis):
    # an excluded pair: u(r) = -k q q erf(beta r)/r; W = -r du/dr u (x) u, du/dr at 30 digits
    q1, q2 = -0.834, 0.417
    u = np.asarray(axis, float) / np.linalg.norm(axis)
    pos = np.array([[10.0, 11.0, 12.0], [10.0, 11.0, 12.0]]) + np.outer([0.0, 1.0], u * r)
    res = O.ewald_corrections(pos, [q1, q2], [0, 1, 1], [1], [40.0, 41.0, 42.0], beta)
    dudr = mp.diff(lambda x: -KE * q1 * q2 * mp.erf(beta * x) / x, mp.mpf(r))
    np.testing.assert_allclose(res["virial"], float(-r * dudr) * np.outer(u, u), rtol=0, atol=1e-11)


def _corr(c, pos=None, box=None):
    return O.ewald_corrections(c["pos"] if pos is None else pos, c["q"], c["off"], c["idx"],
                               c["box"] if box is None else box, 0.34)


def test_ewald_correction_virial_of_an_isolated_cluster():
    c = _isolated_cluster(seed=9)
    r = _corr(c)
    w = c["pos"].T @ r["force"]
    np.testing.assert_allclose(r["virial"], w, rtol=0, atol=1e-10 * np.abs(w).max())
    x0 = c["pos"] - c["pos"].mean(0)
    h = 1e-6
    for a in range(3):
        for b in range(3):
            pp = c["pos"].copy(); pp[:, a] += h * x0[:, b]
            pm = c["pos"].copy(); pm[:, a] -= h * x0[:, b]
            dEdh = (_corr(c, pp)["e_excl"] - _corr(c, pm)["e_excl"]) / (2 * h)
            assert -dEdh == pytest.approx(r["virial"][b, a], rel=1e-6, abs=1e-7), (a, b)


def test_ewald_correction_virial_diagonal_by_scaling_one_box_axis(small_chain):
    s = small_chain
    r = O.ewald_corrections_system(s)
    h = 1e-6
    for a in range(3):
        sc = np.ones(3); sc[a] = 1 + h
        ep = O.ewald_corrections(s.pos * sc, s.charge, s.excl_offset, s.excl_index, s.box * sc, s.beta)["e_excl"]
        sc[a] = 1 - h
        em = O.ewald_corrections(s.pos * sc, s.charge, s.excl_offset, s.excl_index, s.box * sc, s.beta)["e_excl"]
        assert -(ep - em) / (2 * h) == pytest.approx(r["virial"][a, a], rel=1e-6), a


# --- virial of the reciprocal sum under shear ------------------------------------------------

def _triclinic_reciprocal_energy(pos, q, cell, beta, nmax):
    """Plain reciprocal energy of a triclinic cell (columns of `cell` are the cell vectors):
    m = cell^-T n over |n_a| <= nmax, V = det(cell)."""
    inv_t = np.linalg.inv(cell).T
    n = np.stack(np.meshgrid(*[np.arange(-k, k + 1) for k in nmax], indexing="ij"), -1).reshape(-1, 3)
    n = n[np.any(n != 0, axis=1)]
    m = n @ inv_t.T
    m2 = (m * m).sum(1)
    S = (q[:, None] * np.exp(2j * np.pi * (pos @ m.T))).sum(0)
    V = abs(np.linalg.det(cell))
    return float(KE / (2 * np.pi * V) * np.sum(np.exp(-np.pi ** 2 * m2 / beta ** 2) / m2 * np.abs(S) ** 2))


def test_reciprocal_virial_every_component_by_strain_of_the_cell():
    rng = np.random.default_rng(21)
    L = np.array([9.0, 10.0, 11.0])
    n_at = 12
    pos = rng.uniform(0, 1, (n_at, 3)) * L
    q = rng.uniform(-1, 1, n_at)
    q -= q.mean()
    beta, nmax = 0.45, (7, 7, 8)
    ref = PO.ewald_reciprocal_direct(pos, q, L, beta, nmax=nmax)
    cell0 = np.diag(L)
    assert _triclinic_reciprocal_energy(pos, q, cell0, beta, nmax) == pytest.approx(ref["energy"], rel=1e-12)
    h = 1e-6
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3)); e[a, b] = h
            ep = _triclinic_reciprocal_energy(pos @ (np.eye(3) + e).T, q, (np.eye(3) + e) @ cell0, beta, nmax)
            em = _triclinic_reciprocal_energy(pos @ (np.eye(3) - e).T, q, (np.eye(3) - e) @ cell0, beta, nmax)
            assert -(ep - em) / (2 * h) == pytest.approx(ref["virial"][b, a], rel=1e-6, abs=1e-8), (a, b)


def test_spme_virial_off_diagonals_converge_to_the_plain_sum():
    rng = np.random.default_rng(22)
    L = np.array([9.0, 10.0, 11.0])
    pos = rng.uniform(0, 1, (12, 3)) * L
    q = rng.uniform(-1, 1, 12)
    q -= q.mean()
    beta = 0.45
    ref = PO.ewald_reciprocal_direct(pos, q, L, beta, nmax=(7, 7, 8))
    off = ~np.eye(3, dtype=bool)
    errs = []
    for K in (16, 32):
        sp = PO.spme_reciprocal(pos, q, L, beta, (K, K + 2, K + 4))
        errs.append(np.abs(sp["virial"][off] - ref["virial"][off]).max())
    scale = np.abs(ref["virial"]).max()
    assert errs[1] < 1e-4 * scale and errs[1] < errs[0] / 8
