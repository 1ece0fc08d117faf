"""Pins of the molecular-dynamics oracle (oracle/md.py) to what the mathematics fixes:
Philox known answers, the statistics of the thermostat noise, SHAKE and RATTLE against
direct solutions of their equations, bonded forces against finite differences and
closed forms, velocity Verlet against the exact discrete solution of a harmonic bond,
the Langevin update's exact mean and variance, and equipartition of a rigid-water gas
(six degrees of freedom per molecule)."""

import math
import pathlib

import numpy as np
import pytest

from oracle import md as M
from paper_0902_0827_amd import systems as S

GOLDEN = pathlib.Path(__file__).parent / "golden" / "philox4x32_10_kat.txt"


def test_philox_known_answers():
    rows = [l.split() for l in GOLDEN.read_text().splitlines() if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = M.philox4x32_10(np.array(v[:4]), np.array(v[4:6]))
        assert [int(x) for x in out] == v[6:]


def test_noise_is_standard_normal_and_independent():
    n = 200_000
    a = M.normals(12345, 7, 0, np.arange(n))
    b = M.normals(12345, 7, 1, np.arange(n))
    c = M.normals(12345, 8, 0, np.arange(n))
    for z in (a, b, c):
        assert np.all(np.abs(z.mean(0)) < 5 / math.sqrt(n))
        assert np.all(np.abs(z.var(0) - 1) < 5 * math.sqrt(2 / n))
        # fourth moment 3 (Gaussian), sd of the estimate sqrt(96/n)
        assert np.all(np.abs((z ** 4).mean(0) - 3) < 5 * math.sqrt(96 / n))
    for x, y in ((a, b), (a, c), (a[:, 0:1], a[:, 1:2]), (a[:, 0:1], a[:, 2:3])):
        r = np.mean(x * y, 0)
        assert np.all(np.abs(r) < 5 / math.sqrt(n))
    # the counter's fields all enter: another seed, atom or step changes every word
    assert not np.any(M.normals(12346, 7, 0, [5]) == a[5])


def _waters(n, seed):
    s = S.water_lattice(8, 3.1, seed, 9.0, 0.34, n_waters=n)
    mass = np.tile([15.999, 1.008, 1.008], n)
    return s, mass, np.arange(0, 3 * n, 3)


def _constraint_error(x, water_o, abox):
    i, j, d = M._water_constraints(water_o, S.OH_BOND, M_HH)
    r = np.linalg.norm(M._minimage(x[i] - x[j], abox[i]), axis=1)
    return np.max(np.abs(r - d) / d)


M_HH = 2 * S.OH_BOND * math.sin(math.radians(S.HOH_ANGLE_DEG) / 2)


def test_shake_solves_the_constraint_equations():
    """SHAKE's answer satisfies the constraints, moves each pair along its old bond
    (so the result is x_new + sum_p lambda_p s_p / m), keeps the centre of mass, and
    agrees with a Newton solve of the three multipliers per water."""
    s, mass, wo = _waters(40, 3)
    abox = np.broadcast_to(s.box, s.pos.shape)
    rng = np.random.default_rng(1)
    x_new = s.pos + 0.03 * rng.standard_normal(s.pos.shape)
    x = M.shake(s.pos, x_new, mass, wo, S.OH_BOND, M_HH, abox)
    assert _constraint_error(x, wo, abox) < 1e-13
    dm = (mass[:, None] * (x - x_new)).reshape(-1, 3, 3).sum(1)
    assert np.max(np.abs(dm)) < 1e-12
    # Newton on the multipliers of one water, written from the constraint equations
    for w in range(0, 40, 7):
        o = 3 * w
        idx = [(0, 1), (0, 2), (1, 2)]
        d = np.array([S.OH_BOND, S.OH_BOND, M_HH])
        inv = 1.0 / mass[o:o + 3]
        xo = s.pos[o:o + 3].copy()
        xo[1:] = xo[0] + M._minimage(xo[1:] - xo[0], s.box)
        xu = x_new[o:o + 3].copy()
        xu[1:] = xu[0] + M._minimage(xu[1:] - xu[0], s.box)
        sold = [xo[a] - xo[b] for a, b in idx]

        def pos(lam):
            p = xu.copy()
            for k, (a, b) in enumerate(idx):
                p[a] += lam[k] * inv[a] * sold[k]
                p[b] -= lam[k] * inv[b] * sold[k]
            return p

        lam = np.zeros(3)
        for _ in range(30):
            p = pos(lam)
            g = np.array([np.dot(p[a] - p[b], p[a] - p[b]) - d[k] ** 2 for k, (a, b) in enumerate(idx)])
            J = np.zeros((3, 3))
            for q, (a, b) in enumerate(idx):
                for k, (c, e) in enumerate(idx):
                    dv = np.zeros((3, 3))
                    dv[c] += inv[c] * sold[k]
                    dv[e] -= inv[e] * sold[k]
                    J[q, k] = 2 * np.dot(p[a] - p[b], dv[a] - dv[b])
            lam -= np.linalg.solve(J, g)
        ref = pos(lam)
        got = x[o:o + 3].copy()
        got[1:] = got[0] + M._minimage(got[1:] - got[0], s.box)
        shift = got[0] - ref[0]
        shift -= s.box * np.rint(shift / s.box)
        np.testing.assert_allclose(got + 0 * shift, ref + shift, rtol=0, atol=1e-11)


def test_rattle_is_the_exact_projection():
    """RATTLE leaves no relative velocity along any bond, keeps the momentum, and equals
    the direct solution of its linear equations."""
    s, mass, wo = _waters(30, 4)
    abox = np.broadcast_to(s.box, s.pos.shape)
    rng = np.random.default_rng(2)
    v0 = rng.standard_normal(s.pos.shape) * 5.0
    v = M.rattle_velocities(s.pos, v0, mass, wo, S.OH_BOND, M_HH, abox)
    i, j, _ = M._water_constraints(wo, S.OH_BOND, M_HH)
    sv = M._minimage(s.pos[i] - s.pos[j], abox[i])
    assert np.max(np.abs(np.einsum("ij,ij->i", v[i] - v[j], sv))) < 1e-11
    dp = (mass[:, None] * (v - v0)).reshape(-1, 3, 3).sum(1)
    assert np.max(np.abs(dp)) < 1e-11
    idx = [(0, 1), (0, 2), (1, 2)]
    for w in range(0, 30, 5):
        o = 3 * w
        inv = 1.0 / mass[o:o + 3]
        sb = [M._minimage(s.pos[o + a] - s.pos[o + b], s.box) for a, b in idx]
        A = np.zeros((3, 3))
        rhs = np.zeros(3)
        for q, (a, b) in enumerate(idx):
            rhs[q] = -np.dot(v0[o + a] - v0[o + b], sb[q])
            for k, (c, e) in enumerate(idx):
                dv = np.zeros((3, 3))
                dv[c] += inv[c] * sb[k]
                dv[e] -= inv[e] * sb[k]
                A[q, k] = np.dot(dv[a] - dv[b], sb[q])
        mu = np.linalg.solve(A, rhs)
        ref = v0[o:o + 3].copy()
        for k, (a, b) in enumerate(idx):
            ref[a] += mu[k] * inv[a] * sb[k]
            ref[b] -= mu[k] * inv[b] * sb[k]
        np.testing.assert_allclose(v[o:o + 3], ref, rtol=0, atol=1e-11)


def test_bonded_forces_are_minus_the_energy_gradient():
    rng = np.random.default_rng(5)
    box = np.array([12.0, 12.0, 12.0])
    pos = rng.uniform(0, 12, (6, 3))
    pos[1] = pos[0] + [1.4, 0.3, -0.2]
    pos[2] = pos[1] + [0.2, 1.5, 0.1]
    pos[3] = pos[2] + [-11.0, 0.4, 1.2]  # across the boundary: minimum image
    bonds = np.array([[0, 1], [1, 2], [2, 3]])
    angles = np.array([[0, 1, 2], [1, 2, 3]])
    bk, br0 = np.array([300.0, 250.0, 400.0]), np.array([1.5, 1.45, 1.6])
    ak, at0 = np.array([50.0, 70.0]), np.array([1.91, 2.0])
    abox = np.broadcast_to(box, pos.shape)
    f, eb, ea = M.bonded(pos, abox, bonds, bk, br0, angles, ak, at0)
    h = 1e-6
    for a in range(4):
        for c in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[a, c] += h
            pm[a, c] -= h
            ep = sum(x.sum() for x in M.bonded(pp, abox, bonds, bk, br0, angles, ak, at0)[1:])
            em = sum(x.sum() for x in M.bonded(pm, abox, bonds, bk, br0, angles, ak, at0)[1:])
            assert abs(f[a, c] + (ep - em) / (2 * h)) < 1e-6 * max(1.0, abs(f[a, c]))
    assert np.max(np.abs(f.sum(0))) < 1e-10


def test_bonded_closed_forms():
    box = np.array([20.0, 20.0, 20.0])
    pos = np.array([[1.0, 1.0, 1.0], [2.6, 1.0, 1.0], [2.6, 3.0, 1.0]])
    abox = np.broadcast_to(box, pos.shape)
    f, eb, ea = M.bonded(pos, abox, np.array([[0, 1]]), np.array([300.0]), np.array([1.5]),
                         np.array([[0, 1, 2]]), np.array([50.0]), np.array([math.pi / 2]))
    assert eb[0] == pytest.approx(300.0 * 0.1 ** 2, rel=1e-13)
    assert ea[0] == pytest.approx(0.0, abs=1e-20)   # the angle is exactly 90 degrees
    # bond force on atom 0: +2 k (r - r0) toward atom 1 (stretched bond pulls)
    np.testing.assert_allclose(f[0], [2 * 300.0 * 0.1, 0, 0], rtol=1e-12)
    f2, _, ea2 = M.bonded(pos, abox, None, None, None, np.array([[0, 1, 2]]), np.array([50.0]),
                          np.array([math.pi / 3]))
    assert ea2[0] == pytest.approx(50.0 * (math.pi / 6) ** 2, rel=1e-13)
    # torque balance: for the pure angle term the forces on the end atoms are
    # perpendicular to their bonds, with |F_i| = dE/dtheta / |r_ij|
    de = 2 * 50.0 * (math.pi / 2 - math.pi / 3)
    assert np.linalg.norm(f2[0]) == pytest.approx(de / 1.6, rel=1e-12)
    assert np.linalg.norm(f2[2]) == pytest.approx(de / 2.0, rel=1e-12)
    assert abs(np.dot(f2[0], pos[0] - pos[1])) < 1e-12


def test_velocity_verlet_follows_the_exact_discrete_harmonic_solution():
    """Two atoms joined by a bond, no thermostat: the bond length obeys the velocity-Verlet
    recurrence of a harmonic oscillator, whose solution is delta cos(n theta) with
    cos(theta) = 1 - (omega dt)^2 / 2 and omega^2 = 2 k (1/m1 + 1/m2) * 100."""
    k, r0, delta = 300.0, 1.5, 0.05
    m = np.array([12.0, 16.0])
    dt = 0.002
    x = np.array([[5.0, 5.0, 5.0], [5.0 + r0 + delta, 5.0, 5.0]])
    v = np.zeros_like(x)
    abox = np.broadcast_to(np.array([30.0, 30.0, 30.0]), x.shape)
    topo = {}
    bonds, bk, br0 = np.array([[0, 1]]), np.array([k]), np.array([r0])
    force = lambda p: M.bonded(p, abox, bonds, bk, br0)[0]
    f = force(x)
    w2 = 2 * k * (1 / m[0] + 1 / m[1]) * M.ACCEL
    theta = math.acos(1 - w2 * dt * dt / 2)
    for n in range(1, 301):
        x, v, f = M.langevin_step(x, v, f, m, topo, abox, dt, 300.0, 0.0, 1, n, force)
        r = x[1, 0] - x[0, 0]
        assert r - r0 == pytest.approx(delta * math.cos(n * theta), abs=1e-12)
    # the centre of mass does not move
    assert (m @ x[:, 0]) / m.sum() == pytest.approx((m[0] * 5.0 + m[1] * (5.0 + r0 + delta)) / m.sum(), abs=1e-12)


def test_langevin_update_has_the_exact_mean_and_variance():
    """Free atoms (F = 0): after one step v' = c^2 v + noise with Var = (1 - c^4) kT/m * 100
    per component (two half-step updates), for every mass."""
    n = 60_000
    rng = np.random.default_rng(3)
    m = rng.choice([1.008, 12.011, 15.999], n)
    v0 = rng.standard_normal((n, 3)) * 3.0
    x = rng.uniform(0, 50, (n, 3))
    abox = np.broadcast_to(np.array([50.0, 50.0, 50.0]), x.shape)
    dt, T, gamma = 0.002, 300.0, 50.0
    zero = lambda p: np.zeros_like(p)
    x1, v1, _ = M.langevin_step(x, v0, np.zeros_like(x), m, {}, abox, dt, T, gamma, 99, 0, zero)
    c2 = math.exp(-gamma * dt)
    z = (v1 - c2 * v0) / np.sqrt((1 - c2 * c2) * M.ACCEL * M.KB * T / m)[:, None]
    assert np.all(np.abs(z.mean(0)) < 5 / math.sqrt(n))
    assert np.all(np.abs(z.var(0) - 1) < 5 * math.sqrt(2 / n))
    # the drift used the velocity after the first half-step update: x1 = x + dt (c v0 + noise)
    zc = (x1 - x) / dt - math.exp(-gamma * dt / 2) * v0
    sd1 = np.sqrt((1 - math.exp(-gamma * dt)) * M.ACCEL * M.KB * T / m)[:, None]
    assert np.all(np.abs((zc / sd1).var(0) - 1) < 5 * math.sqrt(2 / n))


def test_rigid_water_gas_has_six_degrees_of_freedom_per_molecule():
    """Non-interacting rigid waters under the thermostat: the mean kinetic energy is
    3 kT per molecule (three translational and three rotational degrees of freedom)."""
    n = 1500
    rng = np.random.default_rng(8)
    o = rng.uniform(0, 60, (n, 3))
    rot = S._random_rotations(rng, n)
    half = math.radians(S.HOH_ANGLE_DEG) / 2
    local = np.array([[0, 0, 0], [S.OH_BOND * math.sin(half), 0, S.OH_BOND * math.cos(half)],
                      [-S.OH_BOND * math.sin(half), 0, S.OH_BOND * math.cos(half)]])
    x = (o[:, None, :] + np.einsum("mij,aj->mai", rot, local)).reshape(-1, 3)
    m = np.tile([15.999, 1.008, 1.008], n)
    topo = dict(water_o=np.arange(0, 3 * n, 3), r_oh=S.OH_BOND, r_hh=M_HH)
    abox = np.broadcast_to(np.array([1e4, 1e4, 1e4]), x.shape)
    v = np.zeros_like(x)
    zero = lambda p: np.zeros_like(p)
    f = np.zeros_like(x)
    T, gamma, dt = 300.0, 20.0, 0.002
    ke = []
    for step in range(160):
        x, v, f = M.langevin_step(x, v, f, m, topo, abox, dt, T, gamma, 5, step, zero)
        if step >= 60:
            ke.append(M.kinetic_energy(v, m))
    assert _constraint_error(x, topo["water_o"], abox) < 1e-12
    ratio = np.mean(ke) / (3 * n * M.KB * T)
    assert abs(ratio - 1) < 0.03, ratio
