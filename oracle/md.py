"""FP64 oracle of the molecular-dynamics loop around the force evaluation: bonded terms,
rigid-water constraints, the noise of the thermostat and the velocity-Verlet step with a
Langevin thermostat.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this module; the GPU library never does.  It shares no code
with the GPU library.

ACEMD paper, section 3 ("Molecular dynamics on the GPU"): production runs in the NVT
ensemble evaluate bonded and nonbonded forces, integrate with velocity Verlet under a
Langevin thermostat, use PME electrostatics and constrain bonds to hydrogen; Table 5
reports ns/day at a 4 fs step with PME every step.  The paper names neither the way the
thermostat is split into the Verlet step nor the constraint algorithm.  The readings
taken here (one definition, the same for the GPU library):

* Step (velocity Verlet between two half-step Ornstein-Uhlenbeck velocity updates, the
  Langevin integrator of Bussi and Parrinello, Phys. Rev. E 75, 056707 (2007)), with
  c = exp(-gamma dt/2) and xi, xi' independent standard normal vectors:
      v <- c v + sqrt(1 - c^2) s_i xi                      (s_i^2 = kT/m_i)
      v <- v + (dt/2) F(x)/m
      x' <- x + dt v;  x' <- SHAKE(x, x');  v <- (x' - x)/dt
      v <- v + (dt/2) F(x')/m
      v <- c v + sqrt(1 - c^2) s_i xi'
      v <- RATTLE(x', v)
  gamma = 0 leaves plain velocity Verlet with constraints.
* Constraints: rigid 3-site waters (O-H1, O-H2, H1-H2 at fixed lengths).  Positions by
  SHAKE (Ryckaert, Ciccotti and Berendsen, J. Comput. Phys. 23, 327 (1977)): the
  displacement of each constrained pair is along its bond vector before the move; here
  iterated one constraint at a time until every length holds to 1e-14 relative.
  Velocities by RATTLE's second half (Andersen, J. Comput. Phys. 52, 24 (1983)): the
  component of each bond's relative velocity along the bond removed, iterated likewise.
* Bonded terms (CHARMM form): E = k (r - r0)^2 per bond, k (theta - theta0)^2 per angle.
* Noise: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11) with counter
  (atom, step mod 2^32, step div 2^32, half) and key (seed mod 2^32, seed div 2^32); its
  four words u_k give uniforms (u_k + 1/2)/2^32 and, by the Box-Muller transform, the
  normals xi_x, xi_y from (u_0, u_1) and xi_z from (u_2, u_3).  half = 0 for the first
  thermostat update of a step, 1 for the second.

Units: Angstrom, ps, g/mol, kJ/mol, K.  F/m in (kJ/mol/A)/(g/mol) is 100 A/ps^2, and kT/m
in (kJ/mol)/(g/mol) is 100 A^2/ps^2 of velocity variance.
"""

from __future__ import annotations

import numpy as np

from . import oracle as O
from . import pme as P

ACCEL = 100.0                 # (kJ/mol/A)/(g/mol) in A/ps^2
KB = 8.314462618e-3           # molar gas constant, kJ/mol/K (CODATA 2018, exact)
KE_UNIT = 0.01                # g/mol A^2/ps^2 in kJ/mol

_M0, _M1 = 0xD2511F53, 0xCD9E8D57   # Philox4x32 round multipliers
_W0, _W1 = 0x9E3779B9, 0xBB67AE85   # Philox key increments (Weyl sequence)
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.  ctr [..., 4] and key [..., 2] of uint32 values (any
    integer dtype); returns [..., 4] uint64 holding the 32-bit outputs.  A round takes
    the 64-bit products M0 c0 and M1 c2 and outputs (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2),
    hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key advances by (W0, W1) between rounds."""
    c = np.asarray(ctr, dtype=np.uint64) & _MASK
    k = np.asarray(key, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = (c[..., j].copy() for j in range(4))
    k0, k1 = k[..., 0].copy(), k[..., 1].copy()
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = np.uint64(_M0) * c0
        p1 = np.uint64(_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], -1)


def normals(seed: int, step: int, half: int, atoms) -> np.ndarray:
    """[n, 3] standard normals of the thermostat for global atom indices `atoms`."""
    atoms = np.asarray(atoms, np.int64)
    n = atoms.shape[0]
    ctr = np.zeros((n, 4), np.uint64)
    ctr[:, 0] = atoms.astype(np.uint64)
    ctr[:, 1] = step & _MASK
    ctr[:, 2] = (step >> 32) & _MASK
    ctr[:, 3] = half
    key = np.broadcast_to(np.array([seed & _MASK, (seed >> 32) & _MASK], np.uint64), (n, 2))
    u = (philox4x32_10(ctr, key).astype(np.float64) + 0.5) / 2.0 ** 32
    r01 = np.sqrt(-2.0 * np.log(u[:, 0]))
    r23 = np.sqrt(-2.0 * np.log(u[:, 2]))
    return np.stack([r01 * np.cos(2 * np.pi * u[:, 1]), r01 * np.sin(2 * np.pi * u[:, 1]),
                     r23 * np.cos(2 * np.pi * u[:, 3])], -1)


def _minimage(d, box):
    return d - box * np.rint(d / box)


def _system_box(atom_offset, boxes, n):
    """[n, 3] box of every atom's system."""
    sys_of = np.searchsorted(np.asarray(atom_offset)[1:], np.arange(n), side="right")
    return np.asarray(boxes, np.float64).reshape(-1, 3)[sys_of]


def _water_constraints(water_o, r_oh, r_hh):
    """(i, j, length) of the three constraints of every water."""
    o = np.asarray(water_o, np.int64)
    i = np.concatenate([o, o, o + 1])
    j = np.concatenate([o + 1, o + 2, o + 2])
    d = np.concatenate([np.full(o.size, r_oh), np.full(o.size, r_oh), np.full(o.size, r_hh)])
    return i, j, d


def shake(x_old, x_new, mass, water_o, r_oh, r_hh, abox, tol=1e-14, max_iter=5000):
    """SHAKE: returns x_new moved so that every water constraint holds, each pair moved
    along its bond vector in x_old, in inverse proportion to the masses."""
    x = np.array(x_new, np.float64, copy=True)
    ci, cj, cd = _water_constraints(water_o, r_oh, r_hh)
    if ci.size == 0:
        return x
    s_old = _minimage(x_old[ci] - x_old[cj], abox[ci])
    wi, wj = 1.0 / mass[ci], 1.0 / mass[cj]
    nw = np.asarray(water_o).size
    # a length cannot be resolved below the rounding of the coordinates it comes from
    tol = max(tol, 8.0 * np.finfo(np.float64).eps * float(np.max(np.abs(x))) / float(np.min(cd)))
    for _ in range(max_iter):
        worst = 0.0
        for c in range(3):  # constraint c of every water at once (they share no atoms)
            sl = slice(c * nw, (c + 1) * nw)
            i, j, d = ci[sl], cj[sl], cd[sl]
            s = _minimage(x[i] - x[j], abox[i])
            diff = d * d - np.einsum("ij,ij->i", s, s)
            worst = max(worst, float(np.max(np.abs(diff) / (d * d))))
            g = diff / (2.0 * (wi[sl] + wj[sl]) * np.einsum("ij,ij->i", s, s_old[sl]))
            x[i] += (g * wi[sl])[:, None] * s_old[sl]
            x[j] -= (g * wj[sl])[:, None] * s_old[sl]
        if worst < tol:
            return x
    raise RuntimeError("SHAKE did not converge")


def rattle_velocities(x, v, mass, water_o, r_oh, r_hh, abox, tol=1e-15, max_iter=5000):
    """RATTLE (velocity half): v with every constrained pair's relative velocity along
    its bond removed, the change split in inverse proportion to the masses."""
    v = np.array(v, np.float64, copy=True)
    ci, cj, cd = _water_constraints(water_o, r_oh, r_hh)
    if ci.size == 0:
        return v
    s = _minimage(x[ci] - x[cj], abox[ci])
    wi, wj = 1.0 / mass[ci], 1.0 / mass[cj]
    nw = np.asarray(water_o).size
    vscale = max(float(np.max(np.abs(v))), 1e-300)
    for _ in range(max_iter):
        worst = 0.0
        for c in range(3):
            sl = slice(c * nw, (c + 1) * nw)
            i, j = ci[sl], cj[sl]
            ss = np.einsum("ij,ij->i", s[sl], s[sl])
            rv = np.einsum("ij,ij->i", v[i] - v[j], s[sl])
            worst = max(worst, float(np.max(np.abs(rv) / (np.sqrt(ss) * vscale))))
            k = rv / (ss * (wi[sl] + wj[sl]))
            v[i] -= (k * wi[sl])[:, None] * s[sl]
            v[j] += (k * wj[sl])[:, None] * s[sl]
        if worst < tol:
            return v
    raise RuntimeError("RATTLE did not converge")


def bonded(pos, abox, bonds=None, bond_k=None, bond_r0=None, angles=None, angle_k=None, angle_theta0=None):
    """Harmonic bonds E = k (r - r0)^2 and angles E = k (theta - theta0)^2 (theta at the
    middle atom), minimum image.  Returns (force [N,3], energy per term: bonds, angles)."""
    f = np.zeros_like(pos, dtype=np.float64)
    eb = np.zeros(0)
    ea = np.zeros(0)
    if bonds is not None and len(bonds):
        i, j = bonds[:, 0], bonds[:, 1]
        d = _minimage(pos[i] - pos[j], abox[i])
        r = np.linalg.norm(d, axis=1)
        eb = bond_k * (r - bond_r0) ** 2
        g = (-2.0 * bond_k * (r - bond_r0) / r)[:, None] * d   # force on i
        np.add.at(f, i, g)
        np.add.at(f, j, -g)
    if angles is not None and len(angles):
        i, j, k = angles[:, 0], angles[:, 1], angles[:, 2]
        u = _minimage(pos[i] - pos[j], abox[j])
        w = _minimage(pos[k] - pos[j], abox[j])
        lu, lw = np.linalg.norm(u, axis=1), np.linalg.norm(w, axis=1)
        cos = np.clip(np.einsum("ij,ij->i", u, w) / (lu * lw), -1.0, 1.0)
        th = np.arccos(cos)
        ea = angle_k * (th - angle_theta0) ** 2
        de = 2.0 * angle_k * (th - angle_theta0)          # dE/dtheta
        sin = np.sqrt(np.maximum(1.0 - cos * cos, 1e-300))
        # d(cos)/du = w/(|u||w|) - cos u/|u|^2, dtheta = -d(cos)/sin
        fi = (de / sin)[:, None] * (w / (lu * lw)[:, None] - (cos / lu ** 2)[:, None] * u)
        fk = (de / sin)[:, None] * (u / (lu * lw)[:, None] - (cos / lw ** 2)[:, None] * w)
        np.add.at(f, i, fi)
        np.add.at(f, k, fk)
        np.add.at(f, j, -(fi + fk))
    return f, eb, ea


def total_forces(system, topo, pos, pme_grid=None, ke: float = O.COULOMB_K, nthreads: int = 0, **ff):
    """Every force of the loop at `pos` for one system: the short-range nonbonded term,
    and with a PME grid the Ewald corrections and the reciprocal part, plus the bonded
    terms.  Returns (force [N,3], dict of energies)."""
    s = system
    r = O.evaluate(pos, s.charge, s.type, s.sigma, s.eps, s.excl_offset, s.excl_index, s.box, s.cutoff,
                   s.beta, nthreads=nthreads, ke=ke, pair14_offset=getattr(s, "pair14_offset", None),
                   pair14_index=getattr(s, "pair14_index", None), **ff)
    f = r["force"].copy()
    e = dict(nonbonded=r["energy_total"], corrections=0.0, reciprocal=0.0)
    if pme_grid is not None:
        c = O.ewald_corrections(pos, s.charge, s.excl_offset, s.excl_index, s.box, s.beta, ke=ke,
                                pair14_offset=getattr(s, "pair14_offset", None),
                                pair14_index=getattr(s, "pair14_index", None),
                                scale14_coul=ff.get("scale14_coul", 1.0))
        k = P.spme_reciprocal(pos, s.charge, s.box, s.beta, pme_grid, ke=ke)
        f += c["force"] + k["force"]
        e["corrections"] = c["energy_total"]
        e["reciprocal"] = k["energy"]
    abox = np.broadcast_to(np.asarray(s.box, np.float64), pos.shape)
    fb, eb, ea = bonded(pos, abox, topo.get("bonds"), topo.get("bond_k"), topo.get("bond_r0"),
                        topo.get("angles"), topo.get("angle_k"), topo.get("angle_theta0"))
    e["bonded"] = float(eb.sum() + ea.sum())
    return f + fb, e


def langevin_step(x, v, f, mass, topo, abox, dt, temperature, gamma, seed, step, force_fn):
    """One step of the integrator above from (x, v, F(x)); force_fn(x) -> F(x).
    Returns (x', v', F(x'))."""
    n = x.shape[0]
    c = np.exp(-gamma * dt / 2.0)
    sd = np.sqrt((1.0 - c * c) * ACCEL * KB * temperature / mass)[:, None]
    atoms = np.arange(n)
    m = mass[:, None]
    w_o, r_oh, r_hh = topo.get("water_o", np.zeros(0, np.int64)), topo.get("r_oh", 0.0), topo.get("r_hh", 0.0)
    v = c * v + sd * normals(seed, step, 0, atoms)
    v = v + 0.5 * dt * ACCEL * f / m
    xn = shake(x, x + dt * v, mass, w_o, r_oh, r_hh, abox)
    v = (xn - x) / dt
    fn = force_fn(xn)
    v = v + 0.5 * dt * ACCEL * fn / m
    v = c * v + sd * normals(seed, step, 1, atoms)
    v = rattle_velocities(xn, v, mass, w_o, r_oh, r_hh, abox)
    return xn, v, fn


def kinetic_energy(v, mass) -> float:
    return float(0.5 * KE_UNIT * np.sum(mass[:, None] * v * v))
