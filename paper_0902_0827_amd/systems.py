"""Seeded synthetic workloads: TIP3P-like water boxes with and without a bead-chain solute.

This module only builds inputs (positions, charges, Lennard-Jones type tables and
exclusion lists).  It holds none of the nonbonded arithmetic, so both the HIP
library's tests and the CPU oracle may take their inputs from it.

The paper measures on biomolecular systems solvated in TIP3P water (DHFR, apoA1,
Villin; section 5, Tables 3-5) that are not reproduced here.  These generators
build stand-ins with the same density, charge model and exclusion structure:

* water: rigid TIP3P-like geometry (O-H 0.9572 A, H-O-H 104.52 deg), charges
  O -0.834 e and H +0.417 e, Lennard-Jones on O only (sigma 3.15061 A,
  epsilon 0.6364 kJ/mol), intramolecular O-H1, O-H2, H1-H2 exclusions;
* solute: a self-avoiding bead chain (bond 1.5 A) with random charges shifted to
  a net charge of zero, eight Lennard-Jones types drawn from sigma U[2.5, 3.8] A
  and epsilon U[0.1, 0.9] kJ/mol, and 1-2 / 1-3 exclusions (section 3 describes
  the bonded exclusions the pair kernel must skip).

Atoms are molecule-contiguous (solute first, then O, H1, H2 per water), so every
exclusion sits within a small index window.  Units: Angstrom, e, kJ/mol.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Water model.
OH_BOND = 0.9572
HOH_ANGLE_DEG = 104.52
Q_O = -0.834
Q_H = 0.417
SIGMA_O = 3.15061
EPS_O = 0.6364
MASS_WATER = 15.999 + 2 * 1.008  # g/mol
MASS_BEAD = 14.027  # g/mol (CH2-like united atom; the chain recipe names no mass)
AVOGADRO = 6.02214076e23

# Type table shared by every system: 0 = water O, 1 = water H, 2..9 = solute.  The
# solute types are one fixed draw (a force field), so that any systems can be batched.
FORCE_FIELD_SEED = 20090205
TYPE_O = 0
TYPE_H = 1
N_SOLUTE_TYPES = 8
N_TYPES = 2 + N_SOLUTE_TYPES

BOND = 1.5
MIN_13 = 2.0
MIN_BEAD = 3.0
MIN_WATER_BEAD = 2.5


@dataclasses.dataclass
class System:
    """One periodic system.  Arrays are numpy, positions in float64."""

    name: str
    pos: np.ndarray  # [N, 3] float64, wrapped into [0, L)
    charge: np.ndarray  # [N] float64 (e)
    type: np.ndarray  # [N] int32
    sigma: np.ndarray  # [T] float64 (A)
    eps: np.ndarray  # [T] float64 (kJ/mol)
    excl_offset: np.ndarray  # [N+1] int32, CSR rows (both directions listed)
    excl_index: np.ndarray  # [n_excl] int32, sorted within each row
    box: np.ndarray  # [3] float64
    cutoff: float
    beta: float
    seed: int
    n_solute: int = 0
    # Scaled 1-4 pairs (CSR rows like the exclusions), or None: the solute chain's i, i+3
    # pairs (with_chain_14).  Water has none.
    pair14_offset: Optional[np.ndarray] = None
    pair14_index: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def rounded(self, dtype) -> "System":
        """Copy whose positions and charges are rounded to ``dtype`` and promoted back.

        The oracle is always given exactly the values the device receives.
        """
        s = dataclasses.replace(self)
        s.pos = self.pos.astype(dtype).astype(np.float64)
        s.charge = self.charge.astype(dtype).astype(np.float64)
        return s


def _random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random rotation matrices from normalised Gaussian quaternions."""
    qv = rng.standard_normal((n, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    r = np.empty((n, 3, 3))
    r[:, 0, 0] = 1 - 2 * (y * y + z * z)
    r[:, 0, 1] = 2 * (x * y - z * w)
    r[:, 0, 2] = 2 * (x * z + y * w)
    r[:, 1, 0] = 2 * (x * y + z * w)
    r[:, 1, 1] = 1 - 2 * (x * x + z * z)
    r[:, 1, 2] = 2 * (y * z - x * w)
    r[:, 2, 0] = 2 * (x * z - y * w)
    r[:, 2, 1] = 2 * (y * z + x * w)
    r[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return r


def _water_sites(rng: np.random.Generator, oxygens: np.ndarray) -> np.ndarray:
    """[M,3] oxygen positions -> [3M,3] O,H1,H2 positions with random orientation."""
    half = math.radians(HOH_ANGLE_DEG) / 2
    local = np.array(
        [[0.0, 0.0, 0.0],
         [OH_BOND * math.sin(half), 0.0, OH_BOND * math.cos(half)],
         [-OH_BOND * math.sin(half), 0.0, OH_BOND * math.cos(half)]]
    )
    rot = _random_rotations(rng, oxygens.shape[0])
    atoms = oxygens[:, None, :] + np.einsum("mij,aj->mai", rot, local)
    return atoms.reshape(-1, 3)


def _type_table(rng: Optional[np.random.Generator] = None):
    if rng is None:
        rng = np.random.default_rng(FORCE_FIELD_SEED)
    sig = np.empty(N_TYPES)
    eps = np.empty(N_TYPES)
    sig[TYPE_O], eps[TYPE_O] = SIGMA_O, EPS_O
    sig[TYPE_H], eps[TYPE_H] = 0.0, 0.0
    sig[2:] = rng.uniform(2.5, 3.8, N_SOLUTE_TYPES)
    eps[2:] = rng.uniform(0.1, 0.9, N_SOLUTE_TYPES)
    return sig, eps


def _minimage(d: np.ndarray, box: np.ndarray) -> np.ndarray:
    return d - box * np.rint(d / box)


class _Grid:
    """Bucket grid for neighbour queries while placing beads (generator only)."""

    def __init__(self, box: np.ndarray, width: float):
        self.box = box
        self.n = np.maximum((box // width).astype(int), 1)
        self.w = box / self.n
        self.cells = {}

    def key(self, p):
        c = np.floor(np.mod(p, self.box) / self.w).astype(int) % self.n
        return (int(c[0]), int(c[1]), int(c[2]))

    def add(self, idx, p):
        self.cells.setdefault(self.key(p), []).append(idx)

    def remove(self, idx, p):
        self.cells[self.key(p)].remove(idx)

    def near(self, p):
        c = self.key(p)
        seen = set()
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    k = ((c[0] + dx) % self.n[0], (c[1] + dy) % self.n[1], (c[2] + dz) % self.n[2])
                    if k in seen:
                        continue
                    seen.add(k)
                    yield from self.cells.get(k, ())


def _chain(rng: np.random.Generator, n_beads: int, box: np.ndarray) -> np.ndarray:
    """Self-avoiding bead chain: bond BOND, 1-3 distance >= MIN_13, other pairs >= MIN_BEAD.

    Each step draws a batch of candidate directions and keeps the first candidate that
    satisfies every constraint (minimum image); a trapped chain backs off and regrows."""
    if n_beads == 0:
        return np.zeros((0, 3))
    # Candidates lie BOND from the last bead, so neighbours within MIN_BEAD of a candidate
    # are within MIN_BEAD + BOND of the last bead: the grid cells must be that wide.
    grid = _Grid(box, MIN_BEAD + BOND)
    pos = np.zeros((n_beads, 3))
    pos[0] = rng.uniform(0, 1, 3) * box
    grid.add(0, pos[0])
    k = 1
    fails = 0
    n_try = 32
    while k < n_beads:
        u = rng.standard_normal((n_try, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        cand = pos[k - 1] + BOND * u
        ok = np.ones(n_try, dtype=bool)
        if k >= 2:
            d13 = _minimage(cand - pos[k - 2], box)
            ok &= np.einsum("ij,ij->i", d13, d13) >= MIN_13 ** 2
        near = [j for j in grid.near(pos[k - 1]) if j < k - 2]
        if near:
            d = _minimage(cand[:, None, :] - pos[near][None, :, :], box)
            ok &= (np.einsum("cnk,cnk->cn", d, d) >= MIN_BEAD ** 2).all(axis=1)
        hit = np.flatnonzero(ok)
        if hit.size:
            pos[k] = cand[hit[0]]
            grid.add(k, pos[k])
            k += 1
            fails = 0
        else:
            fails += 1
            if fails % 2 == 0:
                # Trapped: back off a few beads and regrow.
                back = min(k - 1, 2 * fails)
                for j in range(k - back, k):
                    grid.remove(j, pos[j])
                k -= back
    return np.mod(pos, box)


def _free_sites(n_side: int, box: np.ndarray, beads: np.ndarray) -> np.ndarray:
    """Lattice sites (i + 1/2) L / n_side whose minimum-image distance to every bead is
    at least MIN_WATER_BEAD."""
    a = box / n_side
    g = (np.arange(n_side) + 0.5)
    sites = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) * a
    if beads.shape[0] == 0:
        return sites
    from scipy.spatial import cKDTree
    tree = cKDTree(np.mod(beads, box), boxsize=box)
    dist, _ = tree.query(np.mod(sites, box), k=1)
    return sites[dist >= MIN_WATER_BEAD]


def _exclusions_csr(n: int, pairs: np.ndarray):
    """Undirected pairs [P,2] -> CSR listing every pair in both rows, rows sorted."""
    if pairs.size == 0:
        return np.zeros(n + 1, np.int32), np.zeros(0, np.int32)
    a = np.concatenate([pairs[:, 0], pairs[:, 1]])
    b = np.concatenate([pairs[:, 1], pairs[:, 0]])
    order = np.lexsort((b, a))
    a, b = a[order], b[order]
    off = np.zeros(n + 1, np.int64)
    np.add.at(off, a + 1, 1)
    return np.cumsum(off).astype(np.int32), b.astype(np.int32)


def _assemble(name, seed, box, beads, bead_q, bead_t, waters_o, rng, sig, eps, cutoff, beta):
    n_s = beads.shape[0]
    n_w = waters_o.shape[0]
    wat = _water_sites(rng, waters_o)
    pos = np.mod(np.concatenate([beads, wat]), box)
    q = np.concatenate([bead_q, np.tile([Q_O, Q_H, Q_H], n_w)])
    t = np.concatenate([bead_t, np.tile([TYPE_O, TYPE_H, TYPE_H], n_w)]).astype(np.int32)
    pairs = []
    if n_s > 1:
        i = np.arange(n_s - 1)
        pairs.append(np.stack([i, i + 1], 1))
    if n_s > 2:
        i = np.arange(n_s - 2)
        pairs.append(np.stack([i, i + 2], 1))
    if n_w:
        o = n_s + 3 * np.arange(n_w)
        pairs += [np.stack([o, o + 1], 1), np.stack([o, o + 2], 1), np.stack([o + 1, o + 2], 1)]
    pairs = np.concatenate(pairs) if pairs else np.zeros((0, 2), np.int64)
    off, idx = _exclusions_csr(pos.shape[0], pairs)
    return System(name=name, pos=pos, charge=q, type=t, sigma=sig.copy(), eps=eps.copy(),
                  excl_offset=off, excl_index=idx, box=np.asarray(box, float), cutoff=float(cutoff),
                  beta=float(beta), seed=seed, n_solute=n_s)


def water_lattice(n_side: int, spacing: float, seed: int, cutoff: float, beta: float,
                  n_waters: Optional[int] = None, name: str = "water") -> System:
    """Waters with O on an n_side^3 lattice ((i+1/2)*spacing); optionally a random subset."""
    rng = np.random.default_rng(seed)
    sig, eps = _type_table()
    L = n_side * spacing
    box = np.array([L, L, L])
    g = (np.arange(n_side) + 0.5) * spacing
    sites = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    if n_waters is not None and n_waters < sites.shape[0]:
        sites = sites[np.sort(rng.choice(sites.shape[0], n_waters, replace=False))]
    return _assemble(name, seed, box, np.zeros((0, 3)), np.zeros(0), np.zeros(0, np.int32), sites,
                     rng, sig, eps, cutoff, beta)


def solvated_chain(L: float, n_beads: int, n_waters: int, seed: int, cutoff: float, beta: float,
                   n_side: Optional[int] = None, type_seed: Optional[int] = None,
                   name: str = "chain+water") -> System:
    """A self-avoiding bead chain in a cubic box, then waters on free lattice sites."""
    rng = np.random.default_rng(seed)
    sig, eps = _type_table(None if type_seed is None else np.random.default_rng(type_seed))
    box = np.array([L, L, L], float)
    beads = _chain(rng, n_beads, box)
    q = rng.uniform(-0.5, 0.5, n_beads)
    if n_beads:
        q -= q.mean()
    t = rng.integers(2, 2 + N_SOLUTE_TYPES, n_beads).astype(np.int32)
    if n_side is None:
        n_side = max(1, math.ceil(n_waters ** (1 / 3)))
        while True:
            free = _free_sites(n_side, box, beads)
            if free.shape[0] >= n_waters:
                break
            n_side += 1
    else:
        free = _free_sites(n_side, box, beads)
        if free.shape[0] < n_waters:
            raise ValueError("not enough free lattice sites for the requested waters")
    chosen = free[np.sort(rng.choice(free.shape[0], n_waters, replace=False))]
    return _assemble(name, seed, box, beads, q, t, chosen, rng, sig, eps, cutoff, beta)


# --- the five workloads -----------------------------------------------------------------

def config1(seed: int = 1) -> System:
    """216 waters (648 atoms) on a 6^3 lattice of 3.1 A, L = 18.6 A, rc 9 A, beta 0.34 /A."""
    return water_lattice(6, 3.1, seed, 9.0, 0.34, name="water216")


def config2(seed: int = 2) -> System:
    """23,600 atoms, L = 60 A: a 2,000-bead chain plus 7,200 waters; rc 9 A, beta 0.34 /A."""
    return solvated_chain(60.0, 2000, 7200, seed, 9.0, 0.34, n_side=22, name="chain2000+water7200")


def config3(seed: int = 3) -> System:
    """The 23.6k-atom chain-plus-water system used for gradients (same recipe as config 2)."""
    s = solvated_chain(60.0, 2000, 7200, seed, 9.0, 0.34, n_side=22, name="chain2000+water7200")
    return s


def config4(seed: int = 4, n_systems: int = 64) -> List[System]:
    """Uneven replicas: N log-uniform in [3000, 30000], density 0.95-1.05 g/cm^3,
    solute fraction U[0, 0.1]; rc 9 A, beta 0.34 /A.  All share one type table."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n_systems):
        n_b = int(round(math.exp(rng.uniform(math.log(3000), math.log(30000)))))
        frac = rng.uniform(0.0, 0.10)
        n_s = int(round(frac * n_b))
        n_w = int(round((n_b - n_s) / 3))
        rho = rng.uniform(0.95, 1.05)
        mass = n_w * MASS_WATER + n_s * MASS_BEAD
        L = (mass / AVOGADRO / rho) ** (1 / 3) * 1e8
        sub_seed = int(rng.integers(0, 2**31 - 1))
        out.append(solvated_chain(L, n_s, n_w, sub_seed, 9.0, 0.34, name=f"replica{b}"))
    return out


def config5(seed: int = 5) -> System:
    """333,333 waters (999,999 atoms) on a random subset of a 70^3 lattice, L = 215 A,
    rc 12 A, beta 0.26 /A."""
    return water_lattice(70, 215.0 / 70, seed, 12.0, 0.26, n_waters=333_333, name="water333k")


def water_box(n_waters: int, L: float, seed: int, cutoff: float = 9.0, beta: float = 0.34) -> System:
    """Water at the lattice density closest to n_waters in an L box (for scans and tests)."""
    n_side = max(1, math.ceil(n_waters ** (1 / 3)))
    return water_lattice(n_side, L / n_side, seed, cutoff, beta, n_waters=n_waters,
                         name=f"water{n_waters}")


def with_chain_14(s: System) -> System:
    """Copy of a system whose solute chain (the first n_solute atoms, bonded in order) lists
    its 1-4 pairs (i, i + 3), in both rows, as scaled pairs."""
    rows = [[] for _ in range(s.n)]
    for i in range(max(s.n_solute - 3, 0)):
        rows[i].append(i + 3)
        rows[i + 3].append(i)
    off = np.zeros(s.n + 1, np.int32)
    off[1:] = np.cumsum([len(r) for r in rows])
    t = dataclasses.replace(s)
    t.pair14_offset = off
    t.pair14_index = np.array([j for r in rows for j in sorted(r)], np.int32)
    return t


# Stand-in bonded force field of the bead chain for the MD loop (the chain recipe names
# none): harmonic bonds at the chain's bond length and harmonic angles.
MASS_O = 15.999
MASS_H = 1.008
CHAIN_BOND_K = 300.0                     # kJ/mol/A^2
CHAIN_ANGLE_K = 50.0                     # kJ/mol/rad^2
CHAIN_ANGLE_THETA0 = math.radians(109.5)


def water_hh() -> float:
    """H-H distance of the rigid water geometry."""
    return 2.0 * OH_BOND * math.sin(math.radians(HOH_ANGLE_DEG) / 2)


def md_topology(system: System) -> dict:
    """Masses, rigid waters (O indices) and the chain's bonds and angles of one system,
    with atom indices local to it."""
    n, n_s = system.n, system.n_solute
    n_w = (n - n_s) // 3
    mass = np.full(n, MASS_BEAD)
    mass[n_s:] = np.tile([MASS_O, MASS_H, MASS_H], n_w)
    i = np.arange(max(n_s - 1, 0))
    bonds = np.stack([i, i + 1], 1).astype(np.int32).reshape(-1, 2)
    j = np.arange(max(n_s - 2, 0))
    angles = np.stack([j, j + 1, j + 2], 1).astype(np.int32).reshape(-1, 3)
    return dict(mass=mass, water_o=(n_s + 3 * np.arange(n_w)).astype(np.int32), r_oh=OH_BOND, r_hh=water_hh(),
                bonds=bonds, bond_k=np.full(len(bonds), CHAIN_BOND_K), bond_r0=np.full(len(bonds), BOND),
                angles=angles, angle_k=np.full(len(angles), CHAIN_ANGLE_K),
                angle_theta0=np.full(len(angles), CHAIN_ANGLE_THETA0))


def concat_topologies(topos: List[dict], sizes) -> dict:
    """Batch layout of per-system md_topology dicts: atom indices shifted by each system's
    offset."""
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cat = lambda key, shift: np.concatenate([t[key] + (offs[k] if shift else 0) for k, t in enumerate(topos)])
    return dict(mass=cat("mass", False), water_o=cat("water_o", True).astype(np.int32),
                r_oh=topos[0]["r_oh"], r_hh=topos[0]["r_hh"],
                bonds=cat("bonds", True).astype(np.int32).reshape(-1, 2), bond_k=cat("bond_k", False),
                bond_r0=cat("bond_r0", False), angles=cat("angles", True).astype(np.int32).reshape(-1, 3),
                angle_k=cat("angle_k", False), angle_theta0=cat("angle_theta0", False))


def concat_systems(systems: List[System]):
    """Pack systems back to back (batch layout): returns a dict of concatenated arrays.

    The Lennard-Jones type table is shared by a batch, so every system must carry the same one."""
    for s in systems[1:]:
        if not (np.array_equal(s.sigma, systems[0].sigma) and np.array_equal(s.eps, systems[0].eps)):
            raise ValueError("systems in a batch must share one Lennard-Jones type table")
    offs = np.zeros(len(systems) + 1, np.int64)
    offs[1:] = np.cumsum([s.n for s in systems])
    excl_off = [np.zeros(1, np.int64)]
    base = 0
    for s in systems:
        excl_off.append(s.excl_offset[1:].astype(np.int64) + base)
        base += int(s.excl_offset[-1])
    p14_off, p14_idx = None, None
    if any(s.pair14_offset is not None for s in systems):
        p14_off = [np.zeros(1, np.int64)]
        base = 0
        for s in systems:
            o = s.pair14_offset if s.pair14_offset is not None else np.zeros(s.n + 1, np.int32)
            p14_off.append(o[1:].astype(np.int64) + base)
            base += int(o[-1])
        p14_off = np.concatenate(p14_off).astype(np.int32)
        p14_idx = np.concatenate([s.pair14_index for s in systems if s.pair14_index is not None]
                                 + [np.zeros(0, np.int32)]).astype(np.int32)
    return dict(
        atom_offset=offs,
        pair14_offset=p14_off,
        pair14_index=p14_idx,
        pos=np.concatenate([s.pos for s in systems]),
        charge=np.concatenate([s.charge for s in systems]),
        type=np.concatenate([s.type for s in systems]),
        excl_offset=np.concatenate(excl_off).astype(np.int32),
        excl_index=np.concatenate([s.excl_index for s in systems]).astype(np.int32),
        box=np.stack([s.box for s in systems]),
        sigma=systems[0].sigma,
        eps=systems[0].eps,
    )
