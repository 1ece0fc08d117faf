"""FP64 oracle for the reciprocal part of the Ewald sum: the plain k-space sum and its
smooth particle-mesh (SPME) approximation.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this module; the GPU library never does.  It shares no code
with the GPU library.

ACEMD paper, section 3: the long-range electrostatics are particle-mesh Ewald with
fourth-order interpolation on a 64^3 grid (the method of Essmann et al., J. Chem. Phys.
103, 8577 (1995)).  With k_e the Coulomb constant, V the box volume, beta the Ewald
splitting parameter and m = (n1/L1, n2/L2, n3/L3) the reciprocal vectors:

  plain sum     E = k_e/(2 pi V) sum_{m != 0} exp(-pi^2 m^2/beta^2)/m^2 |S(m)|^2,
                S(m) = sum_j q_j exp(2 pi i m.r_j)
  SPME          S(m) is replaced by the discrete Fourier transform of the charge grid
                Q(k) = sum_i q_i prod_a M_n(u_ai - k_a) (periodic in k), u_ai = K_a x_ai/L_a,
                and each term is multiplied by B(m) = prod_a |b_a(m_a)|^2 with
                b_a(m) = exp(2 pi i (n-1) m/K_a) / sum_{k=0}^{n-2} M_n(k+1) exp(2 pi i m k/K_a).

M_n is the cardinal B-spline of order n.  Forces are -dE/dx; the virial is
W_ab = -dE/d(strain_ab) = sum_m E_m [delta_ab - 2 (1 + pi^2 m^2/beta^2) m_a m_b / m^2].
The m = 0 term is omitted (no neutralising-background term for a charged system).
"""

from __future__ import annotations

import numpy as np

from .oracle import COULOMB_K


def cardinal_bspline(x, n: int):
    """M_n(x): M_2(x) = 1 - |x - 1| on [0, 2] and 0 elsewhere;
    M_n(x) = [x M_{n-1}(x) + (n - x) M_{n-1}(x - 1)] / (n - 1)."""
    x = np.asarray(x, np.float64)
    if n == 2:
        return np.where((x >= 0.0) & (x <= 2.0), 1.0 - np.abs(x - 1.0), 0.0)
    return (x * cardinal_bspline(x, n - 1) + (n - x) * cardinal_bspline(x - 1.0, n - 1)) / (n - 1)


def cardinal_bspline_deriv(x, n: int):
    """dM_n/dx = M_{n-1}(x) - M_{n-1}(x - 1)."""
    return cardinal_bspline(x, n - 1) - cardinal_bspline(np.asarray(x, np.float64) - 1.0, n - 1)


def _mvec(K: int, L: float):
    """Reciprocal components n/L of the grid index 0..K-1 (n = i for i <= K/2, else i - K)."""
    i = np.arange(K)
    return np.where(i <= K // 2, i, i - K) / L


def _bmod2(K: int, n: int):
    """|b(m)|^2 for m = 0..K-1."""
    m = np.arange(K)
    k = np.arange(n - 1)
    den = (cardinal_bspline(k + 1.0, n)[None, :] * np.exp(2j * np.pi * np.outer(m, k) / K)).sum(axis=1)
    return 1.0 / np.abs(den) ** 2


def _kspace_terms(m2, mx, my, mz, beta):
    """exp(-pi^2 m^2/beta^2)/m^2 (0 at m = 0) and the virial factor 2 (1 + pi^2 m^2/beta^2)/m^2."""
    with np.errstate(divide="ignore", invalid="ignore"):
        c = np.where(m2 > 0, np.exp(-np.pi ** 2 * m2 / beta ** 2) / m2, 0.0)
        v = np.where(m2 > 0, 2.0 * (1.0 + np.pi ** 2 * m2 / beta ** 2) / m2, 0.0)
    return c, v


def _virial(e_m, v, comps):
    w = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            w[a, b] = np.sum(e_m * ((1.0 if a == b else 0.0) - v * comps[a] * comps[b]))
    return w


def ewald_reciprocal_direct(pos, charge, box, beta, ke: float = COULOMB_K, nmax=(8, 8, 8)) -> dict:
    """The plain reciprocal sum over |n_a| <= nmax[a] (all m != 0).  Returns energy,
    force [N,3] and virial [3,3]."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    q = np.asarray(charge, np.float64)
    L = np.asarray(box, np.float64).reshape(3)
    V = float(np.prod(L))
    axes = [np.arange(-nm, nm + 1) / L[a] for a, nm in enumerate(nmax)]
    mx, my, mz = (g.ravel() for g in np.meshgrid(*axes, indexing="ij"))
    m2 = mx * mx + my * my + mz * mz
    keep = m2 > 0
    mx, my, mz, m2 = mx[keep], my[keep], mz[keep], m2[keep]
    c, v = _kspace_terms(m2, mx, my, mz, beta)
    force = np.zeros_like(pos)
    e_m = np.zeros_like(m2)
    chunk = 4096
    for s in range(0, m2.size, chunk):
        sl = slice(s, s + chunk)
        mvec = np.stack([mx[sl], my[sl], mz[sl]], axis=1)              # [M,3]
        ph = np.exp(2j * np.pi * (pos @ mvec.T))                       # [N,M]
        S = (q[:, None] * ph).sum(axis=0)                              # [M]
        e_m[sl] = ke / (2.0 * np.pi * V) * c[sl] * np.abs(S) ** 2
        # dE/dr_i = sum_m ke/(2 pi V) c 2 Re(conj(S) 2 pi i m q_i e^{2 pi i m r_i})
        im = np.imag(np.conj(S)[None, :] * ph)                         # [N,M]
        force += (2.0 * ke / V) * q[:, None] * ((c[sl] * im[:, :]) @ mvec)
    return {"energy": float(e_m.sum()), "force": force, "virial": _virial(e_m, v, (mx, my, mz))}


def _spline_points(u, K: int, n: int):
    """Grid indices k = floor(u) - j (mod K), j = 0..n-1, with M_n(u - k) and dM_n(u - k)."""
    base = np.floor(u)
    j = np.arange(n)
    x = (u - base)[:, None] + j[None, :]                               # u - k in [0, n)
    idx = (base.astype(np.int64)[:, None] - j[None, :]) % K
    return idx, cardinal_bspline(x, n), cardinal_bspline_deriv(x, n)


def spme_reciprocal(pos, charge, box, beta, grid, order: int = 4, ke: float = COULOMB_K) -> dict:
    """SPME reciprocal energy, force [N,3] and virial [3,3] on a K1 x K2 x K3 grid with
    B-splines of the given order.  Also returns the charge grid Q and the potential grid
    phi = dE/dQ."""
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    q = np.asarray(charge, np.float64)
    L = np.asarray(box, np.float64).reshape(3)
    K = [int(k) for k in grid]
    V = float(np.prod(L))
    n = order
    pts = []
    for a in range(3):
        frac = pos[:, a] / L[a]
        u = K[a] * (frac - np.floor(frac))
        u = np.where(u >= K[a], u - K[a], u)
        pts.append(_spline_points(u, K[a], n))
    (ix, wx, dx), (iy, wy, dy), (iz, wz, dz) = pts
    Q = np.zeros(K)
    for a in range(n):
        for b in range(n):
            for c in range(n):
                np.add.at(Q, (ix[:, a], iy[:, b], iz[:, c]), q * wx[:, a] * wy[:, b] * wz[:, c])
    mx, my, mz = np.meshgrid(_mvec(K[0], L[0]), _mvec(K[1], L[1]), _mvec(K[2], L[2]), indexing="ij")
    m2 = mx * mx + my * my + mz * mz
    c, v = _kspace_terms(m2, mx, my, mz, beta)
    B = _bmod2(K[0], n)[:, None, None] * _bmod2(K[1], n)[None, :, None] * _bmod2(K[2], n)[None, None, :]
    C = c * B
    Fq = np.fft.fftn(Q)
    e_m = ke / (2.0 * np.pi * V) * C * np.abs(Fq) ** 2
    # phi(k) = dE/dQ(k) = ke/(pi V) sum_m C(m) conj(Qhat(m)) exp(2 pi i m.k/K)
    phi = ke / (np.pi * V) * np.real(np.fft.ifftn(C * Fq)) * (K[0] * K[1] * K[2])
    force = np.zeros_like(pos)
    for a in range(n):
        for b in range(n):
            for cc in range(n):
                p = phi[ix[:, a], iy[:, b], iz[:, cc]]
                force[:, 0] -= q * p * (K[0] / L[0]) * dx[:, a] * wy[:, b] * wz[:, cc]
                force[:, 1] -= q * p * (K[1] / L[1]) * wx[:, a] * dy[:, b] * wz[:, cc]
                force[:, 2] -= q * p * (K[2] / L[2]) * wx[:, a] * wy[:, b] * dz[:, cc]
    return {"energy": float(e_m.sum()), "force": force, "virial": _virial(e_m, v, (mx, my, mz)),
            "Q": Q, "phi": phi}


def spme_reciprocal_system(system, grid, order: int = 4, ke: float = COULOMB_K) -> dict:
    """``spme_reciprocal`` on an object with the fields of ``systems.System``."""
    return spme_reciprocal(system.pos, system.charge, system.box, system.beta, grid, order, ke)
