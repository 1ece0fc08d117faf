"""Interpolation error of the paper's tabulated potentials (section 3, Figure 2).

TEST INFRASTRUCTURE ONLY (the test suite and its analyses use it; the GPU library never
does).  ACEMD reads the radial parts of the van der Waals and electrostatic terms from
texture tables with linear interpolation, n = 4096 entries; Figure 2 shows the bounds
(running average) of the relative error (E_interp - E_calc)/E_calc of the van der Waals
potential against direct evaluation, an error whose period is R_max/n.

Reading: the table is uniform in r over [0, R_max] (R_max the largest radius the table
covers: the cutoff), one entry per node r_k = k R_max/n, and E_interp at r in
[r_k, r_k+1] is the linear interpolation of the nodes' values.  The van der Waals
potential is the 12-6 Lennard-Jones form; its r^-12 and r^-6 parts are tabulated
separately (a table of u_LJ itself would depend on the atom types).  The exact values
are evaluated in 30-digit arithmetic (mpmath).

    python -m oracle.table_error      # prints the curve (running-average bounds)
"""

from __future__ import annotations

import mpmath as mp
import numpy as np

mp.mp.dps = 30


def lj_exact(r, sigma, eps):
    """4 eps [(sigma/r)^12 - (sigma/r)^6] at 30 digits, as floats."""
    return np.array([float(4 * mp.mpf(eps) * ((mp.mpf(sigma) / mp.mpf(x)) ** 12 - (mp.mpf(sigma) / mp.mpf(x)) ** 6))
                     for x in np.asarray(r, float)])


def lj_linear_table(r, sigma, eps, n=4096, r_max=9.0):
    """u_LJ at r from linearly interpolated r^-12 and r^-6 tables (nodes k r_max/n; the node
    values are exact doubles of the powers)."""
    r = np.asarray(r, float)
    h = r_max / n
    k = np.floor(r / h)
    u = r / h - k
    a, b = k * h, (k + 1) * h
    e12 = a ** -12.0 + u * (b ** -12.0 - a ** -12.0)
    e6 = a ** -6.0 + u * (b ** -6.0 - a ** -6.0)
    return 4 * eps * (sigma ** 12 * e12 - sigma ** 6 * e6)


def relative_error(r, sigma=3.15061, eps=0.6364, n=4096, r_max=9.0):
    """(E_interp - E_calc)/E_calc of the van der Waals potential at the radii r."""
    exact = lj_exact(r, sigma, eps)
    return (lj_linear_table(r, sigma, eps, n, r_max) - exact) / exact


def figure2_bounds(r_lo=2.5, r_hi=9.0, sigma=3.15061, eps=0.6364, n=4096, r_max=9.0, per_interval=16,
                   window=32):
    """Per table interval in [r_lo, r_hi): the largest and smallest relative error (sampled
    at per_interval points), then their running averages over `window` intervals.
    Returns (interval midpoints, running max, running min)."""
    h = r_max / n
    k0, k1 = int(np.ceil(r_lo / h)), int(np.floor(r_hi / h))
    ks = np.arange(k0, k1)
    t = (np.arange(per_interval) + 0.5) / per_interval
    r = ((ks[:, None] + t[None, :]) * h).ravel()
    err = relative_error(r, sigma, eps, n, r_max).reshape(len(ks), per_interval)
    hi, lo = err.max(axis=1), err.min(axis=1)
    kern = np.ones(window) / window
    mid = (ks + 0.5) * h
    valid = slice(window - 1, None)
    return mid[valid], np.convolve(hi, kern, "full")[:len(hi)][valid], np.convolve(lo, kern, "full")[:len(lo)][valid]


if __name__ == "__main__":
    mid, hi, lo = figure2_bounds(per_interval=8)
    print("| r (A) | running-average upper bound | lower bound |")
    print("|---|---|---|")
    for r in (2.8, 3.0, 3.4, 3.6, 4.0, 5.0, 6.0, 7.0, 8.0, 8.9):
        i = int(np.argmin(np.abs(mid - r)))
        print(f"| {mid[i]:.3f} | {hi[i]:.3e} | {lo[i]:.3e} |")
