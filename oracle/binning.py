"""Plain NumPy reference for cell-list binning and exclusion-window encoding.

TEST INFRASTRUCTURE ONLY (see ``oracle.py``); shares no code with the GPU library.

Binning (ACEMD paper, section 3: atoms are binned by their coordinates into a
cell list whose cells are a fraction of the cutoff R wide, bins of R/2 giving a
halo two cells thick).  The rule written out here, step by step:

1. Box-fraction fixed point, per dimension a:
       t = floor((x_a / L_a) * 2^32)   (one IEEE double division, exact scaling)
       u_a = t mod 2^32                 (unsigned 32-bit; this also wraps x into the box)
2. Grid: with k_a cells per cutoff, n_a = max(1, floor(k_a L_a / (R + 4 L_a 2^-32))),
   so that a cell is at least R/k_a wide plus a margin for the fixed-point rounding.
3. Cell coordinate c_a = floor(u_a * n_a / 2^32) (exact in 64-bit integers);
   linear cell id = (c_x * n_y + c_y) * n_z + c_z  (z fastest: one (x, y) column of
   cells is one contiguous run).
4. Atoms are ordered by (cell id, original index): a stable counting sort.
   cell_start[c] = number of atoms in cells before c (length n_cells + 1).

Exclusions (section 3: excluded pairs stored as bitmaps for any index distance
|i - j| <= 64, with extra bookkeeping beyond that): for each atom i (original
order) a 128-bit window, bit b set when i is excluded with i + delta, where
b = delta + 64 for delta in [-64, -1] and b = delta + 63 for delta in [1, 64].
An exclusion listed in either atom's row counts for both atoms.  An atom with an
exclusion farther than 64 in index gets the ``far`` flag.
"""

from __future__ import annotations

import math

import numpy as np

TWO32 = 4294967296.0


def fixed_point(pos: np.ndarray, box: np.ndarray) -> np.ndarray:
    pos = np.asarray(pos, np.float64).reshape(-1, 3)
    t = np.floor((pos / np.asarray(box, np.float64)) * TWO32).astype(np.int64)
    return (t & 0xFFFFFFFF).astype(np.uint32)


def grid_dims(box, cutoff: float, divs) -> np.ndarray:
    out = []
    for a in range(3):
        L = float(box[a])
        n = math.floor(divs[a] * L / (cutoff + 4.0 * L / TWO32))
        out.append(max(1, n))
    return np.array(out, np.int64)


def cell_ids(fixed: np.ndarray, dims: np.ndarray) -> np.ndarray:
    c = (fixed.astype(np.uint64) * dims.astype(np.uint64)[None, :]) >> np.uint64(32)
    c = c.astype(np.int64)
    return (c[:, 0] * dims[1] + c[:, 1]) * dims[2] + c[:, 2]


def bin_system(pos, box, cutoff, divs):
    """Returns fixed [N,3] uint32, dims [3], cell [N] (per atom), order [N] (sorted -> original),
    cell_start [n_cells+1]."""
    fx = fixed_point(pos, box)
    dims = grid_dims(box, cutoff, divs)
    cell = cell_ids(fx, dims)
    n_cells = int(np.prod(dims))
    # Stable counting sort by cell id.
    counts = np.bincount(cell, minlength=n_cells)
    start = np.zeros(n_cells + 1, np.int64)
    start[1:] = np.cumsum(counts)
    order = np.empty(cell.shape[0], np.int64)
    cursor = start[:-1].copy()
    for i in range(cell.shape[0]):  # in original order: stable by construction
        order[cursor[cell[i]]] = i
        cursor[cell[i]] += 1
    return dict(fixed=fx, dims=dims, cell=cell, order=order, cell_start=start)


def exclusion_windows(n: int, excl_offset, excl_index):
    """Returns masks uint32 [n, 4] (bit b of the window lives in word b // 32) and far bool [n]."""
    masks = np.zeros((n, 4), np.uint32)
    far = np.zeros(n, bool)
    off = np.asarray(excl_offset)
    idx = np.asarray(excl_index)
    for i in range(n):
        for k in range(off[i], off[i + 1]):
            j = int(idx[k])
            for a, b in ((i, j), (j, i)):
                d = b - a
                if d == 0:
                    continue
                if abs(d) > 64:
                    far[a] = True
                    continue
                bit = d + 64 if d < 0 else d + 63
                masks[a, bit // 32] |= np.uint32(1 << (bit % 32))
    return masks, far
