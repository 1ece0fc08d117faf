"""CPU replay of the cluster pair kernel's item setup (the index arithmetic of
k_pair_cluster, restated): for every cluster of a binned system, the neighbour columns,
their z-windows as runs of sorted atoms, and the half-shell column rule.

Checked, at the full size of the 23.6k-atom box and on the small 648-atom box (whose
stencil spans the whole box):
  * bounds: every cell_start index read lies in [0, n_cells], the non-empty runs of an
    item fit the kernel's run table (2 x 9 x 9 entries), including cell divisions
    (4, 16), which the library refuses;
  * coverage: every pair of atoms closer than the cutoff (found independently, by a
    periodic k-d tree) is a candidate of its atoms' clusters, and the half-shell rule
    evaluates it exactly once (the full shell: once from each side).
The binning itself comes from oracle/binning.py, which tests/test_binning_oracle.py pins
and the GPU parity tests hold the build to bit for bit."""

import numpy as np
import pytest

import nbtest_util as U
from oracle import binning as OB
from paper_0902_0827_amd import systems as S

scipy_spatial = pytest.importorskip("scipy.spatial")

K_MAX_RUNS = 2 * 9 * 9  # the kernel's run table


def _items(system, divs, K, half):
    """Per cluster: (first, count, runs [r, 2] of [start, end) sorted indices); and the
    largest cell_start index read."""
    b = OB.bin_system(system.pos, system.box, system.cutoff, divs)
    nx, ny, nz = (int(v) for v in b["dims"])
    kx, ky, kz = divs
    cs = b["cell_start"]
    fz = b["fixed"][b["order"], 2].astype(np.uint64)  # sorted atoms' fixed-point z
    col_count = cs[np.arange(nx * ny) * nz + nz] - cs[np.arange(nx * ny) * nz]
    clusters = (col_count + K - 1) // K
    col_clu_start = np.concatenate([[0], np.cumsum(clusters)])
    allx, ally = 2 * kx + 1 >= nx, 2 * ky + 1 >= ny
    xn, yn = (nx if allx else 2 * kx + 1), (ny if ally else 2 * ky + 1)
    items, max_index = [], 0
    for col in range(nx * ny):
        cx, cy = col // ny, col % ny
        cb0 = col * nz
        for I in range(col_clu_start[col], col_clu_start[col + 1]):
            first = int(cs[cb0] + K * (I - col_clu_start[col]))
            count = int(min(K, cs[cb0 + nz] - first))
            cz0 = int((fz[first] * np.uint64(nz)) >> np.uint64(32))
            cz1 = int((fz[first + count - 1] * np.uint64(nz)) >> np.uint64(32))
            allz = (cz1 - cz0) + 2 * kz + 1 >= nz
            runs = []
            for k in range(xn * yn):
                ox, oy = k // yn, k % yn
                x = ox if allx else cx - kx + ox
                x += nx if x < 0 else (-nx if x >= nx else 0)
                y = oy if ally else cy - ky + oy
                y += ny if y < 0 else (-ny if y >= ny else 0)
                cb = (x * ny + y) * nz
                if allz:
                    idx = [(cb, cb + nz)]
                else:
                    z0, z1 = cz0 - kz, cz1 + kz + 1
                    if z0 < 0:
                        idx = [(cb + z0 + nz, cb + nz), (cb, cb + z1)]
                    elif z1 > nz:
                        idx = [(cb + z0, cb + nz), (cb, cb + z1 - nz)]
                    else:
                        idx = [(cb + z0, cb + z1)]
                # the kernel loads four cell starts for every column: with one run the
                # second pair is (cb, cb), read and discarded
                reads = idx if len(idx) == 2 else idx + [(cb, cb)]
                for a, c in reads:
                    assert 0 <= a <= len(cs) - 1 and 0 <= c <= len(cs) - 1
                    max_index = max(max_index, a, c)
                rr = [[int(cs[a]), int(cs[c])] for a, c in idx]
                if half:
                    rx = int(np.sign(ox - cx)) if allx else int(np.sign(ox - kx))
                    ry = int(np.sign(oy - cy)) if ally else int(np.sign(oy - ky))
                    if rx < 0 or (rx == 0 and ry < 0):
                        rr = []
                    elif rx == 0 and ry == 0:
                        rr = [[max(s0, first), max(max(s0, first), e0)] for s0, e0 in rr]
                runs += [r for r in rr if r[1] > r[0]]
            items.append((first, count, np.array(runs, np.int64).reshape(-1, 2)))
    return b, items, max_index


def _check(system, divs, K, half):
    b, items, max_index = _items(system, divs, K, half)
    assert max_index <= len(b["cell_start"]) - 1
    nrun = max(len(r) for _, _, r in items)
    assert nrun <= K_MAX_RUNS, nrun
    # cluster of every sorted atom
    n = system.n
    clu = np.empty(n, np.int64)
    for c, (first, count, _) in enumerate(items):
        clu[first:first + count] = c
    rank = np.empty(n, np.int64)
    rank[b["order"]] = np.arange(n)  # original -> sorted
    # every pair within the cutoff (a hair beyond it: rounding of the kernel's own test)
    pos = np.mod(system.pos, system.box)
    tree = scipy_spatial.cKDTree(pos, boxsize=system.box)
    pairs = tree.query_pairs(system.cutoff * (1 + 1e-9), output_type="ndarray")
    si, sj = rank[pairs[:, 0]], rank[pairs[:, 1]]
    a = np.concatenate([si, sj])  # ordered pairs: row atom a, candidate c
    c = np.concatenate([sj, si])
    took = np.zeros(a.size, bool)
    order = np.argsort(clu[a], kind="stable")
    bounds = np.searchsorted(clu[a][order], np.arange(len(items) + 1))
    for q, (first, count, runs) in enumerate(items):
        sel = order[bounds[q]:bounds[q + 1]]
        if sel.size == 0:
            continue
        cand = c[sel]
        inside = np.zeros(sel.size, bool)
        for s0, e0 in runs:
            inside |= (cand >= s0) & (cand < e0)
        if half:  # own column from the cluster's first atom on; own atoms only after the row's
            inside &= (cand < first) | (cand > a[sel])
        took[sel] = inside
    once = took[:pairs.shape[0]].astype(int) + took[pairs.shape[0]:].astype(int)
    if half:
        assert np.all(once == 1), f"{np.sum(once != 1)} of {once.size} pairs not evaluated exactly once"
    else:
        assert np.all(once == 2), f"{np.sum(once != 2)} of {once.size} pairs missing from a full shell"
    return nrun, pairs.shape[0]


@pytest.fixture(scope="module")
def box23k():
    return S.config2()


@pytest.mark.parametrize("divs,K,half", [((2, 2, 8), 8, True), ((2, 2, 8), 4, False), ((3, 3, 16), 8, True),
                                         ((4, 4, 16), 8, True)])
def test_stencil_bounds_and_coverage_on_the_23k_box(box23k, divs, K, half):
    nrun, npairs = _check(box23k, divs, K, half)
    assert npairs > 3_900_000
    if divs[0] == 4:
        # (4, 16): 81 neighbour columns, runs fit the table exactly at its 2 x 81 bound
        assert nrun <= K_MAX_RUNS


@pytest.mark.parametrize("half", [True, False])
def test_stencil_on_a_box_the_stencil_spans(half):
    """648 atoms, L = 18.6 A, R = 9 A: 4 cells per axis against a 5-column stencil, so
    every column is visited once (the dedupe case) and the half rule uses column order."""
    _check(S.config1(), (2, 2, 8), 8 if half else 4, half)


@pytest.mark.parametrize("half", [True, False])
@pytest.mark.parametrize("box", [(18.5, 19.0, 90.0), (90.0, 88.0, 18.5)])
def test_stencil_on_elongated_and_slab_boxes(box, half):
    """R = 8 A: the stencil spans the box in x and y but not in z (elongated), or in z
    only (slab); the boxes of the GPU geometry tests."""
    nrun, npairs = _check(U.lattice_system(box, 2.6, seed=31), (2, 2, 8), 8 if half else 4, half)
    assert nrun <= K_MAX_RUNS and npairs > 0
