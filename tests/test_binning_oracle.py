"""Pins for the NumPy binning / exclusion-window references (CPU only)."""

import math
import os

import numpy as np

from oracle import binning as B
from paper_0902_0827_amd import systems as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "binning_tiny.txt")


def _golden():
    d = {"atoms": []}
    for line in open(GOLDEN):
        if not line.strip() or line.startswith("#"):
            continue
        k, *v = line.split()
        if k == "atom":
            d["atoms"].append(v)
        else:
            d[k] = v
    return d


def test_hand_worked_example():
    g = _golden()
    box = np.array([float(x) for x in g["box"]])
    pos = np.array([[float(x) for x in a[:3]] for a in g["atoms"]])
    res = B.bin_system(pos, box, float(g["cutoff"][0]), [int(x) for x in g["divs"]])
    assert list(res["dims"]) == [int(x) for x in g["dims"]]
    np.testing.assert_array_equal(res["fixed"], np.array([[int(x) for x in a[3:6]] for a in g["atoms"]]))
    np.testing.assert_array_equal(res["cell"], [int(a[6]) for a in g["atoms"]])
    np.testing.assert_array_equal(res["order"], [int(x) for x in g["order"]])
    cs = res["cell_start"]
    assert cs[0] == 0 and cs[1] == 2 and cs[27] == 2 and cs[28] == 3 and cs[48] == 3 and cs[49] == 5 and cs[-1] == 5


def test_grid_dims_of_the_workloads():
    assert list(B.grid_dims([18.6] * 3, 9.0, [2, 2, 2])) == [4, 4, 4]
    assert list(B.grid_dims([60.0] * 3, 9.0, [2, 2, 2])) == [13, 13, 13]
    assert list(B.grid_dims([60.0] * 3, 9.0, [2, 2, 8])) == [13, 13, 53]
    assert list(B.grid_dims([215.0] * 3, 12.0, [2, 2, 2])) == [35, 35, 35]
    # every cell is at least R/k wide
    for L in np.linspace(18.1, 90.0, 37):
        for k in (1, 2, 3):
            n = B.grid_dims([L] * 3, 9.0, [k] * 3)[0]
            assert L / n >= 9.0 / k and (n + 1) * 9.0 / k > L - 1e-6


def test_counting_sort_matches_brute_force_sort():
    s = S.solvated_chain(25.0, 40, 400, seed=3, cutoff=9.0, beta=0.34)
    for divs in ([2, 2, 2], [1, 1, 1], [2, 2, 8], [3, 3, 3]):
        res = B.bin_system(s.pos, s.box, s.cutoff, divs)
        # independent: cell from per-atom floor of the wrapped coordinate, sorted by Python
        dims = res["dims"]
        frac = res["fixed"].astype(np.float64) / 2.0**32
        c = np.floor(frac * dims).astype(int)
        lin = (c[:, 0] * dims[1] + c[:, 1]) * dims[2] + c[:, 2]
        np.testing.assert_array_equal(lin, res["cell"])
        order = sorted(range(s.n), key=lambda i: (lin[i], i))
        np.testing.assert_array_equal(res["order"], order)
        counts = np.diff(res["cell_start"])
        assert counts.sum() == s.n
        for cid in np.unique(lin)[:50]:
            members = res["order"][res["cell_start"][cid]:res["cell_start"][cid + 1]]
            assert set(members) == set(np.nonzero(lin == cid)[0])


def test_fixed_point_is_wrap_invariant_and_close_to_the_coordinate():
    rng = np.random.default_rng(1)
    box = np.array([31.0, 17.5, 60.0])
    pos = rng.uniform(0, 1, (500, 3)) * box
    fx = B.fixed_point(pos, box)
    back = fx.astype(np.float64) / 2.0**32 * box
    assert np.all(back <= pos + 1e-12) and np.all(pos - back < box / 2.0**32 + 1e-12)
    shifted = B.fixed_point(pos + box * np.array([3, -2, -7]), box)
    # exact up to the one rounding of the shifted input
    assert np.abs(shifted.astype(np.int64) - fx.astype(np.int64)).max() <= 2**12


def test_exclusion_windows_decode_to_the_symmetric_exclusion_set():
    n = 300
    rng = np.random.default_rng(4)
    pairs = set()
    for _ in range(400):
        i = int(rng.integers(0, n))
        j = int(np.clip(i + rng.integers(-70, 71), 0, n - 1))
        if i != j:
            pairs.add((i, j))  # directed: listed in i's row only
    rows = [[] for _ in range(n)]
    for i, j in pairs:
        rows[i].append(j)
    off = np.zeros(n + 1, np.int32)
    off[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([j for r in rows for j in sorted(r)], np.int32)
    masks, far = B.exclusion_windows(n, off, idx)
    sym = {(i, j) for i, j in pairs} | {(j, i) for i, j in pairs}
    for i in range(n):
        decoded = set()
        for bit in range(128):
            if (int(masks[i, bit // 32]) >> (bit % 32)) & 1:
                d = bit - 64 if bit < 64 else bit - 63
                decoded.add(i + d)
        expect = {j for (a, j) in sym if a == i and abs(j - i) <= 64}
        assert decoded == expect
        assert far[i] == any(a == i and abs(j - i) > 64 for (a, j) in sym)
