"""The CPU model of the paper's table error (Figure 2): linear interpolation of r^-12 and
r^-6 from 4096-entry tables uniform in r over [0, R_max].  Checked against what the
mathematics fixes: the error vanishes at every node (the period R_max/n), it scales as
h^2 (second-order interpolation), and it stays below the paper's 1e-4 except near the
zero of u_LJ at r = sigma, where a relative error has no meaning."""

import numpy as np

from oracle import table_error as TE

SIG, EPS = 3.15061, 0.6364


def test_error_vanishes_at_the_nodes():
    h = 9.0 / 4096
    r = np.arange(1300, 4090, 97) * h
    assert np.abs(TE.relative_error(r)).max() < 1e-12


def test_error_is_second_order_in_the_spacing():
    r = np.linspace(4.0, 8.5, 301) + 1e-3 * np.pi  # not on any node
    e1 = np.abs(TE.relative_error(r, n=1024)).max()
    e2 = np.abs(TE.relative_error(r, n=2048)).max()
    assert 3.6 < e1 / e2 < 4.4


def test_error_bound_of_the_paper_away_from_the_zero_of_u():
    r = np.linspace(2.6, 8.99, 4001)
    r = r[np.abs(r - SIG) > 0.05]
    assert np.abs(TE.relative_error(r)).max() < 1e-4


def test_figure2_bounds_bracket_the_sampled_error():
    mid, hi, lo = TE.figure2_bounds(r_lo=4.0, r_hi=6.0, per_interval=8, window=8)
    assert np.all(hi >= lo)
    assert np.all((mid > 4.0) & (mid < 6.0))
    assert np.abs(hi).max() < 1e-5
