"""Oracle vs multi-precision brute force on tiny inputs.

The brute force (oracle/brute.py) forms trajectories, range offsets and phases
from the physical parameters in exact rational arithmetic, independent of the
integer numerator used by the oracle, and sums in 40-digit arithmetic.  A
wrong lattice anchor, tie rule, phase sign, index order or numerator term in
the oracle fails here.
"""
import numpy as np
import pytest

from oracle.brute import BruteGrid, brute_maps
from oracle.grid import Axis, Radar, make_grid
from oracle.transforms import dsgrft_cell, grft_cell

CASES = [
    # fc, fs, prf, M, N, order, axes, rows
    (6.0e7, 1.0e7, 500.0, 6, 12, 1, [(-2500.0, 2500.0)], [0, 3, 7, 11]),
    (6.0e7, 1.0e7, 500.0, 6, 10, 2, [(-2000.0, 2300.0), (-2.0e4, 1.5e4)],
     [0, 4, 9]),
    (4.0e7, 1.0e7, 400.0, 5, 9, 3,
     [(-1500.0, 1500.0), (-3.0e4, 3.0e4), (-2.0e6, 2.0e6)], [1, 4, 8]),
]


@pytest.mark.parametrize("case", CASES, ids=["P1", "P2", "P3"])
def test_oracle_matches_brute_force(case):
    fc, fs, prf, M, N, P, axes, rows = case
    rng = np.random.default_rng(7 + P)
    echo = (rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N)))
    g = make_grid(Radar(fc, fs, prf), M, N, P, [Axis(*a) for a in axes])
    bg = BruteGrid(fc, fs, prf, 3.0e8, M, N, P, axes)
    assert (bg.R, tuple(bg.i_lo), tuple(bg.K)) == (g.R, g.i_lo, g.K)
    # the walks must actually cross range bins for the test to mean anything
    assert max(abs(i) for i in g.i_lo[:P]) >= g.R
    ds_b, gr_b = brute_maps(echo, bg, rows)
    ds_b = np.array([[[complex(z) for z in r] for r in c] for c in ds_b])
    gr_b = np.array([[[complex(z) for z in r] for r in c] for c in gr_b])
    ds_o = np.stack([dsgrft_cell(echo, g, k, rows=rows) for k in range(g.n_coarse)])
    gr_o = np.stack([grft_cell(echo, g, k, rows=rows) for k in range(g.n_coarse)])
    scale = np.abs(gr_b).max()
    assert np.abs(ds_o - ds_b).max() <= 1e-13 * scale
    assert np.abs(gr_o - gr_b).max() <= 1e-13 * scale
    # DS and GRFT differ somewhere (the coarse walk is not the full walk)
    assert np.abs(ds_o - gr_o).max() > 1e-3 * scale
