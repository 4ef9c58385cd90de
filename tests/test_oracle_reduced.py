"""Pins of the reduced map (oracle.detect.dsgrft_reduced, the ML estimate of
eq. (72) restricted to one coarse cell and range row): it equals the max and
first argmax over the fine axis of the full DS-GRFT power map, whatever the
row chunking, row list, cell list or precomputed fine matrix."""
import numpy as np

from oracle import detect as OD
from oracle import transforms as OT
from oracle.grid import Axis, Radar, make_grid


def _case():
    g = make_grid(Radar(4.0e7, 1.0e7, 400.0), 20, 37, 2, [Axis(-700.0, 700.0), Axis(-9000.0, 9000.0)])
    rng = np.random.default_rng(21)
    e = rng.standard_normal((20, 37)) + 1j * rng.standard_normal((20, 37))
    return g, e


def test_reduced_equals_max_of_full_map_chunked():
    g, e = _case()
    assert g.n_coarse == 12 and g.n_fine == 16 and g.rows == 37
    P = OT.dsgrft_power(e, g)
    # the matrix product's rounding may depend on how many rows it is given
    tol = 1e-13 * P.max()
    for chunk in (1, 5, 16, 37, 1024):
        pm, af = OD.dsgrft_reduced(e, g, chunk=chunk)
        assert pm.shape == (g.n_coarse, 37) and af.dtype == np.int32
        assert np.abs(pm - P.max(-1)).max() <= tol
        assert np.array_equal(af, P.argmax(-1))
    H = OT.fine_matrix(g)
    pm, af = OD.dsgrft_reduced(e, g, chunk=6, H=H)
    assert np.abs(pm - P.max(-1)).max() <= tol and np.array_equal(af, P.argmax(-1))


def test_reduced_cell_and_row_lists():
    g, e = _case()
    P = OT.dsgrft_power(e, g)
    cells = [g.n_coarse - 1, 0, 2]
    rows = [36, 3, 4, 17, 0, 30, 31]
    pm, af = OD.dsgrft_reduced(e, g, cells=cells, rows=rows, chunk=3)
    assert pm.shape == (3, 7)
    for ci, k in enumerate(cells):
        for ri, r in enumerate(rows):
            assert abs(pm[ci, ri] - P[k, r].max()) <= 1e-13 * P.max()
            assert af[ci, ri] == int(np.argmax(P[k, r]))
