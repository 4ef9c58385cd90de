"""TD-GRFT and DS-GRFT evaluated in float64 (oracle).

Test infrastructure only: nothing in the product path imports this module.

Time-domain reading of the paper (the input is the range-compressed echo
y(tau_n, t_m) = s[m][n] of eq. (2)/(4); samples outside [0, N) are zero):

* TD-GRFT, Sec. III-A-1, eq. (13): for a lattice point i,
      Y_G(n0; i) = sum_m S(m, n0 + off(m; i)) * exp(+j 2 pi Num(m; i) / M^3)
  where off is the nearest range bin of the walk (round half up) and the
  phase is H_DFM of eq. (12) times the velocity term of eq. (13).

* DS-GRFT, Sec. IV, Alg. 3: for every coarse cell c_c
    1. mGIFT (eq. (46), Alg. 1): envelope correction along the *coarse*
       trajectory (in the time domain: a gather at the coarse range offset)
       followed by the pre-DFM phase H_pre-DFM(t_m; c_c) of eq. (47);
    2. GFT (eq. (44), Alg. 2): multiply by the fine DFM phase of c_f and sum
       over slow time, for every fine cell of the cell's fine space eq. (52).
  The slow-time sum of step 2 is written as a matrix product over m (a
  library primitive standing for the plain sum; no blocking or reordering of
  the definition beyond that).
"""
from __future__ import annotations

import numpy as np

from .grid import Grid, numerator, phasor, range_offset


def _gather(echo: np.ndarray, rows: np.ndarray, off: np.ndarray) -> np.ndarray:
    """S(m, rows + off[m]) as [M, len(rows)], zero outside [0, N)."""
    M, N = echo.shape
    idx = rows[None, :] + off[:, None]                      # [M, rows]
    ok = (idx >= 0) & (idx < N)
    out = np.zeros(idx.shape, dtype=np.complex128)
    mm = np.broadcast_to(np.arange(M)[:, None], idx.shape)
    out[ok] = echo[mm[ok], idx[ok]]
    return out


def row_index(grid: Grid, rows=None) -> np.ndarray:
    if rows is None:
        return np.arange(grid.n_begin, grid.n_end, dtype=np.int64)
    return np.asarray(rows, dtype=np.int64)


# ---- DS-GRFT ------------------------------------------------------------

def coarse_tables(grid: Grid, k: int):
    """Coarse range offsets off(m; i_c) and pre-DFM phasors for cell k."""
    m = np.arange(grid.M, dtype=np.int64)
    num_c = numerator(grid, m, grid.centre(k))
    return range_offset(grid, num_c), phasor(grid, num_c)


def fine_matrix(grid: Grid, fine=None) -> np.ndarray:
    """[M, F] fine DFM phasors exp(+j 2 pi Num(m; f) / M^3), eq. (44)."""
    fo = grid.fine_offsets()
    if fine is not None:
        fo = fo[np.asarray(fine)]
    m = np.arange(grid.M, dtype=np.int64)
    num_f = numerator(grid, m[:, None], fo[None, :, :])    # [M, F]
    return phasor(grid, num_f)


def mgift(echo: np.ndarray, grid: Grid, k: int, rows=None) -> np.ndarray:
    """Alg. 1 (time-domain reading): y(tau_n, t_m; c_c), shape [M, rows]."""
    off_c, h_pre = coarse_tables(grid, k)
    y = _gather(np.asarray(echo, dtype=np.complex128), row_index(grid, rows), off_c)
    return y * h_pre[:, None]


def gft(y_c: np.ndarray, grid: Grid, fine=None, H=None) -> np.ndarray:
    """Alg. 2 / eq. (44): sum_m y_c[m, n] * H_fine[m, f] -> [rows, F].

    H, if given, is fine_matrix(grid, fine) computed once by the caller (the
    table does not depend on the cell, so a loop over cells may reuse it)."""
    return y_c.T @ (fine_matrix(grid, fine) if H is None else H)


def dsgrft_cell(echo, grid: Grid, k: int, rows=None, fine=None, H=None) -> np.ndarray:
    """Complex DS-GRFT outputs of coarse cell k: [rows, F] complex128."""
    return gft(mgift(echo, grid, k, rows), grid, fine, H)


# ---- TD-GRFT (single scale) ----------------------------------------------

def grft_cell(echo, grid: Grid, k: int, rows=None, fine=None) -> np.ndarray:
    """TD-GRFT, eq. (13), at the fine lattice points of coarse cell k.

    Output layout matches dsgrft_cell: [rows, F] for lattice points
    i = i_c(k) + f, so the two maps can be compared cell by cell.
    """
    echo = np.asarray(echo, dtype=np.complex128)
    r = row_index(grid, rows)
    fo = grid.fine_offsets()
    if fine is not None:
        fo = fo[np.asarray(fine)]
    ic = np.asarray(grid.centre(k), dtype=np.int64)
    m = np.arange(grid.M, dtype=np.int64)
    out = np.empty((len(r), len(fo)), dtype=np.complex128)
    for j, f in enumerate(fo):
        num = numerator(grid, m, ic + f)
        g = _gather(echo, r, range_offset(grid, num))
        out[:, j] = phasor(grid, num) @ g
    return out


# ---- whole maps --------------------------------------------------------

def dsgrft_power(echo, grid: Grid, cells=None) -> np.ndarray:
    """|Y_DS|^2 for the listed coarse cells: [n_cells, rows, F] (small cases)."""
    cells = range(grid.n_coarse) if cells is None else cells
    return np.stack([np.abs(dsgrft_cell(echo, grid, k)) ** 2 for k in cells])


def grft_power(echo, grid: Grid, cells=None) -> np.ndarray:
    cells = range(grid.n_coarse) if cells is None else cells
    return np.stack([np.abs(grft_cell(echo, grid, k)) ** 2 for k in cells])
