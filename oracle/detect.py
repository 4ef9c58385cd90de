"""Reduction, detection and peak parameters (oracle).

Test infrastructure only: nothing in the product path imports this module.

* Reduced map: for every (coarse cell, range row) the largest power over the
  cell's fine space and the smallest fine index attaining it (the ML estimate
  of eq. (72) restricted to one coarse cell and row; the "maximum output of
  each range bin" shown for Experiment 1).
* LRT threshold (Sec. III-C, eqs. (31), (33)): |Y| > gamma with
  gamma^2 = -M K sigma^2 ln P_FA.  The input here is the range-compressed echo,
  whose per-sample noise variance sigma^2 already contains the K frequency
  bins, so the threshold on power is gamma^2 = -M sigma^2 ln P_FA.
* Detections: reduced-map entries above gamma^2, listed in flat order
  (coarse cell major, then row); each carries its argmax fine cell.
* Peak parameters (eq. (72), Alg. 3 with kappa = 1): r0 = n0 dr and
  (v, a, j) = (coarse centre + fine offset) * fine step, in float64.
* Cell-averaging CFAR along range (not in the paper, whose detector is the
  fixed LRT threshold): an entry (cell, row r) is a detection when its power
  exceeds alpha times the mean of the training entries of the same cell,
  rows r' with guard < |r' - r| <= guard + train inside the map.  The mean is
  a float64 sum in increasing r' divided by the number of training entries;
  an entry with no training entry is never a detection.
"""
from __future__ import annotations

import math

import numpy as np

from .grid import Grid
from .transforms import dsgrft_cell


def reduce_power(power: np.ndarray):
    """Max over the last axis and the first index attaining it."""
    return power.max(axis=-1), power.argmax(axis=-1).astype(np.int32)


def dsgrft_reduced(echo, grid: Grid, cells=None, rows=None, chunk=1024, H=None):
    """Reduced DS-GRFT map for the listed coarse cells, rows taken `chunk` at
    a time.  H: the fine matrix (transforms.fine_matrix(grid)) if the caller
    has it, else it is rebuilt for every chunk.

    Returns (pmax [n_cells, rows] float64, argf [n_cells, rows] int32).
    """
    cells = list(range(grid.n_coarse)) if cells is None else list(cells)
    r_all = (np.arange(grid.n_begin, grid.n_end) if rows is None
             else np.asarray(rows))
    pm = np.empty((len(cells), len(r_all)))
    af = np.empty((len(cells), len(r_all)), dtype=np.int32)
    for ci, k in enumerate(cells):
        for s in range(0, len(r_all), chunk):
            y = dsgrft_cell(echo, grid, k, rows=r_all[s:s + chunk], H=H)
            p, a = reduce_power(np.abs(y) ** 2)
            pm[ci, s:s + chunk] = p
            af[ci, s:s + chunk] = a
    return pm, af


def threshold(M: int, sigma2: float, pfa: float) -> float:
    """gamma^2 on |Y|^2, eq. (33) with the K bins folded into sigma^2."""
    return -M * sigma2 * math.log(pfa)


def global_argmax(pmax: np.ndarray):
    """Flat (cell, row) index of the largest reduced power, smallest on ties."""
    flat = int(np.argmax(pmax.reshape(-1)))
    return divmod(flat, pmax.shape[1])


def detections(pmax: np.ndarray, argf: np.ndarray, gamma2: float):
    """(cell, row, fine) triples with power above gamma^2, flat order."""
    k, r = np.nonzero(pmax > gamma2)
    return [(int(a), int(b), int(argf[a, b])) for a, b in zip(k, r)]


def peak_params(grid: Grid, k: int, n0: int, f: int):
    """(r0, v, a, j) in float64 for coarse cell k, range row n0, fine f."""
    i = grid.lattice_point(k, f)
    v, a, j = grid.params(i)
    return n0 * grid.dr, v, a, j


def ca_cfar(pmax: np.ndarray, guard: int, train: int, alpha: float) -> np.ndarray:
    """Cell-averaging CFAR decisions on a reduced map [cells, rows] (float32
    or float64 values): boolean mask of detections.  Rows are visited one at
    a time; the training sum runs over r' in increasing order for all cells
    at once, each step a float64 addition."""
    p = np.asarray(pmax, dtype=np.float64)
    n, rows = p.shape
    hit = np.zeros((n, rows), dtype=bool)
    for r in range(rows):
        train_rows = [q for q in range(r - guard - train, r + guard + train + 1)
                      if 0 <= q < rows and guard < abs(q - r)]
        if not train_rows:
            continue
        acc = np.zeros(n)
        for q in train_rows:
            acc = acc + p[:, q]
        mean = acc / float(len(train_rows))
        hit[:, r] = p[:, r] > alpha * mean
    return hit


def cfar_alpha(n_train: int, pfa: float) -> float:
    """CA-CFAR multiplier for exponentially distributed power with n_train
    training entries: P_FA = (1 + alpha / n_train)^(-n_train)."""
    return n_train * (pfa ** (-1.0 / n_train) - 1.0)
