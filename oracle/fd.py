"""Frequency-domain mGIFT (Alg. 1, eq. (46)) on a range-compressed echo (oracle).

Test infrastructure only: nothing in the product path imports this module.

Alg. 1 compensates the coarse range walk in the range-frequency domain: the
echo spectrum y(f_k, t_m) is multiplied by H_RM(f_k, t_m; c_c) =
exp(+j 4 pi f_k D_c(t_m) / c) (eq. (10)), an IFFT over range frequency
follows, and then the pre-DFM phase of eq. (47).  With a range-compressed
input s[m][n] this reads:

* spectrum: S[m][k] = sum_{n<N} s[m][n] exp(-j 2 pi k n / N'), the row
  zero-padded to N' = the smallest power of two >= N + W, W a bound of the
  coarse walk in bins (so an integer walk never wraps into the window);
* f_k = k_s f_s / N' with the signed index k_s = k for k < N'/2, k - N'
  otherwise; with D_c / dr = x_c(m) = Num_c(m) / (R M^3) (range bins),
  H_RM = exp(+j 2 pi k_s x_c(m) / N');
* y_c[m][n] = (1/N') sum_k S[m][k] H_RM exp(+j 2 pi k n / N'), n in the
  row window, times psi_c(m) = exp(+j 2 pi Num_c(m) / M^3).

For an integer walk this is exactly the time-domain gather s[m][n + x]
(zero outside [0, N)); a fractional walk is shifted by band-limited
(periodic-sinc) interpolation instead of the nearest bin.  The FFTs are
library routines standing for the plain sums above.
"""
from __future__ import annotations

import numpy as np

from .grid import Grid, numerator, phasor
from .transforms import fine_matrix


def walk_bound(grid: Grid) -> int:
    """W = ceil(sum_p max|i_c,p| (M-1)^p M^(3-p) / (R M^3)) + 1."""
    M, R = grid.M, grid.R
    tot = 0
    for p in range(grid.order):
        lo = grid.i_lo[p] + grid.h
        hi = grid.i_lo[p] + (grid.K[p] - 1) * R + grid.h
        tot += max(abs(lo), abs(hi)) * (M - 1) ** (p + 1) * M ** (2 - p)
    return -(-tot // (R * M ** 3)) + 1


def pad_length(grid: Grid) -> int:
    n = grid.N + walk_bound(grid)
    L = 1
    while L < n:
        L *= 2
    return L


def signed_index(Np: int) -> np.ndarray:
    k = np.arange(Np, dtype=np.int64)
    return np.where(k < Np // 2, k, k - Np)


def range_spectrum(echo, Np: int) -> np.ndarray:
    """S[m][k], the zero-padded range DFT of every pulse (complex128)."""
    return np.fft.fft(np.asarray(echo, dtype=np.complex128), Np, axis=1)


def ramp(grid: Grid, num: np.ndarray, Np: int) -> np.ndarray:
    """H_RM[m][k] = exp(+j 2 pi k_s x / N'), x = num / (R M^3), with the
    integer part of x handled exactly: k_s x / N' = (k_s xi mod N') / N'
    + k_s xf / N'."""
    RM3 = np.int64(grid.R) * np.int64(grid.M3)
    num = np.asarray(num, dtype=np.int64)
    xi = np.floor_divide(num, RM3)
    xf = (num - xi * RM3).astype(np.float64) / float(RM3)
    ks = signed_index(Np)
    turns = (np.mod(ks[None, :] * xi[:, None], Np).astype(np.float64)
             + ks[None, :].astype(np.float64) * xf[:, None]) / Np
    return np.exp(2j * np.pi * turns)


def mgift_fd(echo, grid: Grid, k: int, Np: int | None = None, S=None) -> np.ndarray:
    """Alg. 1 in the frequency domain for coarse cell k: [M, rows] complex128."""
    Np = pad_length(grid) if Np is None else Np
    S = range_spectrum(echo, Np) if S is None else S
    m = np.arange(grid.M, dtype=np.int64)
    num = numerator(grid, m, grid.centre(k))
    y = np.fft.ifft(S * ramp(grid, num, Np), axis=1)[:, grid.n_begin:grid.n_end]
    return y * phasor(grid, num)[:, None]


def dsgrft_fd_power(echo, grid: Grid, cells=None) -> np.ndarray:
    """|GFT(mGIFT_FD)|^2 for the listed cells: [n_cells, rows, n_fine]."""
    cells = range(grid.n_coarse) if cells is None else cells
    Np = pad_length(grid)
    S = range_spectrum(echo, Np)
    F = fine_matrix(grid)
    return np.stack([np.abs(mgift_fd(echo, grid, k, Np, S).T @ F) ** 2 for k in cells])
