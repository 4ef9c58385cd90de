"""Dual-scale KT-MFP (Alg. 4, Cor. 1, Prop. 3) on a range-compressed echo,
P = 2 (oracle).

Test infrastructure only: nothing in the product path imports this module.

Reading (kappa = 1, t_m = m / PRF, the motion and lattice of oracle.grid):

* range spectrum: S[m][k] = DFT of row m zero-padded to N' (the frequency-
  domain pad length of oracle.fd), f_k = k_s f_s / N' with the signed index
  k_s (eq. (1) with the carrier split off);
* keystone transform: y_KT(f_k, t) = y(f_k, t f_c / (f_c + f_k)) removes the
  linear range walk of the baseband velocity for every f_k at once (eq. (25));
  with eps_k = f_k / (f_c + f_k) = k_s / (R N' + k_s) (an exact rational, R =
  f_c / f_s) the resampled sequence is the band-limited (sinc) interpolation
  over the M pulses:
      S_KT[m][k] = sum_{m'<M} S[m'][k] sinc(m - m' - m eps_k);
* velocity folding (eq. (23)): v = q V_a + v', V_a = lambda PRF / 2 is M fine
  velocity steps, so a fine velocity index i1 = q M + i1', i1' in [-M/2, M/2);
* coarse cell (q, k2): the coarse RM compensation H_KT,RM of eq. (26),
  exp(+j 4 pi f_k (f_bar q V_a t - c2c t^2) / c), is in turns
      q m eps_k - k_s x2(m) / N',   x2(m) = i2c m^2 M / (R M^3)  (bins),
  then the IFFT over range frequency and the pre-DFM phase of eq. (47), KT
  branch: exp(+j 2 pi i2c m^2 M / M^3);
* fine cells (i1', f2), f2 in [-R/2, R - R/2): the GFT phase
  exp(+j 2 pi (i1' m M^2 + f2 m^2 M) / M^3), i.e. a length-M DFT over slow
  time for the baseband velocities (Prop. 3);
* flat orders: coarse k = k2 N_a + (q - q_lo); fine f = u2 M + u1 with
  u1 = i1' + M/2, u2 = f2 + R/2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import fd as OF
from .grid import Grid, phasor


@dataclass(frozen=True)
class KtLattice:
    q_lo: int
    n_a: int          # folding factors q_lo .. q_lo + n_a - 1
    k2: int           # coarse acceleration cells (the DS-GRFT lattice's K[1])

    @property
    def n_coarse(self) -> int:
        return self.n_a * self.k2


def lattice(grid: Grid) -> KtLattice:
    """Folding factors covering the velocity axis's fine indices."""
    if grid.order != 2:
        raise ValueError("DS-KT-MFP is defined here for P = 2")
    M = grid.M
    i_lo = grid.i_lo[0]
    i_hi = grid.i_lo[0] + grid.K[0] * grid.R - 1
    q_lo = (i_lo + M // 2) // M
    q_hi = (i_hi + M // 2) // M
    return KtLattice(q_lo=q_lo, n_a=q_hi - q_lo + 1, k2=grid.K[1])


def coarse_params(grid: Grid, lat: KtLattice, k: int):
    """(q, i2c) of coarse cell k."""
    q = lat.q_lo + k % lat.n_a
    k2 = k // lat.n_a
    i2c = grid.i_lo[1] + k2 * grid.R + grid.h
    return q, i2c


def eps(grid: Grid, Np: int):
    """(numerator, denominator) of eps_k = k_s / (R N' + k_s), int64."""
    ks = OF.signed_index(Np)
    return ks, np.int64(grid.R) * Np + ks


def keystone(S: np.ndarray, grid: Grid, Np: int) -> np.ndarray:
    """S_KT[m][k] = sum_m' S[m'][k] sinc(m - m' - m eps_k)."""
    M = grid.M
    en, ed = eps(grid, Np)
    e = en.astype(np.float64) / ed.astype(np.float64)            # [Np]
    m = np.arange(M, dtype=np.float64)
    out = np.empty_like(S)
    for k in range(Np):
        d = m[:, None] - m[None, :] - m[:, None] * e[k]          # [M, M']
        out[:, k] = np.sinc(d) @ S[:, k]
    return out


def ramp(grid: Grid, q: int, i2c: int, Np: int) -> np.ndarray:
    """exp(+j 2 pi (q m eps_k - k_s x2(m) / N')) as [M, Np], the integer
    parts reduced exactly."""
    M, R = grid.M, grid.R
    m = np.arange(M, dtype=np.int64)
    en, ed = eps(grid, Np)
    # q m k_s / (R N' + k_s): exact numerator reduced modulo the denominator
    a = np.mod(np.int64(q) * m[:, None] * en[None, :], ed[None, :])
    t1 = a.astype(np.float64) / ed[None, :].astype(np.float64)
    # k_s x2 / N', x2 = i2c m^2 M / (R M^3) = i2c m^2 / (R M^2)
    RM2 = np.int64(R) * M * M
    num = np.int64(i2c) * m * m
    xi = np.floor_divide(num, RM2)
    xf = (num - xi * RM2).astype(np.float64) / float(RM2)
    ks = OF.signed_index(Np)
    t2 = (np.mod(ks[None, :] * xi[:, None], Np).astype(np.float64)
          + ks[None, :].astype(np.float64) * xf[:, None]) / Np
    return np.exp(2j * np.pi * (t1 - t2))


def coarse_rows(echo, grid: Grid, k: int, SK=None, Np=None) -> np.ndarray:
    """mGIFT on the keystoned spectrum for coarse cell k: [M, rows]."""
    Np = OF.pad_length(grid) if Np is None else Np
    if SK is None:
        SK = keystone(OF.range_spectrum(echo, Np), grid, Np)
    lat = lattice(grid)
    q, i2c = coarse_params(grid, lat, k)
    y = np.fft.ifft(SK * ramp(grid, q, i2c, Np), axis=1)[:, grid.n_begin:grid.n_end]
    m = np.arange(grid.M, dtype=np.int64)
    psi = phasor(grid, np.int64(i2c) * m * m * np.int64(grid.M))
    return y * psi[:, None]


def fine_matrix(grid: Grid) -> np.ndarray:
    """[M, M R] GFT phasors for (u1, u2), flat f = u2 M + u1."""
    M, R = grid.M, grid.R
    m = np.arange(M, dtype=np.int64)
    u = np.arange(M * R, dtype=np.int64)
    i1 = u % M - M // 2
    f2 = u // M - R // 2
    num = i1[None, :] * m[:, None] * M * M + f2[None, :] * m[:, None] ** 2 * M
    return phasor(grid, num)


def power(echo, grid: Grid, cells=None) -> np.ndarray:
    """|Y|^2 over [cells, rows, M R]."""
    Np = OF.pad_length(grid)
    SK = keystone(OF.range_spectrum(echo, Np), grid, Np)
    lat = lattice(grid)
    cells = range(lat.n_coarse) if cells is None else cells
    F = fine_matrix(grid)
    return np.stack([np.abs(coarse_rows(echo, grid, k, SK, Np).T @ F) ** 2 for k in cells])


def peak_params(grid: Grid, k: int, row: int, f: int):
    """(r0, v, a) of a map cell."""
    lat = lattice(grid)
    q, i2c = coarse_params(grid, lat, k)
    M, R = grid.M, grid.R
    u1, u2 = f % M, f // M
    i1 = q * M + u1 - M // 2
    i2 = i2c + u2 - R // 2
    return ((grid.n_begin + row) * grid.dr, i1 * grid.steps[0], i2 * grid.steps[1])
