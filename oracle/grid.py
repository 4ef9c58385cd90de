"""Search lattice and exact trajectory arithmetic of the oracle.

Test infrastructure only: nothing in the product path imports this module.

Motion model (Sec. II-B, eq. (7)): R(t) = c0 + c1 t + c2 t^2 + c3 t^3, written
here as r(t) = r0 + v t + a t^2/2 + j t^3/6, i.e. c1 = v, c2 = a/2, c3 = j/6.
Slow time t_m = m / PRF for m = 0..M-1 (the paper counts m = 1..M; starting at
zero makes r0 the range at the first pulse, which does not change |.|).

Step sizes (Sec. III-C, eqs. (39)-(42) with alpha_p = 1 for every order):
  range bin         dr = c / (2 f_s)                       (eq. (39))
  fine (DFM) steps  Delta_DFM,p = c / (2 f_c T^p), T = M/PRF  (eq. (42))
                    -> dv = lambda/(2T), da = lambda/T^2, dj = 3 lambda/T^3
                       in (v, a, j) units
  coarse (RM) steps Delta_RM,p = c / (2 f_s T^p) = R * Delta_DFM,p (eq. (41))
                    with R = f_c / f_s, the DFM-to-RM sensitivity ratio that
                    opens Sec. IV.
The argument called `bandwidth` plays f_s (the range sampling rate).

With integer lattice indices i = (i1, i2, i3), v = i1 dv, a = i2 da, j = i3 dj:
  2 D(t_m) / lambda = Num(m; i) / M^3           (cycles of the DFM phase)
  D(t_m) / dr       = Num(m; i) / (R M^3)       (range walk in bins)
  Num(m; i) = i1 m M^2 + i2 m^2 M + i3 m^3      (an exact integer)
where D(t) = r(t) - r0.  Both are exact rationals, so range offsets (the
`round` of eq. (13)) and phasors are computed without any floating-point
decision.

Dual-scale lattice (Sec. IV-B, eqs. (48)-(52)), read as a half-open tiling:
coarse cell k_p of order p covers the R fine indices
  i_p in [i_lo,p + k_p R, i_lo,p + (k_p + 1) R),
its coarse parameter is the centre i_c,p = i_lo,p + k_p R + h (h = R // 2) and
its fine offsets are f_p in [-h, R - h).  Every fine lattice point belongs to
exactly one coarse cell, so DS-GRFT cells are in one-to-one correspondence with
single-scale GRFT cells.

Flat orders: coarse k = (k3 K2 + k2) K1 + k1; fine f = (u3 R + u2) R + u1 with
u_p = f_p + h in [0, R).  Orders above P have K_p = 1 and index 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 3.0e8  # m/s, the value stated in Sec. II-A


@dataclass(frozen=True)
class Radar:
    fc: float          # carrier frequency f_c [Hz]
    bandwidth: float   # range sampling rate f_s [Hz]; dr = c / (2 f_s)
    prf: float         # pulse repetition frequency [Hz]
    c: float = C_LIGHT
    kappa: float = 1.0  # Prop. 1 scale; only kappa = 1 is supported


@dataclass(frozen=True)
class Axis:
    min: float
    max: float


def _snap(x: float, tol: float = 1e-6):
    """Return the nearest integer when x lies within tol of it, else None."""
    r = round(x)
    return int(r) if abs(x - r) <= tol else None


def index_bounds(lo: float, hi: float, step: float) -> tuple[int, int]:
    """Outward-rounded integer index range [i_lo, i_hi] covering [lo, hi].

    Reading of eq. (32) / eq. (51): the search space [c_min : dc : c_max] is
    anchored on the integer lattice i * step; a bound within 1e-6 of a lattice
    point is taken as that point, otherwise it is rounded outward.
    """
    xl, xh = lo / step, hi / step
    sl, sh = _snap(xl), _snap(xh)
    il = sl if sl is not None else math.floor(xl)
    ih = sh if sh is not None else math.ceil(xh)
    return il, ih


@dataclass
class Grid:
    radar: Radar
    M: int
    N: int
    order: int
    n_begin: int
    n_end: int
    R: int
    lam: float
    dr: float
    T: float
    steps: tuple            # fine steps (dv, da, dj)
    i_lo: tuple             # lowest fine index per order (0 above P)
    K: tuple                # coarse cells per order (1 above P)
    axes: tuple = field(default=())

    # ---- sizes ---------------------------------------------------------
    @property
    def h(self) -> int:
        return self.R // 2

    @property
    def n_coarse(self) -> int:
        return self.K[0] * self.K[1] * self.K[2]

    @property
    def n_fine(self) -> int:
        return self.R ** self.order

    @property
    def rows(self) -> int:
        return self.n_end - self.n_begin

    @property
    def M3(self) -> int:
        return self.M ** 3

    # ---- lattice -------------------------------------------------------
    def coarse_tuple(self, k: int) -> tuple[int, int, int]:
        k1 = k % self.K[0]
        k2 = (k // self.K[0]) % self.K[1]
        k3 = k // (self.K[0] * self.K[1])
        return k1, k2, k3

    def centre(self, k: int) -> tuple[int, int, int]:
        """Coarse parameter indices i_c (eq. (49) on the integer lattice)."""
        kt = self.coarse_tuple(k)
        return tuple(
            (self.i_lo[p] + kt[p] * self.R + self.h) if p < self.order else 0
            for p in range(3))

    def fine_offsets(self) -> np.ndarray:
        """[n_fine, 3] int64 fine offsets f_p in [-h, R-h) in flat order."""
        f = np.arange(self.n_fine, dtype=np.int64)
        out = np.zeros((self.n_fine, 3), dtype=np.int64)
        for p in range(self.order):
            out[:, p] = (f // (self.R ** p)) % self.R - self.h
        return out

    def lattice_point(self, k: int, f: int) -> tuple[int, int, int]:
        fo = self.fine_offsets()[f]
        c = self.centre(k)
        return tuple(int(c[p] + fo[p]) for p in range(3))

    def params(self, i) -> tuple[float, float, float]:
        """Physical (v, a, j) of lattice indices i (float64)."""
        return tuple(float(i[p]) * self.steps[p] for p in range(3))


def make_grid(radar: Radar, M: int, N: int, order: int, axes,
              n_begin: int = 0, n_end: int | None = None) -> Grid:
    """Derive the search lattice from radar parameters and axis extents."""
    if not (1 <= order <= 3):
        raise ValueError("order must be 1, 2 or 3")
    if M < 1 or N < 1:
        raise ValueError("M and N must be positive")
    if radar.kappa != 1.0:
        raise ValueError("only kappa = 1 is supported")
    n_end = N if n_end is None else n_end
    if not (0 <= n_begin < n_end <= N):
        raise ValueError("row range must satisfy 0 <= n_begin < n_end <= N")
    ratio = radar.fc / radar.bandwidth
    R = _snap(ratio, 1e-9 * max(1.0, ratio))
    if R is None or R < 1:
        raise ValueError("f_c / f_s must be a positive integer")
    lam = radar.c / radar.fc                       # Sec. II-A
    dr = radar.c / (2.0 * radar.bandwidth)         # eq. (39)
    T = M / radar.prf                              # eq. (38): T = M PRT
    steps = (lam / (2.0 * T), lam / (T * T), 3.0 * lam / (T * T * T))
    axes = tuple(axes) + (Axis(0.0, 0.0),) * (3 - len(axes))
    i_lo, K = [], []
    for p in range(3):
        if p < order:
            ax = axes[p]
            if not (ax.min <= ax.max):
                raise ValueError("axis min must not exceed max")
            il, ih = index_bounds(ax.min, ax.max, steps[p])
            i_lo.append(il)
            K.append(-(-(ih - il + 1) // R))
        else:
            i_lo.append(0)
            K.append(1)
    g = Grid(radar=radar, M=M, N=N, order=order, n_begin=n_begin, n_end=n_end,
             R=R, lam=lam, dr=dr, T=T, steps=steps, i_lo=tuple(i_lo),
             K=tuple(K), axes=axes)
    # The numerator must stay far inside int64 (it is formed in numpy int64).
    imax = [max(abs(i_lo[p]), abs(i_lo[p] + K[p] * R)) if p < order else 0
            for p in range(3)]
    bound = sum(imax) * M ** 3
    if 2 * bound + R * M ** 3 >= 2 ** 62:
        raise ValueError("search extent too large for the exact integer path")
    return g


# ---- exact trajectory arithmetic ---------------------------------------

def numerator(grid: Grid, m, i) -> np.ndarray:
    """Num(m; i) = i1 m M^2 + i2 m^2 M + i3 m^3 (int64, exact).

    `m` is an int64 array of pulse indices, `i` a length-3 index tuple (or an
    array broadcasting against m with a trailing axis of 3).
    """
    m = np.asarray(m, dtype=np.int64)
    M = np.int64(grid.M)
    i = np.asarray(i, dtype=np.int64)
    return i[..., 0] * m * M * M + i[..., 1] * m * m * M + i[..., 2] * m * m * m


def range_offset(grid: Grid, num) -> np.ndarray:
    """Nearest range bin of the walk, round half up, exactly in integers.

    x = Num / (R M^3); round(x) = floor((2 Num + R M^3) / (2 R M^3)).  This is
    the `round` of eq. (13) with ties taken upward.
    """
    num = np.asarray(num, dtype=np.int64)
    d = np.int64(grid.R) * np.int64(grid.M3)
    return np.floor_divide(2 * num + d, 2 * d)


def phasor(grid: Grid, num) -> np.ndarray:
    """exp(+j 2 pi Num / M^3), the DFM matching phase of eq. (12) with the
    velocity term of eq. (13); the integer part of the cycle count is removed
    exactly before the float64 exponential."""
    num = np.asarray(num, dtype=np.int64)
    M3 = np.int64(grid.M3)
    frac = np.mod(num, M3).astype(np.float64) / float(grid.M3)
    return np.exp(2j * np.pi * frac)
