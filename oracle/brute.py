"""Multi-precision direct evaluation for tiny inputs (oracle cross-check).

Test infrastructure only: nothing in the product path imports this module.

Independent of `grid.numerator`: every quantity is formed from the physical
parameters as exact rationals (fractions.Fraction of the float64 inputs):
  lambda = c / f_c, dr = c / (2 f_s), T = M / PRF, t_m = m / PRF,
  fine steps lambda/(2T), lambda/T^2, 3 lambda/T^3 (eq. (42), alpha_p = 1),
  D(t) = v t + a t^2 / 2 + j t^3 / 6 (eq. (7)),
  range offset = floor(D/dr + 1/2), phase cycles = 2 D / lambda,
and the sums run in mpmath at 40 significant digits.  It evaluates eq. (13)
(TD-GRFT) and the mGIFT -> GFT cascade of Alg. 3 as plain loops.
"""
from __future__ import annotations

import math
from fractions import Fraction as Fr

import mpmath


def _snap_floor_ceil(x: Fr, up: bool) -> int:
    r = round(x)
    if abs(x - r) <= Fr(1, 10 ** 6):
        return int(r)
    return math.ceil(x) if up else math.floor(x)


class BruteGrid:
    def __init__(self, fc, fs, prf, c, M, N, order, axes):
        self.M, self.N, self.P = M, N, order
        fc, fs, prf, c = Fr(fc), Fr(fs), Fr(prf), Fr(c)
        self.lam = c / fc
        self.dr = c / (2 * fs)
        T = Fr(M) / prf
        self.prf = prf
        self.steps = [self.lam / (2 * T), self.lam / T ** 2, 3 * self.lam / T ** 3]
        R = fc / fs
        assert R.denominator == 1
        self.R = int(R)
        self.h = self.R // 2
        self.i_lo, self.K = [], []
        for p in range(3):
            if p < order:
                lo, hi = axes[p]
                il = _snap_floor_ceil(Fr(lo) / self.steps[p], up=False)
                ih = _snap_floor_ceil(Fr(hi) / self.steps[p], up=True)
                self.i_lo.append(il)
                self.K.append(-(-(ih - il + 1) // self.R))
            else:
                self.i_lo.append(0)
                self.K.append(1)

    def walk(self, m: int, par) -> Fr:
        """D(t_m) for parameters par = (v, a, j) as Fractions."""
        t = Fr(m) / self.prf
        return par[0] * t + par[1] * t ** 2 / 2 + par[2] * t ** 3 / 6

    def coarse_cells(self):
        """Coarse parameter tuples in flat order (k1 fastest)."""
        out = []
        for k3 in range(self.K[2]):
            for k2 in range(self.K[1]):
                for k1 in range(self.K[0]):
                    kk = (k1, k2, k3)
                    out.append(tuple(
                        (self.i_lo[p] + kk[p] * self.R + self.h) * self.steps[p]
                        if p < self.P else Fr(0) for p in range(3)))
        return out

    def fine_cells(self):
        """Fine parameter offsets in flat order (u1 fastest)."""
        out = []
        rng = [range(self.R) if p < self.P else range(1) for p in range(3)]
        for u3 in rng[2]:
            for u2 in rng[1]:
                for u1 in rng[0]:
                    uu = (u1, u2, u3)
                    out.append(tuple((uu[p] - self.h) * self.steps[p]
                                     if p < self.P else Fr(0) for p in range(3)))
        return out


def _cis(cycles: Fr):
    frac = cycles - math.floor(cycles)
    return mpmath.expjpi(2 * mpmath.mpf(frac.numerator) / frac.denominator)


def _sample(echo, m, n):
    return mpmath.mpc(complex(echo[m][n])) if 0 <= n < len(echo[m]) else mpmath.mpc(0)


def brute_maps(echo, bg: BruteGrid, rows, dps: int = 40):
    """Return (Y_DS, Y_G) as nested lists [cell][row][fine] of mpmath complex."""
    mpmath.mp.dps = dps
    ds, gr = [], []
    for cpar in bg.coarse_cells():
        ds_c, gr_c = [], []
        for n0 in rows:
            ds_r, gr_r = [], []
            # mGIFT: gather along the coarse walk, pre-DFM phase (Alg. 1)
            yc = []
            for m in range(bg.M):
                Dc = bg.walk(m, cpar)
                off = math.floor(Dc / bg.dr + Fr(1, 2))
                yc.append(_sample(echo, m, n0 + off) * _cis(2 * Dc / bg.lam))
            for fpar in bg.fine_cells():
                # GFT: fine DFM phase and slow-time sum (Alg. 2)
                acc = mpmath.mpc(0)
                for m in range(bg.M):
                    acc += yc[m] * _cis(2 * bg.walk(m, fpar) / bg.lam)
                ds_r.append(acc)
                # TD-GRFT at the same lattice point (eq. (13))
                full = tuple(cpar[p] + fpar[p] for p in range(3))
                acc = mpmath.mpc(0)
                for m in range(bg.M):
                    D = bg.walk(m, full)
                    off = math.floor(D / bg.dr + Fr(1, 2))
                    acc += _sample(echo, m, n0 + off) * _cis(2 * D / bg.lam)
                gr_r.append(acc)
            ds_c.append(ds_r)
            gr_c.append(gr_r)
        ds.append(ds_c)
        gr.append(gr_c)
    return ds, gr
