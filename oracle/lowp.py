"""Reference model of the 8-bit float form of the fine search (oracle).

Test infrastructure only: nothing in the product path imports this module.

The paper evaluates the GFT of eq. (44) exactly.  The library can also run
that slow-time sum with both operands rounded to the OCP 8-bit float E4M3
(1 sign, 4 exponent bits with bias 7, 3 mantissa bits, no infinities, largest
finite 448, subnormal step 2^-9) and power-of-two scales.  This module states
in float64 what that form computes, so that a test can hold the device result
to the accumulation error instead of to the (much larger) rounding error of
8-bit operands.  The rules below are the definition of the form:

* fine phasors F (|F| = 1), per real component:
      x = fl32(256 F),  hi = e4m3(x),  lo = e4m3(16 (x - hi)),
      F ~ hi / 2^8 + lo / 2^12;
* gathered, de-ramped samples G of one unit (coarse cell, and for P = 3 one
  fine jerk offset) and range row n: let mx be the largest |Re S| or |Im S|
  over the raw echo samples S(m, n + off(m)) of the row's walk and e the
  exponent with mx = f 2^e, f in [0.5, 1) (e = 0 when mx = 0), clamped to
  [-100, 100]; then per real component
      x = G 2^(8 - e),  hi = e4m3(x),  lo = e4m3(16 (x - hi)),
      G ~ (hi + lo / 16) 2^(e - 8);
* products summed for split s: 1: Fh Gh; 2: + Fl Gh; 3: + Fh Gl; 4: + Fl Gl.

The device computes G in float32 before rounding it, and this model in
float64, so an element whose scaled value lies within float32 error of an
E4M3 rounding midpoint may round the other way on the device.  `flip_bound`
collects, per row, the largest change that such elements can make.

e4m3 is pinned by exhaustive decoding of all 256 codes, by a hand-worked
example of the scaling rules and by the error bounds of the form.
"""
from __future__ import annotations

import numpy as np

from .grid import Grid, numerator, phasor, range_offset

E4M3_MAX = 448.0


def e4m3_decode(code: int) -> float:
    """Value of an E4M3 code from its bit fields (NaN for S.1111.111)."""
    s, E, m = (code >> 7) & 1, (code >> 3) & 15, code & 7
    if E == 15 and m == 7:
        return float("nan")
    v = (m / 8.0) * 2.0 ** -6 if E == 0 else (1.0 + m / 8.0) * 2.0 ** (E - 7)
    return -v if s else v


def e4m3_spacing(x) -> np.ndarray:
    """Distance between neighbouring E4M3 values around |x| (|x| <= 448)."""
    a = np.abs(np.asarray(x, dtype=np.float64))
    _, ex = np.frexp(a)                    # a = f 2^ex, f in [0.5, 1)
    E = np.maximum(ex - 1, -6)             # binade of a; subnormals share -6
    return np.ldexp(1.0, E - 3)


def e4m3(x) -> np.ndarray:
    """Round to the nearest E4M3 value, ties to even (|x| <= 448)."""
    x = np.asarray(x, dtype=np.float64)
    if np.any(np.abs(x) > E4M3_MAX):
        raise ValueError("value outside the E4M3 range")
    q = e4m3_spacing(x)
    # |x| / q is exact (q is a power of two); np.rint rounds half to even,
    # and an even multiple of q has an even mantissa code.
    return np.sign(x) * np.rint(np.abs(x) / q) * q


def _split(x: np.ndarray):
    hi = e4m3(x)
    lo = e4m3(16.0 * (x - hi))
    return hi, lo


def fine_operands(grid: Grid):
    """Rounded fine phasors of orders 1..min(P, 2): (Fh, Fl) [M, C] complex,
    in real units (hi / 2^8, lo / 2^12).  Order 3 sits in the unit samples."""
    R, h = grid.R, grid.h
    C = R ** min(grid.order, 2)
    f = np.arange(C, dtype=np.int64)
    fo = np.zeros((C, 3), dtype=np.int64)
    fo[:, 0] = f % R - h
    if grid.order >= 2:
        fo[:, 1] = f // R - h
    m = np.arange(grid.M, dtype=np.int64)
    F = phasor(grid, numerator(grid, m[:, None], fo[None, :, :]))
    out = []
    for comp in (F.real, F.imag):
        x = comp * 256.0
        x = x.astype(np.float32).astype(np.float64)
        out.append(_split(x))
    (rh, rl), (ih, il) = out
    return (rh + 1j * ih) / 256.0, (rl + 1j * il) / 4096.0


def _walk(echo, grid: Grid, k: int):
    """Raw echo samples along coarse cell k's walk: S [M, rows] complex128."""
    m = np.arange(grid.M, dtype=np.int64)
    off = range_offset(grid, numerator(grid, m, grid.centre(k)))
    rows = np.arange(grid.n_begin, grid.n_end, dtype=np.int64)
    idx = rows[None, :] + off[:, None]
    ok = (idx >= 0) & (idx < grid.N)
    S = np.zeros(idx.shape, dtype=np.complex128)
    mm = np.broadcast_to(m[:, None], idx.shape)
    S[ok] = np.asarray(echo, dtype=np.complex128)[mm[ok], idx[ok]]
    return S


def row_exponent(S: np.ndarray) -> np.ndarray:
    """e per row (column of S [M, rows]) as defined in the module notes."""
    mx = np.maximum(np.abs(S.real), np.abs(S.imag)).max(axis=0)
    _, e = np.frexp(mx)
    e = np.where(mx > 0, e, 0)
    return np.clip(e, -100, 100).astype(np.int64)


def unit_operands(echo, grid: Grid, k: int, u3: int, split: int):
    """Rounded samples of unit (k, u3): (Gh, Gl) [M, rows] complex in real
    units, and the per-row bound of the change that rounding-midpoint
    elements can make on the device (float32 samples), in real units."""
    S = _walk(echo, grid, k)
    m = np.arange(grid.M, dtype=np.int64)
    f3 = (u3 - grid.h) if grid.order == 3 else 0
    ic = np.asarray(grid.centre(k), dtype=np.int64)
    num = numerator(grid, m, ic) + np.int64(f3) * m * m * m
    G = S * phasor(grid, num)[:, None]
    e = row_exponent(S)
    sc = np.ldexp(1.0, 8 - e)[None, :]
    unit = np.ldexp(1.0, e - 8)[None, :]
    # margin: float32 error of the device's sample, in scaled units (a
    # generous multiple of the bound of one complex product in float32)
    margin = np.ldexp(1.0, -19) * np.abs(S) * sc
    Gh = np.zeros_like(G)
    Gl = np.zeros_like(G)
    D = np.zeros(G.shape[1])
    for part, j in ((G.real, 1.0), (G.imag, 1j)):
        x = part * sc
        hi, lo = _split(x)
        Gh = Gh + j * hi * unit
        Gl = Gl + j * lo / 16.0 * unit
        amb_hi = e4m3(x - margin) != e4m3(x + margin)
        lx = 16.0 * (x - hi)
        amb_lo = e4m3(np.clip(lx - 16 * margin, -E4M3_MAX, E4M3_MAX)) != \
            e4m3(np.clip(lx + 16 * margin, -E4M3_MAX, E4M3_MAX))
        q = e4m3_spacing(x)
        eff_hi = q if split < 3 else q / 8.0
        eff_lo = e4m3_spacing(lx) / 16.0 if split >= 3 else 0.0 * q
        D += ((amb_hi * eff_hi + amb_lo * eff_lo) * unit).sum(axis=0)
    return Gh, Gl, D


def search_power(echo, grid: Grid, k: int, split: int):
    """|Y|^2 of coarse cell k under the 8-bit form with `split` products:
    (P [rows, n_fine], Y [rows, n_fine], D [rows, n_fine]) where D bounds
    |Y_device - Y| from midpoint elements (see the module notes)."""
    if split not in (1, 2, 3, 4):
        raise ValueError("split must be 1..4")
    Fh, Fl = fine_operands(grid)
    C = Fh.shape[1]
    units = grid.R if grid.order == 3 else 1
    Y = np.empty((grid.rows, C * units), dtype=np.complex128)
    D = np.empty((grid.rows, C * units))
    for u3 in range(units):
        Gh, Gl, d = unit_operands(echo, grid, k, u3, split)
        y = Gh.T @ Fh
        if split >= 2:
            y = y + Gh.T @ Fl
        if split >= 3:
            y = y + Gl.T @ Fh
        if split >= 4:
            y = y + Gl.T @ Fl
        Y[:, u3 * C:(u3 + 1) * C] = y
        D[:, u3 * C:(u3 + 1) * C] = d[:, None]
    return np.abs(Y) ** 2, Y, D
