"""Pins of the 8-bit float model (oracle.lowp): E4M3 rounding against an
exhaustive decode of the format, a hand-worked example of the scaling rules,
and element-wise error bounds of the rounded operands."""
import math

import numpy as np
import pytest

from oracle import lowp
from oracle.grid import Axis, Radar, make_grid

FINITE = sorted({lowp.e4m3_decode(c) for c in range(256)
                 if not math.isnan(lowp.e4m3_decode(c))})


def _brute(x: float) -> float:
    """Nearest finite E4M3 value; ties to the code with an even mantissa."""
    best, bd, bcode = None, None, None
    for c in range(256):
        v = lowp.e4m3_decode(c)
        if math.isnan(v) or c == 0x80:
            continue
        d = abs(v - x)
        if bd is None or d < bd or (d == bd and (c & 1) == 0 and (bcode & 1) == 1):
            best, bd, bcode = v, d, c
    return best


def test_e4m3_format_constants():
    assert max(FINITE) == 448.0 and min(FINITE) == -448.0
    assert len(FINITE) == 253          # 254 finite codes, +0 and -0 coincide
    pos = [v for v in FINITE if v > 0]
    assert min(pos) == 2.0 ** -9 and 2.0 ** -6 in pos


def test_e4m3_matches_exhaustive_nearest():
    rng = np.random.default_rng(8)
    xs = list(rng.uniform(-448, 448, 400)) + list(rng.uniform(-1, 1, 300) * 2.0 ** -5)
    # every midpoint between neighbours and every representable value
    xs += [0.5 * (a + b) for a, b in zip(FINITE[:-1], FINITE[1:])] + FINITE
    got = lowp.e4m3(np.array(xs))
    want = np.array([_brute(x) for x in xs])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("x,want", [(1.0625, 1.0), (1.1875, 1.25), (232.0, 224.0),
                                    (2.0 ** -10, 0.0), (3 * 2.0 ** -10, 2.0 ** -8),
                                    (448.0, 448.0), (-0.3, -0.3125)])
def test_e4m3_worked_values(x, want):
    assert float(lowp.e4m3(x)) == want


def _tiny_grid(M=1, N=1):
    return make_grid(Radar(1.0e9, 1.0e7, 500.0), M, N, 1, [Axis(0.0, 0.0)])


def test_scaling_rules_worked_example():
    """One sample 0.3 + 0.7j on a one-pulse grid (zero walk, unit phasors):
    e = 0 (0.7 = 0.7 * 2^0); Re: 76.8 -> hi 80, 16 (76.8 - 80) = -51.2 -> -52;
    Im: 179.2 -> hi 176, 51.2 -> 52."""
    g = _tiny_grid()
    echo = np.array([[0.3 + 0.7j]])
    Gh, Gl, D = lowp.unit_operands(echo, g, 0, 0, split=3)
    assert Gh[0, 0] == (80 + 176j) / 256 and Gl[0, 0] == (-52 + 52j) / 4096
    Fh, Fl = lowp.fine_operands(g)
    assert np.all(Fh == 1.0) and np.all(Fl == 0.0)
    P, Y, _ = lowp.search_power(echo, g, 0, split=3)
    assert np.all(Y == 0.2998046875 + 0.7001953125j)
    P1, Y1, _ = lowp.search_power(echo, g, 0, split=1)
    assert np.all(Y1 == 0.3125 + 0.6875j)


def test_row_exponent_brackets_row_maximum():
    rng = np.random.default_rng(2)
    S = (rng.standard_normal((50, 40)) + 1j * rng.standard_normal((50, 40))) \
        * np.ldexp(1.0, rng.integers(-30, 30, 40))[None, :]
    S[:, 3] = 0
    e = lowp.row_exponent(S)
    mx = np.maximum(np.abs(S.real), np.abs(S.imag)).max(axis=0)
    nz = mx > 0
    assert np.all(mx[nz] < np.ldexp(1.0, e[nz])) and np.all(mx[nz] >= np.ldexp(1.0, e[nz] - 1))
    assert e[3] == 0


def test_rounded_operands_within_format_bounds():
    """|g_q - g| <= 2^-4 |g| + 2^-10 u (hi) and 2^-8 |g| + 2^-13 u (hi + lo)
    per real component, u = 2^(e-8) the row's unit; likewise for F with
    u = 2^-8.  A wrong exponent, scale or lo weight breaks these."""
    g = make_grid(Radar(1.2e8, 1.0e7, 500.0), 40, 64, 2,
                  [Axis(-100.0, 100.0), Axis(-400.0, 400.0)])
    rng = np.random.default_rng(4)
    echo = (rng.standard_normal((40, 64)) + 1j * rng.standard_normal((40, 64))) * 3.0
    echo[:, 10] *= 1e-3
    from oracle import transforms as OT
    for k in (0, g.n_coarse - 1):
        Gh, Gl, _ = lowp.unit_operands(echo, g, k, 0, split=3)
        G = OT.mgift(echo, g, k)
        S = lowp._walk(echo, g, k)
        u = np.ldexp(1.0, lowp.row_exponent(S) - 8)[None, :]
        for part in (np.real, np.imag):
            err1 = np.abs(part(Gh) - part(G))
            err2 = np.abs(part(Gh + Gl) - part(G))
            assert np.all(err1 <= 2.0 ** -4 * np.abs(part(G)) + 2.0 ** -10 * u + 1e-15)
            assert np.all(err2 <= 2.0 ** -8 * np.abs(part(G)) + 2.0 ** -13 * u + 1e-15)
    Fh, Fl = lowp.fine_operands(g)
    F = OT.fine_matrix(g)[:, :Fh.shape[1]]
    for part in (np.real, np.imag):
        assert np.all(np.abs(part(Fh) - part(F)) <= 2.0 ** -4 * np.abs(part(F)) + 2.0 ** -18)
        assert np.all(np.abs(part(Fh + Fl) - part(F)) <= 2.0 ** -8 * np.abs(part(F)) + 2.0 ** -21)


def test_split_passes_reduce_error():
    g = make_grid(Radar(1.2e8, 1.0e7, 500.0), 64, 80, 2,
                  [Axis(-60.0, 60.0), Axis(-200.0, 200.0)])
    rng = np.random.default_rng(6)
    echo = rng.standard_normal((64, 80)) + 1j * rng.standard_normal((64, 80))
    from oracle import transforms as OT
    ref = np.abs(OT.dsgrft_cell(echo, g, 1)) ** 2
    errs, rms = [], []
    for s in (1, 2, 3, 4):
        P, _, _ = lowp.search_power(echo, g, 1, s)
        errs.append(np.abs(P - ref).max() / ref.max())
        rms.append(np.sqrt(np.mean((P - ref) ** 2)) / ref.max())
    # each further product lowers the typical error; the maximum is set by
    # the G rounding until its lo part enters (split 3)
    assert rms[0] > rms[1] > rms[2] > rms[3]
    assert errs[0] < 0.2 and errs[2] < 1e-2 and errs[3] < 1e-2 and errs[2] < errs[1] / 10
