"""Pins of the dual-scale KT-MFP oracle (oracle.ktmfp): the defining sums
evaluated term by term with exact fractions on a tiny input, the keystone
transform holding a baseband target's envelope in one range bin, folded
targets peaking at their own (q, v', a) cell, linearity and the lattice."""
import math
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import fd as OF
from oracle import ktmfp as KT
from oracle.grid import Axis, Radar, make_grid

R1 = synth.RadarParams(1.0e9, 1.0e7, 500.0)


def _grid(M, N, axes=((-150.0, 150.0), (-200.0, 200.0)), radar=R1):
    return make_grid(Radar(radar.fc, radar.fs, radar.prf), M, N, 2, [Axis(*a) for a in axes])


def test_lattice_covers_velocity_axis():
    g = _grid(64, 128)
    lat = KT.lattice(g)
    i_lo, i_hi = g.i_lo[0], g.i_lo[0] + g.K[0] * g.R - 1
    assert lat.q_lo * g.M - g.M // 2 <= i_lo
    assert (lat.q_lo + lat.n_a) * g.M - g.M // 2 > i_hi
    assert lat.n_coarse == lat.n_a * g.K[1]


def test_direct_sums_tiny():
    """M = 4 pulses, N = 5 bins, R = 3: spectrum, keystone, ramp, IFFT,
    pre-DFM and GFT written as plain sums with exact-fraction phases."""
    radar = synth.RadarParams(3.0e7, 1.0e7, 100.0)
    g = _grid(4, 5, ((-80.0, 80.0), (-300.0, 300.0)), radar)
    rng = np.random.default_rng(5)
    e = rng.standard_normal((4, 5)) + 1j * rng.standard_normal((4, 5))
    Np = OF.pad_length(g)
    P = KT.power(e, g)
    lat = KT.lattice(g)
    M, R = g.M, g.R
    Rfr = Fraction(R)

    def ex(turns):
        return complex(math.cos(2 * math.pi * turns), math.sin(2 * math.pi * turns))
    S = [[sum(e[m, n] * ex(-Fraction(k * n, Np) % 1) for n in range(5)) for k in range(Np)]
         for m in range(M)]
    for kc in range(lat.n_coarse):
        q, i2c = KT.coarse_params(g, lat, kc)
        y = np.zeros((M, g.rows), dtype=complex)
        for m in range(M):
            for n in range(g.rows):
                acc = 0j
                for k in range(Np):
                    ks = k if k < Np // 2 else k - Np
                    ek = Fraction(ks, R * Np + ks)
                    skt = sum(S[mp][k] * np.sinc(float(m - mp - m * ek)) for mp in range(M))
                    x2 = Fraction(i2c * m * m, R * M * M)
                    ph = (q * m * ek - ks * x2 / Np + Fraction(k * n, Np)) % 1
                    acc += skt * ex(ph)
                y[m, n] = acc / Np * ex(Fraction(i2c * m * m * M, M ** 3) % 1)
        for f in range(M * R):
            i1, f2 = f % M - M // 2, f // M - R // 2
            for n in range(g.rows):
                Y = sum(y[m, n] * ex(Fraction(i1 * m * M * M + f2 * m * m * M, M ** 3) % 1)
                        for m in range(M))
                assert abs(abs(Y) ** 2 - P[kc, n, f]) <= 1e-9 * (1 + P.max())


def test_keystone_holds_baseband_envelope():
    """A baseband target (q = 0) walking ~2.5 bins: after the keystone and
    the q = 0, zero-acceleration compensation its envelope stays in its range
    bin at every pulse, while the raw echo's peak moves."""
    M, N = 512, 64
    g = _grid(M, N, ((-40.0, 40.0), (0.0, 0.0)))
    v = 37.0
    tg = synth.Target(r0=30.0 * g.dr, v=v, a=0.0, j=0.0, amp=1.0, phase=0.0)
    echo = synth.make_echo(R1, M, N, [tg], 0.0)
    raw_peaks = np.abs(echo).argmax(axis=1)
    assert raw_peaks.max() - raw_peaks.min() >= 2
    Np = OF.pad_length(g)
    SK = KT.keystone(OF.range_spectrum(echo, Np), g, Np)
    y = np.fft.ifft(SK, axis=1)[:, :N]
    inner = np.abs(y[16:M - 16]).argmax(axis=1)
    assert np.all(inner == 30)


@pytest.mark.parametrize("q,i1p,i2,r0b", [(2, -20, 5, 60.0), (1, 31, 11, 40.5), (0, 3, 0, 50.0)])
def test_folded_target_peaks_at_its_cell(q, i1p, i2, r0b):
    M, N = 64, 128
    g = _grid(M, N)
    lat = KT.lattice(g)
    i1 = q * M + i1p
    tg = synth.Target(r0=r0b * g.dr, v=i1 * g.steps[0], a=i2 * g.steps[1], j=0.0,
                      amp=1.0, phase=0.2)
    echo = synth.make_echo(R1, M, N, [tg], 0.0)
    P = KT.power(echo, g)
    k, row, f = np.unravel_index(P.argmax(), P.shape)
    qq, i2c = KT.coarse_params(g, lat, k)
    assert (qq, f % M - M // 2, i2c + f // M - g.R // 2) == (q, i1p, i2)
    assert abs(row - r0b) <= 0.5
    assert math.sqrt(P.max()) >= 0.85 * M
    r0, v, a = KT.peak_params(g, k, row, f)
    assert v == pytest.approx(i1 * g.steps[0]) and a == pytest.approx(i2 * g.steps[1])


def test_linearity():
    g = _grid(16, 40)
    rng = np.random.default_rng(2)
    a, b = (rng.standard_normal((16, 40)) + 1j * rng.standard_normal((16, 40)) for _ in range(2))
    lhs = KT.power(a + 2j * b, g, cells=[0])
    ya = KT.coarse_rows(a, g, 0)
    yb = KT.coarse_rows(b, g, 0)
    F = KT.fine_matrix(g)
    rhs = np.abs((ya + 2j * yb).T @ F) ** 2
    assert np.abs(lhs[0] - rhs).max() <= 1e-9 * rhs.max()
