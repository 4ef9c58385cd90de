"""Pins of the frequency-domain mGIFT (oracle.fd): integer walks reproduce
the time-domain gather, a single impulse gives the closed-form periodic
sinc, a direct evaluation of the defining sums (no FFT) on a tiny input, a
noiseless target at a coarse centre keeps the sampled envelope at every
pulse, linearity, and the walk bound."""
import math
from fractions import Fraction

import numpy as np

import synth
from oracle import fd
from oracle import transforms as OT
from oracle.grid import Axis, Radar, make_grid, numerator, phasor


def _int_walk_grid():
    # R = 2, M = 8: the centre index 16 = R M walks exactly m bins at pulse m
    r = Radar(2.0e7, 1.0e7, 100.0)
    dv = make_grid(r, 8, 40, 1, [Axis(0.0, 0.0)]).steps[0]
    return make_grid(r, 8, 40, 1, [Axis(15 * dv, 18 * dv)])


def test_integer_walk_equals_time_domain():
    g = _int_walk_grid()
    assert g.centre(0) == (16, 0, 0)
    e = np.random.default_rng(1).standard_normal((8, 40)) * (1 + 0.5j)
    assert np.abs(fd.mgift_fd(e, g, 0) - OT.mgift(e, g, 0)).max() <= 1e-12
    # the other cell walks 18 m / 16 bins: fractional, so the two differ
    assert np.abs(fd.mgift_fd(e, g, 1) - OT.mgift(e, g, 1)).max() > 0.1


def test_impulse_gives_periodic_sinc():
    """s[m][n] = delta(n - n0): y[n] = (1/N') sum_{k_s} e^{j2pi k_s t/N'} with
    t = n - n0 + x, i.e. e^{-j pi t/N'} sin(pi t) / (N' sin(pi t / N'))."""
    g = _int_walk_grid()
    M, N = g.M, g.N
    n0 = 17
    e = np.zeros((M, N), dtype=np.complex128)
    e[:, n0] = 1.0
    Np = fd.pad_length(g)
    y = fd.mgift_fd(e, g, 1)
    m = np.arange(M, dtype=np.int64)
    num = numerator(g, m, g.centre(1))
    x = num / (g.R * g.M3)
    n = np.arange(g.n_begin, g.n_end)
    t = n[None, :] - n0 + x[:, None]
    with np.errstate(invalid="ignore", divide="ignore"):
        d = np.exp(-1j * np.pi * t / Np) * np.sin(np.pi * t) / (Np * np.sin(np.pi * t / Np))
    d = np.where(np.abs(t - np.round(t)) < 1e-12, (np.abs(np.round(t)) < 0.5) * 1.0, d)
    ref = d * phasor(g, num)[:, None]
    assert np.abs(y - ref).max() <= 1e-12


def test_direct_sums_tiny():
    """The defining sums evaluated term by term (no FFT), walks from exact
    fractions, on M = 3 pulses, N = 5 bins."""
    r = Radar(3.0e7, 1.0e7, 100.0)            # R = 3
    g = make_grid(r, 3, 5, 2, [Axis(-40.0, 40.0), Axis(-200.0, 200.0)])
    rng = np.random.default_rng(3)
    e = rng.standard_normal((3, 5)) + 1j * rng.standard_normal((3, 5))
    Np = fd.pad_length(g)
    for k in range(g.n_coarse):
        y = fd.mgift_fd(e, g, k)
        ic = g.centre(k)
        for m in range(3):
            num = ic[0] * m * 9 + ic[1] * m * m * 3
            x = Fraction(num, g.R * 27)
            psi = np.exp(2j * np.pi * float(Fraction(num % 27, 27)))
            for n in range(5):
                acc = 0j
                for kk in range(Np):
                    ks = kk if kk < Np // 2 else kk - Np
                    Sk = sum(e[m, q] * np.exp(-2j * np.pi * kk * q / Np) for q in range(5))
                    ph = float((ks * x) % Np) / Np
                    acc += Sk * np.exp(2j * np.pi * ph) * np.exp(2j * np.pi * kk * n / Np)
                assert abs(acc / Np * psi - y[m, n]) <= 1e-11


def test_target_at_coarse_centre_keeps_sampled_envelope():
    """Noiseless sinc-envelope target at a coarse centre, 0.5 bin off the
    range grid: the FD-compensated sum at the centre cell reaches
    M A |sinc(0.5)| = 2 M A / pi (no straddle loss), above the nearest-bin
    gather."""
    c = synth.CONFIGS[2]
    r = c["radar"]
    g = make_grid(Radar(r.fc, r.fs, r.prf), c["M"], c["N"], 2, [Axis(*a) for a in c["axes"]])
    k = 37
    ic = g.centre(k)
    tg = synth.Target(r0=300.5 * g.dr, v=ic[0] * g.steps[0], a=ic[1] * g.steps[1], j=0.0,
                      amp=1.0, phase=0.3)
    echo = synth.make_echo(r, c["M"], c["N"], [tg], 0.0, np.random.Generator(np.random.PCG64(5)))
    F = OT.fine_matrix(g)
    col = g.h * g.R + g.h
    y_fd = (fd.mgift_fd(echo, g, k).T @ F)[300, col]
    y_td = (OT.mgift(echo, g, k).T @ F)[300, col]
    assert abs(abs(y_fd) / c["M"] - 2 / math.pi) <= 2e-3
    assert abs(y_fd) > abs(y_td) * 1.03


def test_linearity():
    g = _int_walk_grid()
    rng = np.random.default_rng(7)
    a, b = (rng.standard_normal((8, 40)) + 1j * rng.standard_normal((8, 40)) for _ in range(2))
    lhs = fd.mgift_fd(2 * a - 3j * b, g, 1)
    rhs = 2 * fd.mgift_fd(a, g, 1) - 3j * fd.mgift_fd(b, g, 1)
    assert np.abs(lhs - rhs).max() <= 1e-12


def test_walk_bound_covers_every_walk():
    for cfg in (1, 2, 3):
        c = synth.CONFIGS[cfg]
        r = c["radar"]
        g = make_grid(Radar(r.fc, r.fs, r.prf), c["M"], c["N"], c["order"],
                      [Axis(*a) for a in c["axes"]])
        m = np.arange(g.M, dtype=np.int64)
        worst = 0.0
        for k in range(0, g.n_coarse, max(1, g.n_coarse // 50)):
            worst = max(worst, float(np.abs(numerator(g, m, g.centre(k))).max()) / (g.R * g.M3))
        for k in (g.n_coarse - 1,):
            worst = max(worst, float(np.abs(numerator(g, m, g.centre(k))).max()) / (g.R * g.M3))
        W = fd.walk_bound(g)
        assert worst <= W
        Np = fd.pad_length(g)
        assert Np >= g.N + W and Np & (Np - 1) == 0 and Np < 2 * (g.N + W)


def test_fd_power_direct_sums_tiny():
    """dsgrft_fd_power on every cell, row and fine cell of a tiny plan against
    the defining sums written out term by term: the frequency-domain shift
    of each pulse (range DFT, ramp, inverse DFT, all as plain sums with the
    walk as an exact fraction) times the whole phase of the lattice point,
    exp(+j 2 pi (i1 m M^2 + i2 m^2 M) / M^3) with i = centre + fine offset
    (no coarse/fine factorisation), summed over pulses.  A transposed
    operand, a conjugated fine table or a wrong fine ordering fails it."""
    r = Radar(3.0e7, 1.0e7, 100.0)            # R = 3, offsets -1, 0, 1
    M, N = 3, 5
    g = make_grid(r, M, N, 2, [Axis(-40.0, 40.0), Axis(-200.0, 200.0)])
    rng = np.random.default_rng(11)
    e = rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))
    Np = fd.pad_length(g)
    P = fd.dsgrft_fd_power(e, g)
    assert P.shape == (g.n_coarse, N, g.R ** 2)
    M3 = M ** 3
    for k in range(g.n_coarse):
        ic = g.centre(k)
        for n in range(N):
            for f in range(g.R ** 2):
                i1 = ic[0] + f % g.R - g.h
                i2 = ic[1] + f // g.R - g.h
                Y = 0j
                for m in range(M):
                    x = Fraction(ic[0] * m * M * M + ic[1] * m * m * M, g.R * M3)
                    acc = 0j
                    for kk in range(Np):
                        ks = kk if kk < Np // 2 else kk - Np
                        Sk = sum(e[m, q] * np.exp(-2j * np.pi * kk * q / Np) for q in range(N))
                        ph = float((ks * x) % Np) / Np
                        acc += Sk * np.exp(2j * np.pi * ph) * np.exp(2j * np.pi * kk * n / Np)
                    turn = Fraction((i1 * m * M * M + i2 * m * m * M) % M3, M3)
                    Y += acc / Np * np.exp(2j * np.pi * float(turn))
                assert abs(abs(Y) ** 2 - P[k, n, f]) <= 1e-10 * max(1.0, abs(Y) ** 2)


def test_fd_power_equals_time_domain_map_on_integer_walk():
    """On the integer-walk cell the frequency-domain map is the time-domain
    DS-GRFT map (transforms.dsgrft_power); on the fractional cell it is not."""
    g = _int_walk_grid()
    e = np.random.default_rng(12).standard_normal((8, 40)) * (0.3 - 1.1j)
    P_fd = fd.dsgrft_fd_power(e, g, cells=[0, 1])
    P_td = OT.dsgrft_power(e, g, cells=[0, 1])
    assert np.abs(P_fd[0] - P_td[0]).max() <= 1e-11 * P_td[0].max()
    assert np.abs(P_fd[1] - P_td[1]).max() > 1e-2 * P_td[1].max()
