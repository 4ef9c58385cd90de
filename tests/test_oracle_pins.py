"""Pins of the oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, an invariant, a library routine, an independent exact evaluation of the
signal model, or numbers printed in the paper.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import detect as D
from oracle import transforms as T
from oracle.grid import Axis, Radar, make_grid, numerator, range_offset
import synth

R1 = Radar(1.0e9, 1.0e7, 500.0)


def small_grid(order=2, M=32, N=96, axes=None, fc=8.0e7):
    """fc/fs = 8 keeps R small while the walks still cross several bins."""
    axes = axes or [(-60.0, 60.0), (-40.0, 40.0), (-300.0, 300.0)][:order]
    return make_grid(Radar(fc, 1.0e7, 500.0), M, N, order,
                     [Axis(*a) for a in axes])


# ---- lattice sizes and steps ------------------------------------------------

@pytest.mark.parametrize("cfg,K,ncoarse", [
    (1, (3, 1, 1), 3), (2, (82, 4, 1), 328), (3, (164, 15, 1), 2460),
    (5, (492, 112, 31), 1708224)])
def test_workload_lattice_sizes(cfg, K, ncoarse):
    c = synth.CONFIGS[cfg]
    r = c["radar"]
    g = make_grid(Radar(r.fc, r.fs, r.prf), c["M"], c["N"], c["order"],
                  [Axis(*a) for a in c["axes"]])
    assert g.K == K and g.n_coarse == ncoarse and g.R == 100


def test_steps_match_stated_coarse_and_fine_grids():
    """Workload grids: fine lambda/(2T), lambda/T^2, 3 lambda/T^3 and coarse
    dr/T, 2 dr/T^2, 6 dr/T^3 -- the coarse step is R times the fine one."""
    g = make_grid(R1, 2048, 8192, 3, [Axis(-900, 900), Axis(-100, 100), Axis(-20, 20)])
    lam, dr, T = 0.3, 15.0, 2048 / 500.0
    fine = (lam / (2 * T), lam / T ** 2, 3 * lam / T ** 3)
    coarse = (dr / T, 2 * dr / T ** 2, 6 * dr / T ** 3)
    for p in range(3):
        assert g.steps[p] == pytest.approx(fine[p], rel=1e-15)
        assert g.R * g.steps[p] == pytest.approx(coarse[p], rel=1e-14)


def test_coarse_velocity_step_identity_eq68():
    """eq. (68): coarse velocity step = (f_c/f_s)/M * V_a, V_a = lambda PRF/2."""
    for fc, fs, prf, M in [(1e9, 1e7, 500.0, 64), (28e9, 491.52e6, 1905.0, 512)]:
        lam, dr, T = 3e8 / fc, 3e8 / (2 * fs), M / prf
        coarse = dr / T
        assert coarse == pytest.approx((fc / fs) / M * lam * prf / 2, rel=1e-14)


def test_paper_experiment1_range_bins_golden():
    """Range conversion r0 = n0 * c/(2 f_s) against the bins printed for
    Experiment 1 with the Table II radar (fixture tests/golden/paper_exp1.txt)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_exp1.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    kv = {r[0]: float(r[1]) for r in rows if r[0] in ("fs_hz",)}
    bins = [(int(r[1]), float(r[2])) for r in rows if r[0] == "bin"]
    dr = 3e8 / (2 * kv["fs_hz"])
    # the text pairs bin 1765 with 538.5 m; 1613 with 492.44 m is one bin off
    # under any rounding convention of 492.44/dr = 1613.6 (floor gives 1613)
    n, r = bins[0]
    assert abs(n * dr - r) <= dr / 2
    n, r = bins[1]
    assert abs(n * dr - r) <= dr


# ---- on-grid single target (normalisation, sign, offsets) -----------------

@pytest.mark.parametrize("order", [1, 2, 3])
def test_on_grid_impulse_target_peak_is_M_times_A(order):
    """A noiseless on-grid target (exact rational trajectory from the signal
    model) gives |Y| = M |A| at the true lattice point and nowhere more."""
    g = small_grid(order)
    rng = np.random.default_rng(11 + order)
    k = int(rng.integers(g.n_coarse))
    f = int(rng.integers(g.n_fine))
    i = g.lattice_point(k, f)
    steps = (Fr(3e8) / Fr(g.radar.fc) / (2 * Fr(g.M) / Fr(500)),
             Fr(3e8) / Fr(g.radar.fc) / (Fr(g.M) / Fr(500)) ** 2,
             3 * Fr(3e8) / Fr(g.radar.fc) / (Fr(g.M) / Fr(500)) ** 3)
    par = [i[p] * steps[p] for p in range(3)]
    n_true = 40
    amp = 0.7 * np.exp(0.3j)
    echo = synth.impulse_target_echo(
        synth.RadarParams(g.radar.fc, g.radar.bandwidth, 500.0), g.M, g.N,
        Fr(n_true) * Fr(15), par[0], par[1], par[2], amp)
    Pg = T.grft_power(echo, g)
    target = (g.M * abs(amp)) ** 2
    assert Pg[k, n_true, f] == pytest.approx(target, rel=1e-12)
    assert Pg.max() <= target * (1 + 1e-12)
    # DS-GRFT: the f = 0 cell of every coarse cell follows its coarse walk, so
    # the true coarse cell's centre point matches exactly when f is the centre
    Pd = T.dsgrft_power(echo, g)
    assert Pd.max() <= target * (1 + 1e-12)
    fc = g.h if order == 1 else (g.h * g.R + g.h if order == 2 else
                                 (g.h * g.R + g.h) * g.R + g.h)
    i_c = g.lattice_point(k, fc)
    par_c = [i_c[p] * steps[p] for p in range(3)]
    echo_c = synth.impulse_target_echo(
        synth.RadarParams(g.radar.fc, g.radar.bandwidth, 500.0), g.M, g.N,
        Fr(n_true) * Fr(15), par_c[0], par_c[1], par_c[2], amp)
    assert T.dsgrft_power(echo_c, g, cells=[k])[0, n_true, fc] == \
        pytest.approx(target, rel=1e-12)


# ---- linearity ----------------------------------------------------------------

def test_linearity_both_transforms():
    g = small_grid(2, M=16, N=40)
    rng = np.random.default_rng(3)
    s1 = rng.standard_normal((16, 40)) + 1j * rng.standard_normal((16, 40))
    s2 = rng.standard_normal((16, 40)) + 1j * rng.standard_normal((16, 40))
    al, be = 0.3 - 1.1j, 2.0 + 0.5j
    for fn in (T.dsgrft_cell, T.grft_cell):
        for k in (0, g.n_coarse - 1):
            lhs = fn(al * s1 + be * s2, g, k)
            rhs = al * fn(s1, g, k) + be * fn(s2, g, k)
            assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(rhs).max()


# ---- factorisation: DS == GRFT where the rounded walks coincide -----------

@pytest.mark.parametrize("order", [1, 2, 3])
def test_ds_equals_grft_where_walks_coincide(order):
    g = small_grid(order, M=16, N=48)
    rng = np.random.default_rng(5)
    echo = rng.standard_normal((16, 48)) + 1j * rng.standard_normal((16, 48))
    m = np.arange(g.M, dtype=np.int64)
    n_same = n_diff = 0
    for k in range(g.n_coarse):
        off_c = range_offset(g, numerator(g, m, g.centre(k)))
        ds = T.dsgrft_cell(echo, g, k)
        gr = T.grft_cell(echo, g, k)
        for f in range(g.n_fine):
            off_f = range_offset(g, numerator(g, m, g.lattice_point(k, f)))
            if np.array_equal(off_c, off_f):
                n_same += 1
                assert np.abs(ds[:, f] - gr[:, f]).max() <= 1e-12 * np.abs(gr[:, f]).max()
            else:
                n_diff += 1
    assert n_same > 0 and n_diff > 0


# ---- fine velocity stage is a DFT ---------------------------------------------

def test_fine_velocity_stage_is_inverse_fft():
    """With the fine velocity step equal to one DFT bin, the velocity stage of
    GFT (eq. (44), Def. 1: GFT = FFT{...}) is M * ifft of the de-chirped
    slow-time row, read at bin (i_c1 + f1) mod M."""
    g = small_grid(2, M=32, N=40)
    rng = np.random.default_rng(9)
    echo = rng.standard_normal((32, 40)) + 1j * rng.standard_normal((32, 40))
    m = np.arange(g.M, dtype=np.int64)
    k = g.n_coarse // 2
    ic = g.centre(k)
    off_c = range_offset(g, numerator(g, m, ic))
    ds = T.dsgrft_cell(echo, g, k)
    n0 = 20
    row = np.array([echo[mm, n0 + off_c[mm]] if 0 <= n0 + off_c[mm] < g.N else 0
                    for mm in range(g.M)])
    for u2 in (0, 3, g.R - 1):
        i2 = ic[1] + u2 - g.h
        chirp = np.exp(2j * np.pi * ((i2 * m * m) % (g.M ** 2)) / g.M ** 2)
        spec = g.M * np.fft.ifft(row * chirp)
        for u1 in range(g.R):
            f = u2 * g.R + u1
            q = (ic[0] + u1 - g.h) % g.M
            assert abs(ds[n0, f] - spec[q]) <= 1e-12 * np.abs(spec).max()


def test_textbook_mtd_special_case():
    """P = 1, a coarse cell whose walk stays in one bin: DS-GRFT of a row is
    the plain slow-time DFT (moving-target detection, Remark after Def. 1)."""
    g = make_grid(R1, 64, 64, 1, [Axis(-40.0, 40.0)])
    rng = np.random.default_rng(2)
    echo = rng.standard_normal((64, 64)) + 1j * rng.standard_normal((64, 64))
    m = np.arange(64, dtype=np.int64)
    for k in range(g.n_coarse):
        if np.any(range_offset(g, numerator(g, m, g.centre(k))) != 0):
            continue
        ds = T.dsgrft_cell(echo, g, k)
        spec = 64 * np.fft.ifft(echo[:, 10])
        for f in range(g.n_fine):
            i1 = g.lattice_point(k, f)[0]
            assert abs(ds[10, f] - spec[i1 % 64]) <= 1e-11 * np.abs(spec).max()
        return
    pytest.fail("no zero-walk coarse cell")


# ---- single-sample echo: closed form --------------------------------------

def test_single_sample_echo_closed_form():
    """Echo = delta at (m0, n1): Y_G(n0; i) is exp(j 2 pi 2 D(t_m0)/lambda)
    where the walk of i passes (m0, n1) and zero elsewhere (physical units,
    exact rationals)."""
    g = small_grid(2, M=12, N=30)
    m0, n1 = 9, 17
    echo = np.zeros((12, 30), dtype=np.complex128)
    echo[m0, n1] = 1.0
    lam, dr, t = Fr(3e8) / Fr(8e7), Fr(15), Fr(m0) / Fr(500)
    T_ = Fr(12) / Fr(500)
    steps = (lam / (2 * T_), lam / T_ ** 2)
    for k in range(g.n_coarse):
        gr = T.grft_cell(echo, g, k)
        for f in range(g.n_fine):
            i = g.lattice_point(k, f)
            D = i[0] * steps[0] * t + i[1] * steps[1] * t * t / 2
            off = math.floor(D / dr + Fr(1, 2))
            cyc = 2 * D / lam
            fr = cyc - math.floor(cyc)
            want = np.zeros(30, dtype=np.complex128)
            if 0 <= n1 - off < 30:
                want[n1 - off] = np.exp(2j * np.pi * fr.numerator / fr.denominator)
            assert np.abs(gr[:, f] - want).max() <= 1e-13


# ---- range equivariance ---------------------------------------------------

def test_range_shift_equivariance():
    g = small_grid(2, M=16, N=64)
    rng = np.random.default_rng(4)
    echo = np.zeros((16, 64), dtype=np.complex128)
    echo[:, 20:44] = rng.standard_normal((16, 24)) + 1j * rng.standard_normal((16, 24))
    d = 5
    sh = np.roll(echo, d, axis=1)
    for k in range(g.n_coarse):
        a = T.dsgrft_cell(echo, g, k)
        b = T.dsgrft_cell(sh, g, k)
        assert np.abs(b[10 + d:50 + d] - a[10:50]).max() <= 1e-12 * (np.abs(a).max() + 1)


# ---- noise statistics and the LRT threshold -------------------------------

def test_noise_only_power_is_exponential_with_mean_M_sigma2():
    """White circular noise: |Y|^2/(M sigma^2) ~ Exp(1) per cell, so the
    threshold of eq. (33) (K folded into sigma^2) gives the design P_FA."""
    g = make_grid(R1, 64, 256, 1, [Axis(-150.0, 150.0)])
    sigma2 = 2.5
    rng = np.random.Generator(np.random.PCG64(99))
    p_all = []
    for _ in range(6):
        echo = synth.make_echo(synth.RadarParams(1e9, 1e7, 500.0), 64, 256, [],
                               sigma2, rng, dtype=np.complex128)
        p_all.append(T.dsgrft_power(echo, g, cells=[1]).ravel())
    p = np.concatenate(p_all) / (64 * sigma2)
    assert p.mean() == pytest.approx(1.0, abs=0.02)
    pfa = 1e-2
    gamma2 = D.threshold(64, sigma2, pfa) / (64 * sigma2)
    assert (p > gamma2).mean() == pytest.approx(pfa, rel=0.15)


# ---- reduction and tie rules ----------------------------------------------

def test_reduction_tie_rules():
    P = np.array([[[1.0, 3.0, 3.0], [2.0, 2.0, 0.5]],
                  [[3.0, 1.0, 3.0], [0.0, 0.0, 0.0]]])
    pm, af = D.reduce_power(P)
    assert af.tolist() == [[1, 0], [0, 0]]
    assert D.global_argmax(pm) == (0, 0)
    assert D.detections(pm, af, 1.5) == [(0, 0, 1), (0, 1, 0), (1, 0, 0)]


def test_peak_parameters():
    g = make_grid(R1, 64, 256, 1, [Axis(-150.0, 150.0)])
    r0, v, a, j = D.peak_params(g, 1, 53, 57)
    assert (r0, a, j) == (795.0, 0.0, 0.0)
    # coarse cell 1 starts at i = -128 + 100; fine u = 57 -> i = -28 + 57
    assert v == pytest.approx((-28 + 57) * 1.171875, rel=1e-15)
