"""Small parity cases shared by the GPU tests (seeded, synthetic).

Each case spans several row/column tiles of the kernels and has ragged tails
in pulses (K), range rows and fine columns.
"""
from __future__ import annotations

import numpy as np

import synth
from oracle.grid import Axis, Radar, make_grid

CASES = {
    # config 1 of the workload table: P = 1, R = 100, M = 64, N = 256
    "cfg1": dict(fc=1.0e9, fs=1.0e7, prf=500.0, M=64, N=256, order=1,
                 axes=[(-150.0, 150.0)], targets=1, snr_db=0.0, rows=None),
    # P = 2, R = 12 (144 fine columns), M = 100 (ragged K), N = 300
    "p2": dict(fc=1.2e8, fs=1.0e7, prf=500.0, M=100, N=300, order=2,
               axes=[(-100.0, 100.0), (-400.0, 400.0)], targets=3, snr_db=-3.0,
               rows=None),
    # P = 2 with a row window of interest [37, 261)
    "p2rows": dict(fc=1.2e8, fs=1.0e7, prf=500.0, M=100, N=300, order=2,
                   axes=[(-100.0, 100.0), (-400.0, 400.0)], targets=3,
                   snr_db=-3.0, rows=(37, 261)),
    # P = 2 with an odd R = 13: every fine cell but the centre has its
    # conjugate partner (169 cells in 85 pair columns)
    "p2odd": dict(fc=1.3e8, fs=1.0e7, prf=500.0, M=64, N=160, order=2,
                  axes=[(-200.0, 200.0), (-300.0, 300.0)], targets=2, snr_db=-3.0,
                  rows=None),
    # P = 3, R = 6 (36 columns x 6 jerk units per coarse cell), M = 72
    "p3": dict(fc=6.0e7, fs=1.0e7, prf=500.0, M=72, N=200, order=3,
               axes=[(-150.0, 150.0), (-600.0, 600.0), (-9000.0, 9000.0)],
               targets=2, snr_db=-3.0, rows=None),
}


def make_case(name: str, seed: int = 123):
    c = CASES[name]
    radar = synth.RadarParams(c["fc"], c["fs"], c["prf"])
    rng = np.random.Generator(np.random.PCG64(seed))
    lam, dr = radar.lam, radar.dr
    T = c["M"] / c["prf"]
    axes = c["axes"] + [(0.0, 0.0)] * (3 - len(c["axes"]))
    tg = synth.draw_targets(rng, radar, c["M"], c["N"], c["targets"], c["snr_db"],
                            1.0, axes[0], axes[1], axes[2])
    echo = synth.make_echo(radar, c["M"], c["N"], tg, 1.0, rng)
    rows = c["rows"]
    g = make_grid(Radar(c["fc"], c["fs"], c["prf"]), c["M"], c["N"], c["order"],
                  [Axis(*a) for a in c["axes"]],
                  *(rows if rows else (0, None)))
    return dict(spec=c, echo=echo, grid=g, targets=tg, lam=lam, dr=dr, T=T)


def plan_for(case, **kw):
    from paper_2403_06788_amd.plan import Plan
    c = case["spec"]
    return Plan(c["fc"], c["fs"], c["prf"], c["M"], c["N"], c["order"], c["axes"],
                rows=c["rows"], **kw)


def near_tie_check(pm_dev, af_dev, P_ref, tol):
    """Reduced-map agreement with the near-tie rule.

    pm_dev/af_dev: [cells, rows] device results (numpy); P_ref: oracle power
    [cells, rows, F].  Powers must agree within tol * max(P_ref).  The device
    argmax must equal the oracle's where the oracle's top-1/top-2 gap exceeds
    2 tol * max, and otherwise lie in the oracle's near-tie set.
    Returns (max relative power error, number of exact-index checks).
    """
    scale = float(P_ref.max())
    pm_ref = P_ref.max(axis=-1)
    af_ref = P_ref.argmax(axis=-1)
    err = float(np.abs(pm_dev.astype(np.float64) - pm_ref).max()) / scale
    assert err <= tol, f"power error {err:.3e} > {tol:.1e}"
    srt = np.sort(P_ref, axis=-1)
    gap = srt[..., -1] - srt[..., -2] if P_ref.shape[-1] > 1 else np.full(pm_ref.shape, np.inf)
    clear = gap > 2 * tol * scale
    assert np.array_equal(af_dev[clear], af_ref[clear]), "argmax mismatch on clear rows"
    amb = np.argwhere(~clear)
    for k, r in amb:
        f = int(af_dev[k, r])
        assert 0 <= f < P_ref.shape[-1]
        assert P_ref[k, r, f] >= pm_ref[k, r] - 2 * tol * scale, "argmax outside near-tie set"
    return err, int(clear.sum())
