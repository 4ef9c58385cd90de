"""Monte-Carlo detection trials (the Pd-vs-SNR sweep of the benchmark): each
detector's statistic and decision against the FP64 oracle on seeded trials
near the detection threshold."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import fd as OF
from oracle import ktmfp as KT
from oracle import transforms as OT
from oracle.grid import Axis, Radar, make_grid

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _oracle_stats(echo, grid, cells, rows, ktc):
    r = np.arange(*rows)
    F = OT.fine_matrix(grid)
    Np = OF.pad_length(grid)
    S = OF.range_spectrum(echo, Np)
    td = max(float((np.abs(OT.dsgrft_cell(echo, grid, k, rows=r + grid.n_begin)) ** 2).max())
             for k in cells)
    fdv = max(float((np.abs(OF.mgift_fd(echo, grid, k, Np, S)[:, r].T @ F) ** 2).max())
              for k in cells)
    gr = max(float((np.abs(OT.grft_cell(echo, grid, k, rows=r + grid.n_begin)) ** 2).max())
             for k in cells)
    ykt = KT.coarse_rows(echo, grid, ktc, Np=Np)[:, r]
    kt = float((np.abs(ykt.T @ KT.fine_matrix(grid)) ** 2).max())
    return {"ds_td": td, "ds_fd": fdv, "ds_kt": kt, "grft": gr}


@pytest.mark.parametrize("snr,seed", [(-16.0, 1), (-15.0, 2), (-14.0, 3), (-13.0, 4)])
def test_trial_statistics_and_decisions_match_oracle(snr, seed):
    from bench import PD_PFA, pd_trial
    from paper_2403_06788_amd.plan import Plan
    sc = synth.PD_SCENARIO
    r = sc["radar"]
    plans = {"ds_td": Plan(r.fc, r.fs, r.prf, sc["M"], sc["N"], sc["order"], sc["axes"]),
             "ds_fd": Plan(r.fc, r.fs, r.prf, sc["M"], sc["N"], sc["order"], sc["axes"],
                           mgift="fd"),
             "ds_kt": Plan(r.fc, r.fs, r.prf, sc["M"], sc["N"], sc["order"], sc["axes"],
                           mgift="kt")}
    grid = make_grid(Radar(r.fc, r.fs, r.prf), sc["M"], sc["N"], sc["order"],
                     [Axis(*a) for a in sc["axes"]])
    gamma2 = plans["ds_td"].threshold(1.0, PD_PFA)
    rng = np.random.Generator(np.random.PCG64(seed))
    tg = synth.draw_targets(rng, r, sc["M"], sc["N"], 1, snr, 1.0, sc["v"], sc["a"], sc["j"])[0]
    echo = synth.make_echo(r, sc["M"], sc["N"], [tg], 1.0, rng)
    res, cells, rows, kt, ktc = pd_trial(plans, torch.from_numpy(echo).cuda(), tg, gamma2)
    assert kt in cells
    q, i2c = KT.coarse_params(grid, KT.lattice(grid), ktc)
    i1 = int(np.floor(tg.v / grid.steps[0] + 0.5))
    assert q * sc["M"] - sc["M"] // 2 <= i1 < q * sc["M"] + sc["M"] // 2
    assert abs(tg.a / grid.steps[1] - i2c) <= grid.R / 2 + 0.5
    ref = _oracle_stats(echo.astype(np.complex128), grid, cells, rows, ktc)
    for d, tol in (("ds_td", 1e-3), ("ds_fd", 1e-3), ("ds_kt", 1e-5), ("grft", 1e-5)):
        stat, hit = res[d]
        assert abs(stat - ref[d]) <= tol * ref[d], (d, stat, ref[d])
        if abs(ref[d] - gamma2) > tol * ref[d]:
            assert hit == (ref[d] > gamma2), d


def test_pd_bench_mode_runs():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "6",
                          "--trials", "3"], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr[-2000:]
    d = json.loads(out.stdout.strip().splitlines()[-1])
    assert set(d["pd"]) == {"ds_td", "ds_fd", "ds_kt", "grft"}
    assert len(d["snr_db"]) == len(d["pd"]["ds_td"])
    assert d["value"] > 0
