"""Writes detect_config2.json and detect_config3.json: the FP64 oracle's LRT
detections (Sec. III-C, eqs. (31), (33); Alg. 3) on the full DS-GRFT search of
the two second-order workloads, for the device detection tests.

  config 2: M=512,  N=2048, P=2, v +-600 m/s, a +-50 m/s^2, 3 targets, -15 dB
  config 3: M=1024, N=4096, P=2, v +-600 m/s, a +-50 m/s^2, 8 targets, -20 dB
  (synth.config_case(cfg) echoes, sigma^2 = 1, R = 100)

For every (coarse cell, range row) the oracle's reduced entry (largest |Y|^2
over the cell's 10^4 fine cells and the smallest fine index attaining it) is
computed; kept are the entries whose power is at least `keep` (0.9 times the
threshold of the largest false-alarm probability listed), each with the other
fine indices of its row within 1% of the row's maximum (the near-tie set of
the index comparison), and the 64 largest entries of the whole map (for the
global maximum).  The thresholds are gamma^2 = -M sigma^2 ln P_FA.

Calls only oracle/ and synth/.  Config 3 evaluates 1.0e11 cells x 1024
pulses in FP64 (about an hour on 8 cores); config 2 a few minutes.

    python tests/golden/make_detect_goldens.py [2] [3]
"""
import os

# one BLAS thread per worker process; the cells are spread over processes
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

import heapq  # noqa: E402
import json  # noqa: E402
import multiprocessing as mp  # noqa: E402
import sys  # noqa: E402
import time  # noqa: E402

import numpy as np  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import detect as OD  # noqa: E402
from oracle import transforms as OT  # noqa: E402
from oracle.grid import Axis, Radar, make_grid  # noqa: E402

PFA = {2: (1e-9, 1e-8, 1e-7), 3: (1e-9, 1e-8)}
SIGMA2 = 1.0
KEEP = 0.9      # kept entries: power >= KEEP * the lowest threshold
NEAR = 0.99     # near-tie set: other fine indices >= NEAR * row maximum
TOP = 64
CHUNK = 512     # range rows per matrix product

_W = {}


def _grid(cfg):
    c = synth.CONFIGS[cfg]
    r = c["radar"]
    return make_grid(Radar(r.fc, r.fs, r.prf), c["M"], c["N"], c["order"],
                     [Axis(*a) for a in c["axes"]])


def _init(cfg, keep):
    g = _grid(cfg)
    _W["g"] = g
    _W["echo"] = synth.config_case(cfg)["echo"].astype(np.complex128)
    _W["H"] = OT.fine_matrix(g)
    _W["keep"] = keep


def _cell(k):
    g, echo, H, keep = _W["g"], _W["echo"], _W["H"], _W["keep"]
    rows = np.arange(g.n_begin, g.n_end)
    kept, top = [], []
    for s in range(0, len(rows), CHUNK):
        r = rows[s:s + CHUNK]
        P = np.abs(OT.dsgrft_cell(echo, g, k, rows=r, H=H)) ** 2
        pm, af = OD.reduce_power(P)
        for i in np.nonzero(pm >= keep)[0]:
            near = np.nonzero(P[i] >= NEAR * pm[i])[0]
            kept.append([int(k), int(r[i]), int(af[i]), float(pm[i]),
                         [[int(f), float(P[i, f])] for f in near if f != af[i]]])
        for i in np.argsort(pm)[-TOP:]:
            top.append((float(pm[i]), int(k), int(r[i]), int(af[i])))
    return kept, heapq.nlargest(TOP, top)


def make(cfg, workers):
    g = _grid(cfg)
    c = synth.CONFIGS[cfg]
    gam = [OD.threshold(g.M, SIGMA2, p) for p in PFA[cfg]]
    keep = KEEP * min(gam)
    t0 = time.time()
    kept, top = [], []
    with mp.get_context("fork").Pool(workers, _init, (cfg, keep)) as pool:
        for i, (kp, tp) in enumerate(pool.imap(_cell, range(g.n_coarse), chunksize=1)):
            kept += kp
            top = heapq.nlargest(TOP, top + tp)
            if (i + 1) % 50 == 0 or i + 1 == g.n_coarse:
                print(f"config {cfg}: {i + 1}/{g.n_coarse} cells, {len(kept)} kept, "
                      f"{time.time() - t0:.0f} s", flush=True)
    kept.sort(key=lambda e: (e[0], e[1]))
    pmax = top[0][0]
    # the near-tie band of the index rule (2 x 1e-3 of the peak power) must lie
    # inside the stored 1% band of every kept row
    assert 2e-3 * pmax <= (1.0 - NEAR) * keep, (pmax, keep)
    out = {"workload": f"DS-GRFT search, M={g.M}, N={g.N}, P={g.order}, "
                       f"axes {c['axes']}, synth.config_case({cfg}) echo",
           "config": cfg, "M": g.M, "N": g.N, "n_coarse": g.n_coarse, "rows": g.rows,
           "n_fine": g.n_fine, "sigma2": SIGMA2, "pfa": list(PFA[cfg]), "gamma2": gam,
           "keep": keep, "near": NEAR, "pmax": pmax,
           "top": [[k, r, f, p] for p, k, r, f in top],
           "entries": kept}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"detect_config{cfg}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, separators=(",", ":"))
    print("wrote", path, f"({len(kept)} entries, {time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    cfgs = [int(a) for a in sys.argv[1:]] or [2, 3]
    for cfg in cfgs:
        make(cfg, os.cpu_count() or 1)
