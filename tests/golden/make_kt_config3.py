"""Writes kt_config3_rows.json: the FP64 oracle's DS-KT-MFP reduced map
(max |Y|^2 and its fine index) on sampled rows of three coarse cells of the
M = 1024, N = 4096 workload (v +-600 m/s, a +-50 m/s^2, N' = 8192, the seeded
8-target echo at -20 dB).  Calls only oracle/ and synth/; takes a few
minutes (the keystone sum over 8192 frequencies x 1024^2 pulse pairs).

    python tests/golden/make_kt_config3.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import fd as OF  # noqa: E402
from oracle import ktmfp as KT  # noqa: E402
from oracle.grid import Axis, Radar, make_grid  # noqa: E402

CELLS = [3, 130, 251]
N_ROWS = 24
ROW_SEED = 17


def main():
    c = synth.CONFIGS[3]
    r = c["radar"]
    g = make_grid(Radar(r.fc, r.fs, r.prf), c["M"], c["N"], c["order"],
                  [Axis(*a) for a in c["axes"]])
    echo = synth.config_case(3)["echo"].astype(np.complex128)
    Np = OF.pad_length(g)
    SK = KT.keystone(OF.range_spectrum(echo, Np), g, Np)
    F = KT.fine_matrix(g)
    rows = sorted(int(x) for x in np.random.default_rng(ROW_SEED).choice(g.rows, N_ROWS,
                                                                          replace=False))
    out = {"workload": "DS-KT-MFP, M=1024, N=4096, P=2, v +-600 m/s, a +-50 m/s^2, "
                       "synth.config_case(3) echo",
           "pad_length": Np, "n_coarse": KT.lattice(g).n_coarse, "rows": rows, "cells": {}}
    for k in CELLS:
        y = KT.coarse_rows(echo, g, k, SK, Np)[:, rows]
        P = np.abs(y.T @ F) ** 2
        srt = np.sort(P, axis=1)
        out["cells"][str(k)] = {"pmax": [float(v) for v in P.max(axis=1)],
                                "argf": [int(v) for v in P.argmax(axis=1)],
                                "second": [float(v) for v in srt[:, -2]]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "kt_config3_rows.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
