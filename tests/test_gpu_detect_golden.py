"""Device LRT detections on the full second-order workloads against the FP64
oracle's detection sets (Sec. III-C, eqs. (31), (33); Alg. 3; eq. (72)).

The goldens (tests/golden/detect_config{2,3}.json, written by
make_detect_goldens.py from oracle/ and synth/ only) hold every reduced-map
entry of the oracle at or above 0.9 of the lowest threshold listed, with its
fine index and the row's other fine cells within 1% of its maximum, and the
64 largest entries of the map.  The device search runs in the configuration
the benchmark times (whole plan, default batching).

Near-tie rule (with tol the form's tolerance and Pmax the oracle's largest
power): an oracle entry more than 2 tol Pmax above the threshold must be
detected, one more than 2 tol Pmax below it must not; every device
detection must be an oracle entry; its power agrees within tol Pmax; its fine
index equals the oracle's unless another fine cell of the row lies within
2 tol Pmax of the row's maximum, in which case it is one of those; the
device's global maximum is one of the oracle's entries within 2 tol Pmax of
the oracle's largest power."""
import json
import os

import numpy as np
import pytest
import torch

import synth
from oracle import detect as OD
from oracle import transforms as OT
from oracle.grid import Axis, Radar, make_grid

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# The two-product bf16 forms keep one operand's bf16 rounding (2^-9
# relative); at M = 512 it reaches 1.03e-3 of the peak power on a detection
# entry, so they are held to 2e-3 here; three products are within 1e-3.
FORMS = {
    2: [("f32", 1, 1e-5), ("f32fft", 1, 1e-5), ("f16_sym", 1, 1e-3), ("f16", 1, 1e-3),
        ("bf16_sym", 3, 1e-3), ("bf16", 3, 1e-3), ("bf16_sym", 2, 2e-3),
        ("bf16_glo", 2, 2e-3), ("fp8", 3, 1e-3), ("fp8_sym", 3, 1e-3)],
    3: [("f32fft", 1, 1e-5), ("f16_sym", 1, 1e-3), ("f16_3m", 1, 1e-3), ("f16", 1, 1e-3),
        ("bf16_sym", 3, 1e-3), ("bf16", 3, 1e-3), ("bf16_sym", 2, 2e-3),
        ("bf16_glo", 2, 2e-3), ("bf16", 2, 2e-3), ("fp8", 3, 1e-3), ("fp8", 4, 1e-3),
        ("fp8_sym", 3, 1e-3), ("fp8_sym", 4, 1e-3)],
}

_cache = {}


def _setup(cfg):
    if cfg in _cache:
        return _cache[cfg]
    path = os.path.join(GOLDEN, f"detect_config{cfg}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    from paper_2403_06788_amd.plan import Plan
    gold = json.load(open(path))
    c = synth.CONFIGS[cfg]
    r = c["radar"]
    plan = Plan(r.fc, r.fs, r.prf, c["M"], c["N"], c["order"], c["axes"])
    grid = make_grid(Radar(r.fc, r.fs, r.prf), c["M"], c["N"], c["order"],
                     [Axis(*a) for a in c["axes"]])
    assert (plan.n_coarse, plan.rows, plan.n_fine) == (gold["n_coarse"], gold["rows"],
                                                       gold["n_fine"])
    echo = torch.from_numpy(synth.config_case(cfg)["echo"]).cuda()
    _cache.clear()
    _cache[cfg] = (gold, plan, grid, echo)
    return _cache[cfg]


def _fine_ok(entry, f_dev, band):
    """Device fine index against an oracle entry under the near-tie rule."""
    _, _, f, p, near = entry
    ties = {int(q) for q, pq in near if pq >= p - band}
    return f_dev == f if not ties else f_dev in ties | {f}


def _compare(plan, grid, pm, af, ents, top, scale, pfas, sigma2, tol, gammas=None):
    band = 2 * tol * scale
    worst = 0.0
    for i, pfa in enumerate(pfas):
        g2 = plan.threshold(sigma2, pfa)
        if gammas is not None:
            assert g2 == gammas[i]
        peaks, cnt, best = plan.detect(pm, af, pfa, sigma2, cap=1 << 16)
        assert cnt == len(peaks)
        got = {(int(q["coarse"]), int(q["row"])): q for q in peaks}
        keys = [(int(q["coarse"]), int(q["row"])) for q in peaks]
        assert keys == sorted(keys)
        must = {k for k, e in ents.items() if e[3] > g2 + band}
        never = {k for k, e in ents.items() if e[3] < g2 - band}
        assert must <= set(got), sorted(must - set(got))[:10]
        assert not (never & set(got)), sorted(never & set(got))[:10]
        assert set(got) <= set(ents), sorted(set(got) - set(ents))[:10]
        for k, q in got.items():
            e = ents[k]
            worst = max(worst, abs(float(q["power"]) - e[3]) / scale)
            assert abs(float(q["power"]) - e[3]) <= tol * scale, (k, float(q["power"]), e[3])
            assert _fine_ok(e, int(q["fine"]), band), (k, int(q["fine"]), e[2], e[4])
            r0, v, a, j = OD.peak_params(grid, k[0], k[1], int(q["fine"]))
            assert (q["r0"], q["v"], q["a"], q["j"]) == pytest.approx((r0, v, a, j), rel=1e-15,
                                                                      abs=1e-12)
    # global maximum
    cand = {(t[0], t[1]) for t in top if t[3] >= top[0][3] - band}
    kb = (int(best["coarse"]), int(best["row"]))
    assert kb in cand, (kb, top[:3])
    assert abs(float(best["power"]) - top[0][3]) <= tol * scale
    if kb in ents:
        assert _fine_ok(ents[kb], int(best["fine"]), band)
    print(f"largest power error on the detections: {worst:.3e} of the peak", flush=True)
    return len(got)


@pytest.mark.parametrize("cfg,form,split,tol",
                         [(c, f, s, t) for c in (2, 3) for f, s, t in FORMS[c]])
def test_detections_match_oracle(cfg, form, split, tol):
    gold, plan, grid, echo = _setup(cfg)
    print(f"config {cfg} {form} x{split}", flush=True)
    pm, af = plan.search(echo, form, split)
    ents = {(e[0], e[1]): e for e in gold["entries"]}
    _compare(plan, grid, pm, af, ents, gold["top"], gold["pmax"], gold["pfa"], gold["sigma2"],
             tol, gold["gamma2"])


@pytest.fixture(scope="module")
def config1():
    """The M = 64 workload: its whole oracle map is computed here (3 coarse
    cells x 256 rows x 100 fine cells), so every reduced entry is known."""
    from paper_2403_06788_amd.plan import Plan
    c = synth.CONFIGS[1]
    r = c["radar"]
    grid = make_grid(Radar(r.fc, r.fs, r.prf), c["M"], c["N"], c["order"],
                     [Axis(*a) for a in c["axes"]])
    e = synth.config_case(1)["echo"]
    P = OT.dsgrft_power(e.astype(np.complex128), grid)
    pm, af = OD.reduce_power(P)
    ents = {}
    for k in range(P.shape[0]):
        for n in range(P.shape[1]):
            near = np.nonzero(P[k, n] >= 0.99 * pm[k, n])[0]
            ents[(k, n)] = [k, n, int(af[k, n]), float(pm[k, n]),
                            [[int(f), float(P[k, n, f])] for f in near if f != af[k, n]]]
    order = sorted(ents.values(), key=lambda x: -x[3])
    top = [[x[0], x[1], x[2], x[3]] for x in order[:64]]
    plan = Plan(r.fc, r.fs, r.prf, c["M"], c["N"], c["order"], c["axes"])
    return dict(plan=plan, grid=grid, echo=torch.from_numpy(e).cuda(), ents=ents, top=top,
                scale=float(P.max()))


@pytest.mark.parametrize("form,split,tol", [("f32", 1, 1e-5), ("f32fft", 1, 1e-5),
                                            ("f16_sym", 1, 1e-3), ("f16_3m", 1, 1e-3),
                                            ("f16", 1, 1e-3), ("bf16_sym", 3, 1e-3),
                                            ("bf16", 3, 1e-3), ("fp8", 3, 1e-2)])
def test_config1_every_entry(config1, form, split, tol):
    """LRT detections of the M = 64 workload at P_FA 1e-9 ... 1e-1 (from the
    target alone to a third of the map) against the complete oracle map."""
    c = config1
    pm, af = c["plan"].search(c["echo"], form, split)
    n = [_compare(c["plan"], c["grid"], pm, af, c["ents"], c["top"], c["scale"], [pfa], 1.0, tol)
         for pfa in (1e-9, 1e-6, 1e-3, 1e-2, 1e-1)]
    assert n[-1] > 100 and n[0] >= 1
