"""Full-size parity at the workload configurations, in the launch
configuration the benchmark times (default plan batching), on sampled
outputs the oracle computes one by one."""
import numpy as np
import pytest
import torch

import synth
from oracle import transforms as OT
from oracle.grid import Axis, Radar, make_grid

pytestmark = pytest.mark.gpu


def _setup(cfg):
    from paper_2403_06788_amd.plan import Plan
    case = synth.config_case(cfg)
    c = synth.CONFIGS[cfg]
    r = c["radar"]
    plan = Plan(r.fc, r.fs, r.prf, c["M"], c["N"], c["order"], c["axes"])
    grid = make_grid(Radar(r.fc, r.fs, r.prf), c["M"], c["N"], c["order"],
                     [Axis(*a) for a in c["axes"]])
    return case, plan, grid, torch.from_numpy(case["echo"]).cuda()


def _check_rows(pm, af, echo, grid, cells, rows, tol):
    scale = 0.0
    refs = {}
    for k in cells:
        P = np.abs(OT.dsgrft_cell(echo, grid, int(k), rows=rows)) ** 2
        refs[k] = P
        scale = max(scale, float(P.max()))
    worst = 0.0
    for k, P in refs.items():
        pm_o, af_o = P.max(-1), P.argmax(-1)
        srt = np.sort(P, -1)
        gap = srt[:, -1] - srt[:, -2]
        for i, r in enumerate(rows):
            worst = max(worst, abs(float(pm[k][r]) - pm_o[i]) / scale)
            if gap[i] > 2 * tol * scale:
                assert af[k][r] == af_o[i], (k, r)
            else:
                assert P[i, af[k][r]] >= pm_o[i] - 2 * tol * scale
    assert worst <= tol, worst
    return worst


@pytest.mark.parametrize("form,split,tol", [("f16", 1, 1e-3), ("bf16", 3, 1e-3)])
def test_config3_full_search_sampled(form, split, tol):
    case, plan, grid, echo = _setup(3)
    pm, af = plan.search(echo, form, split)
    gamma2 = plan.threshold(1.0, 1e-6)
    peaks, cnt, best = plan.detect(pm, af, gamma2, cap=4096)
    pm, af = pm.cpu().numpy(), af.cpu().numpy()
    assert np.isfinite(pm).all() and (af >= 0).all() and (af < plan.n_fine).all()
    rng = np.random.default_rng(31)
    cells = sorted(set([int(best["coarse"])] + [int(x) for x in rng.choice(plan.n_coarse, 3, replace=False)]))
    rows = sorted(set([int(best["row"])] + [int(x) for x in rng.choice(plan.rows, 24, replace=False)]))
    _check_rows(pm, af, case["echo"], grid, cells, rows, tol)
    # global maximum and its parameters
    k, r = int(best["coarse"]), int(best["row"])
    assert best["power"] == pm[k, r] == pm.max()
    # every listed detection is above the threshold and in flat order
    assert cnt == int((pm > gamma2).sum()) and len(peaks) == min(cnt, 4096)
    keys = [(int(q["coarse"]), int(q["row"])) for q in peaks]
    assert keys == sorted(keys)


def test_config2_fp32_plain_and_mfma_sampled():
    case, plan, grid, echo = _setup(2)
    cells = torch.arange(0, plan.n_coarse, 37, dtype=torch.int64)
    pm32, af32 = plan.search(echo, "f32", 1, cells=cells)
    pm16, af16 = plan.search(echo, "f16", 1, cells=cells)
    rows = sorted(np.random.default_rng(5).choice(plan.rows, 24, replace=False).tolist())
    sub = list(range(len(cells)))
    # index the device results by position in the cell list
    idx = {int(c): i for i, c in enumerate(cells.tolist())}

    def remap(a):
        return {c: a[i] for c, i in idx.items()}
    for pm, af, tol in ((pm32, af32, 1e-5), (pm16, af16, 1e-3)):
        pmn, afn = remap(pm.cpu().numpy()), remap(af.cpu().numpy())
        _check_rows(pmn, afn, case["echo"], grid, list(idx), rows, tol)
    assert sub
