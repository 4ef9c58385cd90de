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


@pytest.mark.parametrize("form,split,tol", [("f16", 1, 1e-3), ("bf16", 3, 1e-3),
                                            ("f16_3m", 1, 1e-3), ("bf16_glo", 2, 1e-3),
                                            ("f16_sym", 1, 1e-3), ("bf16_sym", 3, 1e-3),
                                            ("bf16_sym", 2, 1e-3), ("bf16", 2, 1e-3),
                                            ("fp8", 3, 1e-3), ("fp8", 4, 1e-3),
                                            ("fp8_sym", 3, 1e-3), ("fp8_sym", 4, 1e-3)])
def test_config3_full_search_sampled(form, split, tol):
    case, plan, grid, echo = _setup(3)
    pm, af = plan.search(echo, form, split)
    gamma2 = plan.threshold(1.0, 1e-6)
    peaks, cnt, best = plan.detect(pm, af, 1e-6, 1.0, cap=4096)
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


def test_config4_adjoint_full_size():
    """4096 candidates at the M=512, N=2048 workload: analytic gradients vs
    central differences of the device objective, and vs the oracle on a
    sample; J on lattice points equals the search's power map."""
    from oracle import adjoint as OA
    case, plan, grid, echo = _setup(4)
    c = synth.CONFIGS[4]
    rng = np.random.Generator(np.random.PCG64(1004))
    th = synth.adjoint_candidates(rng, c["radar"], c["M"], c["N"], case["targets"],
                                  c["v"], c["a"])
    assert th.shape == (4096, 3)
    theta = torch.from_numpy(th)
    J, saved = plan.adjoint_forward(echo, theta)
    gJ = torch.ones(len(th), dtype=torch.float64, device="cuda")
    gt, _ = plan.adjoint_backward(echo, theta, saved, gJ, want_echo=False)
    gt = gt.cpu().numpy()
    # central differences on the device, candidates away from coarse-cell edges
    hs = np.array([1e-4 * grid.dr, 1e-4 * grid.steps[0], 1e-4 * grid.steps[1]])
    inside = np.ones(len(th), dtype=bool)
    for p in (0, 1):
        u = th[:, p + 1] / grid.steps[p] - grid.i_lo[p] + 0.5
        fr = (u / grid.R) % 1.0
        inside &= (fr > 0.01) & (fr < 0.99)
    idx = np.nonzero(inside)[0]
    assert len(idx) > 3500
    for q in range(3):
        e = np.zeros(3)
        e[q] = hs[q]
        Jp, _ = plan.adjoint_forward(echo, torch.from_numpy(th[idx] + e))
        Jm, _ = plan.adjoint_forward(echo, torch.from_numpy(th[idx] - e))
        fd = (Jp.cpu().numpy() - Jm.cpu().numpy()) / (2 * hs[q])
        scale = np.abs(gt[idx, q]).max()
        assert np.abs(fd - gt[idx, q]).max() <= 1e-4 * scale + 1e-7 * J.cpu().numpy()[idx].max() / hs[q]
    # oracle on a sample
    Jn = J.cpu().numpy()
    for b in np.random.default_rng(3).choice(len(th), 12, replace=False):
        Jo, _, go, _ = OA.gradients(case["echo"], grid, th[b])
        assert Jn[b] == pytest.approx(Jo, rel=1e-9, abs=1e-9 * Jo + 1e-6)
        np.testing.assert_allclose(gt[b], go, rtol=1e-7, atol=1e-9 * np.abs(go).max() + 1e-9)


def test_config5_jerk_search_subset():
    """P = 3 at M=2048, N=8192 on two coarse cells: the reported maximum of
    each sampled row equals the oracle at the reported cell, and no sampled
    fine cell of the row exceeds it (beyond the fp16 tolerance)."""
    case, plan, grid, echo = _setup(5)
    rng = np.random.default_rng(55)
    cells = torch.tensor(sorted(rng.choice(plan.n_coarse, 2, replace=False).tolist()),
                         dtype=torch.int64)
    pm, af = plan.search(echo, "f16", 1, cells=cells)
    pm32, af32 = plan.search(echo, "f32", 1, cells=cells)
    pm, af = pm.cpu().numpy(), af.cpu().numpy()
    pm32, af32 = pm32.cpu().numpy(), af32.cpu().numpy()
    tol = 1e-3
    e = case["echo"].astype(np.complex128)
    for ci, k in enumerate(cells.tolist()):
        rows = rng.choice(plan.rows, 3, replace=False)
        for r in rows:
            probe = np.unique(np.concatenate([rng.choice(plan.n_fine, 3000, replace=False),
                                              [af[ci, r], af32[ci, r]]]))
            y = OT.dsgrft_cell(e, grid, k, rows=[int(r)], fine=probe)[0]
            P = np.abs(y) ** 2
            scale = max(P.max(), float(pm[ci, r]))
            at = P[np.searchsorted(probe, af[ci, r])]
            assert abs(at - pm[ci, r]) <= tol * scale
            assert P.max() <= pm[ci, r] + 2 * tol * scale
            at32 = P[np.searchsorted(probe, af32[ci, r])]
            assert abs(at32 - pm32[ci, r]) <= 1e-5 * scale
            assert P.max() <= pm32[ci, r] + 2e-5 * scale


def test_config3_fft_form_sampled():
    """FFT fine-velocity form at M = 1024: sampled rows of 3 cells against the
    oracle within the FP32 tolerance, and against the GEMM FP32 form."""
    case, plan, grid, echo = _setup(3)
    cells = torch.tensor([0, 1234, plan.n_coarse - 1], dtype=torch.int64)
    pm, af = plan.search(echo, "f32fft", 1, cells=cells)
    pm32, af32 = plan.search(echo, "f32", 1, cells=cells)
    pm, af, pm32 = pm.cpu().numpy(), af.cpu().numpy(), pm32.cpu().numpy()
    rows = sorted(np.random.default_rng(9).choice(plan.rows, 24, replace=False).tolist())
    idx = {int(c): i for i, c in enumerate(cells.tolist())}
    _check_rows({c: pm[i] for c, i in idx.items()}, {c: af[i] for c, i in idx.items()},
                case["echo"], grid, list(idx), rows, 1e-5)
    assert np.abs(pm - pm32).max() <= 2e-5 * pm32.max()


def test_config3_cfar_on_full_map():
    """CA-CFAR over the whole M=1024 reduced map (2460 cells x 4096 rows),
    bit-exact against the oracle's CA-CFAR on the same map."""
    from oracle import detect as OD
    case, plan, grid, echo = _setup(3)
    pm, af = plan.search(echo, "f16_3m", 1)
    guard, train, alpha = 2, 16, 1.5
    hit = OD.ca_cfar(pm.cpu().numpy(), guard, train, alpha)
    cap = int(hit.sum()) + 16
    peaks, cnt, _ = plan.detect_cfar(pm, af, guard, train, alpha, cap=cap)
    assert cnt == int(hit.sum()) and len(peaks) == cnt
    got = np.stack([peaks["coarse"].astype(np.int64), peaks["row"].astype(np.int64)], 1)
    assert np.array_equal(got, np.argwhere(hit))


@pytest.mark.parametrize("form,split,tol", [("bf16_sym", 3, 1e-3), ("f16_sym", 1, 1e-3),
                                            ("f32", 1, 1e-5)])
def test_config5_full_map_on_target_window(form, split, tol):
    """P = 3 at M=2048, N=8192: the full map (10^6 fine cells) of the first
    target's coarse cell on an 8-row window around its range, element by
    element on 2000 sampled fine cells plus each row's reported maximum,
    against the oracle evaluated at those fine cells."""
    from paper_2403_06788_amd.plan import Plan
    case = synth.config_case(5)
    c = synth.CONFIGS[5]
    r = c["radar"]
    tg = case["targets"][0]
    n0 = int(round(tg.r0 / r.dr)) - 4
    rows = (n0, n0 + 8)
    plan = Plan(r.fc, r.fs, r.prf, c["M"], c["N"], c["order"], c["axes"], rows=rows)
    grid = make_grid(Radar(r.fc, r.fs, r.prf), c["M"], c["N"], c["order"],
                     [Axis(*a) for a in c["axes"]], *rows)
    ks = []
    for p, val in enumerate((tg.v, tg.a, tg.j)):
        k = int(np.floor((val / plan.step[p] - plan.i_lo[p] + 0.5) / plan.R))
        ks.append(min(max(k, 0), plan.K[p] - 1))
    kt = (ks[2] * plan.K[1] + ks[1]) * plan.K[0] + ks[0]
    print(f"config 5 {form} x{split}: cell {kt}, rows {rows}", flush=True)
    Pd = plan.search_full(torch.from_numpy(case["echo"]).cuda(), form, split,
                          cc_begin=kt, n=1)[0].cpu().numpy().astype(np.float64)
    assert Pd.shape == (8, grid.n_fine)
    rng = np.random.default_rng(77)
    probe = np.unique(np.concatenate([rng.choice(grid.n_fine, 2000, replace=False),
                                      Pd.argmax(axis=1)]))
    y = OT.dsgrft_cell(case["echo"].astype(np.complex128), grid, kt, fine=probe)
    P = np.abs(y) ** 2
    scale = P.max()
    assert scale > 0.5 * Pd.max()
    assert np.abs(Pd[:, probe] - P).max() <= tol * scale
    plan.close()
