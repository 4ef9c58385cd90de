"""DS-KT-MFP (Alg. 4, Prop. 3) through the C ABI against the FP64 oracle
(oracle.ktmfp): the compensated coarse rows, the full |Y|^2 map and the
reduced map at FP32 tolerance (1e-5 of the peak power), the folded lattice
and peak parameters, sampled rows at M = 1024, and at the full benchmark size
(M = 1024, N = 4096, N' = 8192) the properties that hold at any size."""
import numpy as np
import pytest
import torch

import synth
from cases import near_tie_check
from oracle import fd as OF
from oracle import ktmfp as KT
from oracle.grid import Axis, Radar, make_grid

pytestmark = pytest.mark.gpu

TOL = 1e-5

# M = 64 with R = 100 > M (five folding factors, one coarse acceleration);
# M = 128, R = 12 with a row window (several folds x two coarse accelerations);
# M = 2048, R = 4
KT_CASES = {
    "m64": dict(fc=1.0e9, fs=1.0e7, prf=500.0, M=64, N=128,
                axes=[(-150.0, 150.0), (-200.0, 200.0)], targets=2, snr_db=0.0, rows=None),
    "m128rows": dict(fc=1.2e8, fs=1.0e7, prf=500.0, M=128, N=300,
                     axes=[(-1500.0, 1500.0), (-400.0, 400.0)], targets=3, snr_db=-3.0,
                     rows=(40, 260)),
    # M = 2048: the keystone's 4-frequency tiles and the FFT kernel with 32
    # pulses per lane; R = 4 keeps the oracle's M x MR fine matrix small
    "m2048": dict(fc=4.0e7, fs=1.0e7, prf=500.0, M=2048, N=48,
                  axes=[(-1000.0, 1000.0), (-2.0, 2.0)], targets=1, snr_db=-10.0, rows=None,
                  draw_v=(-50.0, 50.0)),
}


def _plan(c, rows=None):
    from paper_2403_06788_amd.plan import Plan
    return Plan(c["fc"], c["fs"], c["prf"], c["M"], c["N"], 2, c["axes"], rows=rows,
                mgift="kt")


def _grid(c, rows=None):
    return make_grid(Radar(c["fc"], c["fs"], c["prf"]), c["M"], c["N"], 2,
                     [Axis(*a) for a in c["axes"]], *(rows if rows else (0, None)))


def _make(name, seed=77):
    c = KT_CASES[name]
    radar = synth.RadarParams(c["fc"], c["fs"], c["prf"])
    rng = np.random.Generator(np.random.PCG64(seed))
    tg = synth.draw_targets(rng, radar, c["M"], c["N"], c["targets"], c["snr_db"], 1.0,
                            c.get("draw_v", c["axes"][0]), c["axes"][1], (0.0, 0.0))
    echo = synth.make_echo(radar, c["M"], c["N"], tg, 1.0, rng)
    g = _grid(c, c["rows"])
    # the oracle's map, with its keystone (the costly step) computed once and
    # kept for the row test: KT.power is exactly this sequence of calls
    e = echo.astype(np.complex128)
    Np = OF.pad_length(g)
    SK = KT.keystone(OF.range_spectrum(e, Np), g, Np)
    F = KT.fine_matrix(g)
    rows = np.stack([KT.coarse_rows(e, g, k, SK, Np) for k in range(KT.lattice(g).n_coarse)])
    P = np.stack([np.abs(y.T @ F) ** 2 for y in rows])
    return dict(spec=c, grid=g, echo=echo, plan=_plan(c, c["rows"]),
                echo_dev=torch.from_numpy(echo).cuda(), P=P, rows_ref=rows)


@pytest.fixture(scope="module", params=list(KT_CASES))
def kcase(request):
    c = _make(request.param)
    c["name"] = request.param
    return c


def test_kt_lattice_matches_oracle(kcase):
    p, g = kcase["plan"], kcase["grid"]
    lat = KT.lattice(g)
    assert (p.kt_q_lo, p.kt_folds) == (lat.q_lo, lat.n_a)
    assert p.n_coarse == lat.n_coarse and p.n_fine == g.M * g.R
    assert p.fd_pad == OF.pad_length(g)
    assert p.K == tuple(g.K) and p.i_lo == tuple(g.i_lo)


def test_kt_coarse_rows_match_oracle(kcase):
    y = kcase["plan"].mgift(kcase["echo_dev"]).cpu().numpy()
    ref = kcase["rows_ref"]
    err = np.abs(y - ref).max() / np.abs(ref).max()
    assert err <= TOL, f"{kcase['name']}: {err:.3e}"


def test_kt_full_map_matches_oracle(kcase):
    P = kcase["plan"].search_full(kcase["echo_dev"], "f32fft", 1).cpu().numpy()
    ref = kcase["P"]
    err = np.abs(P.astype(np.float64) - ref).max() / ref.max()
    assert err <= TOL, f"{kcase['name']}: {err:.3e}"


def test_kt_reduced_map_matches_oracle(kcase):
    pm, af = kcase["plan"].search(kcase["echo_dev"], "f32fft", 1)
    near_tie_check(pm.cpu().numpy(), af.cpu().numpy(), kcase["P"], TOL)


@pytest.mark.parametrize("Np", [4096, 8192, 16384])
def test_kt_rows_every_large_transform_length(Np):
    """The compensation + IFFT kernel at N' = 4096, 8192 and 16384 (radix
    plans 16/16/16, 32/16/16 and 64/16/16) against the oracle's rows."""
    c = dict(KT_CASES["m64"])
    c["N"] = Np * 3 // 4
    g = _grid(c)
    assert OF.pad_length(g) == Np
    rng = np.random.default_rng(Np)
    e = (rng.standard_normal((c["M"], c["N"])) +
         1j * rng.standard_normal((c["M"], c["N"]))).astype(np.complex64)
    p = _plan(c)
    assert p.fd_pad == Np
    y = p.mgift(torch.from_numpy(e).cuda()).cpu().numpy()
    ee = e.astype(np.complex128)
    SK = KT.keystone(OF.range_spectrum(ee, Np), g, Np)
    ref = np.stack([KT.coarse_rows(ee, g, k, SK, Np) for k in range(KT.lattice(g).n_coarse)])
    assert y.shape == ref.shape
    assert np.abs(y - ref).max() <= TOL * np.abs(ref).max()


def test_kt_cell_list_matches_range(kcase):
    p = kcase["plan"]
    cells = torch.tensor([p.n_coarse - 1, 0, p.n_coarse // 2], dtype=torch.int64)
    pm, af = p.search(kcase["echo_dev"], "f32fft", 1, cells=cells)
    pm_all, af_all = p.search(kcase["echo_dev"], "f32fft", 1)
    idx = cells.cuda()
    assert torch.equal(pm, pm_all[idx]) and torch.equal(af, af_all[idx])


def test_kt_detect_parameters_match_oracle(kcase):
    p, g = kcase["plan"], kcase["grid"]
    pm, af = p.search(kcase["echo_dev"], "f32fft", 1)
    _, _, best = p.detect(pm, af, 1e-300, cap=0)
    k, row, f = int(best["coarse"]), int(best["row"]) - g.n_begin, int(best["fine"])
    assert np.isclose(kcase["P"][k, row, f], kcase["P"].max(), rtol=2 * TOL)
    r0, v, a = KT.peak_params(g, k, row, f)
    assert (best["r0"], best["v"], best["a"]) == pytest.approx((r0, v, a), rel=1e-12,
                                                              abs=1e-9)


@pytest.mark.parametrize("q,i1p,i2,r0b", [(2, -20, 5, 60.0), (1, 31, 11, 40.5),
                                          (-2, -30, -7, 70.0)])
def test_kt_folded_target_detected_at_its_cell(q, i1p, i2, r0b):
    """Noiseless on-lattice target with velocity q V_a + i1' dv: the GPU
    detection lands on its (q, i1', i2) cell with |Y| >= 0.85 M A."""
    c = KT_CASES["m64"]
    p, g = _plan(c), _grid(c)
    M = c["M"]
    radar = synth.RadarParams(c["fc"], c["fs"], c["prf"])
    tg = synth.Target(r0=r0b * g.dr, v=(q * M + i1p) * g.steps[0], a=i2 * g.steps[1], j=0.0,
                      amp=1.0, phase=0.2)
    echo = synth.make_echo(radar, M, c["N"], [tg], 0.0)
    pm, af = p.search(torch.from_numpy(echo).cuda(), "f32fft", 1)
    _, _, best = p.detect(pm, af, 1e-300, cap=0)
    qq, i2c = KT.coarse_params(g, KT.lattice(g), int(best["coarse"]))
    f = int(best["fine"])
    assert (qq, f % M - M // 2, i2c + f // M - g.R // 2) == (q, i1p, i2)
    assert abs(int(best["row"]) - r0b) <= 0.5
    assert np.sqrt(float(best["power"])) >= 0.85 * M
    assert best["v"] == pytest.approx((q * M + i1p) * g.steps[0])


def test_kt_m1024_sampled_rows():
    """M = 1024 (the benchmark's pulse count and keystone tiling), N = 256,
    the benchmark's search axes: three cells, sampled rows, FP32 tolerance."""
    cfg = synth.CONFIGS[3]
    r = cfg["radar"]
    c = dict(fc=r.fc, fs=r.fs, prf=r.prf, M=1024, N=256, axes=list(cfg["axes"]))
    p, g = _plan(c), _grid(c)
    rng = np.random.Generator(np.random.PCG64(9))
    tg = synth.draw_targets(rng, r, 1024, 256, 2, -10.0, 1.0, cfg["axes"][0], cfg["axes"][1],
                            (0.0, 0.0))
    echo = synth.make_echo(r, 1024, 256, tg, 1.0, rng)
    cells = [0, p.n_coarse // 2 + 3, p.n_coarse - 1]
    pm, af = p.search(torch.from_numpy(echo).cuda(), "f32fft", 1,
                      cells=torch.tensor(cells, dtype=torch.int64))
    pm = pm.cpu().numpy()
    e = echo.astype(np.complex128)
    Np = OF.pad_length(g)
    SK = KT.keystone(OF.range_spectrum(e, Np), g, Np)
    F = KT.fine_matrix(g)
    rows = np.random.default_rng(4).choice(g.rows, 16, replace=False)
    P = [np.abs(KT.coarse_rows(e, g, k, SK, Np)[:, rows].T @ F) ** 2 for k in cells]
    scale = max(float(x.max()) for x in P)
    for i in range(len(cells)):
        err = np.abs(pm[i, rows] - P[i].max(axis=1)).max() / scale
        assert err <= TOL, (cells[i], err)


@pytest.fixture(scope="module")
def full3():
    """The benchmark workload: M = 1024, N = 4096 (N' = 8192), v in
    [-600, 600] m/s, a in [-50, 50] m/s^2."""
    from paper_2403_06788_amd.plan import Plan
    cfg = synth.CONFIGS[3]
    r = cfg["radar"]
    p = Plan(r.fc, r.fs, r.prf, cfg["M"], cfg["N"], 2, cfg["axes"], mgift="kt")
    g = make_grid(Radar(r.fc, r.fs, r.prf), cfg["M"], cfg["N"], 2,
                  [Axis(*a) for a in cfg["axes"]])
    return dict(plan=p, grid=g, cfg=cfg)


def test_kt_fullsize_linear(full3):
    """y(a + 2j b) = y(a) + 2j y(b) on the compensated rows of two cells."""
    p, cfg = full3["plan"], full3["cfg"]
    assert p.fd_pad == 8192
    rng = np.random.default_rng(31)
    shape = (cfg["M"], cfg["N"])
    a, b = (torch.from_numpy((rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
                             .astype(np.complex64)).cuda() for _ in range(2))
    for k in (5, p.n_coarse - 2):
        ya, yb = p.mgift(a, k, 1), p.mgift(b, k, 1)
        yab = p.mgift(a + 2j * b, k, 1)
        err = (yab - (ya + 2j * yb)).abs().max().item() / yab.abs().max().item()
        assert err <= 1e-5, (k, err)


@pytest.mark.parametrize("q,i1p,i2,r0b", [(7, 300, -20, 1200.0), (-8, -400, 33, 3001.0)])
def test_kt_fullsize_folded_target(full3, q, i1p, i2, r0b):
    """A noiseless folded target in the full-size search (all cells, the
    benchmark's batching) peaks at its own cell with |Y| >= 0.85 M A."""
    p, g, cfg = full3["plan"], full3["grid"], full3["cfg"]
    M = cfg["M"]
    tg = synth.Target(r0=r0b * g.dr, v=(q * M + i1p) * g.steps[0], a=i2 * g.steps[1], j=0.0,
                      amp=1.0, phase=-0.4)
    echo = synth.make_echo(cfg["radar"], M, cfg["N"], [tg], 0.0)
    pm, af = p.search(torch.from_numpy(echo).cuda(), "f32fft", 1)
    _, _, best = p.detect(pm, af, 1e-300, cap=0)
    qq, i2c = KT.coarse_params(g, KT.lattice(g), int(best["coarse"]))
    f = int(best["fine"])
    assert (qq, f % M - M // 2, i2c + f // M - g.R // 2) == (q, i1p, i2)
    assert int(best["row"]) == round(r0b)
    assert np.sqrt(float(best["power"])) >= 0.85 * M


def test_kt_rejects_what_it_does_not_support():
    from paper_2403_06788_amd._lib import DsgrftError
    from paper_2403_06788_amd.plan import Plan
    c = KT_CASES["m64"]
    with pytest.raises(DsgrftError, match="unsupported"):
        Plan(c["fc"], c["fs"], c["prf"], 64, 128, 1, c["axes"][:1], mgift="kt")
    with pytest.raises(DsgrftError, match="unsupported"):
        Plan(c["fc"], c["fs"], c["prf"], 96, 128, 2, c["axes"], mgift="kt")
    p = _plan(c)
    e = torch.zeros((64, 128), dtype=torch.complex64, device="cuda")
    for form in ("f32", "f16", "bf16", "fp8", "f16_3m", "f16_sym", "bf16_sym"):
        with pytest.raises(DsgrftError, match="unsupported"):
            p.search(e, form, 1)
    with pytest.raises(DsgrftError, match="invalid"):
        p.search(e, "f32fft", 2)
    with pytest.raises(DsgrftError, match="unsupported"):
        p.grft(e)
    with pytest.raises(DsgrftError, match="unsupported"):
        p.coarse_tables()
    th = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(DsgrftError, match="unsupported"):
        p.adjoint_forward(e, th)


def test_kt_config3_sampled_rows_golden(full3):
    """The benchmark workload at full size (its plan and batching) against the
    oracle's reduced map on 24 sampled rows of three coarse cells, stored in
    tests/golden/kt_config3_rows.json by tests/golden/make_kt_config3.py (which
    calls only the oracle): FP32 tolerance, fine index exact where the
    oracle's top-two gap exceeds twice the tolerance."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "kt_config3_rows.json")
    with open(path) as f:
        d = json.load(f)
    p = full3["plan"]
    assert p.fd_pad == d["pad_length"] and p.n_coarse == d["n_coarse"]
    echo = torch.from_numpy(synth.config_case(3)["echo"]).cuda()
    cells = [int(k) for k in d["cells"]]
    pm, af = p.search(echo, "f32fft", 1, cells=torch.tensor(cells, dtype=torch.int64))
    pm, af = pm.cpu().numpy(), af.cpu().numpy()
    rows = np.array(d["rows"])
    scale = max(max(v["pmax"]) for v in d["cells"].values())
    checked = 0
    for i, k in enumerate(cells):
        ref = d["cells"][str(k)]
        err = np.abs(pm[i, rows] - np.array(ref["pmax"])).max() / scale
        assert err <= TOL, (k, err)
        for j, r in enumerate(rows):
            if ref["pmax"][j] - ref["second"][j] > 2 * TOL * scale:
                assert af[i, r] == ref["argf"][j], (k, r)
                checked += 1
    assert checked > 0
