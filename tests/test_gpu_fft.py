"""FFT form of the fine search (fine velocities by a slow-time FFT, Alg. 2),
through the C ABI, against the FP64 oracle (FP32 tolerance 1e-5 of the peak
power) and against the GEMM forms."""
import numpy as np
import pytest
import torch

import synth
from cases import near_tie_check
from oracle import transforms as OT
from oracle.grid import Axis, Radar, make_grid

pytestmark = pytest.mark.gpu

# power-of-two M: P = 1 with M < R (aliased bins), P = 2 (two factorings of M),
# P = 2 with a row window (wavefront-per-row kernel, 8 pulses per lane), P = 2
# at M = 2048 (32 pulses per lane, two wavefronts per workgroup), P = 3.  The
# wavefront kernel forms only the outer eighths of each transform when the R
# wanted fine velocities fit there (R/2 <= M/8: the M >= 512 cases above);
# p2m512wide (R = 150 > M/4) takes every bin of the last pass.
FFT_CASES = {
    "p1alias": dict(fc=1.0e9, fs=1.0e7, prf=500.0, M=64, N=256, order=1,
                    axes=[(-150.0, 150.0)], targets=1, snr_db=0.0, rows=None),
    "p2m128": dict(fc=1.2e8, fs=1.0e7, prf=500.0, M=128, N=300, order=2,
                   axes=[(-100.0, 100.0), (-400.0, 400.0)], targets=3, snr_db=-3.0, rows=None),
    "p2m512rows": dict(fc=2.4e8, fs=1.0e7, prf=1000.0, M=512, N=320, order=2,
                       axes=[(-30.0, 30.0), (-60.0, 60.0)], targets=2, snr_db=-10.0,
                       rows=(40, 300)),
    "p2m2048": dict(fc=1.2e8, fs=1.0e7, prf=1000.0, M=2048, N=96, order=2,
                    axes=[(-20.0, 20.0), (-10.0, 10.0)], targets=2, snr_db=-10.0, rows=None),
    "p2m512wide": dict(fc=1.5e9, fs=1.0e7, prf=1000.0, M=512, N=64, order=2,
                       axes=[(-10.0, 10.0), (-5.0, 5.0)], targets=2, snr_db=-10.0, rows=None),
    "p3m64": dict(fc=6.0e7, fs=1.0e7, prf=500.0, M=64, N=200, order=3,
                  axes=[(-150.0, 150.0), (-600.0, 600.0), (-9000.0, 9000.0)],
                  targets=2, snr_db=-3.0, rows=None),
}


def _make(name, seed=321):
    c = FFT_CASES[name]
    radar = synth.RadarParams(c["fc"], c["fs"], c["prf"])
    rng = np.random.Generator(np.random.PCG64(seed))
    axes = c["axes"] + [(0.0, 0.0)] * (3 - len(c["axes"]))
    tg = synth.draw_targets(rng, radar, c["M"], c["N"], c["targets"], c["snr_db"], 1.0,
                            axes[0], axes[1], axes[2])
    echo = synth.make_echo(radar, c["M"], c["N"], tg, 1.0, rng)
    rows = c["rows"]
    g = make_grid(Radar(c["fc"], c["fs"], c["prf"]), c["M"], c["N"], c["order"],
                  [Axis(*a) for a in c["axes"]], *(rows if rows else (0, None)))
    from paper_2403_06788_amd.plan import Plan
    p = Plan(c["fc"], c["fs"], c["prf"], c["M"], c["N"], c["order"], c["axes"], rows=rows)
    return dict(grid=g, echo=echo, plan=p, echo_dev=torch.from_numpy(echo).cuda(),
                P_ds=OT.dsgrft_power(echo.astype(np.complex128), g))


@pytest.fixture(scope="module", params=list(FFT_CASES))
def fcase(request):
    c = _make(request.param)
    c["name"] = request.param
    return c


def test_fft_full_map_matches_oracle(fcase):
    p = fcase["plan"]
    P = p.search_full(fcase["echo_dev"], "f32fft", 1).cpu().numpy().astype(np.float64)
    ref = fcase["P_ds"]
    err = np.abs(P - ref).max() / ref.max()
    assert err <= 1e-5, f"{fcase['name']}: {err:.3e}"


def test_fft_reduced_map_and_argmax(fcase):
    p = fcase["plan"]
    pm, af = p.search(fcase["echo_dev"], "f32fft", 1)
    near_tie_check(pm.cpu().numpy(), af.cpu().numpy(), fcase["P_ds"], 1e-5)
    P = p.search_full(fcase["echo_dev"], "f32fft", 1).cpu().numpy()
    assert np.array_equal(pm.cpu().numpy(), P.max(axis=-1))
    assert np.array_equal(af.cpu().numpy(), P.argmax(axis=-1))


def test_fft_matches_gemm_forms(fcase):
    p = fcase["plan"]
    a = p.search_full(fcase["echo_dev"], "f32fft", 1).cpu().numpy().astype(np.float64)
    b = p.search_full(fcase["echo_dev"], "f32", 1).cpu().numpy().astype(np.float64)
    assert np.abs(a - b).max() <= 2e-5 * b.max()


def test_fft_aliased_bins_are_identical():
    """M = 64 < R = 100: fine velocities f1 and f1 + 64 share one FFT bin."""
    c = _make("p1alias")
    P = c["plan"].search_full(c["echo_dev"], "f32fft", 1).cpu().numpy()
    assert np.array_equal(P[..., 0:36], P[..., 64:100])


def test_fft_form_rejects_unsupported_lengths():
    from paper_2403_06788_amd._lib import DsgrftError
    from paper_2403_06788_amd.plan import Plan
    p = Plan(1.2e8, 1.0e7, 500.0, 100, 300, 2, [(-100.0, 100.0), (-400.0, 400.0)])
    e = torch.zeros((100, 300), dtype=torch.complex64, device="cuda")
    with pytest.raises(DsgrftError, match="unsupported"):
        p.search(e, "f32fft", 1)
    with pytest.raises(DsgrftError, match="invalid"):
        p.search(e, "f32fft", 3)
