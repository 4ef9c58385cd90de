"""Parity with the FP64 oracle on seeded random small plans: the DS-GRFT map
(GFT eq. (44) after the mGIFT and pre-DFM of eqs. (46)-(47)) reduced over each
cell's fine lattice (eq. (72)).  Order, R, PRF, pulse count, range bins, a row
window and the motion extents (one to three coarse cells per axis) are drawn
from a fixed seed, so the cases cover tile tails the hand-written cases do
not; every main form's reduced map and argmax are checked under the near-tie
rule at its tolerance (FP32 forms 1e-5, fp16 pairs 1e-3, bf16 pairs x3 1e-4,
e4m3 pairs x3 1e-2 as for the other 8-bit small cases).  The same plans with
the frequency-domain mGIFT (Alg. 1) are checked against oracle.fd, and those
of order 2 with a power-of-two pulse count as DS-KT-MFP (Alg. 4, Prop. 3, FFT
fine search) against oracle.ktmfp at 1e-5.  The LRT detections (eqs. (31),
(33), Alg. 3) of the time-domain plans are compared with the oracle's at
P_FA 1e-6 ... 1e-1 under the near-tie rule of the detection goldens, and on
the plans of order 1 and 2 the adjoint of the continuous objective (its value,
theta gradient and echo gradient at random off-grid candidates) with
oracle.adjoint; the single-scale TD-GRFT (eq. (13)) of every plan, full and
reduced map, at 1e-5; cell-averaging CFAR decisions bit for bit on the
device's reduced map with a random window; each form's full map within its
tolerance of the oracle, its reduced map exactly the max / first argmax of
that full map."""
import numpy as np
import pytest
import torch

import synth
from cases import near_tie_check
from oracle import adjoint as OA
from oracle import detect as OD
from oracle import fd as OF
from oracle import ktmfp as KT
from oracle import transforms as OT
from oracle.grid import Axis, Radar, make_grid

pytestmark = pytest.mark.gpu

FS = 1.0e7
MAX_WORK = 1.5e9  # coarse cells x rows x fine cells x pulses of one oracle map


def _draw(seed):
    """One plan: (spec, grid) with its oracle work below MAX_WORK."""
    rng = np.random.Generator(np.random.PCG64(seed))
    while True:
        order = int(rng.choice([1, 2, 2, 2, 3]))
        R = int(rng.choice([6, 11, 12, 24, 100] if order < 3 else [5, 6, 8]))
        fc = R * FS
        prf = float(rng.choice([500.0, 1000.0]))
        M = int(rng.choice([64, 72, 100, 128, 200, 256, 512, 512, 1024, 1024]))
        N = int(rng.integers(40, 321))
        rows = None
        if rng.random() < 0.4:
            a = int(rng.integers(0, N // 3))
            rows = (a, int(rng.integers(a + 1, N + 1)))
        radar = Radar(fc, FS, prf)
        g0 = make_grid(radar, M, N, order, [Axis(0.0, 0.0)] * order)
        axes = []
        for q in range(order):
            c = R * g0.steps[q] * float(rng.uniform(0.3, 2.6))
            axes.append((-c, c * float(rng.uniform(0.5, 1.0))))
        g = make_grid(radar, M, N, order, [Axis(*a) for a in axes],
                      *(rows if rows else (0, None)))
        work = float(g.n_coarse) * g.rows * g.n_fine * M
        if work <= MAX_WORK:
            spec = dict(fc=fc, prf=prf, M=M, N=N, order=order, axes=axes, rows=rows)
            return spec, g


SEEDS = list(range(2024, 2036))

# (form, split, tolerance); the FFT form needs a power-of-two pulse count
FORMS = [("f32", 1, 1e-5), ("f16_sym", 1, 1e-3), ("bf16_sym", 3, 1e-4),
         ("fp8_sym", 3, 1e-2), ("f32fft", 1, 1e-5)]


def _case(seed, mgift):
    spec, g = _draw(seed)
    print(f"seed {seed} ({mgift}): {spec}", flush=True)
    radar = synth.RadarParams(spec["fc"], FS, spec["prf"])
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    axes = spec["axes"] + [(0.0, 0.0)] * (3 - spec["order"])
    tg = synth.draw_targets(rng, radar, spec["M"], spec["N"], 2, -3.0, 1.0,
                            axes[0], axes[1], axes[2])
    echo = synth.make_echo(radar, spec["M"], spec["N"], tg, 1.0, rng)
    from paper_2403_06788_amd.plan import Plan
    p = Plan(spec["fc"], FS, spec["prf"], spec["M"], spec["N"], spec["order"], spec["axes"],
             rows=spec["rows"], mgift=mgift)
    if mgift != "kt":
        assert (p.n_coarse, p.rows, p.n_fine) == (g.n_coarse, g.rows, g.n_fine)
    if mgift == "td":
        P = OT.dsgrft_power(echo.astype(np.complex128), g)
    elif mgift == "fd":
        P = OF.dsgrft_fd_power(echo, g)
    else:
        P = KT.power(echo, g)
    return dict(spec=spec, plan=p, grid=g, echo=echo, echo_dev=torch.from_numpy(echo).cuda(),
                P=P)


@pytest.fixture(scope="module", params=SEEDS)
def rcase(request):
    return _case(request.param, "td")


@pytest.fixture(scope="module", params=SEEDS)
def rcase_fd(request):
    return _case(request.param, "fd")


# DS-KT-MFP takes order 2 and, for its FFT fine search, a power-of-two M
KT_SEEDS = [s for s in SEEDS
            if _draw(s)[0]["order"] == 2 and (_draw(s)[0]["M"] & (_draw(s)[0]["M"] - 1)) == 0]


@pytest.fixture(scope="module", params=KT_SEEDS)
def rcase_kt(request):
    return _case(request.param, "kt")


@pytest.mark.parametrize("form,split,tol", FORMS)
def test_random_plan_reduced_map(rcase, form, split, tol):
    M = rcase["spec"]["M"]
    if form == "f32fft" and (M & (M - 1)) != 0:
        pytest.skip("the FFT form takes a power-of-two pulse count")
    pm, af = rcase["plan"].search(rcase["echo_dev"], form, split)
    err, _ = near_tie_check(pm.cpu().numpy(), af.cpu().numpy(), rcase["P"], tol)
    print(f"{form} x{split}: {err:.3e}", flush=True)


@pytest.mark.parametrize("form,split,tol", FORMS)
def test_random_plan_reduced_map_fd(rcase_fd, form, split, tol):
    """The same plans with the frequency-domain mGIFT against oracle.fd."""
    test_random_plan_reduced_map(rcase_fd, form, split, tol)


def test_random_plan_reduced_map_ktmfp(rcase_kt):
    """The order-2, power-of-two-M plans as DS-KT-MFP against oracle.ktmfp."""
    pm, af = rcase_kt["plan"].search(rcase_kt["echo_dev"], "f32fft", 1)
    assert pm.shape[0] == rcase_kt["P"].shape[0]
    err, _ = near_tie_check(pm.cpu().numpy(), af.cpu().numpy(), rcase_kt["P"], 1e-5)
    print(f"DS-KT-MFP: {err:.3e}", flush=True)


@pytest.mark.parametrize("form,split,tol", [("f32", 1, 1e-5), ("f16_sym", 1, 1e-3)])
def test_random_plan_detections(rcase, form, split, tol):
    """Detection list, global maximum and FP64 peak parameters against the
    oracle's full map (every reduced entry with its near-tie fine cells).  A
    detection's row is the absolute range bin n0 (the window start plus the
    map row)."""
    from test_gpu_detect_golden import _compare
    P = rcase["P"]
    n0 = rcase["grid"].n_begin
    pm_ref, af_ref = P.max(axis=-1), P.argmax(axis=-1)
    ents = {}
    for k in range(P.shape[0]):
        for r in range(P.shape[1]):
            near = np.nonzero(P[k, r] >= 0.99 * pm_ref[k, r])[0]
            ents[(k, n0 + r)] = [k, n0 + r, int(af_ref[k, r]), float(pm_ref[k, r]),
                                 [[int(f), float(P[k, r, f])] for f in near
                                  if f != af_ref[k, r]]]
    order = sorted(ents.values(), key=lambda x: -x[3])
    top = [[x[0], x[1], x[2], x[3]] for x in order[:64]]
    pm, af = rcase["plan"].search(rcase["echo_dev"], form, split)
    _compare(rcase["plan"], rcase["grid"], pm, af, ents, top, float(P.max()),
             [1e-6, 1e-3, 1e-1], 1.0, tol)


def test_random_plan_adjoint(rcase):
    """J, dJ/dtheta and dJ/ds at eight random candidates inside the plan's
    extents against the FP64 oracle (tolerances of the adjoint tests)."""
    spec, g = rcase["spec"], rcase["grid"]
    if spec["order"] > 2:
        pytest.skip("the adjoint's candidates are (r0, v, a)")
    rng = np.random.default_rng(spec["N"])
    n = 8
    va = [spec["axes"][0], spec["axes"][1] if spec["order"] == 2 else (0.0, 0.0)]
    th = np.stack([rng.uniform(2, g.N - 3, n) * g.dr,
                   rng.uniform(*va[0], n), rng.uniform(*va[1], n)], axis=1)
    plan = rcase["plan"]
    J, saved = plan.adjoint_forward(rcase["echo_dev"], torch.from_numpy(th))
    gJ = np.linspace(0.5, 2.0, n)
    gt, ge = plan.adjoint_backward(rcase["echo_dev"], torch.from_numpy(th), saved,
                                   torch.from_numpy(gJ))
    J, gt, ge = J.cpu().numpy(), gt.cpu().numpy(), ge.cpu().numpy()
    for b in range(n):
        Jo, _, go, _ = OA.gradients(rcase["echo"], g, th[b])
        assert J[b] == pytest.approx(Jo, rel=1e-9, abs=1e-9 * (Jo + 1))
        np.testing.assert_allclose(gt[b], gJ[b] * go, rtol=1e-7,
                                   atol=1e-9 * np.abs(gJ[b] * go).max())
    _, _, ref = OA.batch(rcase["echo"], g, th, grad_J=gJ, want_echo_grad=True)
    assert np.abs(ge - ref).max() <= 1e-5 * np.abs(ref).max()


def test_random_plan_grft(rcase):
    """TD-GRFT full map and reduced map against the oracle's eq. (13)."""
    g = rcase["grid"]
    pm, af, P = rcase["plan"].grft(rcase["echo_dev"], full=True)
    ref = OT.grft_power(rcase["echo"].astype(np.complex128), g)
    P = P.cpu().numpy().astype(np.float64)
    assert np.abs(P - ref).max() / ref.max() <= 1e-5
    near_tie_check(pm.cpu().numpy(), af.cpu().numpy(), ref, 1e-5)


def test_random_plan_cfar(rcase):
    """CA-CFAR along range on the fp16-pair device map: the oracle's
    decisions on the same map, the listed powers and fine cells, and the
    global maximum; guard, training length and alpha drawn per plan."""
    g = rcase["grid"]
    rng = np.random.default_rng(rcase["spec"]["N"] + 1)
    guard, train = int(rng.integers(0, 4)), int(rng.integers(1, 24))
    alpha = float(rng.uniform(1.2, 4.0))
    pm, af = rcase["plan"].search(rcase["echo_dev"], "f16_sym", 1)
    pm_h, af_h = pm.cpu().numpy(), af.cpu().numpy()
    want = [(int(k), int(r)) for k, r in np.argwhere(OD.ca_cfar(pm_h, guard, train, alpha))]
    peaks, cnt, best = rcase["plan"].detect_cfar(pm, af, guard, train, alpha, cap=1 << 20)
    got = [(int(q["coarse"]), int(q["row"]) - g.n_begin) for q in peaks]
    assert cnt == len(want) and got == want, (guard, train, alpha)
    for q in peaks[:50]:
        k, r = int(q["coarse"]), int(q["row"]) - g.n_begin
        assert q["power"] == pm_h[k, r] and int(q["fine"]) == af_h[k, r]
    kb, rb = np.unravel_index(np.argmax(pm_h), pm_h.shape)
    assert (int(best["coarse"]), int(best["row"]) - g.n_begin) == (kb, rb)


@pytest.mark.parametrize("form,split,tol", FORMS)
def test_random_plan_full_map(rcase, form, split, tol):
    """Full |Y|^2 map of each form against the oracle, and the reduced map as
    its exact max and first argmax (both variants of a kernel round alike)."""
    M = rcase["spec"]["M"]
    if form == "f32fft" and (M & (M - 1)) != 0:
        pytest.skip("the FFT form takes a power-of-two pulse count")
    p = rcase["plan"]
    P = p.search_full(rcase["echo_dev"], form, split).cpu().numpy()
    ref = rcase["P"]
    assert np.abs(P.astype(np.float64) - ref).max() <= tol * ref.max()
    pm, af = p.search(rcase["echo_dev"], form, split)
    assert np.array_equal(pm.cpu().numpy(), P.max(axis=-1))
    assert np.array_equal(af.cpu().numpy(), P.argmax(axis=-1))
