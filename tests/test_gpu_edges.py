"""Degenerate inputs through the C ABI: an all-zero echo (every fine cell
ties), one pulse, one range bin, one coarse cell, and a single impulse,
against the FP64 oracle."""
import numpy as np
import pytest
import torch

from cases import near_tie_check
from oracle import transforms as OT
from oracle.grid import Axis, Radar, make_grid

pytestmark = pytest.mark.gpu

FORMS = [("f32", 1, 1e-5), ("f16", 1, 1e-3), ("f16_3m", 1, 1e-3), ("f16_sym", 1, 1e-3), ("bf16", 3, 1e-4),
         ("fp8", 3, 1e-2), ("bf16_glo", 2, 1e-2), ("bf16_sym", 3, 1e-4), ("fp8_sym", 3, 1e-2)]

# (fc, fs, prf, M, N, order, axes): one pulse and one bin; two pulses; a
# single coarse cell of order 2 (zero-width acceleration axis) over 5 bins
TINY = {
    "m1n1": (1.0e9, 1.0e7, 500.0, 1, 1, 1, [(0.0, 0.0)]),
    "m2n3": (1.0e9, 1.0e7, 500.0, 2, 3, 1, [(-10.0, 10.0)]),
    "m17n5p2": (1.0e9, 1.0e7, 500.0, 17, 5, 2, [(-30.0, 30.0), (0.0, 0.0)]),
}


def _plan(spec):
    from paper_2403_06788_amd.plan import Plan
    fc, fs, prf, M, N, order, axes = spec
    grid = make_grid(Radar(fc, fs, prf), M, N, order, [Axis(*a) for a in axes])
    return Plan(fc, fs, prf, M, N, order, axes), grid


@pytest.mark.parametrize("form,split,tol", FORMS)
def test_zero_echo_gives_zero_map_and_first_fine_cell(form, split, tol):
    spec = (1.2e8, 1.0e7, 500.0, 100, 300, 2, [(-100.0, 100.0), (-400.0, 400.0)])
    p, g = _plan(spec)
    e = torch.zeros((100, 300), dtype=torch.complex64, device="cuda")
    pm, af = p.search(e, form, split)
    assert torch.count_nonzero(pm).item() == 0
    assert torch.count_nonzero(af).item() == 0      # all cells tie: smallest index
    peaks, cnt, best = p.detect(pm, af, 0.5, 0.0)     # gamma^2 = 0
    assert cnt == 0 and int(best["coarse"]) == 0 and int(best["row"]) == 0
    _, cnt_c, _ = p.detect_cfar(pm, af, 1, 4, 0.0)
    assert cnt_c == 0
    p.close()


@pytest.mark.parametrize("name", list(TINY))
@pytest.mark.parametrize("form,split,tol", FORMS)
def test_tiny_plans_match_oracle(name, form, split, tol):
    spec = TINY[name]
    p, g = _plan(spec)
    M, N = spec[3], spec[4]
    rng = np.random.default_rng(9)
    echo = (rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))).astype(np.complex64)
    ref = OT.dsgrft_power(echo.astype(np.complex128), g)
    P = p.search_full(torch.from_numpy(echo).cuda(), form, split).cpu().numpy()
    assert P.shape == ref.shape
    assert np.abs(P - ref).max() <= tol * ref.max()
    pm, af = p.search(torch.from_numpy(echo).cuda(), form, split)
    near_tie_check(pm.cpu().numpy(), af.cpu().numpy(), ref, tol)
    p.close()


def test_single_impulse_every_form():
    """One sample s[m0][n0] = A: |Y|^2 = |A|^2 at every fine cell of the
    coarse cells whose walk puts pulse m0 on bin n0 - row."""
    spec = (1.2e8, 1.0e7, 500.0, 100, 300, 2, [(-100.0, 100.0), (-400.0, 400.0)])
    p, g = _plan(spec)
    echo = np.zeros((100, 300), dtype=np.complex64)
    echo[37, 150] = 0.6 - 0.8j
    ref = OT.dsgrft_power(echo.astype(np.complex128), g)
    a2 = abs(complex(echo[37, 150])) ** 2
    assert np.all((ref == 0.0) | (np.abs(ref - a2) <= 1e-12)) and ref.max() > 0.0
    # one product term, u the unit roundoff of the operand format: rounding
    # each operand's components moves |Y| by at most u|Y| per operand, so
    # |dP| <= 4u P (f16 u = 2^-11).  Three products: Im also carries
    # (Gr + Gi)(Fr + Fi)(d1 + d2) from rounding the two sums, at most 4u|Y|
    # more, so |dY| <= 6u|Y| and |dP| <= 12u P.  bf16 x3 ~ u^2; bf16 with
    # the rows split keeps the table's rounding only (2u, u = 2^-8); e4m3 x3
    # leaves out Fl Gl and keeps ~2^-8 per operand.  The conjugate-pair form
    # takes the four-product form's operands and products (4u).
    bound = {"f32": 1e-6, "f16": 4 * 2.0 ** -11, "f16_3m": 12 * 2.0 ** -11, "f16_sym": 4 * 2.0 ** -11,
             "bf16_glo": 4 * 2.0 ** -8,
             "bf16": 1e-4, "bf16_sym": 1e-4, "fp8": 8 * 2.0 ** -8, "fp8_sym": 8 * 2.0 ** -8}
    for form, split, _ in FORMS:
        P = p.search_full(torch.from_numpy(echo).cuda(), form, split).cpu().numpy()
        assert np.array_equal(P == 0.0, ref == 0.0), (form, split)
        assert np.abs(P - ref).max() <= bound[form] * a2, (form, split, np.abs(P - ref).max())
    p.close()
