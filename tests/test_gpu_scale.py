"""Echo scale: every form's reduced map and argmax scale exactly with the
echo.  Multiplying the echo by 2^k multiplies |Y|^2 by 2^(2k) in exact
arithmetic; the fp16 forms store the gathered rows with one power-of-two
shift per echo (largest component in [2^9, 2^10)), the 8-bit form with one
per (unit, row), and bf16/FP32 keep FP32's exponent range, so the device
results must be bit-identical after the 2^(2k) factor.  Without the shift an
echo of 2^20 overflows fp16 (65504) and one of 2^-20 underflows it."""
import numpy as np
import pytest
import torch

from cases import make_case, near_tie_check, plan_for
from oracle import transforms as OT

pytestmark = pytest.mark.gpu

FORMS = [("f32", 1), ("f16", 1), ("f16", 3), ("f16_3m", 1), ("f16_sym", 1), ("bf16", 3),
         ("bf16_sym", 3), ("fp8", 3), ("fp8_sym", 3)]


@pytest.fixture(scope="module")
def case():
    c = make_case("p2")
    c["plan"] = plan_for(c)
    c["P_ds"] = OT.dsgrft_power(c["echo"].astype(np.complex128), c["grid"])
    return c


@pytest.mark.parametrize("form,split", FORMS)
@pytest.mark.parametrize("k", [20, -20, 40, -40])
def test_scaled_echo_scales_the_map_exactly(case, form, split, k):
    p = case["plan"]
    e = case["echo"]
    pm0, af0 = p.search(torch.from_numpy(e).cuda(), form, split)
    es = (e.astype(np.complex128) * 2.0 ** k).astype(np.complex64)
    assert np.array_equal(es.astype(np.complex128) * 2.0 ** -k, e.astype(np.complex128))
    pm1, af1 = p.search(torch.from_numpy(es).cuda(), form, split)
    pm0, pm1 = pm0.cpu().numpy().astype(np.float64), pm1.cpu().numpy().astype(np.float64)
    assert np.isfinite(pm1).all()
    assert np.array_equal(pm1, pm0 * 2.0 ** (2 * k)), (form, split, k)
    assert torch.equal(af0, af1)


@pytest.mark.parametrize("form,split,tol", [("f16", 1, 1e-3), ("f16_3m", 1, 1e-3),
                                            ("f16_sym", 1, 1e-3)])
def test_large_echo_fp16_forms_match_oracle(case, form, split, tol):
    """An echo whose components reach ~3e5 (beyond fp16's 65504) still gives
    the oracle's map within the fp16 tolerance."""
    p = case["plan"]
    s = 2.0 ** 16
    es = (case["echo"].astype(np.complex128) * s).astype(np.complex64)
    assert np.abs(es.real).max() > 65504.0
    pm, af = p.search(torch.from_numpy(es).cuda(), form, split)
    near_tie_check(pm.cpu().numpy().astype(np.float64) / s ** 2, af.cpu().numpy(),
                   case["P_ds"], tol)
