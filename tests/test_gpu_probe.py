"""The matrix-core probe used for the attainable roofline: a plausible rate
(below the published peak) and shader clock, for fp16, bf16 and e4m3."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("form,peak", [("f16", 2500.0), ("bf16", 2500.0), ("fp8", 5000.0)])
def test_mfma_probe_rate_and_clock(form, peak):
    from paper_2403_06788_amd.plan import Plan
    tf, ghz = Plan.mfma_probe(form, 20.0)
    print(f"{form}: {tf:.1f} TFLOP/s at {ghz:.3f} GHz", flush=True)
    assert 0.2 * peak < tf <= 1.02 * peak
    assert 0.5 < ghz < 3.0
    # the rate follows the clock: at most the published peak scaled by it
    assert tf <= peak * ghz / 2.4 * 1.05


def test_mfma_probe_rejects_other_forms():
    from paper_2403_06788_amd._lib import DsgrftError
    from paper_2403_06788_amd.plan import Plan
    with pytest.raises(DsgrftError, match="invalid"):
        Plan.mfma_probe("f32", 10.0)
