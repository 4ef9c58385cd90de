"""The search's two-stream pipeline (producer stream for tables, coarse
compensation and gathers; fine search on the caller's stream, two gathered
slots): one gathered unit per batch, so every slot is reused many times, must
give bit-identical maps to the default batching, for each coarse-stage mode
and for order 3 (several gathered units per coarse cell)."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

R1 = synth.CONFIGS[1]["radar"]


def _plans(mgift, order=2, M=128, N=300, axes=((-1500.0, 1500.0), (-400.0, 400.0))):
    from paper_2403_06788_amd.plan import Plan
    fc, fs, prf = 1.2e8, 1.0e7, 500.0
    kw = dict(mgift=mgift)
    big = Plan(fc, fs, prf, M, N, order, axes[:order], **kw)
    one = Plan(fc, fs, prf, M, N, order, axes[:order], batch=1, **kw)
    radar = synth.RadarParams(fc, fs, prf)
    rng = np.random.Generator(np.random.PCG64(41))
    ax = list(axes[:order]) + [(0.0, 0.0)] * (3 - order)
    tg = synth.draw_targets(rng, radar, M, N, 2, -5.0, 1.0, *ax)
    echo = torch.from_numpy(synth.make_echo(radar, M, N, tg, 1.0, rng)).cuda()
    return big, one, echo


@pytest.mark.parametrize("mgift,form,split", [("td", "f16", 1), ("td", "bf16", 3), ("td", "f16_3m", 1),
                                              ("td", "f16_sym", 1), ("td", "bf16_sym", 3),
                                              ("td", "bf16_sym", 2), ("td", "fp8_sym", 3),
                                              ("fd", "f16", 1),
                                              ("kt", "f32fft", 1)])
def test_single_unit_batches_match_default_batching(mgift, form, split):
    big, one, echo = _plans(mgift)
    assert one.n_coarse >= 6
    pa, fa = big.search(echo, form, split)
    pb, fb = one.search(echo, form, split)
    assert torch.equal(pa, pb) and torch.equal(fa, fb)
    # again, with the same plans (slots left from the previous call)
    pc, fc_ = one.search(echo, form, split)
    assert torch.equal(pa, pc) and torch.equal(fa, fc_)


def test_order3_units_across_batches():
    big, one, echo = _plans("td", order=3, M=64, N=200,
                            axes=((-150.0, 150.0), (-600.0, 600.0), (-9000.0, 9000.0)))
    cells = torch.tensor([0, big.n_coarse - 1, big.n_coarse // 2], dtype=torch.int64)
    pa, fa = big.search(echo, "f16", 1, cells=cells)
    pb, fb = one.search(echo, "f16", 1, cells=cells)
    assert torch.equal(pa, pb) and torch.equal(fa, fb)


def test_two_plans_on_two_streams():
    """A plan is used by one stream at a time, but separate plans may run
    concurrently: two plans searching on two streams at once give the
    results of the same searches run one after the other, bit for bit."""
    big, one, echo = _plans("td")
    ref_a = big.search(echo, "f16_sym", 1)
    ref_b = one.search(echo, "bf16_sym", 3)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.current_stream().synchronize()
    outs = []
    for _ in range(3):
        with torch.cuda.stream(s1):
            a = big.search(echo, "f16_sym", 1)
        with torch.cuda.stream(s2):
            b = one.search(echo, "bf16_sym", 3)
        outs.append((a, b))
    torch.cuda.synchronize()
    for a, b in outs:
        assert torch.equal(a[0], ref_a[0]) and torch.equal(a[1], ref_a[1])
        assert torch.equal(b[0], ref_b[0]) and torch.equal(b[1], ref_b[1])
