"""dsgrft_noise_power_noalloc (the entry point that allocates nothing; its
partial sums live in a static device array) against dsgrft_noise_power of a
plan on the same echo: identical doubles (same kernels and summation order),
on two calls in a row, the second with a smaller echo."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _noalloc(L, echo):
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    M, N = echo.shape
    st = L.dsgrft_noise_power_noalloc(C.c_void_p(echo.data_ptr()), M, N,
                                      C.c_void_p(out.data_ptr()),
                                      C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, st
    return out


def test_noalloc_noise_power_matches_plan_entry_point():
    from paper_2403_06788_amd import _lib
    from paper_2403_06788_amd.plan import Plan
    L = _lib.lib()
    big = synth.config_case(3)["echo"]                  # 1024 x 4096: 64 partial sums
    rng = np.random.default_rng(5)
    small = (rng.standard_normal((70, 300)) * 3.0 + 1j * rng.standard_normal((70, 300))
             ).astype(np.complex64)                     # 21000 samples: one partial sum
    results = []
    for e in (big, small):
        M, N = e.shape
        print(f"noalloc noise power on {M} x {N}", flush=True)
        dev = torch.from_numpy(e).cuda()
        got = _noalloc(L, dev)
        plan = Plan(1.0e9, 1.0e7, 500.0, M, N, 1, [(0.0, 0.0)])
        want = plan.noise_power(dev, as_tensor=True)
        torch.cuda.synchronize()
        assert got.item() == want.item()
        assert got.item() == pytest.approx(np.mean(np.abs(e.astype(np.complex128)) ** 2),
                                           rel=1e-12)
        results.append(got.item())
        plan.close()
    assert results[0] != results[1]
