"""Adjoint kernels (forward J, gradients, echo gradient, refinement) vs the
FP64 oracle and finite differences, through the C ABI and the autograd
Function."""
import numpy as np
import pytest
import torch

from cases import make_case, plan_for
from oracle import adjoint as OA
from oracle import transforms as OT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def p2():
    c = make_case("p2", seed=7)
    c["plan"] = plan_for(c)
    c["echo_dev"] = torch.from_numpy(c["echo"]).cuda()
    return c


def _thetas(c, n, seed):
    g = c["grid"]
    rng = np.random.default_rng(seed)
    th = np.stack([rng.uniform(2, g.N - 3, n) * g.dr,
                   rng.uniform(-90, 90, n), rng.uniform(-350, 350, n)], axis=1)
    return th


def test_forward_matches_oracle(p2):
    th = _thetas(p2, 24, 1)
    J, saved = p2["plan"].adjoint_forward(p2["echo_dev"], torch.from_numpy(th))
    J = J.cpu().numpy()
    for b in range(len(th)):
        Jo, Yo = OA.objective(p2["echo"], p2["grid"], th[b])
        assert J[b] == pytest.approx(Jo, rel=1e-9, abs=1e-9 * (Jo + 1))


def test_forward_equals_power_map_on_grid(p2):
    g = p2["grid"]
    P = OT.dsgrft_power(p2["echo"].astype(np.complex128), g)
    rng = np.random.default_rng(3)
    pts, ref = [], []
    for _ in range(16):
        k, f, n0 = int(rng.integers(g.n_coarse)), int(rng.integers(g.n_fine)), int(rng.integers(g.N))
        v, a, _ = g.params(g.lattice_point(k, f))
        pts.append((n0 * g.dr, v, a))
        ref.append(P[k, n0, f])
    J, _ = p2["plan"].adjoint_forward(p2["echo_dev"], torch.tensor(pts, dtype=torch.float64))
    # the echo is complex64; the map is FP64 of the same samples
    np.testing.assert_allclose(J.cpu().numpy(), ref, rtol=1e-9, atol=1e-9 * max(ref))


def test_theta_gradient_matches_oracle(p2):
    th = _thetas(p2, 16, 2)
    plan = p2["plan"]
    J, saved = plan.adjoint_forward(p2["echo_dev"], torch.from_numpy(th))
    gJ = torch.ones(len(th), dtype=torch.float64, device="cuda")
    gt, _ = plan.adjoint_backward(p2["echo_dev"], torch.from_numpy(th), saved, gJ,
                                  want_echo=False)
    gt = gt.cpu().numpy()
    for b in range(len(th)):
        _, _, go, _ = OA.gradients(p2["echo"], p2["grid"], th[b])
        np.testing.assert_allclose(gt[b], go, rtol=1e-7, atol=1e-9 * np.abs(go).max())


def test_echo_gradient_matches_oracle(p2):
    th = _thetas(p2, 8, 4)
    plan = p2["plan"]
    gJ = np.linspace(0.5, 2.0, len(th))
    J, saved = plan.adjoint_forward(p2["echo_dev"], torch.from_numpy(th))
    _, ge = plan.adjoint_backward(p2["echo_dev"], torch.from_numpy(th), saved,
                                  torch.from_numpy(gJ), want_theta=False)
    ge = ge.cpu().numpy()
    _, _, ref = OA.batch(p2["echo"], p2["grid"], th, grad_J=gJ, want_echo_grad=True)
    assert np.abs(ge - ref).max() <= 1e-5 * np.abs(ref).max()


def test_autograd_function_and_central_differences(p2):
    from paper_2403_06788_amd.autograd import objective
    plan = p2["plan"]
    th0 = _thetas(p2, 6, 5)
    theta = torch.tensor(th0, dtype=torch.float64, device="cuda", requires_grad=True)
    echo = p2["echo_dev"].clone().requires_grad_(True)
    J = objective(plan, echo, theta)
    J.sum().backward()
    g = theta.grad.cpu().numpy()
    g_dev = p2["grid"]
    hs = np.array([1e-4 * g_dev.dr, 1e-4 * g_dev.steps[0], 1e-4 * g_dev.steps[1]])
    for b in range(len(th0)):
        for q in range(3):
            e = np.zeros(3)
            e[q] = hs[q]
            tp = torch.from_numpy(np.stack([th0[b] + e, th0[b] - e])).to(torch.float64)
            Jp, _ = plan.adjoint_forward(p2["echo_dev"], tp)
            Jp = Jp.cpu().numpy()
            fd = (Jp[0] - Jp[1]) / (2 * hs[q])
            assert fd == pytest.approx(g[b, q], rel=1e-4, abs=1e-6 * abs(J[b].item()) / hs[q] * 1e-3)
    assert echo.grad is not None and echo.grad.dtype == torch.complex64


def test_refine_increases_objective(p2):
    plan = p2["plan"]
    th0 = _thetas(p2, 32, 6)
    J0, _ = plan.adjoint_forward(p2["echo_dev"], torch.from_numpy(th0))
    th, J = plan.refine(p2["echo_dev"], torch.from_numpy(th0), iters=20)
    J0, J = J0.cpu().numpy(), J.cpu().numpy()
    assert np.all(J >= J0 * (1 - 1e-12))
    Jc, _ = plan.adjoint_forward(p2["echo_dev"], th)
    np.testing.assert_allclose(Jc.cpu().numpy(), J, rtol=1e-12)


def test_autograd_cpu_float32_theta(p2):
    """theta on the CPU in float32 with requires_grad: the gradient comes back
    on the CPU in float32 (and equals the FP64 gradient of the same points)."""
    from paper_2403_06788_amd.autograd import objective
    plan = p2["plan"]
    th0 = _thetas(p2, 4, 8).astype(np.float32)
    theta = torch.tensor(th0, dtype=torch.float32, requires_grad=True)
    J = objective(plan, p2["echo_dev"], theta)
    J.sum().backward()
    assert theta.grad.device.type == "cpu" and theta.grad.dtype == torch.float32
    th64 = torch.from_numpy(th0.astype(np.float64))
    J64, saved = plan.adjoint_forward(p2["echo_dev"], th64)
    gt, _ = plan.adjoint_backward(p2["echo_dev"], th64, saved,
                                  torch.ones(4, dtype=torch.float64), want_echo=False)
    np.testing.assert_allclose(theta.grad.numpy(), gt.cpu().numpy().astype(np.float32),
                               rtol=1e-6)
