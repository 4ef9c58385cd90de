"""Pins of the continuous objective and its gradients (oracle/adjoint.py)."""
import numpy as np
import pytest

from oracle import adjoint as A
from oracle import transforms as T
from oracle.grid import Axis, Radar, make_grid


def grid_and_echo(M=24, N=48, seed=0):
    g = make_grid(Radar(8.0e7, 1.0e7, 500.0), M, N, 2,
                  [Axis(-60.0, 60.0), Axis(-40.0, 40.0)])
    rng = np.random.default_rng(seed)
    echo = rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))
    return g, echo


def test_objective_equals_power_map_on_grid():
    g, echo = grid_and_echo()
    P = T.dsgrft_power(echo, g)
    rng = np.random.default_rng(1)
    for _ in range(20):
        k = int(rng.integers(g.n_coarse))
        f = int(rng.integers(g.n_fine))
        n0 = int(rng.integers(g.N))
        i = g.lattice_point(k, f)
        v, a, _ = g.params(i)
        J, _ = A.objective(echo, g, (n0 * g.dr, v, a))
        assert A.coarse_cell_of(g, v, a) == k
        assert J == pytest.approx(P[k, n0, f], rel=1e-11, abs=1e-11 * P.max())


def _inside(g, v, a, margin=0.05):
    for p, val in enumerate((v, a)):
        u = val / g.steps[p] - g.i_lo[p] + 0.5
        frac = (u / g.R) % 1.0
        if frac < margin or frac > 1 - margin:
            return False
    return True


def test_theta_gradient_matches_central_differences():
    g, echo = grid_and_echo(seed=2)
    rng = np.random.default_rng(3)
    hs = (1e-4 * g.dr, 1e-4 * g.steps[0], 1e-4 * g.steps[1])
    checked = 0
    while checked < 12:
        th = np.array([rng.uniform(5, g.N - 5) * g.dr,
                       rng.uniform(-50, 50), rng.uniform(-30, 30)])
        if not _inside(g, th[1], th[2]):
            continue
        J, _, grad, _ = A.gradients(echo, g, th)
        for p in range(3):
            e = np.zeros(3)
            e[p] = hs[p]
            fd = (A.objective(echo, g, th + e)[0] - A.objective(echo, g, th - e)[0]) / (2 * hs[p])
            scale = abs(grad[p]) + 1e-6 * J / hs[p] * 1e-4
            assert abs(fd - grad[p]) <= 1e-5 * max(abs(grad[p]), 1.0) + 1e-7 * scale
        checked += 1


def test_echo_gradient_matches_central_differences():
    g, echo = grid_and_echo(M=12, N=20, seed=4)
    th = np.array([9.3 * g.dr, 7.0, -3.0])
    J, Y, _, ge = A.gradients(echo, g, th)
    rng = np.random.default_rng(5)
    h = 1e-6
    for _ in range(10):
        m, n = int(rng.integers(12)), int(rng.integers(20))
        d = np.zeros_like(echo)
        d[m, n] = h
        fre = (A.objective(echo + d, g, th)[0] - A.objective(echo - d, g, th)[0]) / (2 * h)
        fim = (A.objective(echo + 1j * d, g, th)[0] - A.objective(echo - 1j * d, g, th)[0]) / (2 * h)
        assert ge[m, n].real == pytest.approx(fre, rel=1e-6, abs=1e-8)
        assert ge[m, n].imag == pytest.approx(fim, rel=1e-6, abs=1e-8)


def test_sinc_derivative_series_branch_is_continuous():
    u = np.array([-1e-4 - 1e-12, -1e-4 + 1e-12, 0.0, 1e-4 - 1e-12, 1e-4 + 1e-12, 0.37])
    d = A._dsinc(u)
    assert d[2] == 0.0
    assert d[0] == pytest.approx(d[1], rel=1e-7)
    assert d[3] == pytest.approx(d[4], rel=1e-7)
    h = 1e-6
    fd = (np.sinc(0.37 + h) - np.sinc(0.37 - h)) / (2 * h)
    assert d[5] == pytest.approx(fd, rel=1e-8)


def test_batch_weighted_echo_gradient_two_candidates():
    """batch(): J and dJ/dtheta per candidate equal objective()/gradients(),
    and the echo gradient is the grad_J-weighted sum over candidates, checked
    against central differences of L(s) = sum_b grad_J[b] J_b(s) in the real
    and imaginary part of each sampled echo entry (a dropped or misapplied
    weight changes L's gradient)."""
    g, echo = grid_and_echo(M=12, N=20, seed=6)
    thetas = np.array([[9.3 * g.dr, 7.0, -3.0], [4.6 * g.dr, -11.0, 5.5]])
    gJ = np.array([0.7, -1.9])
    J, G, ge = A.batch(echo, g, thetas, grad_J=gJ, want_echo_grad=True)
    for b in range(2):
        jb, _, gb, _ = A.gradients(echo, g, thetas[b])
        assert J[b] == jb and np.array_equal(G[b], gb)
        assert J[b] == pytest.approx(A.objective(echo, g, thetas[b])[0], rel=1e-13)

    def L(s):
        return sum(gJ[b] * A.objective(s, g, thetas[b])[0] for b in range(2))

    rng = np.random.default_rng(8)
    h = 1e-6
    for _ in range(12):
        m, n = int(rng.integers(12)), int(rng.integers(20))
        d = np.zeros_like(echo)
        d[m, n] = h
        fre = (L(echo + d) - L(echo - d)) / (2 * h)
        fim = (L(echo + 1j * d) - L(echo - 1j * d)) / (2 * h)
        assert ge[m, n].real == pytest.approx(fre, rel=1e-6, abs=1e-8)
        assert ge[m, n].imag == pytest.approx(fim, rel=1e-6, abs=1e-8)
    # unit weights when grad_J is omitted; no echo gradient unless asked
    _, _, ge1 = A.batch(echo, g, thetas, want_echo_grad=True)
    ref = A.gradients(echo, g, thetas[0])[3] + A.gradients(echo, g, thetas[1])[3]
    assert np.abs(ge1 - ref).max() <= 1e-12 * np.abs(ref).max()
    assert A.batch(echo, g, thetas)[2] is None
