"""Continuous DS-GRFT objective and its analytic gradients (oracle).

Test infrastructure only: nothing in the product path imports this module.

The paper defines the transforms only on the search lattice.  The off-grid
objective used for peak refinement is a reading of its own, not the paper's:
for theta = (r0, v, a),

  coarse cell   k_p = clamp(floor((theta_p / d_p - i_lo,p + 1/2) / R)),
                i_c = its centre (Sec. IV-B lattice), p = v, a
  envelope      x_m = r0 / dr + off(m; i_c)        (coarse RM correction,
                                                  mGIFT of eq. (46))
  interpolant   s~_m(x) = sum_{n=0}^{N-1} s[m][n] sinc(x - n),
                sinc(u) = sin(pi u) / (pi u)
  phase         cyc_m = 2 (v t_m + a t_m^2 / 2) / lambda  (eq. (12)-(13)
                with the continuous parameters)
  Y(theta) = sum_m s~_m(x_m) exp(+j 2 pi cyc_m),   J = |Y|^2.

At lattice points (r0 = n0 dr, (v, a) on the fine grid) sinc reduces to a
Kronecker delta and J equals the DS-GRFT power map.  Inside a coarse cell J is
smooth; the gradients below are exact derivatives there (the coarse offsets
are piecewise constant and contribute nothing).

Gradient of the echo follows PyTorch's convention for a real loss of a
complex input (dJ/dRe + j dJ/dIm):
  dJ/ds[m][n] = 2 Y conj(sinc(x_m - n) exp(j 2 pi cyc_m)).
"""
from __future__ import annotations

import math

import numpy as np

from .grid import Grid, numerator, range_offset


def coarse_cell_of(grid: Grid, v: float, a: float) -> int:
    ks = []
    for p, val in enumerate((v, a)):
        if p >= grid.order:
            ks.append(0)
            continue
        u = val / grid.steps[p]
        k = math.floor((u - grid.i_lo[p] + 0.5) / grid.R)
        ks.append(min(max(k, 0), grid.K[p] - 1))
    return ks[0] + grid.K[0] * ks[1]


def _dsinc(u: np.ndarray) -> np.ndarray:
    """d/du sinc(u) with sinc(u) = sin(pi u)/(pi u)."""
    out = np.empty_like(u)
    small = np.abs(u) < 1e-4
    us = u[~small]
    out[~small] = (np.cos(np.pi * us) - np.sinc(us)) / us
    ul = u[small]
    out[small] = -(np.pi ** 2) * ul / 3.0 + (np.pi ** 4) * ul ** 3 / 30.0
    return out


def _terms(echo: np.ndarray, grid: Grid, theta):
    r0, v, a = (float(t) for t in theta)
    if grid.order > 2:
        raise ValueError("the continuous objective covers orders 1 and 2")
    k = coarse_cell_of(grid, v, a)
    m = np.arange(grid.M, dtype=np.int64)
    off = range_offset(grid, numerator(grid, m, grid.centre(k)))
    x = r0 / grid.dr + off.astype(np.float64)                   # [M]
    t = m.astype(np.float64) / grid.radar.prf
    cyc = 2.0 * (v * t + a * t * t / 2.0) / grid.lam
    frac = cyc - np.floor(cyc)
    e = np.exp(2j * np.pi * frac)                               # [M]
    u = x[:, None] - np.arange(grid.N, dtype=np.float64)[None, :]  # [M, N]
    w = np.sinc(u)
    return k, t, e, u, w


def objective(echo, grid: Grid, theta):
    """(J, Y) at one candidate theta = (r0, v, a)."""
    echo = np.asarray(echo, dtype=np.complex128)
    _, _, e, _, w = _terms(echo, grid, theta)
    st = (echo * w).sum(axis=1)                                 # s~_m(x_m)
    Y = (st * e).sum()
    return float(abs(Y) ** 2), complex(Y)


def gradients(echo, grid: Grid, theta):
    """(J, Y, dJ/dtheta [3], dJ/ds [M, N]) at one candidate."""
    echo = np.asarray(echo, dtype=np.complex128)
    _, t, e, u, w = _terms(echo, grid, theta)
    st = (echo * w).sum(axis=1)
    dst = (echo * _dsinc(u)).sum(axis=1)
    Y = (st * e).sum()
    dY_dr0 = (dst * e).sum() / grid.dr
    dY_dv = (st * e * (2j * np.pi * 2.0 * t / grid.lam)).sum()
    dY_da = (st * e * (2j * np.pi * t * t / grid.lam)).sum()
    cY = np.conj(Y)
    g = np.array([2.0 * (cY * d).real for d in (dY_dr0, dY_dv, dY_da)])
    g_echo = 2.0 * Y * np.conj(w * e[:, None])
    return float(abs(Y) ** 2), complex(Y), g, g_echo


def batch(echo, grid: Grid, thetas, grad_J=None, want_echo_grad=False):
    """Vector versions over candidates: J [B], grad_theta [B, 3] and,
    optionally, sum_b grad_J[b] * dJ_b/ds [M, N]."""
    B = len(thetas)
    J = np.empty(B)
    G = np.empty((B, 3))
    ge = np.zeros(np.shape(echo), dtype=np.complex128) if want_echo_grad else None
    for b, th in enumerate(thetas):
        j, _, g, gs = gradients(echo, grid, th)
        J[b] = j
        G[b] = g
        if want_echo_grad:
            ge += (1.0 if grad_J is None else float(grad_J[b])) * gs
    return J, G, ge
