"""Range-compressed echo generator (received-signal model of Sec. II).

s[m][n] = sum_targets A exp(j phi0) env(n - r(t_m)/dr) exp(-j 4 pi r(t_m)/lambda)
          + w[m][n]
with r(t) = r0 + v t + a t^2/2 + j t^3/6 (eq. (7) with c2 = a/2, c3 = j/6),
t_m = m / PRF (m = 0..M-1), dr = c/(2 f_s), lambda = c/f_c, and w circular
complex Gaussian with E|w|^2 = sigma2 (re and im each of variance sigma2/2).

Envelopes:
  'sinc'    the usual range-compressed response of eqs. (4)-(5)
            (sinc(u) = sin(pi u)/(pi u)); default for the workload configs.
  'impulse' a unit sample at the nearest range bin (ties upward), with
            range bin and phase evaluated exactly in rational arithmetic;
            used for on-grid pins.

Draw order (numpy PCG64, one generator per case): for each target in turn
v, a, j (only for axes of non-zero width), then r0 uniform over the bins that
keep the whole trajectory inside the window, then phi0 ~ U[0, 2 pi); then the
noise, real parts before imaginary parts.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from fractions import Fraction as Fr

import numpy as np


@dataclass(frozen=True)
class RadarParams:
    fc: float
    fs: float
    prf: float
    c: float = 3.0e8

    @property
    def lam(self) -> float:
        return self.c / self.fc

    @property
    def dr(self) -> float:
        return self.c / (2.0 * self.fs)


@dataclass(frozen=True)
class Target:
    r0: float
    v: float
    a: float
    j: float
    amp: float
    phase: float


_R1 = RadarParams(fc=1.0e9, fs=1.0e7, prf=500.0)

# The five workload configurations (radar, sizes, search axes, targets).
# Detection-probability scenario (Monte-Carlo sweep): one target per trial,
# range walk up to ~10 bins, noise sigma^2 = 1.
PD_SCENARIO = dict(radar=_R1, M=256, N=512, order=2,
                   axes=((-300.0, 300.0), (-50.0, 50.0)),
                   v=(-300.0, 300.0), a=(-50.0, 50.0), j=(0.0, 0.0))

CONFIGS = {
    1: dict(radar=_R1, M=64, N=256, order=1, axes=((-150.0, 150.0),),
            n_targets=1, snr_db=0.0, r0_bins=(50.0, 200.0),
            v=(-150.0, 150.0), a=(0.0, 0.0), j=(0.0, 0.0)),
    2: dict(radar=_R1, M=512, N=2048, order=2,
            axes=((-600.0, 600.0), (-50.0, 50.0)),
            n_targets=3, snr_db=-15.0, r0_bins=None,
            v=(-600.0, 600.0), a=(-50.0, 50.0), j=(0.0, 0.0)),
    3: dict(radar=_R1, M=1024, N=4096, order=2,
            axes=((-600.0, 600.0), (-50.0, 50.0)),
            n_targets=8, snr_db=-20.0, r0_bins=None,
            v=(-600.0, 600.0), a=(-50.0, 50.0), j=(0.0, 0.0)),
    4: dict(radar=_R1, M=512, N=2048, order=2,
            axes=((-600.0, 600.0), (-50.0, 50.0)),
            n_targets=16, snr_db=-10.0, r0_bins=None,
            v=(-600.0, 600.0), a=(-50.0, 50.0), j=(0.0, 0.0)),
    5: dict(radar=_R1, M=2048, N=8192, order=3,
            axes=((-900.0, 900.0), (-100.0, 100.0), (-20.0, 20.0)),
            n_targets=4, snr_db=-25.0, r0_bins=None,
            v=(-900.0, 900.0), a=(-100.0, 100.0), j=(-20.0, 20.0)),
}


def _walk(t, v, a, j):
    return v * t + a * t * t / 2.0 + j * t * t * t / 6.0


def _uniform(rng, lo, hi):
    return float(lo) if lo == hi else float(rng.uniform(lo, hi))


def draw_targets(rng, radar: RadarParams, M: int, N: int, n: int,
                 snr_db: float, sigma2: float, v, a, j, r0_bins=None):
    """Draw n targets; amplitude from the per-pulse SNR |A|^2 / sigma2."""
    amp = math.sqrt(sigma2 * 10.0 ** (snr_db / 10.0))
    t = np.arange(M) / radar.prf
    out = []
    for _ in range(n):
        tv = _uniform(rng, *v)
        ta = _uniform(rng, *a)
        tj = _uniform(rng, *j)
        walk = np.abs(_walk(t, tv, ta, tj)).max() / radar.dr
        margin = math.ceil(walk) + 1
        lo, hi = (0.0, N - 1.0) if r0_bins is None else r0_bins
        lo, hi = max(lo, margin), min(hi, N - 1 - margin)
        if lo > hi:
            raise ValueError("window too small for the drawn trajectory")
        r0 = float(rng.uniform(lo, hi)) * radar.dr
        ph = float(rng.uniform(0.0, 2.0 * math.pi))
        out.append(Target(r0, tv, ta, tj, amp, ph))
    return out


def make_echo(radar: RadarParams, M: int, N: int, targets, sigma2: float,
              rng=None, dtype=np.complex64) -> np.ndarray:
    """Sinc-envelope echo of the targets plus (if rng is given) noise."""
    t = np.arange(M) / radar.prf
    n = np.arange(N, dtype=np.float64)
    s = np.zeros((M, N), dtype=np.complex128)
    for tg in targets:
        r = tg.r0 + _walk(t, tg.v, tg.a, tg.j)                   # [M]
        cyc = 2.0 * r / radar.lam
        ph = np.exp(-2j * np.pi * (cyc - np.floor(cyc)))
        env = np.sinc(n[None, :] - (r / radar.dr)[:, None])      # [M, N]
        s += tg.amp * np.exp(1j * tg.phase) * env * ph[:, None]
    if rng is not None and sigma2 > 0:
        sd = math.sqrt(sigma2 / 2.0)
        re = rng.standard_normal((M, N))
        im = rng.standard_normal((M, N))
        s += sd * (re + 1j * im)
    return s.astype(dtype)


def impulse_target_echo(radar: RadarParams, M: int, N: int, r0, v, a=0, j=0,
                        amp: complex = 1.0) -> np.ndarray:
    """Noiseless echo with one unit-sample trajectory, exact in rationals.

    r0, v, a, j may be Fractions (exact lattice values) or floats.  The
    envelope sits at floor(r(t_m)/dr + 1/2); the phase is exp(-j 4 pi r/lambda).
    """
    lam = Fr(radar.c) / Fr(radar.fc)
    dr = Fr(radar.c) / (2 * Fr(radar.fs))
    prf = Fr(radar.prf)
    r0, v, a, j = (Fr(x) for x in (r0, v, a, j))
    s = np.zeros((M, N), dtype=np.complex128)
    for m in range(M):
        tm = Fr(m) / prf
        r = r0 + v * tm + a * tm * tm / 2 + j * tm * tm * tm / 6
        n = math.floor(r / dr + Fr(1, 2))
        cyc = 2 * r / lam
        fr = cyc - math.floor(cyc)
        if 0 <= n < N:
            s[m, n] = amp * np.exp(-2j * np.pi * (fr.numerator / fr.denominator))
    return s


def adjoint_candidates(rng, radar: RadarParams, M: int, N: int, targets,
                       v_rng, a_rng, per_target=16, n_uniform=3840):
    """Candidate (r0, v, a) points: jitter around each target, then uniform.

    Jitter: r0 +- 1 range bin, v +- 2 fine velocity steps, a +- 2 fine
    acceleration steps (fine steps lambda/(2T) and lambda/T^2, T = M/PRF).
    Uniform points lie in [0, N-1] bins x v_rng x a_rng.
    """
    T = M / radar.prf
    dv, da = radar.lam / (2.0 * T), radar.lam / (T * T)
    out = []
    for tg in targets:
        for _ in range(per_target):
            out.append((tg.r0 + rng.uniform(-1, 1) * radar.dr,
                        tg.v + rng.uniform(-2, 2) * dv,
                        tg.a + rng.uniform(-2, 2) * da))
    for _ in range(n_uniform):
        out.append((rng.uniform(0, N - 1) * radar.dr,
                    rng.uniform(*v_rng), rng.uniform(*a_rng)))
    return np.asarray(out, dtype=np.float64)


def config_case(cfg: int, seed: int | None = None, sigma2: float = 1.0,
                noise: bool = True, dtype=np.complex64) -> dict:
    """Echo and metadata of workload config `cfg` (seed defaults to 1000+cfg)."""
    c = CONFIGS[cfg]
    seed = 1000 + cfg if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    tg = draw_targets(rng, c["radar"], c["M"], c["N"], c["n_targets"],
                      c["snr_db"], sigma2, c["v"], c["a"], c["j"], c["r0_bins"])
    echo = make_echo(c["radar"], c["M"], c["N"], tg, sigma2,
                     rng if noise else None, dtype=dtype)
    return dict(cfg=cfg, seed=seed, radar=c["radar"], M=c["M"], N=c["N"],
                order=c["order"], axes=c["axes"], targets=tg, echo=echo,
                sigma2=sigma2, rng=rng)
