"""Python face of the DS-GRFT library: one `Plan` per radar/lattice setup.

Methods take and return torch tensors on the plan's GPU and pass their
device pointers and the current HIP stream straight to the C ABI; torch is
used for device memory and streams only.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import FORMS, PEAK_DTYPE, check

CFG_FIELDS = ("M", "N", "order")


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _echo(echo: torch.Tensor) -> torch.Tensor:
    if echo.dtype != torch.complex64 or not echo.is_cuda or not echo.is_contiguous():
        raise ValueError("echo must be a contiguous complex64 CUDA tensor [M][N]")
    return echo


class Plan:
    """Dual-scale lattice, fine tables and workspace for one search setup.

    fc, fs, prf: carrier [Hz], range sampling rate [Hz], PRF [Hz];
    axes: [(vmin, vmax), (amin, amax), (jmin, jmax)][:order];
    rows: optional (n_begin, n_end) range rows of interest;
    mgift: "td" (nearest-bin gather along the coarse walk), "fd"
    (frequency-domain coarse compensation of Alg. 1) or "kt" (DS-KT-MFP,
    Alg. 4: keystone transform and folded velocity lattice; order 2, FFT
    form only).
    """

    def __init__(self, fc, fs, prf, M, N, order, axes, rows=None, c=3.0e8,
                 kappa=1.0, batch=0, mgift="td"):
        L = _lib.lib()
        radar = _lib.Radar(fc, fs, prf, c, kappa)
        cfg = _lib.Config()
        cfg.M, cfg.N, cfg.order = M, N, order
        cfg.n_begin, cfg.n_end = (0, 0) if rows is None else rows
        for p, ax in enumerate(axes):
            cfg.axis[p].min, cfg.axis[p].max = float(ax[0]), float(ax[1])
        cfg.batch = batch
        modes = {"td": 0, "fd": 1, "kt": 2}
        if mgift not in modes:
            raise ValueError('mgift must be "td", "fd" or "kt"')
        cfg.mgift = modes[mgift]
        h = C.c_void_p()
        check("dsgrft_plan_create", L.dsgrft_plan_create(C.byref(radar), C.byref(cfg), C.byref(h)))
        self._h = h
        self._L = L
        info = _lib.PlanInfo()
        check("dsgrft_plan_get_info", L.dsgrft_plan_get_info(h, C.byref(info)))
        self.M, self.N, self.order = M, N, order
        self.R = info.R
        self.K = tuple(info.K)
        self.i_lo = tuple(info.i_lo)
        self.rows = info.rows
        self.n_begin = cfg.n_begin
        self.n_coarse = info.n_coarse
        self.n_fine = info.n_fine
        self.lam, self.dr, self.T = info.lambda_, info.dr, info.T
        self.step = tuple(info.step)
        self.workspace_bytes = info.workspace_bytes
        self.fd_pad = info.fd_pad
        self.kt_q_lo, self.kt_folds = info.kt_q_lo, info.kt_folds
        self.prf = prf
        self.mgift_mode = mgift

    def close(self):
        if getattr(self, "_h", None):
            self._L.dsgrft_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- stage a0 / a1+a2 readback --------------------------------------
    def coarse_tables(self, cc_begin=0, n=None):
        n = self.n_coarse - cc_begin if n is None else n
        off = torch.empty((n, self.M), dtype=torch.int32, device="cuda")
        psi = torch.empty((n, self.M), dtype=torch.complex64, device="cuda")
        check("dsgrft_coarse_tables", self._L.dsgrft_coarse_tables(
            self._h, cc_begin, n, _ptr(off), _ptr(psi), _stream()))
        return off, psi

    def mgift(self, echo, cc_begin=0, n=None):
        echo = _echo(echo)
        n = self.n_coarse - cc_begin if n is None else n
        out = torch.empty((n, self.M, self.rows), dtype=torch.complex64, device="cuda")
        check("dsgrft_mgift", self._L.dsgrft_mgift(
            self._h, _ptr(echo), cc_begin, n, _ptr(out), _stream()))
        return out

    # ---- search -----------------------------------------------------------
    def search(self, echo, form="f16", split=1, cells=None, cc_begin=0, n=None,
               out=None):
        """Reduced DS-GRFT map: (pmax [n, rows] float32, argf [n, rows] int32).

        form/split: "f32" (vector ALUs) and "f32fft" (slow-time FFT) with
        split 1; "f16", "bf16", "fp8" with split 1-4 products; "f16_3m"
        (three real products per complex product) with split 1; "f16_sym"
        (fine cells in conjugate pairs, four real products per pair) with
        split 1; "bf16_glo" (the gathered rows split) with split 2;
        "bf16_sym" over conjugate pairs with split 2 (bf16_glo's products)
        or 3 (bf16 split 3's products); "fp8_sym" over conjugate pairs with
        split 3 or 4 (fp8's products)."""
        echo = _echo(echo)
        if cells is not None:
            cells = cells.to(device="cuda", dtype=torch.int64).contiguous()
            n = cells.numel()
        else:
            n = self.n_coarse - cc_begin if n is None else n
        if out is None:
            pmax = torch.empty((n, self.rows), dtype=torch.float32, device="cuda")
            argf = torch.empty((n, self.rows), dtype=torch.int32, device="cuda")
        else:
            pmax, argf = out
        check("dsgrft_search", self._L.dsgrft_search(
            self._h, FORMS[form], split, _ptr(echo), _ptr(cells), cc_begin, n,
            _ptr(pmax), _ptr(argf), _stream()))
        return pmax, argf

    def search_full(self, echo, form="f32", split=1, cc_begin=0, n=None):
        echo = _echo(echo)
        n = self.n_coarse - cc_begin if n is None else n
        pw = torch.empty((n, self.rows, self.n_fine), dtype=torch.float32, device="cuda")
        check("dsgrft_search_full", self._L.dsgrft_search_full(
            self._h, FORMS[form], split, _ptr(echo), cc_begin, n, _ptr(pw), _stream()))
        return pw

    def grft(self, echo, cc_begin=0, n=None, full=False):
        echo = _echo(echo)
        n = self.n_coarse - cc_begin if n is None else n
        pmax = torch.empty((n, self.rows), dtype=torch.float32, device="cuda")
        argf = torch.empty((n, self.rows), dtype=torch.int32, device="cuda")
        pw = (torch.empty((n, self.rows, self.n_fine), dtype=torch.float32, device="cuda")
              if full else None)
        check("dsgrft_grft", self._L.dsgrft_grft(
            self._h, _ptr(echo), cc_begin, n, _ptr(pmax), _ptr(argf), _ptr(pw), _stream()))
        return (pmax, argf, pw) if full else (pmax, argf)

    # ---- detection ----------------------------------------------------------
    def noise_power(self, echo, as_tensor=False):
        """Mean |s|^2 of the echo (sigma^2 of eq. (33)): a float, or with
        as_tensor a one-element float64 CUDA tensor (no synchronisation)."""
        echo = _echo(echo)
        out = torch.empty(1, dtype=torch.float64, device="cuda")
        check("dsgrft_noise_power", self._L.dsgrft_noise_power(
            self._h, _ptr(echo), _ptr(out), _stream()))
        return out if as_tensor else float(out.item())

    def _detect_out(self, cap):
        peaks = torch.empty((max(cap, 1), PEAK_DTYPE.itemsize), dtype=torch.uint8, device="cuda")
        best = torch.empty((1, PEAK_DTYPE.itemsize), dtype=torch.uint8, device="cuda")
        count = torch.zeros(1, dtype=torch.int32, device="cuda")
        return peaks, best, count

    @staticmethod
    def _detect_result(fn, status, peaks, best, hc, cap):
        # E_CAPACITY still delivers the first `cap` entries and the true count
        if status != 5:
            check(fn, status)
        cnt = int(hc.value)
        pk = peaks[:min(cnt, cap)].cpu().numpy().view(PEAK_DTYPE).reshape(-1)
        bp = best.cpu().numpy().view(PEAK_DTYPE).reshape(-1)[0]
        return pk, cnt, bp

    def detect(self, pmax, argf, pfa, sigma2=1.0, cap=1024, cells=None, cc_begin=0):
        """LRT test (eq. (33)) on a reduced map at false-alarm probability
        `pfa`; sigma2 is a float or a one-element float64 CUDA tensor (e.g.
        noise_power(..., as_tensor=True)).  Returns (peaks structured numpy
        array [min(count, cap)], count, best peak); count > cap means the
        list was truncated."""
        n = pmax.shape[0]
        if cells is not None:
            cells = cells.to(device="cuda", dtype=torch.int64).contiguous()
        dev = isinstance(sigma2, torch.Tensor)
        peaks, best, count = self._detect_out(cap)
        hc = C.c_int32(0)
        st = self._L.dsgrft_detect(
            self._h, _ptr(pmax), _ptr(argf), _ptr(cells), cc_begin, n,
            0.0 if dev else float(sigma2), _ptr(sigma2) if dev else None, float(pfa),
            _ptr(peaks), cap, _ptr(count), _ptr(best), C.byref(hc), _stream())
        return self._detect_result("dsgrft_detect", st, peaks, best, hc, cap)

    def detect_cfar(self, pmax, argf, guard, train, alpha, cap=1024, cells=None, cc_begin=0):
        """Cell-averaging CFAR along range on a reduced map.  Returns (peaks
        structured numpy array [min(count, cap)], count, best peak)."""
        n = pmax.shape[0]
        if cells is not None:
            cells = cells.to(device="cuda", dtype=torch.int64).contiguous()
        peaks, best, count = self._detect_out(cap)
        hc = C.c_int32(0)
        st = self._L.dsgrft_detect_cfar(
            self._h, _ptr(pmax), _ptr(argf), _ptr(cells), cc_begin, n, int(guard), int(train),
            float(alpha), _ptr(peaks), cap, _ptr(count), _ptr(best), C.byref(hc), _stream())
        return self._detect_result("dsgrft_detect_cfar", st, peaks, best, hc, cap)

    def threshold(self, sigma2, pfa):
        """LRT threshold gamma^2 on |Y|^2 (eq. (33)), from the library."""
        g = C.c_double()
        check("dsgrft_lrt_threshold", self._L.dsgrft_lrt_threshold(
            self._h, float(sigma2), float(pfa), C.byref(g)))
        return g.value

    # ---- measurement -----------------------------------------------------
    def profile_begin(self, capacity=4096):
        check("dsgrft_profile_begin", self._L.dsgrft_profile_begin(self._h, capacity))

    def profile_end(self) -> dict:
        pr = _lib.Profile()
        check("dsgrft_profile_end", self._L.dsgrft_profile_end(self._h, C.byref(pr)))
        return {k: getattr(pr, k) for k, _ in pr._fields_}

    @staticmethod
    def mfma_probe(form="f16", ms=50.0):
        """Attainable matrix-core rate on random operands: (TFLOP/s, GHz)."""
        t, g = C.c_double(), C.c_double()
        check("dsgrft_mfma_probe", _lib.lib().dsgrft_mfma_probe(FORMS[form], float(ms),
                                                                C.byref(t), C.byref(g)))
        return t.value, g.value

    # ---- adjoint --------------------------------------------------------------
    def adjoint_forward(self, echo, theta):
        echo = _echo(echo)
        theta = theta.to(device="cuda", dtype=torch.float64).contiguous()
        B = theta.shape[0]
        J = torch.empty(B, dtype=torch.float64, device="cuda")
        saved = torch.empty((B, 8), dtype=torch.float64, device="cuda")
        check("dsgrft_adjoint_forward", self._L.dsgrft_adjoint_forward(
            self._h, _ptr(echo), _ptr(theta), B, _ptr(J), _ptr(saved), _stream()))
        return J, saved

    def adjoint_backward(self, echo, theta, saved, gJ, want_theta=True, want_echo=True):
        echo = _echo(echo)
        theta = theta.to(device="cuda", dtype=torch.float64).contiguous()
        gJ = gJ.to(device="cuda", dtype=torch.float64).contiguous()
        B = theta.shape[0]
        gt = torch.empty((B, 3), dtype=torch.float64, device="cuda") if want_theta else None
        ge = torch.empty((self.M, self.N), dtype=torch.complex64, device="cuda") if want_echo else None
        check("dsgrft_adjoint_backward", self._L.dsgrft_adjoint_backward(
            self._h, _ptr(echo), _ptr(theta), B, _ptr(saved), _ptr(gJ), _ptr(gt),
            _ptr(ge), _stream()))
        return gt, ge

    def refine(self, echo, theta, iters=30):
        echo = _echo(echo)
        th = theta.to(device="cuda", dtype=torch.float64).clone().contiguous()
        B = th.shape[0]
        J = torch.empty(B, dtype=torch.float64, device="cuda")
        check("dsgrft_refine", self._L.dsgrft_refine(
            self._h, _ptr(echo), _ptr(th), B, iters, _ptr(J), _stream()))
        return th, J
