"""ctypes binding of libdsgrft.so (argument marshalling only).

Every computation runs in the library's HIP kernels; this module only passes
device pointers (torch tensors' data_ptr()), sizes and the current HIP stream,
and checks status codes.  If the in-tree library is missing the import fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsgrft.so")

STATUS = {0: "ok", 1: "invalid argument", 2: "out of device memory",
          3: "HIP runtime error", 4: "unsupported request",
          5: "output capacity exceeded"}

FORMS = {"f32": 0, "f16": 1, "bf16": 2, "fp8": 3, "f32fft": 4, "f16_3m": 5, "bf16_glo": 6, "f16_sym": 7,
         "bf16_sym": 8, "fp8_sym": 9}


class DsgrftError(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn}: {STATUS.get(code, code)} (status {code})")
        self.code = code


class Radar(C.Structure):
    _fields_ = [("fc", C.c_double), ("fs", C.c_double), ("prf", C.c_double),
                ("c", C.c_double), ("kappa", C.c_double)]


class Axis(C.Structure):
    _fields_ = [("min", C.c_double), ("max", C.c_double)]


class Config(C.Structure):
    _fields_ = [("M", C.c_int32), ("N", C.c_int32), ("order", C.c_int32),
                ("n_begin", C.c_int32), ("n_end", C.c_int32),
                ("axis", Axis * 3), ("batch", C.c_int32), ("mgift", C.c_int32)]


class PlanInfo(C.Structure):
    _fields_ = [("R", C.c_int32), ("K", C.c_int32 * 3), ("i_lo", C.c_int32 * 3),
                ("rows", C.c_int32), ("n_coarse", C.c_int64),
                ("n_fine", C.c_int64), ("lambda_", C.c_double),
                ("dr", C.c_double), ("T", C.c_double),
                ("step", C.c_double * 3), ("workspace_bytes", C.c_size_t),
                ("fd_pad", C.c_int32), ("kt_q_lo", C.c_int32), ("kt_folds", C.c_int32)]


class Profile(C.Structure):
    _fields_ = [("gather_launches", C.c_int64), ("fine_launches", C.c_int64),
                ("gather_ms", C.c_double), ("fine_ms", C.c_double),
                ("gather_bytes", C.c_double), ("fine_flops", C.c_double),
                ("fine_cell_pulses", C.c_double), ("fine_mfma_flops", C.c_double)]


PEAK_DTYPE = np.dtype({
    "names": ["coarse", "row", "fine", "power", "pad", "r0", "v", "a", "j"],
    "formats": [np.int64, np.int32, np.int32, np.float32, np.float32,
                np.float64, np.float64, np.float64, np.float64],
    "offsets": [0, 8, 12, 16, 20, 24, 32, 40, 48], "itemsize": 56})

_lib = None


def lib():
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2403_06788_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "dsgrft_plan_create": [C.POINTER(Radar), C.POINTER(Config), C.POINTER(vp)],
        "dsgrft_plan_get_info": [vp, C.POINTER(PlanInfo)],
        "dsgrft_coarse_tables": [vp, i64, i64, vp, vp, vp],
        "dsgrft_mgift": [vp, vp, i64, i64, vp, vp],
        "dsgrft_search": [vp, C.c_int, i32, vp, vp, i64, i64, vp, vp, vp],
        "dsgrft_search_full": [vp, C.c_int, i32, vp, i64, i64, vp, vp],
        "dsgrft_grft": [vp, vp, i64, i64, vp, vp, vp, vp],
        "dsgrft_noise_power": [vp, vp, vp, vp],
        "dsgrft_lrt_threshold": [vp, dbl, dbl, C.POINTER(dbl)],
        "dsgrft_noise_power_noalloc": [vp, i32, i32, vp, vp],
        "dsgrft_detect": [vp, vp, vp, vp, i64, i64, dbl, vp, dbl, vp, i32, vp, vp,
                          C.POINTER(i32), vp],
        "dsgrft_detect_cfar": [vp, vp, vp, vp, i64, i64, i32, i32, dbl, vp, i32, vp, vp,
                               C.POINTER(i32), vp],
        "dsgrft_adjoint_forward": [vp, vp, vp, i32, vp, vp, vp],
        "dsgrft_adjoint_backward": [vp, vp, vp, i32, vp, vp, vp, vp, vp],
        "dsgrft_refine": [vp, vp, vp, i32, i32, vp, vp],
        "dsgrft_profile_begin": [vp, i32],
        "dsgrft_profile_end": [vp, C.POINTER(Profile)],
        "dsgrft_mfma_probe": [C.c_int, dbl, C.POINTER(dbl), C.POINTER(dbl)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    L.dsgrft_plan_destroy.argtypes = [vp]
    L.dsgrft_plan_destroy.restype = None
    L.dsgrft_status_string.argtypes = [C.c_int]
    L.dsgrft_status_string.restype = C.c_char_p
    _lib = L
    return L


def check(fn: str, code: int):
    if code != 0:
        raise DsgrftError(fn, code)


def exported_symbols():
    """Names declared in include/dsgrft.h (checked by the ABI test)."""
    return ["dsgrft_plan_create", "dsgrft_plan_destroy", "dsgrft_plan_get_info",
            "dsgrft_status_string", "dsgrft_coarse_tables", "dsgrft_mgift",
            "dsgrft_search", "dsgrft_search_full", "dsgrft_grft",
            "dsgrft_noise_power", "dsgrft_noise_power_noalloc", "dsgrft_lrt_threshold",
            "dsgrft_detect",
            "dsgrft_detect_cfar",
            "dsgrft_adjoint_forward",
            "dsgrft_adjoint_backward", "dsgrft_refine",
            "dsgrft_profile_begin", "dsgrft_profile_end", "dsgrft_mfma_probe"]
