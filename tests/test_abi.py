"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/dsgrft.h, and rejects invalid arguments before touching
the device."""
import ctypes as C
import os
import re

import pytest

from paper_2403_06788_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dsgrft.h")

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH),
                                reason="libdsgrft.so not built")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dsgrft_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_binding_surface():
    assert declared_functions() == sorted(_lib.exported_symbols())


def test_every_declared_symbol_is_exported():
    L = _lib.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_status_strings():
    L = _lib.lib()
    assert L.dsgrft_status_string(0) == b"ok"
    assert L.dsgrft_status_string(4) == b"unsupported request"
    assert L.dsgrft_status_string(99) == b"unknown status"


def _create(fc=1e9, fs=1e7, prf=500.0, M=64, N=256, order=1, axes=((-150, 150),),
            kappa=1.0, rows=(0, 0), batch=0, c=3e8, mgift=0):
    L = _lib.lib()
    r = _lib.Radar(fc, fs, prf, c, kappa)
    cfg = _lib.Config()
    cfg.M, cfg.N, cfg.order = M, N, order
    cfg.n_begin, cfg.n_end = rows
    for p, ax in enumerate(axes):
        cfg.axis[p].min, cfg.axis[p].max = ax
    cfg.batch = batch
    cfg.mgift = mgift
    h = C.c_void_p()
    return L.dsgrft_plan_create(C.byref(r), C.byref(cfg), C.byref(h))


@pytest.mark.parametrize("kw", [
    dict(M=0), dict(N=0), dict(order=0), dict(order=4),
    dict(fs=3e7),                       # f_c / f_s not an integer
    dict(fc=-1.0), dict(prf=0.0), dict(c=float("nan")),
    dict(axes=((150, -150),)),          # min > max
    dict(rows=(10, 5)), dict(rows=(0, 300)), dict(rows=(-1, 10)),
    dict(batch=-1),
    dict(M=2048, order=3, axes=((-1e12, 1e12), (-1, 1), (-1, 1))),  # numerator overflow
    dict(mgift=3), dict(mgift=-1),      # no such coarse stage
])
def test_plan_create_rejects_invalid(kw):
    assert _create(**kw) == 1


def test_plan_create_kappa_unsupported():
    assert _create(kappa=0.995) == 4


@pytest.mark.parametrize("kw", [
    dict(order=1),                                                 # DS-KT-MFP needs P = 2
    dict(order=2, M=96, axes=((-150, 150), (-200, 200))),          # M not a power of two
    dict(order=2, M=4096, axes=((-150, 150), (-200, 200))),        # M above 2048
])
def test_ktmfp_plan_limits(kw):
    assert _create(mgift=2, **kw) == 4


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of dsgrft_radar, dsgrft_config, dsgrft_plan_info and
    dsgrft_peak have the C header's sizes and field offsets (a host C program
    built with gcc prints them)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    mirrors = {"dsgrft_radar": _lib.Radar, "dsgrft_config": _lib.Config,
               "dsgrft_plan_info": _lib.PlanInfo, "dsgrft_profile": _lib.Profile}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "dsgrft.h"',
             "int main(void) {"]
    for cname, cls in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            cf = "lambda" if fname == "lambda_" else fname
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {cf}));')
    lines.append('  printf("dsgrft_peak size %zu\\n", sizeof(dsgrft_peak));')
    for fname in _lib.PEAK_DTYPE.names:
        cf = "pad_" if fname == "pad" else fname
        lines.append(f'  printf("dsgrft_peak {fname} %zu\\n", offsetof(dsgrft_peak, {cf}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for ln in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        s, f, v = ln.split()
        got[(s, f)] = int(v)
    for cname, cls in mirrors.items():
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
    assert got[("dsgrft_peak", "size")] == _lib.PEAK_DTYPE.itemsize
    for fname in _lib.PEAK_DTYPE.names:
        assert got[("dsgrft_peak", fname)] == _lib.PEAK_DTYPE.fields[fname][1], fname


def test_null_pointers_rejected():
    L = _lib.lib()
    h = C.c_void_p()
    assert L.dsgrft_plan_create(None, None, C.byref(h)) == 1
    assert L.dsgrft_search(None, 1, 1, None, None, 0, 1, None, None, None) == 1
    assert L.dsgrft_detect(None, None, None, None, 0, 1, 1.0, None, 1e-6, None, 0, None, None,
                           None, None) == 1
    assert L.dsgrft_detect_cfar(None, None, None, None, 0, 1, 2, 8, 5.0, None, 0, None, None,
                                None, None) == 1
    g = C.c_double()
    assert L.dsgrft_lrt_threshold(None, 1.0, 1e-6, C.byref(g)) == 1
    # the MFMA probe checks its arguments before any HIP call
    t, gh = C.c_double(), C.c_double()
    assert L.dsgrft_mfma_probe(0, 10.0, C.byref(t), C.byref(gh)) == 1        # FP32: no
    assert L.dsgrft_mfma_probe(1, 0.0, C.byref(t), C.byref(gh)) == 1         # ms < 1
    assert L.dsgrft_mfma_probe(1, 10.0, None, C.byref(gh)) == 1
    # the no-allocation noise power checks its arguments before any HIP call
    fake = C.c_void_p(256)
    assert L.dsgrft_noise_power_noalloc(None, 4, 4, fake, None) == 1
    assert L.dsgrft_noise_power_noalloc(fake, 0, 4, fake, None) == 1
    assert L.dsgrft_noise_power_noalloc(fake, 1 << 15, 1 << 14, fake, None) == 1  # > 2^28
    assert L.dsgrft_adjoint_forward(None, None, None, 1, None, None, None) == 1
    info = _lib.PlanInfo()
    assert L.dsgrft_plan_get_info(None, C.byref(info)) == 1
    L.dsgrft_plan_destroy(None)  # accepted
