"""Host-side checks of the C ABI (no GPU needed).

* the shared library loads and exports every function the header declares;
* argument validation rejects bad descriptors, bins and sizes on the host,
  before anything is launched, with a message in cnpc_last_error().
"""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cnpc.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cnpc_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported():
    from paper_2605_04864_amd import _lib as L
    names = _declared()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L.lib, n)]
    assert not missing, missing
    assert set(names) == set(L.EXPORTED)


def test_version_and_empty_error():
    from paper_2605_04864_amd import _lib as L
    assert b"gfx950" in L.lib.cnpc_version()


def _desc(**kw):
    from paper_2605_04864_amd import _lib as L
    d = L.mesh_desc(kw.get("n", 64), kw.get("box", 1000.0), assign=kw.get("assign", L.TSC),
                    interlace=kw.get("interlace", True), dtype=kw.get("dtype", L.F32),
                    observer=kw.get("observer"), los=kw.get("los"))
    return d


@pytest.mark.parametrize("kw,msg", [
    ({"n": 100}, "power of two"),
    ({"n": 8}, "power of two"),
    ({"n": 2048}, "power of two"),
    ({"assign": 4}, "assign"),
    ({"dtype": 7}, "dtype"),
    ({"box": -1.0}, "boxsize"),
    ({"observer": (10.0, 10.0, 10.0)}, "outside"),
    ({"los": (0.0, 0.0, 2.0)}, "unit vector"),
])
def test_descriptor_validation(kw, msg):
    from paper_2605_04864_amd import _lib as L
    d = _desc(**kw)
    st = L.lib.cnpc_fft_r2c(C.byref(d), 1, 0, C.c_void_p(16), C.c_void_p(32), None, 0, None)
    assert st == -1
    assert msg in L.last_error()


def test_bins_and_band_validation():
    from paper_2605_04864_amd import _lib as L
    d = _desc(n=64, box=1000.0)
    b = L.kbins(0.0, 0.05, 10)  # top edge 0.5 > k_N = 0.201
    st = L.lib.cnpc_bin_pk(C.byref(d), C.byref(b), 32, 0, None, None, 0, None, None, None, None,
                           C.c_void_p(64), None, C.c_void_p(64), 1 << 20, None)
    assert st == -1 and "Nyquist" in L.last_error()
    b = L.kbins(0.0, 0.01, 20)
    st = L.lib.cnpc_bin_pk(C.byref(d), C.byref(b), 8, 0, None, None, 0, None, None, None, None,
                           C.c_void_p(64), None, C.c_void_p(64), 1 << 20, None)
    assert st == -1 and "does not cover" in L.last_error()
    st = L.lib.cnpc_fft_r2c(C.byref(d), 1, 12, C.c_void_p(16), C.c_void_p(32), None, 0, None)
    assert st == -1 and "band" in L.last_error()
    assert L.lib.cnpc_band_for(C.byref(d), 0.2) == 32


def test_paint_and_bispec_validation():
    from paper_2605_04864_amd import _lib as L
    d = _desc(n=64, box=1000.0)
    st = L.lib.cnpc_paint(C.byref(d), C.c_void_p(16), None, 0, C.c_void_p(16), None, 10,
                          C.c_void_p(16), C.c_void_p(16), None, C.c_void_p(16), 1 << 30, None)
    assert st == -1 and "ngal" in L.last_error()
    st = L.lib.cnpc_paint(C.byref(d), C.c_void_p(16), C.c_void_p(16), 10, C.c_void_p(16), None, 10,
                          C.c_void_p(16), C.c_void_p(16), None, C.c_void_p(16), 1 << 30, None)
    assert st == -1 and "weights" in L.last_error()
    h = C.c_void_p()
    b = L.kbins(0.01, 0.01, 5)
    st = L.lib.cnpc_bispec_plan_create(C.byref(h), C.byref(d), C.byref(b), L.EST_SCOCCIMARRO, 0,
                                       L.PREC_F32, C.c_void_p(16), 1 << 20, None)
    assert st == -1 and "k = 0" in L.last_error()
    b = L.kbins(0.0, 0.01, 5)
    st = L.lib.cnpc_bispec_plan_create(C.byref(h), C.byref(d), C.byref(b), L.EST_SCOCCIMARRO, 0,
                                       L.PREC_F64, C.c_void_p(16), 1 << 20, None)
    assert st == -1 and "FP64" in L.last_error()
    assert L.lib.cnpc_paint_workspace_size(C.byref(d), 1000, 10000) > 0
    assert L.lib.cnpc_bispec_workspace_size(C.byref(d), C.byref(b), 0, 0) > 0
