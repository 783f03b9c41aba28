"""The C-ABI library loads and exports every declared entry point; argument
errors are reported before any device work (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

from paper_2304_08232_amd import mgpcg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+char\s*\*|mgpcg_status)\s*(mgpcg_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    L = C.CDLL(mgpcg.LIB_PATH)
    decl = declared_functions()
    assert len(decl) >= 15
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(mgpcg.ABI_FUNCTIONS) == decl


def _cfg(dims, levels=4, nrhs=1, dtype=0, order=0, smoother=0, sweeps=0):
    flat = [v for d in dims for v in d]
    arr = (C.c_int * len(flat))(*flat)
    cfg = mgpcg._Config(len(dims), arr, levels, nrhs, dtype, order, None, smoother, sweeps)
    cfg._keep = arr
    return cfg


def test_argument_errors_without_device():
    L = mgpcg.lib()
    h = C.c_void_p()
    assert L.mgpcg_create(None, None, C.byref(h)) == -1
    assert L.mgpcg_create(C.byref(_cfg([(16, 16, 16)])), None, None) == -1
    assert L.mgpcg_create(C.byref(_cfg([(12, 16, 16)])), None, C.byref(h)) == -2  # 12 % 8 != 0
    assert b"not divisible" in L.mgpcg_last_error()
    assert L.mgpcg_create(C.byref(_cfg([(0, 16, 16)], levels=1)), None, C.byref(h)) == -2
    assert L.mgpcg_create(C.byref(_cfg([(16, 16, 16)], levels=9)), None, C.byref(h)) == -2
    assert L.mgpcg_create(C.byref(_cfg([(16, 16, 16)], nrhs=3)), None, C.byref(h)) == -1
    assert L.mgpcg_create(C.byref(_cfg([(16, 16, 16)], smoother=2)), None, C.byref(h)) == -1
    # the sequential smoother: FP64 V-cycle and one right-hand side only
    assert L.mgpcg_create(C.byref(_cfg([(16, 16, 16)], dtype=1, smoother=1)), None, C.byref(h)) == -1
    assert L.mgpcg_create(C.byref(_cfg([(16, 16, 16)], nrhs=2, smoother=1)), None, C.byref(h)) == -1
    assert b"sequential smoother" in L.mgpcg_last_error()
    # the 32-bit row-index limit: 27 n < 2^31
    assert L.mgpcg_create(C.byref(_cfg([(448, 448, 448)], levels=1)), None, C.byref(h)) == -2
    assert b"too large" in L.mgpcg_last_error()
    assert L.mgpcg_create(C.byref(_cfg([(16, 16, 16)], sweeps=-1)), None, C.byref(h)) == -1
    assert L.mgpcg_create(C.byref(_cfg([(16, 16, 16)], sweeps=17)), None, C.byref(h)) == -1
    assert b"sweeps" in L.mgpcg_last_error()
    assert L.mgpcg_create(C.byref(_cfg([(16, 16, 16)], dtype=2)), None, C.byref(h)) == -1
    assert L.mgpcg_create(C.byref(_cfg([(16, 16, 16)], order=2)), None, C.byref(h)) == -1
    assert h.value is None
    # NULL handles
    assert L.mgpcg_destroy(None) == 0
    n = C.c_int64()
    assert L.mgpcg_info(None, 0, C.byref(n), None, None) == -1
    assert L.mgpcg_spmv(None, 0, None, None, 0, None) == -1
    assert L.mgpcg_colour_pass(None, 0, 0, None, None, 0, None) == -1
    assert L.mgpcg_pcg_solve(None, None, None, 10, C.c_double(0.0), None, None, 0, None) == -1
    sch = mgpcg._Schedule()
    assert L.mgpcg_get_schedule(None, C.byref(sch)) == -1
    assert L.mgpcg_set_schedule(None, C.byref(sch), None) == -1
    assert L.mgpcg_autotune(None, None, 10, 3, None, C.byref(sch), None) == -1
    assert L.mgpcg_last_error()


@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="a GPU device is present")
def test_no_device_reported():
    L = mgpcg.lib()
    h = C.c_void_p()
    assert L.mgpcg_create(C.byref(_cfg([(16, 16, 16)])), None, C.byref(h)) == -6
