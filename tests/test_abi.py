"""The C-ABI library loads and exports every entry point include/acr.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

import paper_1701_00182_amd as acr

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "acr.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(acr_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = _declared()
    for n in ("acr_factor", "acr_solve", "acr_solve_transpose", "acr_free"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = acr.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def _opts(**kw):
    o = acr.Options()
    acr.lib().acr_options_default(ctypes.byref(o))
    o.nx, o.ny, o.nplanes, o.leaf = 4, 4, 4, 4
    for k, v in kw.items():
        setattr(o, k, v)
    return o


@pytest.mark.parametrize("kw", [dict(nx=0), dict(ny=-1), dict(nplanes=0), dict(leaf=0), dict(eps=-1.0),
                                dict(eps=float("nan")), dict(max_rank=-2), dict(precision=9),
                                dict(stencil_points=9), dict(stencil_points=-1), dict(gemm_tiles=2),
                                dict(gemm_tiles=-1)])
def test_invalid_options_rejected_before_device_work(kw):
    L = acr.lib()
    h = ctypes.c_void_p(123)
    code = L.acr_factor(ctypes.byref(_opts(**kw)), ctypes.c_void_p(16), None, ctypes.byref(h))
    assert code == 1 and not h.value


def test_release_cached_memory_without_device_work():
    # nothing was allocated in this process: the cache is empty
    assert acr.release_cached_memory() == 0


def test_null_arguments_rejected():
    L = acr.lib()
    h = ctypes.c_void_p()
    assert L.acr_factor(ctypes.byref(_opts()), None, None, ctypes.byref(h)) == 1
    assert L.acr_solve(None, 1, None, 0, None, 0, None) == 1
    assert L.acr_solve_transpose(None, 1, None, 0, None, 0, None) == 1
    L.acr_free(None)
    assert L.acr_status_string(0) == b"success"
    r = acr.TuneResult()
    assert L.acr_autotune(None, ctypes.c_void_p(16), 8, None, None, ctypes.byref(r)) == 1
    assert L.acr_autotune(ctypes.byref(_opts()), None, 8, None, None, ctypes.byref(r)) == 1
    assert L.acr_autotune(ctypes.byref(_opts()), ctypes.c_void_p(16), -1, None, None, ctypes.byref(r)) == 1
    assert L.acr_autotune(ctypes.byref(_opts()), ctypes.c_void_p(16), 8, None, None, None) == 1
