"""The C-ABI library loads and exports every symbol the header declares;
host-side argument validation works without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "adc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(adc_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_2012_06714_amd as adc
    declared = _header_symbols()
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(adc.lib, name), name
    assert set(declared) == set(adc.ABI_SYMBOLS)


def test_host_validation_without_gpu():
    import paper_2012_06714_amd as adc
    lib = adc.lib
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(8)
    assert lib.adc_setup(None, dummy, 2, 3, 4, 2, 1, ctypes.byref(h)) == adc.ADC_E_ARG
    assert "NULL" in adc.last_error()
    assert lib.adc_setup(dummy, dummy, 0, 3, 4, 2, 1, ctypes.byref(h)) == adc.ADC_E_ARG
    assert lib.adc_setup(dummy, dummy, 2, 3, 4, 4, 1, ctypes.byref(h)) == adc.ADC_E_ARG
    assert "order" in adc.last_error()
    assert lib.adc_setup(dummy, dummy, 2, 3, 4, 3, 7, ctypes.byref(h)) == adc.ADC_E_ARG
    assert lib.adc_setup(dummy, dummy, 2, 3, 4, 3, 1, None) == adc.ADC_E_ARG
    assert lib.adc_set_option(None, b"tol_e", 1e-8) == adc.ADC_E_ARG
    assert lib.adc_sigma(None, dummy, dummy, 1) == adc.ADC_E_ARG
    assert lib.adc_davidson(None, 1, None, None, None, None) == adc.ADC_E_ARG
    assert lib.adc_dim(None) == -1
    used, peak = ctypes.c_longlong(-7), ctypes.c_longlong(-7)
    assert lib.adc_workspace(None, ctypes.byref(used), ctypes.byref(peak)) == adc.ADC_E_ARG
    assert used.value == -7 and peak.value == -7
    arr = (ctypes.c_void_p * 1)(8)
    e = (ctypes.c_double * 1)()
    # flag bits outside graph/concurrent/stats/thread count, and more than 64 threads
    assert lib.adc_batch_davidson(arr, 1, 1, 8, e, None, None, None, None) == adc.ADC_E_ARG
    assert lib.adc_batch_davidson(arr, 1, 1, 1 << 16, e, None, None, None, None) == adc.ADC_E_ARG
    assert lib.adc_batch_davidson(arr, 1, 1, 2 | (65 << 8), e, None, None, None, None) == adc.ADC_E_ARG
    lib.adc_destroy(None)
    # the unrestricted setup: argument checks before any device work
    su = lib.adc_setup_u
    assert su(None, dummy, dummy, dummy, 2, 1, 6, 4, 2, 1, ctypes.byref(h)) == adc.ADC_E_ARG
    assert su(dummy, dummy, dummy, dummy, 2, 1, 6, 4, 3, 1, ctypes.byref(h)) == adc.ADC_E_ARG
    assert "order 2" in adc.last_error()
    assert su(dummy, dummy, dummy, dummy, 6, 1, 6, 4, 2, 1, ctypes.byref(h)) == adc.ADC_E_ARG
    assert su(dummy, dummy, dummy, dummy, 2, 0, 6, 4, 2, 1, ctypes.byref(h)) == adc.ADC_E_ARG
    assert su(dummy, dummy, dummy, dummy, 2, 1, 6, 4, 2, 5, ctypes.byref(h)) == adc.ADC_E_ARG
    assert su(dummy, dummy, dummy, dummy, 2, 1, 6, 4, 2, 1, None) == adc.ADC_E_ARG
    # the batch object: argument checks before any device work
    assert lib.adc_setup_batch(1, None, ctypes.byref(h)) == adc.ADC_E_ARG
    assert lib.adc_setup_batch(0, dummy, ctypes.byref(h)) == adc.ADC_E_ARG
    assert lib.adc_setup_batch(1, dummy, None) == adc.ADC_E_ARG
    desc = adc._SystemDesc(None, 8, 2, 3, 4, 2, 1)
    assert lib.adc_setup_batch(1, ctypes.byref(desc), ctypes.byref(h)) == adc.ADC_E_ARG
    assert "system 0" in adc.last_error() and "NULL" in adc.last_error()
    assert h.value is None
    assert lib.adc_davidson_batch(None, 1, 0, e, None, None, None, None) == adc.ADC_E_ARG
    assert lib.adc_batch_set_option(None, b"tol_e", 1e-8) == adc.ADC_E_ARG
    assert lib.adc_batch_context(None, 0) is None
    lib.adc_batch_destroy(None)


def test_gemm_configs_and_argument_checks_without_gpu():
    """The tile configurations each product type offers (a static list), and
    adc_gemm's argument checks, which run before any device work."""
    import paper_2012_06714_amd as adc
    lib = adc.lib
    ids = (ctypes.c_int * 8)()
    assert lib.adc_gemm_configs(4, ids) == adc.ADC_E_ARG
    assert lib.adc_gemm_configs(0, None) == adc.ADC_E_ARG
    got = {}
    for dtype in range(4):
        n = lib.adc_gemm_configs(dtype, ids)
        assert 1 <= n <= 8
        got[dtype] = [ids[k] for k in range(n)]
    assert got[0] == [0, 2, 3] and got[1] == [0, 1, 2]
    # BF16 products: the LDS-DMA tile (8) beside the register-staged ones
    assert got[2] == got[3] == [0, 1, 6, 7, 8]
    dummy = ctypes.c_void_p(256)
    g = lib.adc_gemm
    ll = ctypes.c_longlong
    args = lambda **kw: dict(dict(dtype=3, ta=0, tb=1, M=ll(4), N=ll(4), K=ll(8), alpha=1.0,
                                  A=dummy, lda=ll(8), B=dummy, ldb=ll(8), beta=0.0, C=dummy,
                                  ldc=ll(4), map=None, config=-1, stream=None), **kw)
    call = lambda **kw: g(*args(**kw).values())
    assert call(config=9) == adc.ADC_E_ARG and "config" in adc.last_error()
    assert call(config=-2) == adc.ADC_E_ARG
    assert call(dtype=4) == adc.ADC_E_ARG
    assert call(M=ll(0)) == adc.ADC_E_ARG
    assert call(A=None) == adc.ADC_E_ARG
    assert call(lda=ll(7)) == adc.ADC_E_ARG and "leading" in adc.last_error()
    assert call(ldc=ll(3)) == adc.ADC_E_ARG
