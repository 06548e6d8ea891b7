"""Host-side checks of the C ABI library that need no GPU: it loads, it
exports every function the public headers declare, and argument errors are
reported before any device work."""
import ctypes
import os
import re

import pytest

from paper_2108_11932_amd import tlr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("tlr.h", "tlr_kernels.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(tlrk?_[a-z_0-9]+)\s*\(", src))
    return names


def test_library_loads_and_exports_every_declared_symbol():
    l = tlr.lib()
    declared = _declared()
    assert "tlr_potrf" in declared and "tlrk_ara" in declared
    for name in sorted(declared):
        assert hasattr(l, name), name
    # and the binding wraps exactly the declared functions
    assert declared == set(tlr.SIGNATURES)


def test_default_options():
    o = tlr.opts()
    assert (o.bs, o.eps_mode, o.precision, o.shift, o.max_active, o.r_min) == (16, 0, 0, 0.0, 0, 0)


@pytest.mark.parametrize("n,m", [(0, 16), (-5, 16), (100, 0), (100, -1), (100, 100000)])
def test_create_rejects_bad_sizes(n, m):
    h = ctypes.c_void_p()
    st = tlr.lib().tlr_create(n, m, None, None, None, ctypes.byref(h))
    assert st == tlr.TLR_ERR_ARG
    assert h.value is None
    assert tlr.lib().tlr_last_error()


def test_null_handles_are_argument_errors():
    l = tlr.lib()
    o = tlr.opts()
    st = tlr.Stats()
    assert l.tlr_potrf(None, 1e-6, ctypes.byref(o), ctypes.byref(st), None) == tlr.TLR_ERR_ARG
    assert l.tlr_ldlt(None, 1e-6, ctypes.byref(o), None, ctypes.byref(st), None) == tlr.TLR_ERR_ARG
    assert l.tlr_solve(None, 1, None, 10, None) == tlr.TLR_ERR_ARG
    assert l.tlr_matvec(None, 1, None, 10, None, 10, None) == tlr.TLR_ERR_ARG
    assert l.tlr_destroy(None) == tlr.TLR_OK


def test_compress_rejects_bad_threshold_and_options():
    l = tlr.lib()
    h = ctypes.c_void_p()
    o = tlr.opts()
    fake = ctypes.c_void_p(16)
    assert l.tlr_compress(fake, 10, 10, 4, 0.0, ctypes.byref(o), None, None,
                          ctypes.byref(h)) == tlr.TLR_ERR_ARG
    assert l.tlr_compress(fake, 5, 10, 4, 1e-3, ctypes.byref(o), None, None,
                          ctypes.byref(h)) == tlr.TLR_ERR_ARG
    bad = tlr.opts(bs=64)
    assert l.tlr_compress(fake, 10, 10, 4, 1e-3, ctypes.byref(bad), None, None,
                          ctypes.byref(h)) == tlr.TLR_ERR_ARG
    assert b"bs" in l.tlr_last_error()
    assert l.tlr_compress_kernel(fake, 4, 10, 0, 0.1, 0.0, 4, 1e-3, None, None, None,
                                 ctypes.byref(h)) == tlr.TLR_ERR_ARG
    assert l.tlr_compress_kernel(fake, 2, 10, 7, 0.1, 0.0, 4, 1e-3, None, None, None,
                                 ctypes.byref(h)) == tlr.TLR_ERR_ARG


def test_kernel_entry_points_check_arguments():
    l = tlr.lib()
    info = ctypes.c_int()
    assert l.tlrk_potrf(0, None, 1, ctypes.byref(info), None) == tlr.TLR_ERR_ARG
    assert l.tlrk_trsm(4, 2, None, 4, None, 4, 0, 0, None) == tlr.TLR_ERR_ARG
    p = (tlr.GemmProblem * 1)(tlr.GemmProblem(4, 4, 4, 16, 2, 16, 4, 16, 4, 1.0, 0.0))
    assert l.tlrk_gemm_batched(0, 0, 1, p, None) == tlr.TLR_ERR_ARG
    r = ctypes.c_int()
    assert l.tlrk_ara(8, 1, ctypes.c_void_p(16), 0.0, 16, 1, 1, ctypes.c_void_p(16),
                      ctypes.c_void_p(16), ctypes.byref(r), ctypes.byref(r), None) == tlr.TLR_ERR_ARG
