"""Host-side checks of the C-ABI library: it loads, exports every function
include/ngd.h declares, and rejects invalid arguments before any device
work (these calls never reach the GPU)."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2405_20067_amd import ngd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ngd.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(ngd_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ngd.LIB_PATH):
        pytest.fail("libngd.so is not built (python -m paper_2405_20067_amd.build)")
    return ngd.lib()


def test_header_and_binding_agree():
    assert _declared() == sorted(ngd.EXPORTED)


def test_library_exports_every_declared_symbol(L):
    out = subprocess.run(["nm", "-D", "--defined-only", ngd.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [s for s in _declared() if s not in syms]
    assert not missing, missing
    for name in _declared():
        assert hasattr(L, name)


def test_version_and_defaults(L):
    assert L.ngd_version() == 10000
    p = ngd.CullParams()
    assert L.ngd_cull_params_default(ctypes.byref(p)) == 0
    assert (p.n_proj, p.tile, p.key_proj, p.key_bits) == (16, 256, 16, 2)
    assert p.tau == pytest.approx(1e-4)
    assert L.ngd_cull_params_default(None) == ngd.E_INVAL
    assert b"NULL" in L.ngd_last_error()


@pytest.mark.parametrize("n,k", [(0, 10), (13, 10), (-1, 10), (4, -1), (4, 1 << 31)])
def test_mixture_create_rejects_bad_sizes(L, n, k):
    h = ctypes.c_void_p(1234)
    assert L.ngd_mixture_create(n, k, ctypes.byref(h)) == ngd.E_INVAL
    assert h.value is None
    assert L.ngd_last_error().startswith(b"ngd_mixture_create")
    assert L.ngd_mixture_create(4, 10, None) == ngd.E_INVAL


def test_null_handles_are_rejected(L):
    assert L.ngd_mixture_update(None, None, None, None, None, None) == ngd.E_INVAL
    assert L.ngd_mixture_validate(None, None) == ngd.E_INVAL
    assert L.ngd_mixture_info(None, None, None, None) == ngd.E_INVAL
    assert L.ngd_mixture_destroy(None) == 0
    assert L.ngd_cull_destroy(None) == 0
    assert L.ngd_cull_stats(None, None, None, None) == ngd.E_INVAL
    assert L.ngd_cull_export(None, *([None] * 8)) == ngd.E_INVAL
    assert L.ngd_eval(None, None, None, 0, 0, None, None) == ngd.E_INVAL
    assert L.ngd_eval_backward(None, None, None, 0, None, 0, *([None] * 5)) == ngd.E_INVAL
    h = ctypes.c_void_p()
    p = ngd.CullParams()
    L.ngd_cull_params_default(ctypes.byref(p))
    assert L.ngd_cull_build(None, None, 0, ctypes.byref(p), None, None,
                            ctypes.byref(h)) == ngd.E_INVAL


def test_l2_loss_argument_checks(L):
    assert L.ngd_l2_loss(None, None, -1, None, None, None) == ngd.E_INVAL
    assert L.ngd_l2_loss(None, None, 5, ctypes.c_void_p(16), None, None) == ngd.E_INVAL
    assert L.ngd_l2_loss(ctypes.c_void_p(2), ctypes.c_void_p(16), 5, ctypes.c_void_p(16),
                         ctypes.c_void_p(16), None) == ngd.E_INVAL   # misaligned


def test_l2_loss_noalloc_argument_checks(L):
    one = ctypes.c_void_p(16)
    assert L.ngd_l2_loss_noalloc(None, None, -1, one, one, None) == ngd.E_INVAL
    assert L.ngd_l2_loss_noalloc(one, one, 1 << 31, one, one, None) == ngd.E_INVAL
    assert b"outside" in L.ngd_last_error()
    assert L.ngd_l2_loss_noalloc(None, None, 5, one, None, None) == ngd.E_INVAL
    assert L.ngd_l2_loss_noalloc(ctypes.c_void_p(2), one, 5, one, one,
                                 None) == ngd.E_INVAL   # misaligned


def test_rel_l2_loss_argument_checks(L):
    one = ctypes.c_void_p(16)
    for eps in (0.0, -0.01, float("nan"), float("inf")):
        assert L.ngd_rel_l2_loss(one, one, 5, eps, one, one, None) == ngd.E_INVAL
    assert L.ngd_rel_l2_loss(None, None, -1, 0.01, None, None, None) == ngd.E_INVAL
    assert L.ngd_rel_l2_loss(None, None, 5, 0.01, one, None, None) == ngd.E_INVAL
    assert L.ngd_rel_l2_loss(ctypes.c_void_p(2), one, 5, 0.01, one, one,
                             None) == ngd.E_INVAL   # misaligned


def test_allocator_failure_is_reported_as_nomem(L):
    calls = []

    @ngd.ALLOC_FN
    def failing_alloc(nbytes, ctx):
        calls.append(nbytes)
        return None

    @ngd.FREE_FN
    def never_free(ptr, ctx):
        raise AssertionError("nothing was allocated")

    assert L.ngd_set_allocator(failing_alloc, never_free, None) == 0
    try:
        h = ctypes.c_void_p()
        assert L.ngd_mixture_create(10, 1000, ctypes.byref(h)) == ngd.E_NOMEM
        assert h.value is None
        assert calls and calls[0] >= 1000 * 72 * 4
        assert b"allocation" in L.ngd_last_error()
    finally:
        assert L.ngd_set_allocator(ngd.ALLOC_FN(), ngd.FREE_FN(), None) == 0


def test_allocator_misaligned_memory_is_returned_and_reported(L):
    """A workspace pointer not aligned to 256 bytes is handed back to the
    allocator's free at once (never used: the value below is no real
    allocation) and the call fails with NGD_E_NOMEM."""
    freed = []

    @ngd.ALLOC_FN
    def misaligned_alloc(nbytes, ctx):
        return 0x10010

    @ngd.FREE_FN
    def record_free(ptr, ctx):
        freed.append(ptr)

    assert L.ngd_set_allocator(misaligned_alloc, record_free, None) == 0
    try:
        h = ctypes.c_void_p()
        assert L.ngd_mixture_create(4, 100, ctypes.byref(h)) == ngd.E_NOMEM
        assert h.value is None
        assert freed and all(f == 0x10010 for f in freed)
    finally:
        assert L.ngd_set_allocator(ngd.ALLOC_FN(), ngd.FREE_FN(), None) == 0


def test_allocator_must_be_given_in_pairs(L):
    @ngd.ALLOC_FN
    def a(nbytes, ctx):
        return None

    assert L.ngd_set_allocator(a, ngd.FREE_FN(), None) == ngd.E_INVAL


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(ngd, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(ngd, "_lib", None)
    with pytest.raises(ImportError):
        ngd.lib()
