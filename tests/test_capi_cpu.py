"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every entry point the public header declares; argument validation
that happens before any device work."""
import ctypes
import os
import re

import pytest

from paper_1305_5120_amd import chfsi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chfsi.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(chfsi_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("chfsi_create", "chfsi_reduce", "chfsi_solve", "chfsi_release", "chfsi_last_error",
                     "chfsi_filter", "chfsi_qr", "chfsi_eigh", "chfsi_rayleigh_ritz", "chfsi_residuals",
                     "chfsi_lanczos"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(chfsi.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_defaults():
    lib = chfsi.load()
    assert lib.chfsi_status_string(0) == b"CHFSI_OK"
    assert lib.chfsi_status_string(-3) == b"CHFSI_ENOCONV"
    o = chfsi.default_opts()
    assert (o.degree, o.max_iter, o.lanczos_steps, o.precision) == (20, 1000, 10, 0)


def test_create_rejects_bad_arguments_before_touching_the_device():
    lib = chfsi.load()
    h = ctypes.c_void_p()
    o = chfsi.default_opts()
    assert lib.chfsi_create(ctypes.byref(h), 0, ctypes.byref(o), None) == -1
    o.degree = 0
    assert lib.chfsi_create(ctypes.byref(h), 10, ctypes.byref(o), None) == -1
    o = chfsi.default_opts(precision=7)
    assert lib.chfsi_create(ctypes.byref(h), 10, ctypes.byref(o), None) == -1
    o = chfsi.default_opts(lanczos_steps=500)
    assert lib.chfsi_create(ctypes.byref(h), 10, ctypes.byref(o), None) == -1
    for bad in (-1, 13):
        o = chfsi.default_opts(mixed_switch_digits=bad)
        assert lib.chfsi_create(ctypes.byref(h), 10, ctypes.byref(o), None) == -1
    assert lib.chfsi_create(None, 10, None, None) == -1
    lib.chfsi_release(None)  # NULL-safe


def test_null_context_is_rejected():
    lib = chfsi.load()
    assert lib.chfsi_solve(None, None, 0, None, 0, 1, 0, None, 0, 0, 1e-10, None, None, 0, None) == -1
    assert lib.chfsi_last_error(None) == b"null context"


def test_solve_argument_validation_without_device_work():
    """Invalid sizes fail before any allocation or launch."""
    lib = chfsi.load()
    h = ctypes.c_void_p()
    o = chfsi.default_opts()
    assert lib.chfsi_create(ctypes.byref(h), 16, ctypes.byref(o), None) == 0
    try:
        ev = (ctypes.c_double * 16)()
        fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
        # nev + nex > n
        assert lib.chfsi_solve(h, fake, 16, fake, 16, 10, 10, None, 16, 0, 1e-10, ev, None, 16, None) == -1
        assert b"nev" in lib.chfsi_last_error(h)
        # no extra column while the block is not the whole space
        assert lib.chfsi_solve(h, fake, 16, fake, 16, 4, 0, None, 16, 0, 1e-10, ev, None, 16, None) == -1
        assert b"nex >= 1" in lib.chfsi_last_error(h)
        # tol <= 0
        assert lib.chfsi_solve(h, fake, 16, fake, 16, 4, 2, None, 16, 0, 0.0, ev, None, 16, None) == -1
        # leading dimension too small
        assert lib.chfsi_solve(h, fake, 8, fake, 16, 4, 2, None, 16, 0, 1e-10, ev, None, 16, None) == -1
        # null H
        assert lib.chfsi_solve(h, None, 16, fake, 16, 4, 2, None, 16, 0, 1e-10, ev, None, 16, None) == -1
        # kw > k
        assert lib.chfsi_solve(h, fake, 16, fake, 16, 4, 2, fake, 16, 9, 1e-10, ev, None, 16, None) == -1
        # a later valid-argument error message replaces the earlier one
        assert lib.chfsi_filter(h, fake, 16, fake, 16, 3, 5, 2.0, 1.0, 0.0) == -1
        assert b"b > a" in lib.chfsi_last_error(h)
        assert lib.chfsi_zgemm(h, 2, 0, 1, 1, 1, 1.0, fake, 1, fake, 1, 0.0, None, 1, 0.0, None, 1, fake, 1, 0) == -1
    finally:
        lib.chfsi_release(h)


def test_static_gemm_validation_without_device_work():
    """The allocation-free GEMM rejects bad arguments, and an explicit K
    split whose partial tiles exceed its fixed scratch, before touching the
    device; its message is the thread's context-free error."""
    lib = chfsi.load()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    assert lib.chfsi_zgemm_static(None, 2, 0, 1, 1, 1, 1.0, fake, 1, fake, 1, 0.0, None, 1, 0.0, None, 1, fake, 1,
                                  0) == -1
    assert b"bad sizes" in lib.chfsi_last_error(None)
    M = N = 2000  # two splits of 2000 x 2000 complex numbers: 128 MB > 64 MiB
    assert lib.chfsi_zgemm_static(None, 0, 0, M, N, 64, 1.0, fake, M, fake, 64, 0.0, None, M, 0.0, None, M, fake, M,
                                  (1 << 8) | (2 << 16)) == -1
    assert b"static scratch" in lib.chfsi_last_error(None)
    assert lib.chfsi_zgemm_static(None, 0, 0, M, N, 64, 1.0, fake, M - 1, fake, 64, 0.0, None, M, 0.0, None, M, fake,
                                  M, 0) == -1
    assert b"lda" in lib.chfsi_last_error(None)
    # an empty product succeeds without work and clears the message
    assert lib.chfsi_zgemm_static(None, 0, 0, 0, 5, 5, 1.0, None, 1, None, 1, 0.0, None, 1, 0.0, None, 1, None, 1,
                                  0) == 0
    assert lib.chfsi_last_error(None) == b"null context"


def test_batch_create_and_solve_validation_without_device_work():
    """Batch creation rejects bad member counts, sizes and tile shapes before
    any device call; a null batch is rejected by every entry point."""
    lib = chfsi.load()
    chfsi._load_batch(lib)
    h = ctypes.c_void_p()
    o = chfsi.default_opts()
    sizes = (ctypes.c_int64 * 2)(64, 80)
    assert lib.chfsi_batch_create(None, 2, sizes, ctypes.byref(o), 0) == -1
    assert lib.chfsi_batch_create(ctypes.byref(h), 0, sizes, ctypes.byref(o), 0) == -1
    assert lib.chfsi_batch_create(ctypes.byref(h), 2, None, ctypes.byref(o), 0) == -1
    assert lib.chfsi_batch_create(ctypes.byref(h), 2, sizes, ctypes.byref(o), 2) == -1
    bad = (ctypes.c_int64 * 2)(64, 0)
    assert lib.chfsi_batch_create(ctypes.byref(h), 2, bad, ctypes.byref(o), 0) == -1
    o6 = chfsi.default_opts(filter_tile=6)  # 128 x 128 has no grouped kernel
    assert lib.chfsi_batch_create(ctypes.byref(h), 2, sizes, ctypes.byref(o6), 0) == -1
    assert not h.value
    assert lib.chfsi_batch_solve(None, None, None, None, None, None, None, 1e-10, None, None, None, None, None,
                                 None) == -1
    assert lib.chfsi_batch_reset(None) == -1
    assert lib.chfsi_batch_last_error(None) == b"null batch"
    lib.chfsi_batch_release(None)
