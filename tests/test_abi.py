"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every function include/ldq.h declares; argument errors are reported, not crashed."""
import ctypes

import pytest

from paper_1105_5256_amd import ldq


def test_library_exports_every_declared_function():
    lib = ldq.load()
    names = ldq.header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(ldq._SIGNATURES) == set(names)


def test_status_strings_and_defaults():
    lib = ldq.load()
    assert lib.ldq_status_string(0) == b"LDQ_OK"
    assert lib.ldq_status_string(2) == b"LDQ_E_NOT_SPD"
    assert lib.ldq_status_string(99) == b"LDQ_E_UNKNOWN"
    o = ldq.ldq_options_default()
    assert (o.k, o.nshifts, o.tol, o.max_iter, o.precision) == (2, 20, 1e-10, 100000, ldq.LDQ_FP64)


def test_null_arguments_are_rejected():
    lib = ldq.load()
    assert lib.ldq_create(0, None, None) == ldq.LDQ_E_INVALID
    assert lib.ldq_op_lattice(None, 2, None, 1, 0.1, None, 1.0, 0, None) == ldq.LDQ_E_INVALID
    assert lib.ldq_logdet(None, None, None, None, None) == ldq.LDQ_E_INVALID
    assert b"NULL" in lib.ldq_last_error()
    lib.ldq_destroy(None)
    lib.ldq_op_destroy(None)


def test_create_without_device_fails_cleanly():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    h = ctypes.c_void_p()
    assert ldq.load().ldq_create(0, None, ctypes.byref(h)) == ldq.LDQ_E_DEVICE
