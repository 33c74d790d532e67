"""The C ABI without a GPU: the library loads, exports every function that
include/psvd.h declares, and its host-only calls behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psvd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(psvd_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2108_08845_amd import _lib
    return _lib.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("psvd_initialize", "psvd_incorporate_data", "psvd_singular_values", "psvd_modes",
                 "psvd_apmos_batched", "psvd_rsvd", "psvd_save_state", "psvd_load_state", "psvd_loss_grad",
                 "psvd_stream_backward", "psvd_finalize"):
        assert must in names


def test_library_exports_every_declared_function(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2108_08845_amd import _lib
    assert sorted(_lib.EXPORTS) == declared_functions()


def test_status_strings(lib):
    lib.psvd_status_string.restype = ctypes.c_char_p
    assert lib.psvd_status_string(0) == b"PSVD_OK"
    for code in range(-1, -10, -1):
        s = lib.psvd_status_string(code)
        assert s.startswith(b"PSVD_E_")


def test_default_options(lib):
    from paper_2108_08845_amd import _lib
    o = _lib.Options()
    ctypes.memset(ctypes.byref(o), 0xFF, ctypes.sizeof(o))
    lib.psvd_default_options(ctypes.byref(o))
    assert o.method == _lib.DETERMINISTIC and o.precision == _lib.PREC_FP64
    assert o.seed == 0 and o.stream is None and o.max_sweeps == 60
    assert o.flags == 0 and o.tile_rows == 0 and o.wg_per_cu == 0


def test_invalid_arguments_rejected_before_any_device_work(lib):
    from paper_2108_08845_amd import _lib
    h = ctypes.c_void_p()
    o = _lib.Options()
    lib.psvd_default_options(ctypes.byref(o))
    bad = [
        (0, 5, 1.0, 0, 0),      # M < 1
        (100, 0, 1.0, 0, 0),    # K < 1
        (100, 101, 1.0, 0, 0),  # K > M
        (100, 5, 0.0, 0, 0),    # ff <= 0
        (100, 5, 1.5, 0, 0),    # ff > 1
        (100, 5, 1.0, -1, 0),   # p < 0
        (100, 5, 1.0, 0, -1),   # q < 0
    ]
    for M, K, ff, p, q in bad:
        rc = lib.psvd_initialize(ctypes.byref(h), M, K, ff, p, q, ctypes.byref(o))
        assert rc == _lib.PSVD_E_INVAL, (M, K, ff, p, q)
        assert not h.value
    for field, value in (("tile_rows", 48), ("wg_per_cu", 9), ("precision", 7), ("method", 5)):
        o2 = _lib.Options()
        lib.psvd_default_options(ctypes.byref(o2))
        setattr(o2, field, value)
        rc = lib.psvd_initialize(ctypes.byref(h), 100, 5, 1.0, 0, 0, ctypes.byref(o2))
        assert rc == _lib.PSVD_E_INVAL, field
    # handle-less call: argument errors carry a message for psvd_last_error(NULL)
    rc = lib.psvd_rsvd(None, 10, 10, 10, _lib.PSVD_F32, 3, 2, 1, 0, _lib.PREC_FP32, None, 10, None, 10,
                       _lib.PSVD_F32, None, None, None)
    assert rc == _lib.PSVD_E_INVAL
    assert lib.psvd_last_error(None).startswith(b"PSVD_E_INVAL")
    lib.psvd_finalize(None)


def test_null_handle_calls(lib):
    from paper_2108_08845_amd import _lib
    assert lib.psvd_incorporate_data(None, None, 1, 1, 1, _lib.PSVD_F32) == _lib.PSVD_E_INVAL
    assert lib.psvd_save_state(None, None, 0, None) == _lib.PSVD_E_INVAL
    assert lib.psvd_load_state(None, None, 0) == _lib.PSVD_E_INVAL
