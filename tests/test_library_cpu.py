"""The C-ABI library loads on the CPU host and exports what include/sts.h declares.

No compute call is made here (there is no GPU in this container); only calls
that are pure host logic (sizes, argument checks, error strings) run.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sts.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sts_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2607_07816_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2607_07816_amd import build
        build.build(verbose=False)
    return _lib.load()


def test_header_declares_the_core_calls():
    syms = declared_symbols()
    for s in ("sts_init", "sts_apply_gate", "sts_truncate", "sts_peak"):
        assert s in syms


def test_every_declared_symbol_is_exported(lib):
    from paper_2607_07816_amd import _lib
    syms = declared_symbols()
    assert set(syms) == set(_lib.EXPORTS)
    for s in syms:
        assert hasattr(lib, s), s


def test_strerror_and_sizes(lib):
    from paper_2607_07816_amd import _lib
    assert _lib.strerror(0) == "ok"
    assert "capacity" in _lib.strerror(-3)
    b128 = _lib.required_bytes(1 << 20, _lib.STS_C128)
    b64 = _lib.required_bytes(1 << 20, _lib.STS_C64)
    # three term buffers and the side buffer dominate
    assert b128 - b64 >= 3 * 8 * (1 << 20)
    assert b64 >= (3 * 16 + 4 * 16) * (1 << 20)
    with pytest.raises(_lib.StsError):
        _lib.required_bytes(0, _lib.STS_C64)


def test_init_rejects_bad_arguments_before_any_device_work(lib):
    ctx = ctypes.c_void_p(0)
    for n, prec in ((0, 0), (65, 0), (10, 7)):
        rc = lib.sts_init(ctypes.byref(ctx), n, 16, 0.0, prec, None, None, 0, 0)
        assert rc == -1 and not ctx.value
    # K larger than the capacity asked for (and below 2^n, so it can cut)
    rc = lib.sts_init(ctypes.byref(ctx), 30, 1 << 20, 0.0, 0, None, None, 0, 1024)
    assert rc == -3 and not ctx.value


def test_calls_on_null_context_fail_cleanly(lib):
    u = (ctypes.c_double * 8)()
    q = (ctypes.c_int * 1)(0)
    assert lib.sts_apply_gate(None, 1, q, u) == -1
    assert lib.sts_truncate(None) == -1
    lib.sts_free(None)


def test_batch_rejects_bad_config_without_running(lib):
    import ctypes

    from paper_2607_07816_amd import _lib
    res = (_lib.CircuitResult * 1)()
    circ = (_lib.Circuit * 1)()
    m = (ctypes.c_int * 1)(2)
    q = (ctypes.c_int * 2)(0, 1)
    u = (ctypes.c_double * 32)()
    t = (ctypes.c_uint8 * 1)(1)
    circ[0] = _lib.Circuit(4, 16, 0.0, 1, ctypes.addressof(m), ctypes.addressof(q), ctypes.addressof(u),
                           ctypes.addressof(t))
    for cfg in (_lib.BatchConfig(_lib.STS_C64, 0, 0), _lib.BatchConfig(_lib.STS_C64, 65, 0),
                _lib.BatchConfig(7, 2, 0), _lib.BatchConfig(_lib.STS_C64, 2, -1)):
        assert lib.sts_batch_run(1, circ, ctypes.byref(cfg), res) == _lib.STS_E_ARG
    # a gate of 6 qubits, or 0 qubits, is refused before anything runs
    for bad in (6, 0):
        m[0] = bad
        assert lib.sts_batch_run(1, circ, ctypes.byref(_lib.BatchConfig(_lib.STS_C64, 2, 0)), res) == _lib.STS_E_ARG
    assert lib.sts_batch_run(0, None, ctypes.byref(_lib.BatchConfig(_lib.STS_C64, 2, 0)), None) == _lib.STS_OK


def test_server_rejects_bad_config_without_running(lib):
    import ctypes

    from paper_2607_07816_amd import _lib
    h = ctypes.c_void_p(0)
    for cfg in (_lib.ServerConfig(_lib.STS_C64, 0, 1, 1, 0), _lib.ServerConfig(_lib.STS_C64, 1, 0, 1, 0),
                _lib.ServerConfig(_lib.STS_C64, 1, 1, 0, 0), _lib.ServerConfig(9, 1, 1, 1, 0),
                _lib.ServerConfig(_lib.STS_C64, 65, 1, 1, 0)):
        assert lib.sts_server_create(ctypes.byref(h), ctypes.byref(cfg)) == _lib.STS_E_ARG and not h.value
    lib.sts_server_destroy(None)  # NULL is a no-op
