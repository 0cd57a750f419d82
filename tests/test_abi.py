"""The C interface: the built library loads and exports every declared entry point.

No GPU call is made here (host-only functions only).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "asjoin.h")
LIB = os.path.join(ROOT, "paper_2411_18183_amd", "libasjoin.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(asj_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2411_18183_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("asj_signature", "asj_build", "asj_probe", "asj_join", "asj_table_free", "asj_strerror",
                     "asj_table_status"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_is_host_only_and_total(lib):
    lib.asj_strerror.restype = ctypes.c_char_p
    lib.asj_strerror.argtypes = [ctypes.c_int]
    assert lib.asj_strerror(0) == b"ok"
    for code in range(-1, -8, -1):
        assert lib.asj_strerror(code)


def test_invalid_arguments_are_rejected_before_any_device_work(lib):
    lib.asj_signature.restype = ctypes.c_int
    # NULL keys -> ASJ_EINVAL without touching the device
    assert lib.asj_signature(None, ctypes.c_uint64(0), None, None) == -1
    lib.asj_table_free.restype = ctypes.c_int
    assert lib.asj_table_free(None) == 0
    lib.asj_table_capacity.restype = ctypes.c_int64
    assert lib.asj_table_capacity(None) == -1
    lib.asj_autotune.restype = ctypes.c_int
    assert lib.asj_autotune(None, None, None, None, ctypes.c_int64(0), None, None, None) == -1
    lib.asj_autotune_batch.restype = ctypes.c_int
    assert lib.asj_autotune_batch(None, None, None, None) == -1
    lib.asj_autotune_clear.restype = None
    lib.asj_autotune_clear()
