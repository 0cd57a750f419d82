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


class _Keys(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("ids", ctypes.c_void_p),
                ("n", ctypes.c_int64)]


class _Opts(ctypes.Structure):
    _fields_ = [("f", ctypes.c_int32), ("nsym", ctypes.c_int32), ("load_factor", ctypes.c_float),
                ("flags", ctypes.c_uint32), ("keys_per_window", ctypes.c_int32), ("grid_rounds", ctypes.c_int32)]


class _HostOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_int64), ("partitions", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def test_host_join_checks_its_arguments_on_the_host(lib):
    """asj_join_host validates pointers, host offsets, partition counts and flags before any device work."""
    f = lib.asj_join_host
    f.restype = ctypes.c_int
    data = (ctypes.c_uint8 * 8)(*b"abcdefgh")
    good = (ctypes.c_int64 * 3)(0, 4, 8)
    bad = (ctypes.c_int64 * 3)(0, 6, 4)  # decreasing
    cnt = ctypes.c_int64(-7)
    out = (ctypes.c_int32 * 8)()
    R = _Keys(ctypes.cast(data, ctypes.c_void_p), ctypes.cast(good, ctypes.c_void_p), None, 2)
    Sbad = _Keys(ctypes.cast(data, ctypes.c_void_p), ctypes.cast(bad, ctypes.c_void_p), None, 2)
    P = ctypes.byref
    # missing out_count, negative capacity, capacity without a buffer
    assert f(P(R), P(R), None, None, out, ctypes.c_int64(4), None, None, None) == -1
    assert f(P(R), P(R), None, None, out, ctypes.c_int64(-1), P(cnt), None, None) == -1
    assert f(P(R), P(R), None, None, None, ctypes.c_int64(4), P(cnt), None, None) == -1
    # offsets that decrease, a NULL relation
    assert f(P(R), P(Sbad), None, None, out, ctypes.c_int64(4), P(cnt), None, None) == -1
    assert f(None, P(R), None, None, out, ctypes.c_int64(4), P(cnt), None, None) == -1
    # partitions must be 0 or a power of two up to 1024; the budget must not be negative
    for parts, budget in ((3, 0), (2048, 0), (-1, 0), (0, -5)):
        ho = _HostOpts(budget, parts, 0)
        assert f(P(R), P(R), None, P(ho), out, ctypes.c_int64(4), P(cnt), None, None) == -1
    # sorted output is not offered for host joins
    o = _Opts(16, 2, 0.0, 0x10, 0, 0)
    assert f(P(R), P(R), P(o), None, out, ctypes.c_int64(4), P(cnt), None, None) == -6
    assert cnt.value == -7  # never written on a rejected call


def test_header_constants_match_the_binding():
    """Every #define ASJ_* value of the header (flags and status codes) is the
    binding's constant of the same name."""
    from paper_2411_18183_amd import asjoin as A
    text = open(HEADER).read()
    defs = dict(re.findall(r"^#define\s+(ASJ_[A-Z0-9_]+)\s+\(?(-?(?:0x[0-9a-fA-F]+|\d+))u?\)?", text, flags=re.M))
    assert "ASJ_RIGHT_OUTER" in defs and "ASJ_GLOBAL_TABLES" in defs and "ASJ_EINVAL" in defs
    for name, val in defs.items():
        assert hasattr(A, name), name
        assert getattr(A, name) == int(val, 0), name


def test_noalloc_refuses_oversized_build_side_before_device_work(lib):
    """asj_join_noalloc rejects a build side beyond its fixed scratch array
    (and NULL arguments) on the host, before any device call."""
    class Keys(ctypes.Structure):
        _fields_ = [("data", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("ids", ctypes.c_void_p),
                    ("n", ctypes.c_int64)]
    lib.asj_join_noalloc.restype = ctypes.c_int
    dummy = ctypes.c_int64(0)
    r = Keys(None, ctypes.addressof(dummy), None, 10241)  # pointers are never dereferenced
    s = Keys(None, ctypes.addressof(dummy), None, 1)
    cnt = ctypes.c_int64(0)
    assert lib.asj_join_noalloc(ctypes.byref(r), ctypes.byref(s), None, None, ctypes.c_int64(0),
                                ctypes.byref(cnt), None, None) == -1
    assert lib.asj_join_noalloc(None, None, None, None, ctypes.c_int64(0), None, None, None) == -1


def test_batch_workspace_sizing_on_the_host(lib):
    """asj_batch_workspace_bytes is host arithmetic: it grows with the
    relations, refuses bad arguments (-1), and leaves the table-build scratch
    (8 bytes per build row at least) out for ASJ_LOCAL_ONLY batches, whose
    workspace is then too small for the same batch without the flag."""
    lib.asj_batch_workspace_bytes.restype = ctypes.c_int64
    lib.asj_batch_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
    ws = lambda J, m, n, **kw: lib.asj_batch_workspace_bytes(J, m, n, ctypes.byref(_Opts(**{
        "f": 16, "nsym": 2, "load_factor": 0.5, "flags": 0, "keys_per_window": 32, "grid_rounds": 0, **kw})))
    small, large = ws(3, 100000, 120000), ws(3, 200000, 120000)
    assert 0 < small < large
    local = ws(3, 100000, 120000, flags=0x1000)  # ASJ_LOCAL_ONLY
    assert 0 < local and small - local >= 8 * 100000
    assert ws(0, 10, 10) == -1                     # no joins
    assert ws(3, -1, 10) == -1                     # negative row count
    assert ws(3, 10, 10, load_factor=1.5) == -1    # load factor out of (0, 1)
    assert ws(3, 10, 10, flags=0x1000 | 0x400) == -1  # ASJ_LOCAL_ONLY with ASJ_GLOBAL_TABLES
