"""Oracle for the signature-accelerated equi-join -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never links,
loads or calls it, and it shares no code with the HIP path.

The arithmetic lives in ``asj_oracle.c`` (plain single-threaded C written
from Section 3.1 and Section 3.2 of Mokadem, Hameurlain, Morvan, "Equi join
query acceleration using algebraic signatures").  This module compiles it
with gcc and exposes numpy-friendly wrappers.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "asj_oracle.c")
_LIB = os.path.join(_HERE, "_asj_oracle.so")

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_u64p = ctypes.POINTER(ctypes.c_uint64)

METHOD_DEFINITION = 0  # per-term log/antilog (Section 3.1)
METHOD_HORNER = 1      # Horner's rule with multiplication by alpha only
METHOD_POLY = 2        # P(alpha^j) with carry-less multiplication


def build() -> str:
    """Compile the oracle into ``oracle/_asj_oracle.so`` (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.or_init.restype = ctypes.c_int
        for name in ("or_gf_exp", "or_gf_log", "or_mul_table", "or_mul_clmul"):
            fn = getattr(L, name)
            fn.restype = ctypes.c_uint32
        L.or_gf_exp.argtypes = [ctypes.c_int, ctypes.c_uint32]
        L.or_gf_log.argtypes = [ctypes.c_int, ctypes.c_uint32]
        L.or_mul_table.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32]
        L.or_mul_clmul.argtypes = [ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32]
        L.or_alpha_order.restype = ctypes.c_uint32
        L.or_alpha_order.argtypes = [ctypes.c_int]
        L.or_signature.restype = ctypes.c_int
        L.or_signature.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _u8p, _i64p, ctypes.c_int64, _u64p]
        rel = [_u8p, _i64p, _i32p, ctypes.c_int64]
        for name in ("or_join_nested", "or_join_hash"):
            fn = getattr(L, name)
            fn.restype = ctypes.c_int64
            fn.argtypes = rel + rel + [_i32p, ctypes.c_int64]
        L.or_join_sig.restype = ctypes.c_int64
        L.or_join_sig.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int] + rel + rel + [_i32p, ctypes.c_int64, _i64p]
        if L.or_init() != 0:
            raise RuntimeError("oracle: alpha is not primitive for the chosen field polynomial")
        _lib = L
    return _lib


# ---------------------------------------------------------------------------
# small helpers
# ---------------------------------------------------------------------------

def _ptr(a, typ):
    return a.ctypes.data_as(typ) if a is not None else None


def _arena(keys):
    """list of bytes -> (data uint8, offsets int64)"""
    lens = np.fromiter((len(k) for k in keys), dtype=np.int64, count=len(keys))
    off = np.zeros(len(keys) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    data = np.frombuffer(b"".join(keys), dtype=np.uint8).copy() if off[-1] else np.zeros(1, np.uint8)
    return data, off


def _as_rel(rel):
    """Accept (data, offsets[, ids]) tuples or an object with .data/.offsets/.ids."""
    if hasattr(rel, "data"):
        data, off, ids = rel.data, rel.offsets, getattr(rel, "ids", None)
    elif isinstance(rel, (list, tuple)) and len(rel) and isinstance(rel[0], (bytes, bytearray)):
        data, off = _arena(list(rel))
        ids = None
    else:
        data, off = rel[0], rel[1]
        ids = rel[2] if len(rel) > 2 else None
    data = np.ascontiguousarray(data, dtype=np.uint8)
    if data.size == 0:
        data = np.zeros(1, np.uint8)
    off = np.ascontiguousarray(off, dtype=np.int64)
    ids = None if ids is None else np.ascontiguousarray(ids, dtype=np.int32)
    return data, off, ids, len(off) - 1


# ---------------------------------------------------------------------------
# field
# ---------------------------------------------------------------------------

def gf_exp(f, e):
    return lib().or_gf_exp(f, e)


def gf_log(f, v):
    return lib().or_gf_log(f, v)


def mul_table(f, a, b):
    return lib().or_mul_table(f, a, b)


def mul_clmul(f, a, b):
    return lib().or_mul_clmul(f, a, b)


def alpha_order(f):
    return lib().or_alpha_order(f)


# ---------------------------------------------------------------------------
# signatures
# ---------------------------------------------------------------------------

def signatures(keys, f=16, nsym=2, method=METHOD_DEFINITION):
    """Packed signatures (uint64) of every key in `keys` (list of bytes or a relation)."""
    data, off, _, n = _as_rel(keys)
    out = np.zeros(max(n, 1), dtype=np.uint64)
    rc = lib().or_signature(method, f, nsym, _ptr(data, _u8p), _ptr(off, _i64p), n, _ptr(out, _u64p))
    if rc != 0:
        raise ValueError("oracle: bad signature parameters")
    return out[:n]


def signature(key: bytes, f=16, nsym=2, method=METHOD_DEFINITION) -> int:
    return int(signatures([key], f, nsym, method)[0])


# ---------------------------------------------------------------------------
# joins; return (pairs int32[k, 2] sorted by (r_id, s_id), full count)
# ---------------------------------------------------------------------------

def _run_join(fn, R, S, extra_front=(), extra_back=(), cap=None):
    rd, ro, ri, m = _as_rel(R)
    sd, so, si, n = _as_rel(S)
    args_r = [_ptr(rd, _u8p), _ptr(ro, _i64p), _ptr(ri, _i32p), m]
    args_s = [_ptr(sd, _u8p), _ptr(so, _i64p), _ptr(si, _i32p), n]
    if cap is None:
        cap = 1 << 16
    while True:
        pairs = np.zeros((max(cap, 1), 2), dtype=np.int32)
        cnt = fn(*extra_front, *args_r, *args_s, _ptr(pairs, _i32p), cap, *extra_back)
        if cnt < 0:
            raise MemoryError("oracle join failed to allocate")
        if cnt <= cap:
            break
        cap = int(cnt)
    return sort_pairs(pairs[:cnt]), int(cnt)


def sort_pairs(pairs):
    pairs = np.asarray(pairs, dtype=np.int32).reshape(-1, 2)
    if len(pairs) == 0:
        return pairs
    order = np.lexsort((pairs[:, 1], pairs[:, 0]))
    return pairs[order]


def join_nested(R, S):
    """The equi-join by definition (all byte-equal pairs); tiny inputs only."""
    pairs, _ = _run_join(lib().or_join_nested, R, S)
    return pairs


def join_hash(R, S, cap=None):
    """Simple hash join on the key bytes (Section 2)."""
    pairs, _ = _run_join(lib().or_join_hash, R, S, cap=cap)
    return pairs


def join_signature(R, S, f=16, nsym=2, verify=True, cap=None):
    """Signature hash join (Section 3.2, Figure 2).

    Returns (pairs, n_candidates).  With verify=False the output is the
    paper-literal one: every pair whose signatures are equal.
    """
    ncand = np.zeros(1, dtype=np.int64)
    pairs, _ = _run_join(lib().or_join_sig, R, S, extra_front=(f, nsym, 1 if verify else 0),
                         extra_back=(_ptr(ncand, _i64p),), cap=cap)
    return pairs, int(ncand[0])


# ---------------------------------------------------------------------------
# Join variants beyond the inner equi-join (the paper names outer joins and
# the semi-join as future work, Section 5).  Each is its plain definition
# over the inner join T (pairs of key-equal rows) and the probe relation S:
#   semi   S |x R : one pair (-1, s_id) per probe row with at least one match
#   anti   S |> R : one pair (-1, s_id) per probe row with no match
#   left   S =x R : T plus (-1, s_id) for every probe row with no match
#   right  S x= R : T plus (r_id, -1) for every build row that no probe row
#                   matches
#   full   S =x= R: T plus both kinds of unmatched row
# Matches are exact key equality (or, with verify=False, signature equality,
# the paper-literal reading).
# ---------------------------------------------------------------------------

def _probe_ids(S):
    _, _, ids, n = _as_rel(S)
    return np.arange(n, dtype=np.int32) if ids is None else np.asarray(ids, dtype=np.int32)


def _matched_rows(R, S, verify=True):
    """Boolean per probe row: does it match some build row?  Probe row i is
    matched exactly when it occurs in the inner join (computed with row
    indexes as ids, so repeated ids cannot hide a row)."""
    data, off, _, n = _as_rel(S)
    rows = (data, off, np.arange(n, dtype=np.int32))
    pairs = join_hash(R, rows, cap=n + 1024) if verify else join_signature(R, rows, verify=False)[0]
    matched = np.zeros(n, dtype=bool)
    matched[pairs[:, 1]] = True
    return matched


def _matched_build_rows(R, S, verify=True):
    """Boolean per build row: does some probe row match it?  (Row indexes as
    build ids, as in _matched_rows.)"""
    data, off, _, m = _as_rel(R)
    rows = (data, off, np.arange(m, dtype=np.int32))
    pairs = join_hash(rows, S) if verify else join_signature(rows, S, verify=False)[0]
    matched = np.zeros(m, dtype=bool)
    matched[pairs[:, 0]] = True
    return matched


def join_variant(R, S, kind: str, verify=True):
    """Semi ('semi'), anti ('anti'), left outer ('left'), right outer
    ('right') or full outer ('full') join of S with R, as sorted (r_id, s_id)
    pairs (r_id = -1 for the probe-only rows, s_id = -1 for the build-only
    rows)."""
    ids = _probe_ids(S)
    matched = _matched_rows(R, S, verify)
    lonely = np.stack([np.full(int((~matched).sum()), -1, np.int32), ids[~matched]], axis=1)
    if kind == "semi":
        return sort_pairs(np.stack([np.full(int(matched.sum()), -1, np.int32), ids[matched]], axis=1))
    if kind == "anti":
        return sort_pairs(lonely)
    if kind in ("left", "right", "full"):
        inner = join_nested(R, S) if verify else join_signature(R, S, verify=False)[0]
        parts = [inner.reshape(-1, 2)]
        if kind in ("left", "full"):
            parts.append(lonely)
        if kind in ("right", "full"):
            rids = _probe_ids(R)
            rm = _matched_build_rows(R, S, verify)
            parts.append(np.stack([rids[~rm], np.full(int((~rm).sum()), -1, np.int32)], axis=1))
        return sort_pairs(np.concatenate(parts))
    raise ValueError(kind)
