"""Seeded synthetic relations for the equi-join workloads.

This module is the only thing the oracle side and the HIP side share: it
makes inputs and holds none of the join or signature arithmetic.  Every
relation is a columnar key arena::

    data    uint8[total]      the key bytes, packed back to back
    offsets int64[n + 1]      key k is data[offsets[k] : offsets[k + 1]]
    ids     int32[n]          tuple id carried into the output pairs

Row plans (lengths, which rows copy which) come from numpy's PCG64 seeded by
(seed, config, part); the bytes come from ``fill.c`` (SplitMix64 per row).
Both are deterministic for a given seed, on any machine with this numpy.

Workloads (sizes at scale = 1):

* ``tiny``    R = S = 10,000 keys of 256 printable bytes; R distinct; exactly
              20% of S rows copy uniformly chosen R rows, the rest are fresh.
* ``large``   R = 1M, S = 4M; lengths log-uniform over [64, 4096]; every key
              starts with one fixed 48-byte printable prefix; 50% of S rows
              copy an R row chosen by Zipf(1.0) rank through a seeded
              permutation of R, the rest are fresh.
* ``dna``     keys over {A,C,G,T}, lengths uniform in [1000, 10000];
              R = 200k, S = 1M: 30% exact copies, 40% copies with one base
              substituted by one of the other three, 30% fresh.
* ``batch``   256 independent joins; |R_k| log-uniform [100, 200000],
              |S_k| = round(U(1, 8) |R_k|); lengths log-uniform [16, 2048] of
              XML-like text over a 64-name seeded vocabulary; 25% of S_k rows
              copy R_k rows.
* ``served``  resident R = 10M keys of 256 printable bytes; probe requests of
              log-uniform size [10k, 1M]: 30% copies of R rows, 70% fresh keys
              of log-uniform length [64, 1024].
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fill.c")
_LIB = os.path.join(_HERE, "_fill.so")

PRINTABLE = np.arange(0x20, 0x7F, dtype=np.uint8)  # 95 printable ASCII bytes
DNA = np.frombuffer(b"ACGT", dtype=np.uint8).copy()

_STREAM = {"R": 1, "S": 2, "prefix": 3, "vocab": 4}


def build() -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", _LIB + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.fill_alphabet.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, P, ctypes.c_int,
                                    P, ctypes.c_int64]
        L.fill_alphabet.restype = None
        L.fill_xml.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint64, P, P, ctypes.c_int]
        L.fill_xml.restype = None
        L.copy_rows.argtypes = [P, P, P, P, P, P, ctypes.c_int64]
        L.copy_rows.restype = None
        _lib = L
    return _lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


@dataclass
class Relation:
    data: np.ndarray
    offsets: np.ndarray
    ids: np.ndarray

    @property
    def n(self) -> int:
        return len(self.offsets) - 1

    @property
    def nbytes(self) -> int:
        return int(self.offsets[-1] - self.offsets[0])

    def key(self, k: int) -> bytes:
        return self.data[self.offsets[k]:self.offsets[k + 1]].tobytes()

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def subset(self, rows) -> "Relation":
        """A new packed relation holding the given rows (ids carried along)."""
        rows = np.asarray(rows, dtype=np.int64)
        lens = self.lengths()[rows]
        off = np.zeros(len(rows) + 1, dtype=np.int64)
        np.cumsum(lens, out=off[1:])
        data = np.zeros(max(int(off[-1]), 1), dtype=np.uint8)
        if len(rows):
            dst_rows = np.arange(len(rows), dtype=np.int64)
            _L().copy_rows(_p(data), _p(off), _p(dst_rows), _p(self.data), _p(self.offsets), _p(rows), len(rows))
        return Relation(data, off, self.ids[rows].copy())


@dataclass
class Workload:
    name: str
    R: Relation
    S: Relation
    meta: dict = field(default_factory=dict)


def _offsets(lens: np.ndarray) -> np.ndarray:
    off = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return off


def _alloc(lens: np.ndarray):
    off = _offsets(np.asarray(lens, dtype=np.int64))
    # padded so that a reader may touch the 16-byte unit holding the last byte
    data = np.zeros(int(off[-1]) + 16, dtype=np.uint8)
    return data, off


def _fill(data, off, rows, seed, stream, alphabet, prefix=None):
    rows = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nrows = (len(off) - 1) if rows is None else len(rows)
    pre = np.zeros(1, np.uint8) if prefix is None else np.ascontiguousarray(prefix, dtype=np.uint8)
    _L().fill_alphabet(_p(data), _p(off), _p(rows), nrows, seed, stream, _p(alphabet), len(alphabet),
                       _p(pre), 0 if prefix is None else len(prefix))


def _copy(dst_data, dst_off, dst_rows, src: Relation, src_rows):
    dst_rows = np.ascontiguousarray(dst_rows, dtype=np.int64)
    src_rows = np.ascontiguousarray(src_rows, dtype=np.int64)
    _L().copy_rows(_p(dst_data), _p(dst_off), _p(dst_rows), _p(src.data), _p(src.offsets), _p(src_rows),
                   len(dst_rows))


def _loguniform_int(rng, lo, hi, size):
    """floor(exp(U(ln lo, ln(hi + 1)))) clipped to [lo, hi]."""
    x = np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi + 1), size=size))).astype(np.int64)
    return np.clip(x, lo, hi)


def _row_ids(n):
    return np.arange(n, dtype=np.int32)


def _scaled(x, scale, lo=1):
    return max(lo, int(round(x * scale)))


# ---------------------------------------------------------------------------
# tiny: R = S = 10k, 256-byte printable keys, 20% of S copied from R
# ---------------------------------------------------------------------------

def tiny(seed: int = 1, scale: float = 1.0, key_len: int = 256) -> Workload:
    rng = np.random.default_rng([seed, 1])
    m = _scaled(10_000, scale)
    n = _scaled(10_000, scale)
    rd, ro = _alloc(np.full(m, key_len))
    _fill(rd, ro, None, seed, _STREAM["R"], PRINTABLE)
    R = Relation(rd, ro, _row_ids(m))
    ncopy = int(round(0.2 * n))
    copy_rows = np.sort(rng.permutation(n)[:ncopy])
    copy_src = rng.integers(0, m, size=ncopy)
    sd, so = _alloc(np.full(n, key_len))
    fresh = np.setdiff1d(np.arange(n), copy_rows)
    _fill(sd, so, fresh, seed, _STREAM["S"], PRINTABLE)
    _copy(sd, so, copy_rows, R, copy_src)
    S = Relation(sd, so, _row_ids(n))
    return Workload("tiny", R, S, {"copies": ncopy, "expected_matches": ncopy, "seed": seed, "scale": scale})


def fixed_length(seed: int, m: int, n: int, key_len: int, copy_frac: float = 0.2,
                 alphabet: np.ndarray | None = None) -> Workload:
    """Keys of one length (the key-length sweep): R = m random keys, S = n
    keys of which round(copy_frac * n) copy uniformly drawn R rows.  Bytes
    are uniform over `alphabet` (default: all 256 values, so short keys stay
    nearly distinct)."""
    alphabet = np.arange(256, dtype=np.uint8) if alphabet is None else alphabet
    rng = np.random.default_rng([seed, 8, key_len])
    rd, ro = _alloc(np.full(m, key_len))
    _fill(rd, ro, None, seed, _STREAM["R"], alphabet)
    R = Relation(rd, ro, _row_ids(m))
    ncopy = int(round(copy_frac * n))
    copy_rows = np.sort(rng.permutation(n)[:ncopy])
    copy_src = rng.integers(0, m, size=ncopy)
    sd, so = _alloc(np.full(n, key_len))
    fresh = np.setdiff1d(np.arange(n), copy_rows)
    _fill(sd, so, fresh, seed, _STREAM["S"], alphabet)
    _copy(sd, so, copy_rows, R, copy_src)
    S = Relation(sd, so, _row_ids(n))
    return Workload(f"fixed{key_len}", R, S, {"copies": ncopy, "seed": seed, "key_len": key_len})


# ---------------------------------------------------------------------------
# large: R = 1M, S = 4M, log-uniform [64, 4096], 48-byte shared prefix, Zipf(1)
# ---------------------------------------------------------------------------

def zipf_ranks(rng, n_items: int, size: int, s: float = 1.0) -> np.ndarray:
    """0-based ranks drawn with P(rank k) proportional to 1/(k+1)^s (inverse CDF)."""
    w = 1.0 / np.power(np.arange(1, n_items + 1, dtype=np.float64), s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.uniform(0.0, 1.0, size=size)
    return np.minimum(np.searchsorted(cdf, u, side="right"), n_items - 1).astype(np.int64)


def large(seed: int = 2, scale: float = 1.0) -> Workload:
    rng = np.random.default_rng([seed, 2])
    m = _scaled(1_000_000, scale)
    n = _scaled(4_000_000, scale)
    prefix = rng.integers(0x20, 0x7F, size=48).astype(np.uint8)
    lr = _loguniform_int(rng, 64, 4096, m)
    rd, ro = _alloc(lr)
    _fill(rd, ro, None, seed, _STREAM["R"], PRINTABLE, prefix)
    R = Relation(rd, ro, _row_ids(m))
    ncopy = n // 2
    copy_rows = np.sort(rng.permutation(n)[:ncopy])
    perm = rng.permutation(m)
    copy_src = perm[zipf_ranks(rng, m, ncopy, 1.0)]
    ls = _loguniform_int(rng, 64, 4096, n)
    ls[copy_rows] = lr[copy_src]
    sd, so = _alloc(ls)
    is_copy = np.zeros(n, dtype=bool)
    is_copy[copy_rows] = True
    _fill(sd, so, np.flatnonzero(~is_copy), seed, _STREAM["S"], PRINTABLE, prefix)
    _copy(sd, so, copy_rows, R, copy_src)
    S = Relation(sd, so, _row_ids(n))
    return Workload("large", R, S, {"copies": ncopy, "expected_matches": ncopy, "seed": seed, "scale": scale})


# ---------------------------------------------------------------------------
# dna: R = 200k distinct, S = 1M (30% copies, 40% one-base substitutions, 30% fresh)
# ---------------------------------------------------------------------------

def dna(seed: int = 3, scale: float = 1.0, min_len: int = 1000, max_len: int = 10000) -> Workload:
    rng = np.random.default_rng([seed, 3])
    m = _scaled(200_000, scale)
    n = _scaled(1_000_000, scale)
    lr = rng.integers(min_len, max_len + 1, size=m)
    rd, ro = _alloc(lr)
    _fill(rd, ro, None, seed, _STREAM["R"], DNA)
    R = Relation(rd, ro, _row_ids(m))
    kind = np.zeros(n, dtype=np.int8)  # 0 fresh, 1 exact copy, 2 near-duplicate
    order = rng.permutation(n)
    n_copy, n_near = int(round(0.3 * n)), int(round(0.4 * n))
    kind[order[:n_copy]] = 1
    kind[order[n_copy:n_copy + n_near]] = 2
    src = rng.integers(0, m, size=n)
    ls = rng.integers(min_len, max_len + 1, size=n)
    dup = kind > 0
    ls[dup] = lr[src[dup]]
    sd, so = _alloc(ls)
    _fill(sd, so, np.flatnonzero(~dup), seed, _STREAM["S"], DNA)
    _copy(sd, so, np.flatnonzero(dup), R, src[dup])
    near = np.flatnonzero(kind == 2)
    pos = (rng.uniform(size=len(near)) * ls[near]).astype(np.int64)
    shift = rng.integers(1, 4, size=len(near))  # one of the three other bases
    at = so[near] + pos
    base_idx = np.searchsorted(DNA, sd[at])
    sd[at] = DNA[(base_idx + shift) % 4]
    S = Relation(sd, so, _row_ids(n))
    return Workload("dna", R, S, {"copies": n_copy, "near": n_near, "expected_matches": n_copy,
                                  "kind": kind, "src": src, "seed": seed, "scale": scale})


# ---------------------------------------------------------------------------
# batch: 256 independent joins of XML-like keys
# ---------------------------------------------------------------------------

def vocabulary(seed: int, nnames: int = 64):
    rng = np.random.default_rng([seed, _STREAM["vocab"]])
    names = []
    seen = set()
    while len(names) < nnames:
        L = int(rng.integers(3, 11))
        nm = bytes((rng.integers(0, 26, size=L) + ord("a")).astype(np.uint8).tolist())
        if nm not in seen:
            seen.add(nm)
            names.append(nm)
    voff = np.zeros(nnames + 1, dtype=np.int64)
    voff[1:] = np.cumsum([len(x) for x in names])
    vocab = np.frombuffer(b"".join(names), dtype=np.uint8).copy()
    return names, vocab, voff


@dataclass
class BatchWorkload:
    name: str
    R: Relation          # all joins' build rows, join k at rows r_seg[k]:r_seg[k+1]
    S: Relation          # all joins' probe rows, join k at rows s_seg[k]:s_seg[k+1]
    r_seg: np.ndarray    # int64[J + 1]
    s_seg: np.ndarray    # int64[J + 1]
    meta: dict = field(default_factory=dict)

    @property
    def njoins(self) -> int:
        return len(self.r_seg) - 1

    def join(self, k: int) -> Workload:
        """Join k as a stand-alone workload (row-local ids)."""
        R = self.R.subset(np.arange(self.r_seg[k], self.r_seg[k + 1]))
        S = self.S.subset(np.arange(self.s_seg[k], self.s_seg[k + 1]))
        return Workload(f"{self.name}[{k}]", R, S)


def batch(seed: int = 4, scale: float = 1.0, njoins: int = 256, max_r: int = 200_000,
          min_len: int = 16, max_len: int = 2048) -> BatchWorkload:
    rng = np.random.default_rng([seed, 4])
    _, vocab, voff = vocabulary(seed)
    rsz = np.maximum(1, np.round(_loguniform_int(rng, 100, max_r, njoins) * scale)).astype(np.int64)
    ssz = np.maximum(1, np.round(rng.uniform(1.0, 8.0, size=njoins) * rsz)).astype(np.int64)
    r_seg = _offsets(rsz)
    s_seg = _offsets(ssz)
    M, N = int(r_seg[-1]), int(s_seg[-1])
    lr = _loguniform_int(rng, min_len, max_len, M)
    rd, ro = _alloc(lr)
    _L().fill_xml(_p(rd), _p(ro), None, M, seed, _STREAM["R"], _p(vocab), _p(voff), len(voff) - 1)
    # ids are row-local within each join
    rid = (np.arange(M, dtype=np.int64) - np.repeat(r_seg[:-1], rsz)).astype(np.int32)
    R = Relation(rd, ro, rid)
    join_of_s = np.repeat(np.arange(njoins), ssz)
    is_copy = rng.uniform(size=N) < 0.25
    src = r_seg[join_of_s] + np.floor(rng.uniform(size=N) * rsz[join_of_s]).astype(np.int64)
    ls = _loguniform_int(rng, min_len, max_len, N)
    ls[is_copy] = lr[src[is_copy]]
    sd, so = _alloc(ls)
    fresh = np.ascontiguousarray(np.flatnonzero(~is_copy), dtype=np.int64)
    _L().fill_xml(_p(sd), _p(so), _p(fresh), len(fresh), seed,
                  _STREAM["S"], _p(vocab), _p(voff), len(voff) - 1)
    _copy(sd, so, np.flatnonzero(is_copy), R, src[is_copy])
    sid = (np.arange(N, dtype=np.int64) - np.repeat(s_seg[:-1], ssz)).astype(np.int32)
    S = Relation(sd, so, sid)
    return BatchWorkload("batch", R, S, r_seg, s_seg, {"seed": seed, "scale": scale, "copies": int(is_copy.sum())})


# ---------------------------------------------------------------------------
# served: resident R = 10M x 256 B; probe requests of 10k..1M keys
# ---------------------------------------------------------------------------

def served_build_side(seed: int = 5, scale: float = 1.0, key_len: int = 256) -> Relation:
    m = _scaled(10_000_000, scale)
    rd, ro = _alloc(np.full(m, key_len))
    _fill(rd, ro, None, seed, _STREAM["R"], PRINTABLE)
    return Relation(rd, ro, _row_ids(m))


def served_request(R: Relation, seed: int, request: int, size: int | None = None,
                   hit_rate: float = 0.3, min_size: int = 10_000, max_size: int = 1_000_000,
                   min_len: int = 64, max_len: int = 1024) -> Relation:
    rng = np.random.default_rng([seed, 5, request])
    n = int(size) if size is not None else int(_loguniform_int(rng, min_size, max_size, 1)[0])
    is_copy = rng.uniform(size=n) < hit_rate
    src = rng.integers(0, R.n, size=n)
    ls = _loguniform_int(rng, min_len, max_len, n)
    ls[is_copy] = R.lengths()[src[is_copy]]
    sd, so = _alloc(ls)
    fresh = np.flatnonzero(~is_copy)
    _fill(sd, so, fresh, seed ^ (request << 20), _STREAM["S"], PRINTABLE)
    _copy(sd, so, np.flatnonzero(is_copy), R, src[is_copy])
    return Relation(sd, so, _row_ids(n))


def poisson_arrivals(seed: int, rate_per_s: float, count: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process."""
    rng = np.random.default_rng([seed, 6])
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))


# ---------------------------------------------------------------------------
# small adversarial relations for parity tests
# ---------------------------------------------------------------------------

def from_keys(keys, ids=None) -> Relation:
    lens = np.array([len(k) for k in keys], dtype=np.int64)
    data, off = _alloc(lens)
    if off[-1]:
        data[:off[-1]] = np.frombuffer(b"".join(keys), dtype=np.uint8)
    ids = _row_ids(len(keys)) if ids is None else np.asarray(ids, dtype=np.int32)
    return Relation(data, off, ids)


def random_small(seed: int, m: int, n: int, max_len: int = 40, alphabet: bytes = b"ab\x00",
                 dup_rate: float = 0.3, lengths=None) -> Workload:
    """Tiny relations with duplicates, empty keys, odd lengths and NUL bytes."""
    rng = np.random.default_rng([seed, 7])
    alpha = np.frombuffer(alphabet, dtype=np.uint8)

    def mk(count):
        out = []
        for _ in range(count):
            L = int(rng.integers(0, max_len + 1)) if lengths is None else int(rng.choice(lengths))
            out.append(alpha[rng.integers(0, len(alpha), size=L)].tobytes())
        return out

    rk = mk(m)
    sk = mk(n)
    for i in range(n):
        if rk and rng.uniform() < dup_rate:
            sk[i] = rk[int(rng.integers(0, m))]
    return Workload("small", from_keys(rk), from_keys(sk))


def unaligned_copy(rel: Relation, shift: int) -> Relation:
    """The same keys in an arena that starts `shift` bytes later (tests byte alignment)."""
    data = np.zeros(len(rel.data) + shift + 16, dtype=np.uint8)
    data[shift:shift + len(rel.data)] = rel.data
    return Relation(data, rel.offsets + shift, rel.ids.copy())
