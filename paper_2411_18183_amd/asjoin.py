"""Python binding of libasjoin: the C entry points under the same names.

Argument marshalling only -- every step of the join runs in the library's
HIP kernels.  PyTorch supplies device memory (tensors) and streams.  The
library must have been built (``python -m paper_2411_18183_amd.build``);
importing this module without it raises, there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import torch  # loads the HIP runtime that libasjoin then shares

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libasjoin.so")

ASJ_OK = 0
ASJ_EINVAL = -1
ASJ_ENOMEM = -2
ASJ_EOVERFLOW = -3
ASJ_ETABLEFULL = -4
ASJ_EHIP = -5
ASJ_EUNSUPPORTED = -6

ASJ_NO_VERIFY = 0x1
ASJ_PLAIN = 0x2
ASJ_PROBE_FUSED = 0x4
ASJ_PROBE_SPLIT = 0x8
ASJ_SORTED = 0x10
ASJ_VALIDATE = 0x20
ASJ_SEMI = 0x40
ASJ_ANTI = 0x80
ASJ_LEFT_OUTER = 0x100
ASJ_RIGHT_OUTER = 0x800
ASJ_FINGERPRINT = 0x200
ASJ_GLOBAL_TABLES = 0x400
ASJ_LOCAL_ONLY = 0x1000


class AsjError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


class asj_keys(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("offsets", ctypes.c_void_p), ("ids", ctypes.c_void_p),
                ("n", ctypes.c_int64)]


class asj_sig_params(ctypes.Structure):
    _fields_ = [("f", ctypes.c_int32), ("nsym", ctypes.c_int32)]


class asj_opts(ctypes.Structure):
    _fields_ = [("sig", asj_sig_params), ("load_factor", ctypes.c_float), ("flags", ctypes.c_uint32),
                ("keys_per_window", ctypes.c_int32), ("grid_rounds", ctypes.c_int32)]


class asj_batch(ctypes.Structure):
    _fields_ = [("r", asj_keys), ("s", asj_keys), ("r_seg", ctypes.c_void_p), ("s_seg", ctypes.c_void_p),
                ("njoins", ctypes.c_int32), ("out", ctypes.c_void_p), ("out_seg", ctypes.c_void_p),
                ("out_count", ctypes.c_void_p), ("cand_count", ctypes.c_void_p), ("done_clock", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_int64)]


class asj_tune_result(ctypes.Structure):
    _fields_ = [("best", asj_opts), ("best_ms", ctypes.c_float), ("default_ms", ctypes.c_float),
                ("trials", ctypes.c_int32)]


class asj_host_opts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_int64), ("partitions", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class asj_host_stats(ctypes.Structure):
    _fields_ = [("partitions", ctypes.c_int32), ("reserved", ctypes.c_int32), ("chunks", ctypes.c_int64),
                ("pieces", ctypes.c_int64), ("bytes_h2d", ctypes.c_int64), ("bytes_d2h", ctypes.c_int64),
                ("device_peak", ctypes.c_int64), ("ms_partition", ctypes.c_double), ("ms_join", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libasjoin is not built ({LIB_PATH} missing); run python -m paper_2411_18183_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P, I64 = ctypes.c_void_p, ctypes.c_int64
        L.asj_signature.argtypes = [ctypes.POINTER(asj_keys), asj_sig_params, P, P]
        L.asj_build.argtypes = [ctypes.POINTER(asj_keys), ctypes.POINTER(asj_opts), ctypes.POINTER(P), P]
        L.asj_probe.argtypes = [P, ctypes.POINTER(asj_keys), P, I64, P, P, P]
        L.asj_join.argtypes = [ctypes.POINTER(asj_keys), ctypes.POINTER(asj_keys), ctypes.POINTER(asj_opts), P, I64,
                               P, P, P]
        L.asj_join_noalloc.argtypes = L.asj_join.argtypes
        L.asj_table_status.argtypes = [P]
        L.asj_table_capacity.argtypes = [P]
        L.asj_table_capacity.restype = I64
        L.asj_table_free.argtypes = [P]
        L.asj_strerror.argtypes = [ctypes.c_int]
        L.asj_strerror.restype = ctypes.c_char_p
        L.asj_timing_enable.argtypes = [ctypes.c_int]
        L.asj_timing_read.argtypes = [P, P, ctypes.c_int]
        L.asj_util_copy.argtypes = [P, P, I64, P]
        L.asj_batch_workspace_bytes.argtypes = [ctypes.c_int32, I64, I64, ctypes.POINTER(asj_opts)]
        L.asj_batch_workspace_bytes.restype = I64
        L.asj_join_batch.argtypes = [ctypes.POINTER(asj_batch), ctypes.POINTER(asj_opts), P]
        L.asj_autotune.argtypes = [ctypes.POINTER(asj_keys), ctypes.POINTER(asj_keys), ctypes.POINTER(asj_opts), P,
                                   I64, P, ctypes.POINTER(asj_tune_result), P]
        L.asj_autotune_batch.argtypes = [ctypes.POINTER(asj_batch), ctypes.POINTER(asj_opts),
                                         ctypes.POINTER(asj_tune_result), P]
        L.asj_autotune_clear.argtypes = []
        L.asj_autotune_clear.restype = None
        L.asj_join_host.argtypes = [ctypes.POINTER(asj_keys), ctypes.POINTER(asj_keys), ctypes.POINTER(asj_opts),
                                    ctypes.POINTER(asj_host_opts), P, I64, P, ctypes.POINTER(asj_host_stats), P]
        L.asj_join_host_release.argtypes = []
        L.asj_clock_khz.argtypes = []
        L.asj_clock_khz.restype = I64
        for name in ("asj_signature", "asj_build", "asj_probe", "asj_join", "asj_join_noalloc", "asj_table_status",
                     "asj_table_free",
                     "asj_timing_enable", "asj_timing_read", "asj_util_copy", "asj_join_batch", "asj_autotune",
                     "asj_autotune_batch", "asj_join_host", "asj_join_host_release"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().asj_strerror(code).decode()


def _check(rc: int, where: str):
    if rc != ASJ_OK:
        raise AsjError(rc, where)


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _need_dev(t, dtype, numel, what):
    """Raise ValueError unless t is a contiguous device tensor of dtype with at
    least numel elements (the library writes through its pointer)."""
    if t is None or not isinstance(t, torch.Tensor):
        raise ValueError(f"{what}: a device tensor is required")
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{what}: must be a contiguous cuda {dtype} tensor")
    if t.numel() < numel:
        raise ValueError(f"{what}: holds {t.numel()} elements, needs at least {numel}")


def _need_pairs(out, what):
    """out must be a contiguous cuda int32 tensor of shape [cap, 2]; returns cap."""
    if out is None or not isinstance(out, torch.Tensor) or out.dim() != 2 or out.shape[1] != 2:
        raise ValueError(f"{what}: must be an int32 tensor of shape [cap, 2]")
    _need_dev(out, torch.int32, 0, what)
    return out.shape[0]


@dataclass
class DeviceKeys:
    """A relation's join attributes in device memory (see asj_keys)."""
    data: torch.Tensor              # uint8
    offsets: torch.Tensor           # int64, n + 1
    ids: Optional[torch.Tensor]     # int32, n (None -> row index)

    @property
    def n(self) -> int:
        return self.offsets.numel() - 1

    @classmethod
    def from_host(cls, rel, device="cuda", with_ids=True) -> "DeviceKeys":
        """Copy a host relation (numpy data/offsets/ids) to the device."""
        data = torch.from_numpy(rel.data).to(device)
        off = torch.from_numpy(rel.offsets).to(device)
        ids = torch.from_numpy(rel.ids).to(device) if (with_ids and rel.ids is not None) else None
        return cls(data, off, ids)

    def c(self) -> asj_keys:
        for t, dt in ((self.data, torch.uint8), (self.offsets, torch.int64)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError("keys: data must be contiguous cuda uint8, offsets contiguous cuda int64")
        if self.ids is not None and (self.ids.dtype != torch.int32 or not self.ids.is_cuda or
                                     not self.ids.is_contiguous() or self.ids.numel() != self.n):
            raise ValueError("keys: ids must be a contiguous cuda int32 tensor of n elements")
        return asj_keys(self.data.data_ptr() if self.data.numel() else None, self.offsets.data_ptr(),
                        self.ids.data_ptr() if self.ids is not None else None, self.n)


def asj_signature(keys: DeviceKeys, f: int = 16, nsym: int = 2, out: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    """Signatures of every key (int32 tensor holding the uint32 bit patterns;
    2 words per key, the low word first, for 64-bit signatures f * nsym = 64)."""
    words = 2 if f * nsym == 64 else 1
    if out is None:
        out = torch.empty(max(keys.n, 0) * words, dtype=torch.int32, device=keys.offsets.device)
    else:
        _need_dev(out, torch.int32, keys.n * words, "asj_signature out")
    k = keys.c()
    _check(lib().asj_signature(ctypes.byref(k), asj_sig_params(f, nsym),
                               ctypes.c_void_p(out.data_ptr() if out.numel() else None), _stream(stream)),
           "asj_signature")
    return out


class Table:
    """asj_table handle; keeps the borrowed build relation alive."""

    def __init__(self, handle: ctypes.c_void_p, keys: DeviceKeys):
        self.handle = handle
        self.keys = keys

    @property
    def capacity(self) -> int:
        return int(lib().asj_table_capacity(self.handle))

    def status(self) -> int:
        return lib().asj_table_status(self.handle)

    def free(self):
        if self.handle:
            _check(lib().asj_table_free(self.handle), "asj_table_free")
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _opts(f, nsym, load_factor, flags, keys_per_window=0, grid_rounds=0) -> asj_opts:
    return asj_opts(asj_sig_params(f, nsym), float(load_factor), int(flags), int(keys_per_window), int(grid_rounds))


def asj_build(R: DeviceKeys, f: int = 16, nsym: int = 2, load_factor: float = 0.0, flags: int = 0,
              keys_per_window: int = 0, grid_rounds: int = 0, stream=None) -> Table:
    k = R.c()
    o = _opts(f, nsym, load_factor, flags, keys_per_window, grid_rounds)
    h = ctypes.c_void_p()
    _check(lib().asj_build(ctypes.byref(k), ctypes.byref(o), ctypes.byref(h), _stream(stream)), "asj_build")
    return Table(h, R)


def asj_probe(t: Table, S: DeviceKeys, out: torch.Tensor, counts: torch.Tensor, stream=None):
    """Launch the probe.  out: int32 [cap, 2]; counts: int64 [2] -> (|T|, candidates)."""
    k = S.c()
    cap = _need_pairs(out, "asj_probe out")
    _need_dev(counts, torch.int64, 2, "asj_probe counts")
    _check(lib().asj_probe(t.handle, ctypes.byref(k), ctypes.c_void_p(out.data_ptr() if cap else None), cap,
                           ctypes.c_void_p(counts.data_ptr()), ctypes.c_void_p(counts.data_ptr() + 8),
                           _stream(stream)), "asj_probe")


def asj_join(R: DeviceKeys, S: DeviceKeys, out: torch.Tensor, counts: torch.Tensor, f: int = 16, nsym: int = 2,
             load_factor: float = 0.0, flags: int = 0, keys_per_window: int = 0, grid_rounds: int = 0, stream=None):
    """Launch a whole join.  out: int32 [cap, 2]; counts: int64 [2] -> (|T|, candidates)."""
    kr, ks = R.c(), S.c()
    o = _opts(f, nsym, load_factor, flags, keys_per_window, grid_rounds)
    cap = _need_pairs(out, "asj_join out")
    _need_dev(counts, torch.int64, 2, "asj_join counts")
    _check(lib().asj_join(ctypes.byref(kr), ctypes.byref(ks), ctypes.byref(o),
                          ctypes.c_void_p(out.data_ptr() if cap else None), cap, ctypes.c_void_p(counts.data_ptr()),
                          ctypes.c_void_p(counts.data_ptr() + 8), _stream(stream)), "asj_join")


ASJ_NOALLOC_MAX_BUILD_ROWS = 10240
ASJ_NOALLOC_SCRATCH_BYTES = 65536


def asj_join_noalloc(R: DeviceKeys, S: DeviceKeys, out: torch.Tensor, counts: torch.Tensor, f: int = 16,
                     nsym: int = 2, load_factor: float = 0.0, flags: int = 0, keys_per_window: int = 0,
                     grid_rounds: int = 0, stream=None):
    """asj_join for at most ASJ_NOALLOC_MAX_BUILD_ROWS build rows without any device allocation (the
    library's fixed scratch array; calls overlapping on one device race).  out: int32 [cap, 2];
    counts: int64 [2] -> (|T|, candidates)."""
    kr, ks = R.c(), S.c()
    o = _opts(f, nsym, load_factor, flags, keys_per_window, grid_rounds)
    cap = _need_pairs(out, "asj_join_noalloc out")
    _need_dev(counts, torch.int64, 2, "asj_join_noalloc counts")
    _check(lib().asj_join_noalloc(ctypes.byref(kr), ctypes.byref(ks), ctypes.byref(o),
                                  ctypes.c_void_p(out.data_ptr() if cap else None), cap,
                                  ctypes.c_void_p(counts.data_ptr()), ctypes.c_void_p(counts.data_ptr() + 8),
                                  _stream(stream)), "asj_join_noalloc")


def join(R: DeviceKeys, S: DeviceKeys, cap: Optional[int] = None, **kw):
    """Convenience two-call join: returns (pairs int32 [|T|, 2] on the device, |T|, candidates)."""
    dev = S.offsets.device
    if cap is None:
        cap = max(1024, S.n)
    counts = torch.zeros(2, dtype=torch.int64, device=dev)
    out = torch.empty((cap, 2), dtype=torch.int32, device=dev)
    asj_join(R, S, out, counts, **kw)
    total, ncand = (int(x) for x in counts.tolist())
    if total > cap:
        out = torch.empty((total, 2), dtype=torch.int32, device=dev)
        asj_join(R, S, out, counts, **kw)
        total, ncand = (int(x) for x in counts.tolist())
    return out[:max(total, 0)], total, ncand


@dataclass
class HostKeys:
    """A relation's join attributes in host memory (CPU tensors; pinned ones
    give asj_join_host the full host-link rate)."""
    data: torch.Tensor              # uint8
    offsets: torch.Tensor           # int64, n + 1
    ids: Optional[torch.Tensor]     # int32, n (None -> row index)

    @property
    def n(self) -> int:
        return self.offsets.numel() - 1

    @classmethod
    def from_host(cls, rel, pin=True, with_ids=True) -> "HostKeys":
        """Wrap (and by default pin) a host relation's numpy data/offsets/ids."""
        def t(a):
            x = torch.from_numpy(a)
            return x.pin_memory() if pin else x
        ids = t(rel.ids) if (with_ids and rel.ids is not None) else None
        return cls(t(rel.data), t(rel.offsets), ids)

    def c(self) -> asj_keys:
        for t, dt in ((self.data, torch.uint8), (self.offsets, torch.int64)):
            if t.dtype != dt or t.is_cuda or not t.is_contiguous():
                raise ValueError("host keys: data must be contiguous cpu uint8, offsets contiguous cpu int64")
        if self.ids is not None and (self.ids.dtype != torch.int32 or self.ids.is_cuda or
                                     not self.ids.is_contiguous() or self.ids.numel() != self.n):
            raise ValueError("host keys: ids must be a contiguous cpu int32 tensor of n elements")
        return asj_keys(self.data.data_ptr() if self.data.numel() else None, self.offsets.data_ptr(),
                        self.ids.data_ptr() if self.ids is not None else None, self.n)


def asj_join_host(R: HostKeys, S: HostKeys, out: torch.Tensor, f: int = 16, nsym: int = 2,
                  load_factor: float = 0.0, flags: int = 0, keys_per_window: int = 0, grid_rounds: int = 0, hbm_budget: int = 0,
                  partitions: int = 0, stream=None):
    """Join host-resident relations within a device-memory budget.  out: cpu int32 [cap, 2].
    Returns (|T|, stats dict); the first min(|T|, cap) rows of out hold pairs."""
    if out.is_cuda or out.dtype != torch.int32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous cpu int32 tensor [cap, 2]")
    kr, ks = R.c(), S.c()
    o = _opts(f, nsym, load_factor, flags, keys_per_window, grid_rounds)
    ho = asj_host_opts(int(hbm_budget), int(partitions), 0)
    st = asj_host_stats()
    cnt = ctypes.c_int64(0)
    cap = out.shape[0]
    _check(lib().asj_join_host(ctypes.byref(kr), ctypes.byref(ks), ctypes.byref(o), ctypes.byref(ho),
                               ctypes.c_void_p(out.data_ptr() if cap else None), cap, ctypes.byref(cnt),
                               ctypes.byref(st), _stream(stream)), "asj_join_host")
    stats = {name: getattr(st, name) for name, _ in asj_host_stats._fields_ if name != "reserved"}
    return int(cnt.value), stats


def asj_join_host_release():
    """Free the pinned host regions asj_join_host keeps between calls."""
    _check(lib().asj_join_host_release(), "asj_join_host_release")


def timing_enable(on: bool = True):
    _check(lib().asj_timing_enable(1 if on else 0), "asj_timing_enable")


def timing_read(cap: int = 16):
    ms = (ctypes.c_float * cap)()
    names = (ctypes.c_char_p * cap)()
    n = lib().asj_timing_read(ctypes.cast(ms, ctypes.c_void_p), ctypes.cast(names, ctypes.c_void_p), cap)
    if n < 0:
        raise AsjError(n, "asj_timing_read")
    return [(names[i].decode(), float(ms[i])) for i in range(min(n, cap))]


def asj_util_read(src: torch.Tensor, nbytes: int, out_word: torch.Tensor, grid: int = 0, stream=None):
    _need_dev(out_word, torch.int32, 1, "asj_util_read out_word")
    if not src.is_cuda or not src.is_contiguous() or nbytes < 0 or nbytes > src.numel() * src.element_size():
        raise ValueError("asj_util_read: src must be a contiguous cuda tensor of at least nbytes bytes")
    L = lib()
    L.asj_util_read.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    L.asj_util_read.restype = ctypes.c_int
    _check(L.asj_util_read(ctypes.c_void_p(src.data_ptr()), int(nbytes), ctypes.c_void_p(out_word.data_ptr()),
                           int(grid), _stream(stream)), "asj_util_read")


def asj_util_copy(dst: torch.Tensor, src: torch.Tensor, nbytes: int, stream=None):
    for t, what in ((dst, "dst"), (src, "src")):
        if not t.is_cuda or not t.is_contiguous() or nbytes < 0 or nbytes > t.numel() * t.element_size():
            raise ValueError(f"asj_util_copy: {what} must be a contiguous cuda tensor of at least nbytes bytes")
    _check(lib().asj_util_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), int(nbytes),
                               _stream(stream)), "asj_util_copy")


# ---------------------------------------------------------------------------
# batches of independent joins
# ---------------------------------------------------------------------------

def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


def asj_batch_workspace_bytes(njoins: int, n_build: int, n_probe: int, f: int = 16, nsym: int = 2,
                              load_factor: float = 0.0, flags: int = 0, keys_per_window: int = 0, grid_rounds: int = 0) -> int:
    o = _opts(f, nsym, load_factor, flags, keys_per_window, grid_rounds)
    v = lib().asj_batch_workspace_bytes(int(njoins), int(n_build), int(n_probe), ctypes.byref(o))
    if v < 0:
        raise AsjError(ASJ_EINVAL, "asj_batch_workspace_bytes")
    return int(v)


def asj_join_batch(R: DeviceKeys, S: DeviceKeys, r_seg: torch.Tensor, s_seg: torch.Tensor, out: torch.Tensor,
                   out_seg: torch.Tensor, out_count: torch.Tensor, cand_count: Optional[torch.Tensor] = None,
                   done_clock: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None, f: int = 16,
                   nsym: int = 2, load_factor: float = 0.0, flags: int = 0, keys_per_window: int = 0, grid_rounds: int = 0, stream=None):
    """Launch a batch of joins (see asj_batch in the header).  All tensors on the device:
    r_seg/s_seg/out_seg int64 [J+1], out int32 [*, 2], out_count (and cand_count) int64 [J],
    done_clock int64 [J+1] (device clock ticks), workspace uint8 (optional)."""
    J = r_seg.numel() - 1
    for t in (r_seg, s_seg, out_seg, out_count, cand_count, done_clock):
        if t is not None and (not t.is_cuda or t.dtype != torch.int64 or not t.is_contiguous()):
            raise ValueError("batch: segment, count and clock tensors must be contiguous cuda int64")
    if J < 1 or s_seg.numel() != J + 1 or out_seg.numel() != J + 1:
        raise ValueError("batch: r_seg, s_seg and out_seg must each hold njoins + 1 entries")
    _need_dev(out_count, torch.int64, J, "batch out_count")
    if cand_count is not None:
        _need_dev(cand_count, torch.int64, J, "batch cand_count")
    if done_clock is not None:
        _need_dev(done_clock, torch.int64, J + 1, "batch done_clock")
    _need_pairs(out, "batch out")  # out_seg (read on the device) must stay within out.shape[0]
    if workspace is not None:
        _need_dev(workspace, torch.uint8, 0, "batch workspace")
    b = asj_batch(R.c(), S.c(), _ptr(r_seg), _ptr(s_seg), J, _ptr(out), _ptr(out_seg), _ptr(out_count),
                  _ptr(cand_count), _ptr(done_clock), _ptr(workspace),
                  int(workspace.numel()) if workspace is not None else 0)
    o = _opts(f, nsym, load_factor, flags, keys_per_window, grid_rounds)
    _check(lib().asj_join_batch(ctypes.byref(b), ctypes.byref(o), _stream(stream)), "asj_join_batch")


def _tune_dict(r: asj_tune_result) -> dict:
    b = r.best
    sched = "split" if b.flags & ASJ_PROBE_SPLIT else "fused"
    return {"load_factor": round(float(b.load_factor), 4), "keys_per_window": int(b.keys_per_window),
            "grid_rounds": int(b.grid_rounds), "schedule": sched, "best_ms": round(float(r.best_ms), 4), "default_ms": round(float(r.default_ms), 4),
            "trials": int(r.trials)}


def autotune(R: DeviceKeys, S: DeviceKeys, out: torch.Tensor, out_count: torch.Tensor, f: int = 16, nsym: int = 2,
             flags: int = 0, stream=None) -> dict:
    """Run the library's autotuner on these relations (see asj_autotune); later calls that leave the load
    factor, keys per window, grid rounds and schedule at 0 use its choice."""
    _need_pairs(out, "autotune out")
    _need_dev(out_count, torch.int64, 1, "autotune out_count")
    rk, sk = R.c(), S.c()
    o = _opts(f, nsym, 0.0, flags)
    res = asj_tune_result()
    _check(lib().asj_autotune(ctypes.byref(rk), ctypes.byref(sk), ctypes.byref(o), _ptr(out), out.shape[0],
                              _ptr(out_count), ctypes.byref(res), _stream(stream)), "asj_autotune")
    return _tune_dict(res)


def autotune_batch(R: DeviceKeys, S: DeviceKeys, r_seg: torch.Tensor, s_seg: torch.Tensor, out: torch.Tensor,
                   out_seg: torch.Tensor, out_count: torch.Tensor, f: int = 16, nsym: int = 2, flags: int = 0,
                   stream=None) -> dict:
    J = r_seg.numel() - 1
    for t, what in ((r_seg, "r_seg"), (s_seg, "s_seg"), (out_seg, "out_seg")):
        _need_dev(t, torch.int64, J + 1, f"autotune_batch {what}")
    _need_dev(out_count, torch.int64, J, "autotune_batch out_count")
    _need_pairs(out, "autotune_batch out")
    b = asj_batch(R.c(), S.c(), _ptr(r_seg), _ptr(s_seg), J, _ptr(out), _ptr(out_seg), _ptr(out_count), None,
                  None, None, 0)
    o = _opts(f, nsym, 0.0, flags)
    res = asj_tune_result()
    _check(lib().asj_autotune_batch(ctypes.byref(b), ctypes.byref(o), ctypes.byref(res), _stream(stream)),
           "asj_autotune_batch")
    return _tune_dict(res)


def autotune_clear():
    lib().asj_autotune_clear()


def clock_khz() -> int:
    return int(lib().asj_clock_khz())


def join_batch(R: DeviceKeys, S: DeviceKeys, r_seg_host, s_seg_host, caps=None, **kw):
    """Convenience batch join with the two-call pattern.

    Returns (out int32 [*, 2] on the device, out_seg int64 numpy [J+1],
    counts numpy [J], candidates numpy [J], done_clock numpy [J+1])."""
    import numpy as np
    dev = S.offsets.device
    r_seg_host = np.asarray(r_seg_host, dtype=np.int64)
    s_seg_host = np.asarray(s_seg_host, dtype=np.int64)
    J = len(r_seg_host) - 1
    if caps is None:
        caps = np.diff(s_seg_host) + 16
    r_seg = torch.from_numpy(r_seg_host).to(dev)
    s_seg = torch.from_numpy(s_seg_host).to(dev)
    for _ in range(2):
        out_seg_host = np.zeros(J + 1, dtype=np.int64)
        out_seg_host[1:] = np.cumsum(caps)
        out_seg = torch.from_numpy(out_seg_host).to(dev)
        out = torch.empty((max(int(out_seg_host[-1]), 1), 2), dtype=torch.int32, device=dev)
        counts = torch.zeros(J, dtype=torch.int64, device=dev)
        cands = torch.zeros(J, dtype=torch.int64, device=dev)
        clock = torch.zeros(J + 1, dtype=torch.int64, device=dev)
        asj_join_batch(R, S, r_seg, s_seg, out, out_seg, counts, cands, clock, **kw)
        c = counts.cpu().numpy()
        if (c <= caps).all():
            break
        caps = np.maximum(caps, c)
    return out, out_seg_host, c, cands.cpu().numpy(), clock.cpu().numpy()


# ---------------------------------------------------------------------------
# serving: probe requests against a resident table
# ---------------------------------------------------------------------------

class asj_server_opts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("hbm_budget", ctypes.c_int64), ("max_batch_keys", ctypes.c_int64),
                ("max_batch_requests", ctypes.c_int32), ("dry_run", ctypes.c_int32),
                ("dry_ns_per_key", ctypes.c_double)]


class asj_request_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("count", ctypes.c_int64), ("t_arrive_ms", ctypes.c_double),
                ("t_launch_ms", ctypes.c_double), ("t_done_ms", ctypes.c_double), ("batch_id", ctypes.c_int32),
                ("batch_requests", ctypes.c_int32), ("t_device_ms", ctypes.c_double),
                ("t_kernel_ms", ctypes.c_double)]


class asj_server_stats_t(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int64), ("busy_slots", ctypes.c_int64), ("budget_used", ctypes.c_int64),
                ("peak_budget_used", ctypes.c_int64), ("launches", ctypes.c_int64), ("now_ms", ctypes.c_double)]


def _server_lib():
    L = lib()
    if not getattr(L, "_server_ready", False):
        P, I64 = ctypes.c_void_p, ctypes.c_int64
        L.asj_server_create.argtypes = [P, ctypes.POINTER(asj_server_opts), ctypes.POINTER(P)]
        L.asj_server_submit.argtypes = [P, P, P, I64, P, I64, ctypes.POINTER(I64)]
        L.asj_server_wait.argtypes = [P, I64, ctypes.POINTER(asj_request_info)]
        L.asj_server_stats.argtypes = [P, ctypes.POINTER(asj_server_stats_t)]
        L.asj_server_destroy.argtypes = [P]
        for name in ("asj_server_create", "asj_server_submit", "asj_server_wait", "asj_server_stats",
                     "asj_server_destroy"):
            getattr(L, name).restype = ctypes.c_int
        L._server_ready = True
    return L


def _host_ptr(a):
    """Address of a host buffer: a numpy array or a CPU torch tensor (pinned or not)."""
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        if a.is_cuda or not a.is_contiguous():
            raise ValueError("server buffers must be contiguous host tensors")
        return ctypes.c_void_p(a.data_ptr()) if a.numel() else None
    if not a.flags["C_CONTIGUOUS"]:
        raise ValueError("server buffers must be contiguous")
    return ctypes.c_void_p(a.ctypes.data) if a.size else None


class Server:
    """asj_server: continuous-batching probe server over a resident table."""

    def __init__(self, table: Optional[Table], slots: int = 4, hbm_budget: int = 0, max_batch_keys: int = 0,
                 max_batch_requests: int = 0, dry_run: bool = False, dry_ns_per_key: float = 0.0):
        L = _server_lib()
        o = asj_server_opts(slots, int(hbm_budget), int(max_batch_keys), int(max_batch_requests),
                            1 if dry_run else 0, float(dry_ns_per_key))
        h = ctypes.c_void_p()
        _check(L.asj_server_create(table.handle if table is not None else None, ctypes.byref(o), ctypes.byref(h)),
               "asj_server_create")
        self.handle = h
        self.table = table
        self._live = {}

    def submit(self, data, offsets, out, out_cap: Optional[int] = None) -> int:
        """Queue a request; data uint8 / offsets int64 / out int32 [cap, 2] host buffers kept alive until wait()."""
        def dtype_of(a):
            return a.dtype if isinstance(a, torch.Tensor) else torch.from_numpy(a[:0]).dtype
        if dtype_of(offsets) != torch.int64 or (data is not None and dtype_of(data) != torch.uint8):
            raise ValueError("server request: data must be uint8 and offsets int64")
        n = (offsets.numel() if isinstance(offsets, torch.Tensor) else offsets.size) - 1
        rows = 0
        if out is not None:
            if dtype_of(out) != torch.int32 or len(out.shape) != 2 or out.shape[1] != 2:
                raise ValueError("server request: out must be an int32 buffer of shape [cap, 2]")
            rows = out.shape[0]
        cap = rows if out_cap is None else int(out_cap)
        if cap < 0 or cap > rows:
            raise ValueError(f"server request: out_cap {cap} exceeds the {rows} rows of out")
        t = ctypes.c_int64()
        _check(_server_lib().asj_server_submit(self.handle, _host_ptr(data), _host_ptr(offsets), n, _host_ptr(out),
                                               int(cap), ctypes.byref(t)), "asj_server_submit")
        self._live[t.value] = (data, offsets, out)
        return t.value

    def wait(self, ticket: int) -> dict:
        info = asj_request_info()
        rc = _server_lib().asj_server_wait(self.handle, int(ticket), ctypes.byref(info))
        if rc != ASJ_EINVAL:  # EINVAL: another caller waits on the ticket and still needs its buffers
            self._live.pop(ticket, None)
        return {"status": rc, "count": int(info.count), "t_arrive_ms": info.t_arrive_ms,
                "t_launch_ms": info.t_launch_ms, "t_done_ms": info.t_done_ms, "batch_id": info.batch_id,
                "batch_requests": info.batch_requests, "t_device_ms": info.t_device_ms,
                "t_kernel_ms": info.t_kernel_ms}

    def stats(self) -> dict:
        st = asj_server_stats_t()
        _check(_server_lib().asj_server_stats(self.handle, ctypes.byref(st)), "asj_server_stats")
        return {k: getattr(st, k) for k, _ in st._fields_}

    def close(self):
        if self.handle:
            _check(_server_lib().asj_server_destroy(self.handle), "asj_server_destroy")
            self.handle = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
