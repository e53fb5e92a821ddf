"""ctypes binding to libhiputf.so (C ABI in include/hiputf.h).

Argument marshalling only: torch supplies device memory and the current HIP
stream; every step of the transcoding runs in the library's gfx950 kernels.
There is no fallback: importing this module without the built library, or
calling it on CPU tensors, raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import NamedTuple

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhiputf.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2109_10433_amd.build`")

OK = 0
BAD_LEAD = 1
TRUNCATED = 2
STRAY_CONTINUATION = 3
OVERLONG = 4
TOO_LARGE = 5
SURROGATE = 6
UNPAIRED_SURROGATE = 7
OUTPUT_TOO_SMALL = 16
INVALID_ARGUMENT = 17
DEVICE = 18
EXCEEDS_SCRATCH = 19
NOALLOC_MAX_BYTES = 1 << 28

OP_VALIDATE_UTF8 = 0
OP_UTF16_LENGTH_FROM_UTF8 = 1
OP_CONVERT_UTF8_TO_UTF16LE = 2
OP_VALIDATE_UTF16LE = 3
OP_UTF8_LENGTH_FROM_UTF16LE = 4
OP_CONVERT_UTF16LE_TO_UTF8 = 5


class HuResult(ctypes.Structure):
    _fields_ = [("error", ctypes.c_int32), ("reserved", ctypes.c_int32), ("count", ctypes.c_uint64)]


class Result(NamedTuple):
    error: int
    count: int


lib = ctypes.CDLL(LIB_PATH)
_p, _sz, _i = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
for _name, _args in [
    ("validate_utf8", [_p, _sz, _p]),
    ("utf16_length_from_utf8", [_p, _sz, _p]),
    ("convert_utf8_to_utf16le", [_p, _sz, _p, _sz, _p]),
    ("validate_utf16le", [_p, _sz, _p]),
    ("utf8_length_from_utf16le", [_p, _sz, _p]),
    ("convert_utf16le_to_utf8", [_p, _sz, _p, _sz, _p]),
    ("convert_valid_utf8_to_utf16le", [_p, _sz, _p, _sz, _p]),
    ("convert_valid_utf16le_to_utf8", [_p, _sz, _p, _sz, _p]),
    ("validate_utf16be", [_p, _sz, _p]),
    ("utf8_length_from_utf16be", [_p, _sz, _p]),
    ("convert_utf16be_to_utf8", [_p, _sz, _p, _sz, _p]),
    ("convert_utf8_to_utf16be", [_p, _sz, _p, _sz, _p]),
]:
    getattr(lib, _name).argtypes = _args
    getattr(lib, _name).restype = HuResult
for _name, _args in [
    ("validate_utf8_async", [_p, _sz, _p, _p, _sz, _p]),
    ("utf16_length_from_utf8_async", [_p, _sz, _p, _p, _sz, _p]),
    ("convert_utf8_to_utf16le_async", [_p, _sz, _p, _sz, _p, _p, _sz, _p]),
    ("validate_utf16le_async", [_p, _sz, _p, _p, _sz, _p]),
    ("utf8_length_from_utf16le_async", [_p, _sz, _p, _p, _sz, _p]),
    ("convert_utf16le_to_utf8_async", [_p, _sz, _p, _sz, _p, _p, _sz, _p]),
    ("convert_valid_utf8_to_utf16le_async", [_p, _sz, _p, _sz, _p, _p, _sz, _p]),
    ("convert_valid_utf16le_to_utf8_async", [_p, _sz, _p, _sz, _p, _p, _sz, _p]),
    ("validate_utf16be_async", [_p, _sz, _p, _p, _sz, _p]),
    ("utf8_length_from_utf16be_async", [_p, _sz, _p, _p, _sz, _p]),
    ("convert_utf16be_to_utf8_async", [_p, _sz, _p, _sz, _p, _p, _sz, _p]),
    ("convert_utf8_to_utf16be_async", [_p, _sz, _p, _sz, _p, _p, _sz, _p]),
    ("convert_utf8_to_utf16le_noalloc", [_p, _sz, _p, _sz, _p, _p]),
]:
    getattr(lib, _name).argtypes = _args
    getattr(lib, _name).restype = _i
class HuBom(ctypes.Structure):
    _fields_ = [("encoding", ctypes.c_int32), ("length", ctypes.c_int32)]


BOM_NONE, BOM_UTF8, BOM_UTF16LE, BOM_UTF16BE = 0, 1, 2, 3
lib.hu_detect_bom.argtypes = [_p, _sz]
lib.hu_detect_bom.restype = HuBom
lib.hu_workspace_bytes.argtypes = [_i, _sz]
lib.hu_workspace_bytes.restype = _sz
lib.hu_tile_bytes.argtypes = [_i, _sz]
lib.hu_tile_bytes.restype = _sz
lib.hu_workspace_init.argtypes = [_p, _sz, _p]
lib.hu_workspace_init.restype = _i
lib.hu_batch_workspace_bytes.argtypes = [ctypes.c_uint32, ctypes.c_uint64]
lib.hu_batch_workspace_bytes.restype = _sz
lib.hu_batch_run.argtypes = [_p, ctypes.c_uint32, ctypes.c_uint64, _p, _p, _p, _p, _p, _sz, _p]
lib.hu_batch_run.restype = _i
lib.hu_batch_graph_create.argtypes = [_p, ctypes.c_uint32, ctypes.c_uint64, _p, _p, _p, _p, _p, _sz,
                                      ctypes.POINTER(ctypes.c_void_p)]
lib.hu_batch_graph_create.restype = _i
lib.hu_graph_launch.argtypes = [_p, _p]
lib.hu_graph_launch.restype = _i
lib.hu_graph_destroy.argtypes = [_p]
lib.hu_graph_destroy.restype = None
lib.hu_tune_batch.argtypes = [_p, ctypes.c_uint32, ctypes.c_uint64, _p, _p, _p, _p, _sz, ctypes.c_char_p, _p,
                              ctypes.POINTER(ctypes.c_double), _p]
lib.hu_tune_batch.restype = _i
lib.hu_tuning_lookup.argtypes = [ctypes.c_char_p, _p]
lib.hu_tuning_lookup.restype = _i
lib.hu_error_name.argtypes = [_i]
lib.hu_error_name.restype = ctypes.c_char_p
lib.hu_shutdown.argtypes = []
lib.hu_shutdown.restype = None

lib.hu_server_create.argtypes = [_p, ctypes.POINTER(_p)]
lib.hu_server_create.restype = _i
lib.hu_server_submit.argtypes = [_p, _p]
lib.hu_server_submit.restype = _i
lib.hu_server_poll.argtypes = [_p, _p, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32), ctypes.c_int64]
lib.hu_server_poll.restype = _i
lib.hu_server_replay.argtypes = [_p, _p, _p, ctypes.c_uint64, _p]
lib.hu_server_replay.restype = _i
lib.hu_server_stats_get.argtypes = [_p, _p]
lib.hu_server_stats_get.restype = _i
lib.hu_server_stats_reset.argtypes = [_p]
lib.hu_server_stats_reset.restype = _i
lib.hu_server_destroy.argtypes = [_p]
lib.hu_server_destroy.restype = None

EXPORTED_BATCH = ["hu_batch_workspace_bytes", "hu_batch_run", "hu_batch_graph_create", "hu_graph_launch",
                  "hu_graph_destroy", "hu_tune_batch", "hu_tuning_lookup"]
EXPORTED_SERVER = ["hu_server_create", "hu_server_submit", "hu_server_poll", "hu_server_replay",
                   "hu_server_stats_get", "hu_server_stats_reset", "hu_server_destroy"]
EXPORTED = EXPORTED_BATCH + EXPORTED_SERVER + [
    "validate_utf8", "utf16_length_from_utf8", "convert_utf8_to_utf16le",
    "validate_utf16le", "utf8_length_from_utf16le", "convert_utf16le_to_utf8",
    "validate_utf8_async", "utf16_length_from_utf8_async", "convert_utf8_to_utf16le_async",
    "validate_utf16le_async", "utf8_length_from_utf16le_async", "convert_utf16le_to_utf8_async",
    "convert_valid_utf8_to_utf16le", "convert_valid_utf16le_to_utf8",
    "convert_valid_utf8_to_utf16le_async", "convert_valid_utf16le_to_utf8_async",
    "validate_utf16be", "utf8_length_from_utf16be", "convert_utf16be_to_utf8", "convert_utf8_to_utf16be",
    "validate_utf16be_async", "utf8_length_from_utf16be_async", "convert_utf16be_to_utf8_async",
    "convert_utf8_to_utf16be_async", "hu_detect_bom", "convert_utf8_to_utf16le_noalloc",
    "hu_workspace_bytes", "hu_tile_bytes", "hu_workspace_init", "hu_error_name", "hu_shutdown",
]


def detect_bom(head: bytes) -> tuple[int, int]:
    """(BOM_* encoding, BOM length in bytes) of a host buffer's first bytes."""
    buf = ctypes.create_string_buffer(bytes(head[:4]), max(len(head[:4]), 1))
    b = lib.hu_detect_bom(ctypes.cast(buf, ctypes.c_void_p), len(head[:4]))
    return int(b.encoding), int(b.length)


def error_name(code: int) -> str:
    return lib.hu_error_name(int(code)).decode()


def stream_handle(stream: torch.cuda.Stream | None = None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check(t: torch.Tensor, dtypes, what: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{what} must have dtype in {dtypes}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t


_U8 = (torch.uint8,)
_U16 = (torch.int16, torch.uint16)


def _res(r: HuResult) -> Result:
    return Result(int(r.error), int(r.count))


def validate_utf8(src: torch.Tensor, stream=None) -> Result:
    _check(src, _U8, "src")
    with torch.cuda.device(src.device):
        return _res(lib.validate_utf8(src.data_ptr(), src.numel(), stream_handle(stream)))


def utf16_length_from_utf8(src: torch.Tensor, stream=None) -> Result:
    _check(src, _U8, "src")
    with torch.cuda.device(src.device):
        return _res(lib.utf16_length_from_utf8(src.data_ptr(), src.numel(), stream_handle(stream)))


def convert_utf8_to_utf16le(src: torch.Tensor, out: torch.Tensor | None = None, stream=None,
                            validate: bool = True):
    """Returns (int16 tensor holding the UTF-16LE words, Result). With `out`
    the words go there (capacity = out.numel()) and `out` is returned whole.
    validate=False: the non-validating call, for input known to be valid."""
    _check(src, _U8, "src")
    fn = lib.convert_utf8_to_utf16le if validate else lib.convert_valid_utf8_to_utf16le
    with torch.cuda.device(src.device):
        dst = out if out is not None else torch.empty(max(src.numel(), 1), dtype=torch.int16, device=src.device)
        _check(dst, _U16, "out")
        r = _res(fn(src.data_ptr(), src.numel(), dst.data_ptr(),
                    dst.numel() if out is not None else src.numel(), stream_handle(stream)))
    if out is not None:
        return out, r
    return dst[: r.count] if r.error == OK else dst[:0], r


def validate_utf16le(src: torch.Tensor, stream=None) -> Result:
    _check(src, _U16, "src")
    with torch.cuda.device(src.device):
        return _res(lib.validate_utf16le(src.data_ptr(), src.numel(), stream_handle(stream)))


def utf8_length_from_utf16le(src: torch.Tensor, stream=None) -> Result:
    _check(src, _U16, "src")
    with torch.cuda.device(src.device):
        return _res(lib.utf8_length_from_utf16le(src.data_ptr(), src.numel(), stream_handle(stream)))


def convert_utf16le_to_utf8(src: torch.Tensor, out: torch.Tensor | None = None, stream=None,
                            validate: bool = True):
    """Returns (uint8 tensor holding the UTF-8 bytes, Result).
    validate=False: the non-validating call, for input known to be valid."""
    _check(src, _U16, "src")
    fn = lib.convert_utf16le_to_utf8 if validate else lib.convert_valid_utf16le_to_utf8
    with torch.cuda.device(src.device):
        dst = out if out is not None else torch.empty(max(3 * src.numel(), 1), dtype=torch.uint8, device=src.device)
        _check(dst, _U8, "out")
        r = _res(fn(src.data_ptr(), src.numel(), dst.data_ptr(),
                    dst.numel() if out is not None else 3 * src.numel(), stream_handle(stream)))
    if out is not None:
        return out, r
    return dst[: r.count] if r.error == OK else dst[:0], r


def workspace(op: int, n_units: int, device=None) -> torch.Tensor:
    """A zero-filled workspace tensor for the *_async calls (256-byte aligned)."""
    nbytes = int(lib.hu_workspace_bytes(op, n_units))
    return torch.zeros(nbytes + 256, dtype=torch.uint8, device=device or "cuda")


def workspace_ptr(ws: torch.Tensor) -> tuple[int, int]:
    """(aligned device pointer, usable bytes) of a workspace tensor."""
    p = ws.data_ptr()
    a = (p + 255) & ~255
    return a, ws.numel() - (a - p)


def result_from_device(rec: torch.Tensor) -> Result:
    """Decode a 16-byte device result record (uint8 tensor) on the host."""
    b = rec.cpu().numpy().tobytes()[:16]
    r = HuResult.from_buffer_copy(b)
    return _res(r)


# ---------------------------------------------------------------- batches

class HuTuning(ctypes.Structure):
    _fields_ = [("sub_tiles", ctypes.c_uint32), ("groups_per_cu", ctypes.c_uint32)]


try:
    import numpy as _np
    DOC_DTYPE = _np.dtype([("src_off", "<u8"), ("n_units", "<u8"), ("dst_off", "<u8"), ("dst_cap", "<u8"),
                           ("op", "<u4"), ("reserved", "<u4")])
except ImportError:  # pragma: no cover
    DOC_DTYPE = None


class Batch:
    """A document table on the device plus its workspace and result records.

    docs: numpy array of DOC_DTYPE (offsets into src / dst). src, dst: device
    tensors holding all inputs / outputs (dst may be None without convert
    operations)."""

    def __init__(self, docs, src: torch.Tensor, dst: torch.Tensor | None = None,
                 total_input_bytes: int | None = None):
        import numpy as np
        self.docs_host = np.ascontiguousarray(docs, dtype=DOC_DTYPE)
        self.n = int(self.docs_host.size)
        self.device = src.device
        self.src = src
        self.dst = dst
        if total_input_bytes is None:
            unit = np.where(self.docs_host["op"] >= OP_VALIDATE_UTF16LE, 2, 1).astype(np.uint64)
            total_input_bytes = int((self.docs_host["n_units"] * unit).sum())
        self.total = int(total_input_bytes)
        self.docs = torch.from_numpy(self.docs_host.view(np.uint8).copy()).to(self.device)
        self.results = torch.zeros((max(self.n, 1), 16), dtype=torch.uint8, device=self.device)
        nbytes = int(lib.hu_batch_workspace_bytes(self.n, self.total))
        self.ws = torch.zeros(nbytes + 256, dtype=torch.uint8, device=self.device)
        self.ws_ptr, self.ws_bytes = workspace_ptr(self.ws)

    def update_docs(self, docs):
        """Rewrite the device document table in place (same count)."""
        import numpy as np
        d = np.ascontiguousarray(docs, dtype=DOC_DTYPE)
        assert d.size == self.n
        self.docs.copy_(torch.from_numpy(d.view(np.uint8).copy()).to(self.device))
        self.docs_host = d

    def _args(self):
        return (self.docs.data_ptr(), self.n, self.total, self.src.data_ptr(),
                self.dst.data_ptr() if self.dst is not None else None, self.results.data_ptr())

    def run(self, tuning: HuTuning | None = None, stream=None) -> int:
        a = self._args()
        return lib.hu_batch_run(*a, ctypes.byref(tuning) if tuning is not None else None,
                                self.ws_ptr, self.ws_bytes, stream_handle(stream))

    def graph(self, tuning: HuTuning | None = None):
        a = self._args()
        h = ctypes.c_void_p()
        rc = lib.hu_batch_graph_create(*a, ctypes.byref(tuning) if tuning is not None else None,
                                       self.ws_ptr, self.ws_bytes, ctypes.byref(h))
        if rc != OK:
            raise RuntimeError(f"graph capture failed: {error_name(rc)}")
        return h

    def tune(self, key: str | None = None, stream=None):
        a = self._args()
        best = HuTuning()
        us = ctypes.c_double()
        rc = lib.hu_tune_batch(*a, self.ws_ptr, self.ws_bytes, key.encode() if key else None,
                               ctypes.byref(best), ctypes.byref(us), stream_handle(stream))
        if rc != OK:
            raise RuntimeError(f"tuning failed: {error_name(rc)}")
        return best, us.value

    def results_host(self):
        """(errors int32 array, counts uint64 array) after synchronising."""
        import numpy as np
        torch.cuda.synchronize(self.device)
        h = self.results[: self.n].cpu().numpy().reshape(-1).view(np.uint8)
        rec = h.view([("error", "<i4"), ("reserved", "<i4"), ("count", "<u8")])
        return rec["error"].copy(), rec["count"].copy()


def graph_launch(handle, stream=None) -> int:
    return lib.hu_graph_launch(handle, stream_handle(stream))


def graph_destroy(handle) -> None:
    lib.hu_graph_destroy(handle)


def tuning_lookup(key: str):
    t = HuTuning()
    rc = lib.hu_tuning_lookup(key.encode(), ctypes.byref(t))
    return t if rc == OK else None


# ---------------------------------------------------------------- server

class HuServerConfig(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_uint64), ("batch_bytes", ctypes.c_uint64),
                ("batch_requests", ctypes.c_uint32), ("max_in_flight", ctypes.c_uint32),
                ("slots", ctypes.c_uint32), ("plain", ctypes.c_uint32), ("tuning", HuTuning)]


class HuServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("input_bytes", ctypes.c_uint64), ("output_bytes", ctypes.c_uint64),
                ("p50_ns", ctypes.c_int64), ("p99_ns", ctypes.c_int64), ("max_ns", ctypes.c_int64),
                ("device_ns", ctypes.c_int64), ("mean_batch", ctypes.c_double)]


def _np_dtypes():
    import numpy as np
    req = np.dtype([("tag", "<u8"), ("op", "<u4"), ("reserved", "<u4"), ("src", "<u8"), ("n_units", "<u8"),
                    ("dst", "<u8"), ("dst_cap", "<u8")])
    comp = np.dtype([("tag", "<u8"), ("error", "<i4"), ("reserved", "<i4"), ("count", "<u8"),
                     ("latency_ns", "<i8")])
    assert req.itemsize == 48 and comp.itemsize == 32
    return req, comp


REQUEST_DTYPE, COMPLETION_DTYPE = _np_dtypes()


class Server:
    """hu_server_*: requests from host (numpy) buffers, batched on the device.

    Buffers handed to submit/replay must stay alive until their requests have
    completed (the caller keeps references)."""

    def __init__(self, pool_bytes=0, batch_bytes=0, batch_requests=0, max_in_flight=0, slots=0, plain=False,
                 tuning: HuTuning | None = None):
        cfg = HuServerConfig(pool_bytes, batch_bytes, batch_requests, max_in_flight, slots, 1 if plain else 0,
                             tuning if tuning is not None else HuTuning(0, 0))
        h = ctypes.c_void_p()
        rc = lib.hu_server_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != OK:
            raise RuntimeError(f"hu_server_create failed: {error_name(rc)}")
        self.h = h

    def close(self):
        if self.h:
            lib.hu_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        self.close()

    @staticmethod
    def request(tag, op, src, dst=None, dst_cap=None):
        """One REQUEST_DTYPE record for numpy buffers src (and dst)."""
        import numpy as np
        r = np.zeros(1, dtype=REQUEST_DTYPE)[0]
        r["tag"], r["op"] = tag, op
        r["src"] = src.ctypes.data if src.size else 0
        r["n_units"] = src.size
        if dst is not None:
            r["dst"] = dst.ctypes.data
            r["dst_cap"] = dst.size if dst_cap is None else dst_cap
        elif dst_cap is not None:
            r["dst_cap"] = dst_cap
        return r

    def submit(self, rec) -> int:
        import numpy as np
        a = np.ascontiguousarray(np.asarray(rec, dtype=REQUEST_DTYPE).reshape(1))
        return lib.hu_server_submit(self.h, a.ctypes.data)

    def poll(self, max_n=1024, timeout_s=0.0):
        import numpy as np
        out = np.zeros(max_n, dtype=COMPLETION_DTYPE)
        n = ctypes.c_uint32()
        rc = lib.hu_server_poll(self.h, out.ctypes.data, max_n, ctypes.byref(n), int(timeout_s * 1e9))
        if rc != OK:
            raise RuntimeError(error_name(rc))
        return out[:n.value]

    def replay(self, reqs, arrival_ns):
        """Open-loop replay of REQUEST_DTYPE records at the given offsets (ns)."""
        import numpy as np
        reqs = np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
        arr = np.ascontiguousarray(arrival_ns, dtype=np.int64)
        out = np.zeros(reqs.size, dtype=COMPLETION_DTYPE)
        rc = lib.hu_server_replay(self.h, reqs.ctypes.data, arr.ctypes.data, reqs.size, out.ctypes.data)
        if rc != OK:
            raise RuntimeError(f"replay failed: {error_name(rc)}")
        return out

    def stats(self) -> dict:
        st = HuServerStats()
        lib.hu_server_stats_get(self.h, ctypes.byref(st))
        return {f: getattr(st, f) for f, _ in HuServerStats._fields_}

    def reset_stats(self):
        lib.hu_server_stats_reset(self.h)
