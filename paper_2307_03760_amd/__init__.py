"""Chunk-parallel decompression on AMD Instinct MI355X (gfx950).

Thin Python binding of ``libcodag.so`` (C ABI declared in ``include/codag.h``):
argument marshalling only.  Every decoding step runs in the library's HIP
kernels; PyTorch supplies device memory and streams.  There is no CPU
fallback: if the library is missing, the functions raise.
"""
from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcodag.so")

RLE_V1, RLE_V2, DEFLATE = 1, 2, 3
OK = 0
E_INVALID_ARGUMENT, E_HIP, E_CORRUPT, E_TRUNCATED, E_OVERFLOW, E_UNDERFLOW = -1, -2, -3, -4, -5, -6

_lib = None
_lock = threading.Lock()


class CodagError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})" if what else status_string(status))


class Opts(ctypes.Structure):
    _fields_ = [("waves_per_block", ctypes.c_int), ("lit_table_bits", ctypes.c_int),
                ("chunk_ticks", ctypes.c_void_p), ("history_kib", ctypes.c_int),
                ("reserved", ctypes.c_int * 7)]


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
            L = ctypes.CDLL(LIB_PATH)
            vp, u64, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
            L.codag_decompress.argtypes = [i32, vp, vp, vp, vp, u64, vp]
            L.codag_decompress.restype = i32
            L.codag_decompress_ex.argtypes = [i32, vp, vp, vp, vp, u64, vp, vp, ctypes.POINTER(Opts)]
            L.codag_decompress_ex.restype = i32
            L.codag_get_error.argtypes = [vp, ctypes.POINTER(u64)]
            L.codag_get_error.restype = i32
            L.codag_status_string.argtypes = [i32]
            L.codag_status_string.restype = ctypes.c_char_p
            L.codag_shutdown.argtypes = []
            L.codag_shutdown.restype = None
            _lib = L
    return _lib


def status_string(status: int) -> str:
    try:
        return lib().codag_status_string(int(status)).decode()
    except ImportError:
        return f"status {status}"


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream))


def _check_dev(t, name, dtype=None, n=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype not in dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected one of {dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


def decompress(codec: int, comp, chunk_offsets, out, out_offsets, *, status=None,
               waves_per_block: int = 0, lit_table_bits: int = 0, history_kib: int = 0,
               chunk_ticks=None, stream=None) -> None:
    """Enqueue codag_decompress_ex on `stream` (default: torch's current stream).

    comp: uint8 device tensor; chunk_offsets/out_offsets: int64 device tensors of
    n_chunks + 1 offsets; out: uint8 device tensor; status: optional int32 device
    tensor of n_chunks; chunk_ticks: optional int64 device tensor of n_chunks.
    """
    import torch
    n = chunk_offsets.numel() - 1
    if n < 0 or out_offsets.numel() != n + 1:
        raise ValueError("offset arrays must hold n_chunks + 1 entries")
    offs = (torch.int64, torch.uint64) if hasattr(torch, "uint64") else (torch.int64,)
    a = _check_dev(comp, "comp", (torch.uint8,))
    b = _check_dev(chunk_offsets, "chunk_offsets", offs)
    c = _check_dev(out, "out", (torch.uint8,))
    d = _check_dev(out_offsets, "out_offsets", offs)
    s = _check_dev(status, "status", (torch.int32,), n)
    t = _check_dev(chunk_ticks, "chunk_ticks", (torch.int64,), n)
    opts = Opts(waves_per_block, lit_table_bits, t, history_kib, (ctypes.c_int * 7)())
    rc = lib().codag_decompress_ex(int(codec), a, b, c, d, n, _stream_handle(stream), s,
                                   ctypes.byref(opts))
    if rc != OK:
        raise CodagError(rc, "codag_decompress_ex")


def get_error(stream=None):
    """(status, first bad chunk or None) since the last call; synchronizes `stream`."""
    first = ctypes.c_uint64(0)
    rc = lib().codag_get_error(_stream_handle(stream), ctypes.byref(first))
    return rc, (None if first.value == 0xFFFFFFFFFFFFFFFF else int(first.value))


def shutdown() -> None:
    lib().codag_shutdown()
