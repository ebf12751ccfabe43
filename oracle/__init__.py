"""Oracle: TEST INFRASTRUCTURE ONLY.

Plain, slow CPU implementations of what the GPU path computes, used to prove
parity.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import this package; the GPU library and its Python
binding never do, and share no code, header, table or constant with it.

* ``oracle.c`` -- sequential decoders for ORC integer RLE v1/v2 (signed or
  unsigned, 1/2/4/8-byte elements), ORC byte RLE and Deflate (CODAG,
  Section II-A and Section V-A; bit layouts from the Apache ORC
  run-length encodings and RFC 1951), and ORC's compressed-stream framing.
* ``mlp.py`` -- float64 forward/backward/Adam of the 16-64-64-1 cost model.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

RLE_V1, RLE_V2, DEFLATE, BYTE_RLE, LZ4 = 1, 2, 3, 4, 5
OK, E_INVALID_ARGUMENT, E_CORRUPT, E_TRUNCATED, E_OVERFLOW, E_UNDERFLOW = 0, -1, -3, -4, -5, -6

_lib = None
_lock = threading.Lock()


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no intrinsics)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC",
                               "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            u8p = ctypes.POINTER(ctypes.c_uint8)
            u64p = ctypes.POINTER(ctypes.c_uint64)
            lib.oracle_decode_chunk.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64,
                                                ctypes.c_void_p, ctypes.c_uint64, u64p]
            lib.oracle_decode_chunk.restype = ctypes.c_int
            lib.oracle_decompress.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                              ctypes.c_void_p]
            lib.oracle_decompress.restype = ctypes.c_int
            lib.oracle_decompress_ex.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                                 ctypes.c_void_p]
            lib.oracle_decompress_ex.restype = ctypes.c_int
            lib.oracle_decode_chunk_ex.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                   ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                                   ctypes.c_uint64, u64p]
            lib.oracle_decode_chunk_ex.restype = ctypes.c_int
            lib.oracle_orc_inflate_stream.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                                      ctypes.c_void_p, ctypes.c_uint64, u64p]
            lib.oracle_orc_inflate_stream.restype = ctypes.c_int
            lib.oracle_orc_decompress_stream.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64,
                                                         ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint64,
                                                         u64p]
            lib.oracle_orc_decompress_stream.restype = ctypes.c_int
            del u8p
            _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data if a.size else 0


def decode_chunk(codec: int, data: bytes | np.ndarray, out_cap: int):
    """Decode one chunk; returns (status, output bytes produced before stopping)."""
    lib = _load()
    src = np.frombuffer(bytes(data), dtype=np.uint8) if not isinstance(data, np.ndarray) else data
    src = np.ascontiguousarray(src, dtype=np.uint8)
    # 8-byte aligned output storage (RLE values are aligned int64s).
    store = np.zeros((out_cap + 7) // 8 + 1, dtype=np.uint64)
    out = store.view(np.uint8)[:out_cap]
    produced = ctypes.c_uint64(0)
    st = lib.oracle_decode_chunk(codec, _ptr(src), src.size, out.ctypes.data, out_cap,
                                 ctypes.byref(produced))
    return st, bytes(out[: produced.value])


def decompress(codec: int, comp: np.ndarray, chunk_offsets: np.ndarray,
               out_offsets: np.ndarray, threads: int = 1):
    """Chunk-array decode on the host.  Returns (out uint8 array, status int32 array).

    With threads > 1 the chunks are split into contiguous ranges decoded
    concurrently (ctypes releases the GIL); each chunk is still decoded by the
    same sequential code.
    """
    lib = _load()
    comp = np.ascontiguousarray(comp, dtype=np.uint8)
    co = np.ascontiguousarray(chunk_offsets, dtype=np.uint64)
    oo = np.ascontiguousarray(out_offsets, dtype=np.uint64)
    n = co.size - 1
    total = int(oo[-1]) if n >= 0 and oo.size else 0
    store = np.zeros(total // 8 + 2, dtype=np.uint64)
    out = store.view(np.uint8)[:total]
    status = np.zeros(max(n, 0), dtype=np.int32)
    if n <= 0:
        return out, status
    if threads <= 1 or n < 2:
        rc = lib.oracle_decompress(codec, _ptr(comp), co.ctypes.data, out.ctypes.data if total else 0,
                                   oo.ctypes.data, n, status.ctypes.data)
        if rc != 0:
            raise ValueError("oracle_decompress rejected its arguments")
        return out, status
    bounds = np.linspace(0, n, min(threads, n) + 1).astype(np.int64)

    def work(i):
        a, b = int(bounds[i]), int(bounds[i + 1])
        if b <= a:
            return 0
        return lib.oracle_decompress(codec, _ptr(comp), co[a:].ctypes.data,
                                     out.ctypes.data if total else 0, oo[a:].ctypes.data,
                                     b - a, status[a:].ctypes.data)

    with ThreadPoolExecutor(max_workers=len(bounds) - 1) as ex:
        rcs = list(ex.map(work, range(len(bounds) - 1)))
    if any(rcs):
        raise ValueError("oracle_decompress rejected its arguments")
    return out, status


def decompress_ex(codec: int, comp: np.ndarray, chunk_offsets: np.ndarray,
                  out_offsets: np.ndarray, *, elem_bytes: int = 8, unsigned: bool = False,
                  capacity: bool = False):
    """decompress() with the element type of the RLE codecs, byte RLE, and
    Deflate output ranges as capacities.  Returns (out, status, produced)."""
    lib = _load()
    comp = np.ascontiguousarray(comp, dtype=np.uint8)
    co = np.ascontiguousarray(chunk_offsets, dtype=np.uint64)
    oo = np.ascontiguousarray(out_offsets, dtype=np.uint64)
    n = co.size - 1
    total = int(oo[-1]) if n >= 0 and oo.size else 0
    store = np.zeros(total // 8 + 2, dtype=np.uint64)
    out = store.view(np.uint8)[:total]
    status = np.zeros(max(n, 0), dtype=np.int32)
    produced = np.zeros(max(n, 0), dtype=np.uint64)
    if n <= 0:
        return out, status, produced
    rc = lib.oracle_decompress_ex(codec, elem_bytes, int(unsigned), int(capacity), _ptr(comp),
                                  co.ctypes.data, store.ctypes.data, oo.ctypes.data, n,
                                  status.ctypes.data, produced.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_decompress_ex rejected its arguments")
    return out, status, produced


def orc_inflate_stream(framed: bytes | np.ndarray, block_size: int, out_cap: int, codec: int = DEFLATE):
    """One compressed ORC stream (ZLIB codec, or LZ4 with codec=LZ4):
    (status, decompressed bytes)."""
    lib = _load()
    src = np.frombuffer(bytes(framed), dtype=np.uint8) if not isinstance(framed, np.ndarray) else framed
    src = np.ascontiguousarray(src, dtype=np.uint8)
    out = np.zeros(max(out_cap, 1), dtype=np.uint8)
    made = ctypes.c_uint64(0)
    st = lib.oracle_orc_decompress_stream(codec, _ptr(src), src.size, block_size, out.ctypes.data,
                                          out_cap, ctypes.byref(made))
    return st, bytes(out[: made.value])
