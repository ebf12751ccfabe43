"""ctypes binding of the CPU encoders in ``encoders.c`` (input production only)."""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "encoders.c")
_LIB_PATH = os.path.join(_HERE, "libencoders.so")
_lib = None
_lock = threading.Lock()

# RLE v2 sub-encoding choices for encode_rle_v2's seg_kind.
AUTO, SHORT_REPEAT, DIRECT, PATCHED_BASE, DELTA = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", _SRC,
                               "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            vp, sz = ctypes.c_void_p, ctypes.c_size_t
            lib.enc_rle_v1.argtypes = [vp, sz, vp]
            lib.enc_rle_v1.restype = sz
            lib.enc_rle_v2.argtypes = [vp, vp, vp, sz, vp]
            lib.enc_rle_v2.restype = sz
            lib.enc_bound.argtypes = [sz]
            lib.enc_bound.restype = sz
            _lib = lib
    return _lib


def encode_rle_v1(values: np.ndarray) -> bytes:
    """Greedy ORC integer RLE v1 encoding of a signed int64 array."""
    lib = _load()
    v = np.ascontiguousarray(values, dtype=np.int64)
    out = np.empty(lib.enc_bound(v.size), dtype=np.uint8)
    n = lib.enc_rle_v1(v.ctypes.data, v.size, out.ctypes.data)
    return out[:n].tobytes()


def encode_rle_v2(values: np.ndarray, seg_len=None, seg_kind=None) -> bytes:
    """ORC integer RLE v2 encoding.

    ``seg_len``/``seg_kind`` split the values into consecutive segments, each
    encoded with the given sub-encoding (AUTO, SHORT_REPEAT, DIRECT,
    PATCHED_BASE or DELTA; a segment that does not suit its sub-encoding falls
    back to DIRECT).  Without them the whole array uses the automatic choice.
    """
    lib = _load()
    v = np.ascontiguousarray(values, dtype=np.int64)
    if seg_len is None:
        seg_len = np.array([v.size], dtype=np.int64)
        seg_kind = np.array([AUTO], dtype=np.uint8)
    sl = np.ascontiguousarray(seg_len, dtype=np.int64)
    sk = np.ascontiguousarray(seg_kind, dtype=np.uint8)
    assert int(sl.sum()) == v.size and sl.size == sk.size
    out = np.empty(lib.enc_bound(v.size), dtype=np.uint8)
    n = lib.enc_rle_v2(v.ctypes.data, sl.ctypes.data if sl.size else 0,
                       sk.ctypes.data if sk.size else 0, sl.size, out.ctypes.data)
    return out[:n].tobytes()


def encode_byte_rle(data: bytes) -> bytes:
    """ORC byte RLE, greedy: a stretch of 3 or more equal bytes becomes runs
    of up to 130 (header = length - 3, then the byte); everything else goes
    out as literal lists of up to 128 bytes (header = -count)."""
    b = bytes(data)
    out = bytearray()
    lit = bytearray()

    def flush_lit():
        while lit:
            k = min(len(lit), 128)
            out.append(256 - k)
            out.extend(lit[:k])
            del lit[:k]

    i, n = 0, len(b)
    while i < n:
        j = i
        while j < n and b[j] == b[i] and j - i < 130:
            j += 1
        if j - i >= 3:
            flush_lit()
            out.append(j - i - 3)
            out.append(b[i])
            i = j
        else:
            lit.append(b[i])
            i += 1
    flush_lit()
    return bytes(out)
