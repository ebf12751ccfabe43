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

ORDER_INDEX, ORDER_GIVEN, ORDER_LEARNED, ORDER_CODEC = 0, 1, 2, 3
SCHED_BLOB_BYTES = 8 + 16 + 4 * (5313 + 34) + 8
SCHED_FEATURES, SCHED_PARAMS, SCHED_NORM = 16, 5313, 34
OK = 0
RLE_V1, RLE_V2, DEFLATE, BYTE_RLE, LZ4 = 1, 2, 3, 4, 5
VARIANT_DEFAULT, VARIANT_LEADER_LANE, VARIANT_PREFETCH_WAVE, VARIANT_BLOCK_LEADER = 0, 1, 2, 3
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
                ("group_parallel", ctypes.c_int), ("variant", ctypes.c_int),
                ("elem_bytes", ctypes.c_int), ("unsigned_values", ctypes.c_int),
                ("reserved", ctypes.c_int * 3)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("waves_per_cu", ctypes.c_int), ("waves_per_block", ctypes.c_int),
                ("lit_table_bits", ctypes.c_int), ("history_kib", ctypes.c_int),
                ("order", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("chunks_per_claim", ctypes.c_int), ("reserved", ctypes.c_int * 9)]


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
            L.codag_decompress_noalloc.argtypes = [i32, vp, vp, vp, vp, u64, vp, vp, ctypes.POINTER(Opts)]
            L.codag_decompress_noalloc.restype = i32
            L.codag_orc_inflate_stream.argtypes = [vp, u64, ctypes.c_uint32, vp, u64, vp, vp, vp]
            L.codag_orc_inflate_stream.restype = i32
            L.codag_orc_decompress_stream.argtypes = [i32, vp, u64, ctypes.c_uint32, vp, u64, vp, vp, vp]
            L.codag_orc_decompress_stream.restype = i32
            L.codag_get_error.argtypes = [vp, ctypes.POINTER(u64)]
            L.codag_get_error.restype = i32
            L.codag_status_string.argtypes = [i32]
            L.codag_status_string.restype = ctypes.c_char_p
            L.codag_shutdown.argtypes = []
            L.codag_shutdown.restype = None
            bo = ctypes.POINTER(BatchOpts)
            fp, dp = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)
            sigs = {
                "codag_plan_create": [ctypes.POINTER(vp), bo],
                "codag_plan_get_opts": [vp, bo],
                "codag_plan_set_opts": [vp, bo],
                "codag_decompress_batch": [vp, vp, vp, vp, vp, vp, u64, vp, vp, vp, vp],
                "codag_autotune": [vp, vp, vp, vp, vp, vp, u64, vp, i32, dp, vp],
                "codag_sched_features": [vp, vp, vp, vp, vp, u64, vp, vp],
                "codag_sched_set_params": [vp, fp, fp],
                "codag_sched_get_params": [vp, fp, fp],
                "codag_sched_train": [vp, vp, vp, u64, i32, ctypes.c_float, u64, fp, vp],
                "codag_sched_grad": [vp, vp, vp, u64, fp, fp, vp],
                "codag_sched_predict": [vp, vp, u64, vp, vp],
                "codag_sched_order": [vp, vp, vp, vp, vp, u64, vp, vp],
                "codag_sched_save": [vp, vp, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
                "codag_sched_load": [vp, vp, ctypes.c_size_t],
                "codag_autotune_cache_save": [ctypes.c_char_p, ctypes.c_size_t,
                                              ctypes.POINTER(ctypes.c_size_t)],
                "codag_autotune_cache_load": [ctypes.c_char_p],
            }
            for name, args in sigs.items():
                fn = getattr(L, name)
                fn.argtypes = args
                fn.restype = i32
            L.codag_plan_destroy.argtypes = [vp]
            L.codag_plan_destroy.restype = None
            L.codag_autotune_cache_clear.argtypes = []
            L.codag_autotune_cache_clear.restype = None
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
               group_parallel: int = 0, chunk_ticks=None, variant: int = 0, elem_bytes: int = 0,
               unsigned_values: bool = False, stream=None) -> None:
    """Enqueue codag_decompress_ex on `stream` (default: torch's current stream).

    comp: uint8 device tensor; chunk_offsets/out_offsets: int64 device tensors of
    n_chunks + 1 offsets; out: uint8 device tensor; status: optional int32 device
    tensor of n_chunks; chunk_ticks: optional int64 device tensor of n_chunks.
    """
    _decompress("codag_decompress_ex", codec, comp, chunk_offsets, out, out_offsets, status,
                waves_per_block, lit_table_bits, history_kib, group_parallel, chunk_ticks, variant,
                elem_bytes, unsigned_values, stream)


def _decompress(entry, codec, comp, chunk_offsets, out, out_offsets, status, waves_per_block,
                lit_table_bits, history_kib, group_parallel, chunk_ticks, variant, elem_bytes,
                unsigned_values, stream):
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
    opts = Opts(waves_per_block, lit_table_bits, t, history_kib, group_parallel, variant,
                elem_bytes, int(unsigned_values), (ctypes.c_int * 3)())
    rc = getattr(lib(), entry)(int(codec), a, b, c, d, n, _stream_handle(stream), s,
                               ctypes.byref(opts))
    if rc != OK:
        raise CodagError(rc, entry)


def decompress_noalloc(codec: int, comp, chunk_offsets, out, out_offsets, *, status=None,
                       waves_per_block: int = 0, lit_table_bits: int = 0, history_kib: int = 0,
                       group_parallel: int = 0, chunk_ticks=None, variant: int = 0,
                       elem_bytes: int = 0, unsigned_values: bool = False, stream=None) -> None:
    """Enqueue codag_decompress_noalloc (arguments as decompress()): the same
    decode with every workspace in the library's static per-device scratch
    array; calls that overlap in time on one device must not be made."""
    _decompress("codag_decompress_noalloc", codec, comp, chunk_offsets, out, out_offsets, status,
                waves_per_block, lit_table_bits, history_kib, group_parallel, chunk_ticks, variant,
                elem_bytes, unsigned_values, stream)


def orc_inflate_stream(framed, block_size: int, out, out_len, status, *, stream=None) -> None:
    """Enqueue codag_orc_inflate_stream: framed (uint8 device tensor, the
    compressed ORC stream), out (uint8 device tensor, capacity out.numel()),
    out_len (int64 device tensor of 1), status (int32 device tensor of 1)."""
    import torch
    a = _check_dev(framed, "framed", (torch.uint8,))
    b = _check_dev(out, "out", (torch.uint8,))
    c = _check_dev(out_len, "out_len", (torch.int64,), 1)
    d = _check_dev(status, "status", (torch.int32,), 1)
    rc = lib().codag_orc_inflate_stream(a, framed.numel(), int(block_size), b, out.numel(), c, d,
                                        _stream_handle(stream))
    if rc != OK:
        raise CodagError(rc, "codag_orc_inflate_stream")


def orc_decompress_stream(codec: int, framed, block_size: int, out, out_len, status, *,
                          stream=None) -> None:
    """Enqueue codag_orc_decompress_stream: as orc_inflate_stream for a
    stream of ORC's ZLIB (codec DEFLATE) or LZ4 (codec LZ4) codec."""
    import torch
    a = _check_dev(framed, "framed", (torch.uint8,))
    b = _check_dev(out, "out", (torch.uint8,))
    c = _check_dev(out_len, "out_len", (torch.int64,), 1)
    d = _check_dev(status, "status", (torch.int32,), 1)
    rc = lib().codag_orc_decompress_stream(int(codec), a, framed.numel(), int(block_size), b,
                                           out.numel(), c, d, _stream_handle(stream))
    if rc != OK:
        raise CodagError(rc, "codag_orc_decompress_stream")


def autotune_cache_save() -> str:
    """codag_autotune_cache_save: the process's autotune cache as text."""
    n = ctypes.c_size_t(0)
    lib().codag_autotune_cache_save(None, 0, ctypes.byref(n))
    buf = ctypes.create_string_buffer(n.value)
    _check(lib().codag_autotune_cache_save(buf, n.value, ctypes.byref(n)), "codag_autotune_cache_save")
    return buf.value.decode()


def autotune_cache_load(text: str) -> None:
    """codag_autotune_cache_load."""
    _check(lib().codag_autotune_cache_load(text.encode()), "codag_autotune_cache_load")


def autotune_cache_clear() -> None:
    lib().codag_autotune_cache_clear()


def get_error(stream=None):
    """(status, first bad chunk or None) since the last call; synchronizes `stream`."""
    first = ctypes.c_uint64(0)
    rc = lib().codag_get_error(_stream_handle(stream), ctypes.byref(first))
    return rc, (None if first.value == 0xFFFFFFFFFFFFFFFF else int(first.value))


def shutdown() -> None:
    lib().codag_shutdown()


def _check(rc, what):
    if rc != OK:
        raise CodagError(rc, what)


def _offsets_dtypes():
    import torch
    return (torch.int64, torch.uint64) if hasattr(torch, "uint64") else (torch.int64,)


def _floats(n, values=None):
    arr = (ctypes.c_float * n)()
    if values is not None:
        import numpy as np
        v = np.ascontiguousarray(np.asarray(values, dtype=np.float32).reshape(-1))
        if v.size != n:
            raise ValueError(f"expected {n} floats, got {v.size}")
        ctypes.memmove(arr, v.ctypes.data, 4 * n)
    return arr


class Plan:
    """A batched-launch plan (codag_plan_*) on the current device.

    Holds the persistent kernel's queue, a captured graph per argument set and
    the learned cost model.  Calls on one plan must not overlap in time.
    """

    def __init__(self, *, waves_per_cu: int = 0, waves_per_block: int = 0, lit_table_bits: int = 0,
                 history_kib: int = 0, order: int = ORDER_INDEX, use_graph: bool = False,
                 chunks_per_claim: int = 0):
        self._h = ctypes.c_void_p()
        o = BatchOpts(waves_per_cu, waves_per_block, lit_table_bits, history_kib, order,
                      int(use_graph), chunks_per_claim)
        _check(lib().codag_plan_create(ctypes.byref(self._h), ctypes.byref(o)), "codag_plan_create")

    def close(self) -> None:
        if self._h:
            lib().codag_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def opts(self) -> dict:
        o = BatchOpts()
        _check(lib().codag_plan_get_opts(self._h, ctypes.byref(o)), "codag_plan_get_opts")
        return {k: getattr(o, k) for k, _ in BatchOpts._fields_ if k != "reserved"}

    def set_opts(self, **kw) -> None:
        cur = self.opts
        cur.update(kw)
        o = BatchOpts(*(int(cur[k]) for k, _ in BatchOpts._fields_ if k != "reserved"))
        _check(lib().codag_plan_set_opts(self._h, ctypes.byref(o)), "codag_plan_set_opts")

    def _args(self, codecs, comp, chunk_offsets, out, out_offsets):
        import torch
        n = chunk_offsets.numel() - 1
        if n < 0 or out_offsets.numel() != n + 1:
            raise ValueError("offset arrays must hold n_chunks + 1 entries")
        offs = _offsets_dtypes()
        return n, [_check_dev(codecs, "codecs", (torch.uint8,), n),
                   _check_dev(comp, "comp", (torch.uint8,)),
                   _check_dev(chunk_offsets, "chunk_offsets", offs),
                   _check_dev(out, "out", (torch.uint8,)) if out is not None else None,
                   _check_dev(out_offsets, "out_offsets", offs)]

    def decompress(self, codecs, comp, chunk_offsets, out, out_offsets, *, status=None,
                   order=None, chunk_ticks=None, stream=None) -> None:
        """Enqueue codag_decompress_batch; tensors as in decompress(), plus
        codecs (uint8, n), order (int32 permutation, n) and chunk_ticks (int64, n)."""
        import torch
        n, (a, b, c, d, e) = self._args(codecs, comp, chunk_offsets, out, out_offsets)
        st = _check_dev(status, "status", (torch.int32,), n)
        od = _check_dev(order, "order", (torch.int32,), n)
        tk = _check_dev(chunk_ticks, "chunk_ticks", (torch.int64,), n)
        _check(lib().codag_decompress_batch(self._h, a, b, c, d, e, n, st, od, tk,
                                            _stream_handle(stream)), "codag_decompress_batch")

    def autotune(self, codecs, comp, chunk_offsets, out, out_offsets, *, order=None,
                 reps: int = 3, stream=None) -> float:
        """Run codag_autotune; returns the best time per launch in ms."""
        import torch
        n, (a, b, c, d, e) = self._args(codecs, comp, chunk_offsets, out, out_offsets)
        od = _check_dev(order, "order", (torch.int32,), n)
        best = ctypes.c_double(0)
        _check(lib().codag_autotune(self._h, a, b, c, d, e, n, od, int(reps), ctypes.byref(best),
                                    _stream_handle(stream)), "codag_autotune")
        return best.value

    # -- cost model -------------------------------------------------------

    def features(self, codecs, comp, chunk_offsets, out_offsets, *, stream=None):
        """n x 16 float32 device tensor of header features."""
        import torch
        n, (a, b, c, _, e) = self._args(codecs, comp, chunk_offsets, None, out_offsets)
        feat = torch.empty((n, SCHED_FEATURES), dtype=torch.float32, device=comp.device)
        _check(lib().codag_sched_features(self._h, a, b, c, e, n, ctypes.c_void_p(feat.data_ptr()),
                                          _stream_handle(stream)), "codag_sched_features")
        return feat

    def set_params(self, params, norm) -> None:
        _check(lib().codag_sched_set_params(self._h, _floats(SCHED_PARAMS, params),
                                            _floats(SCHED_NORM, norm)), "codag_sched_set_params")

    def get_params(self):
        import numpy as np
        p, q = _floats(SCHED_PARAMS), _floats(SCHED_NORM)
        _check(lib().codag_sched_get_params(self._h, p, q), "codag_sched_get_params")
        return np.ctypeslib.as_array(p).copy(), np.ctypeslib.as_array(q).copy()

    def save_model(self) -> bytes:
        """codag_sched_save: the model as SCHED_BLOB_BYTES bytes."""
        buf = ctypes.create_string_buffer(SCHED_BLOB_BYTES)
        n = ctypes.c_size_t(0)
        _check(lib().codag_sched_save(self._h, buf, SCHED_BLOB_BYTES, ctypes.byref(n)),
               "codag_sched_save")
        return buf.raw[: n.value]

    def load_model(self, blob: bytes) -> None:
        """codag_sched_load."""
        b = bytes(blob)
        _check(lib().codag_sched_load(self._h, ctypes.c_char_p(b), len(b)), "codag_sched_load")

    def _feat_target(self, feat, target):
        import torch
        n = feat.shape[0]
        if feat.dim() != 2 or feat.shape[1] != SCHED_FEATURES:
            raise ValueError("feat must be n x 16")
        return n, _check_dev(feat, "feat", (torch.float32,)), \
            _check_dev(target, "target", (torch.float32,), n)

    def train(self, feat, target, *, steps: int, lr: float = 1e-3, seed: int = 0, stream=None):
        """codag_sched_train; returns the loss before each step (numpy)."""
        import numpy as np
        n, f, t = self._feat_target(feat, target)
        losses = _floats(max(steps, 1))
        _check(lib().codag_sched_train(self._h, f, t, n, int(steps), float(lr), int(seed), losses,
                                       _stream_handle(stream)), "codag_sched_train")
        return np.ctypeslib.as_array(losses)[:steps].copy()

    def grad(self, feat, target, *, stream=None):
        """(loss, gradient over the packed parameters) at the current model."""
        import numpy as np
        n, f, t = self._feat_target(feat, target)
        g, l = _floats(SCHED_PARAMS), _floats(1)
        _check(lib().codag_sched_grad(self._h, f, t, n, g, l, _stream_handle(stream)),
               "codag_sched_grad")
        return float(l[0]), np.ctypeslib.as_array(g).copy()

    def predict(self, feat, *, stream=None):
        import torch
        n = feat.shape[0]
        pred = torch.empty(n, dtype=torch.float32, device=feat.device)
        _check(lib().codag_sched_predict(self._h, _check_dev(feat, "feat", (torch.float32,)), n,
                                         ctypes.c_void_p(pred.data_ptr()), _stream_handle(stream)),
               "codag_sched_predict")
        return pred

    def order(self, codecs, comp, chunk_offsets, out_offsets, *, stream=None):
        """The learned queue order (int32 device tensor)."""
        import torch
        n, (a, b, c, _, e) = self._args(codecs, comp, chunk_offsets, None, out_offsets)
        order = torch.empty(n, dtype=torch.int32, device=comp.device)
        _check(lib().codag_sched_order(self._h, a, b, c, e, n, ctypes.c_void_p(order.data_ptr()),
                                       _stream_handle(stream)), "codag_sched_order")
        return order
