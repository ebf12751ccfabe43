"""Seeded synthetic workloads: generators and CPU encoders.

This module only produces inputs.  It holds no decoding arithmetic; both the
oracle (in tests) and the GPU path consume what it produces.

The paper's real datasets (CODAG Section V-B, the dataset table) are not
available, so each workload stands in for them with seeded synthetic columns
of the stated shapes:

* ``rle_v1``  -- alternating run groups (length 3..130, delta -128..127,
  base uniform in +-2^40) and literal groups (length 1..128, values uniform in
  +-2^40), cut into 128 KiB chunks of int64 (16,384 values).
* ``rle_v2``  -- segments giving ~25% of values each to SHORT_REPEAT (3..10
  repeats), DIRECT (512 values, widths 1..64), DELTA (512 monotone values,
  steps 1..1000) and PATCHED_BASE (512 values < 2^12 with 2% outliers up to
  2^48), cut into 256 KiB chunks (32,768 values).
* ``deflate`` -- 64 KiB chunks: 50% Zipf(s=1.1) text over a 4,096-word
  random lowercase vocabulary, 30% little-endian int32 columns of 64 distinct
  values, 20% uniform random bytes; zlib level 9 raw deflate (window 32 KiB),
  a seeded third of the compressible chunks with fixed Huffman codes only.
* ``lz4`` -- the ``deflate`` workload's chunks (same classes, same bytes)
  as LZ4 blocks from the reference LZ4 compressor (through pyarrow).
* ``batched`` -- mixed codecs (40/30/30) with log-normal chunk sizes
  (median 64 KiB, clipped to 4 KiB..1 MiB).
* ``learned`` -- Deflate chunks with skewed ratios: random, Zipf text and
  run-heavy int32 thirds; log-normal sizes as in ``batched``.

Chunk j of workload k draws from ``numpy.random.default_rng([seed, k, j])``.
"""
from __future__ import annotations

import multiprocessing as mp
import os
import zlib
from dataclasses import dataclass, field

import numpy as np

from . import enc
from .enc import AUTO, DELTA, DIRECT, PATCHED_BASE, SHORT_REPEAT  # noqa: F401

RLE_V1, RLE_V2, DEFLATE, LZ4 = 1, 2, 3, 5
WL_RLE_V1, WL_RLE_V2, WL_DEFLATE, WL_BATCHED, WL_LEARNED = 1, 2, 3, 4, 5


@dataclass
class Chunked:
    """Compressed chunks laid out back to back (CSR offsets)."""
    codecs: np.ndarray          # uint8 per chunk
    comp: np.ndarray            # uint8, all compressed chunks
    chunk_offsets: np.ndarray   # uint64, n + 1
    out_offsets: np.ndarray     # uint64, n + 1
    info: dict = field(default_factory=dict)

    @property
    def n_chunks(self) -> int:
        return int(self.chunk_offsets.size - 1)

    @property
    def out_bytes(self) -> int:
        return int(self.out_offsets[-1])

    @property
    def comp_bytes(self) -> int:
        return int(self.chunk_offsets[-1])


def workers() -> int:
    """Worker processes for generation: the host's cores, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _pack(codecs, blobs, out_sizes, info=None) -> Chunked:
    n = len(blobs)
    co = np.zeros(n + 1, dtype=np.uint64)
    oo = np.zeros(n + 1, dtype=np.uint64)
    if n:
        co[1:] = np.cumsum([len(b) for b in blobs], dtype=np.uint64)
        oo[1:] = np.cumsum(np.asarray(out_sizes, dtype=np.uint64), dtype=np.uint64)
    comp = np.frombuffer(b"".join(blobs), dtype=np.uint8).copy() if n else np.zeros(0, np.uint8)
    return Chunked(np.asarray(codecs, dtype=np.uint8), comp, co, oo, dict(info or {}))


# ---------------------------------------------------------------------------
# Value generators
# ---------------------------------------------------------------------------

def rle_v1_values(n: int, rng: np.random.Generator) -> np.ndarray:
    """Alternating run groups and literal groups, starting with a run."""
    est = 2 * (n // 66 + 8)
    run_len = rng.integers(3, 131, est)
    lit_len = rng.integers(1, 129, est)
    lens = np.empty(2 * est, dtype=np.int64)
    lens[0::2] = run_len
    lens[1::2] = lit_len
    while lens.sum() < n:  # pragma: no cover - est is generous
        lens = np.concatenate([lens, lens])
    ends = np.cumsum(lens)
    g = int(np.searchsorted(ends, n)) + 1
    lens = lens[:g].copy()
    lens[-1] -= int(ends[g - 1] - n)
    gid = np.repeat(np.arange(g), lens)
    pos = np.arange(n, dtype=np.int64) - np.repeat(np.cumsum(lens) - lens, lens)
    is_run = (gid % 2) == 0
    base = rng.integers(-(1 << 40), (1 << 40) + 1, g)
    delta = rng.integers(-128, 128, g)
    lit = rng.integers(-(1 << 40), (1 << 40) + 1, n)
    vals = np.where(is_run, base[gid] + pos * delta[gid], lit)
    return vals.astype(np.int64)


def _u64(rng, size):
    return rng.integers(0, np.iinfo(np.uint64).max, size, dtype=np.uint64, endpoint=True)


def _unzigzag(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64)
    mag = (z >> np.uint64(1)).astype(np.int64)
    return np.where((z & np.uint64(1)) != 0, ~mag, mag).astype(np.int64)


def rle_v2_segments(n: int, rng: np.random.Generator):
    """Segments giving each sub-encoding about a quarter of the values.

    Returns (values int64[n], seg_len int64[m], seg_kind uint8[m]).
    """
    kinds = np.array([SHORT_REPEAT, DIRECT, DELTA, PATCHED_BASE], dtype=np.uint8)
    w = np.array([1 / 6.5, 1 / 512, 1 / 512, 1 / 512])
    w /= w.sum()
    est = int(n / (w @ np.array([6.5, 512, 512, 512])) * 1.1) + 16
    cls = rng.choice(4, size=est, p=w)
    lens = np.where(cls == 0, rng.integers(3, 11, est), 512).astype(np.int64)
    ends = np.cumsum(lens)
    while ends[-1] < n:  # pragma: no cover
        cls = np.concatenate([cls, cls])
        lens = np.concatenate([lens, lens])
        ends = np.cumsum(lens)
    m = int(np.searchsorted(ends, n)) + 1
    cls, lens = cls[:m].copy(), lens[:m].copy()
    lens[-1] -= int(ends[m - 1] - n)
    sid = np.repeat(np.arange(m), lens)
    starts = np.cumsum(lens) - lens
    pos = np.arange(n, dtype=np.int64) - np.repeat(starts, lens)
    c = cls[sid]
    vals = np.zeros(n, dtype=np.int64)

    # SHORT_REPEAT: a zigzag value needing exactly W bytes, W uniform in 1..8.
    wb = rng.integers(1, 9, m)
    lo = np.where(wb == 1, 0, np.left_shift(np.uint64(1), (8 * (wb - 1)).astype(np.uint64)))
    span = np.where(wb == 8, np.uint64(0) - lo.astype(np.uint64),
                    np.left_shift(np.uint64(1), (8 * wb).astype(np.uint64)) - lo.astype(np.uint64))
    zsr = lo.astype(np.uint64) + _u64(rng, m) % span
    sr_val = _unzigzag(zsr)
    mask = c == 0
    vals[mask] = sr_val[sid[mask]]

    # DIRECT: zigzag values uniform below 2^b, the top bit set once.
    b = rng.integers(1, 65, m).astype(np.uint64)
    mask = c == 1
    if mask.any():
        bb = b[sid[mask]]
        z = _u64(rng, int(mask.sum()))
        z = np.where(bb == 64, z, z & ((np.uint64(1) << bb) - np.uint64(1)))
        top_pos = rng.integers(0, 512, m)
        hit = pos[mask] == np.minimum(top_pos[sid[mask]], lens[sid[mask]] - 1)
        z = np.where(hit, z | (np.uint64(1) << (bb - np.uint64(1))), z)
        vals[mask] = _unzigzag(z)

    # DELTA: monotone timestamps, start uniform in [0, 2^40], steps 1..1000.
    mask = c == 2
    if mask.any():
        start = rng.integers(0, (1 << 40) + 1, m)
        step = rng.integers(1, 1001, n)
        step = np.where(pos == 0, 0, step)
        step = np.where(mask, step, 0)
        cs = np.cumsum(step)
        seg_cs0 = cs[starts]  # cumulative sum at each segment's first value
        vals[mask] = start[sid[mask]] + (cs[mask] - seg_cs0[sid[mask]])

    # PATCHED_BASE: values below 2^12, 2% of them outliers in [2^12, 2^48].
    mask = c == 3
    if mask.any():
        k = int(mask.sum())
        base_v = rng.integers(0, 4096, k)
        out_v = rng.integers(1 << 12, (1 << 48) + 1, k)
        vals[mask] = np.where(rng.random(k) < 0.02, out_v, base_v)

    return vals, lens, kinds[cls]


def _split_segments(seg_len: np.ndarray, seg_kind: np.ndarray, n: int, chunk: int):
    """Split segments at chunk boundaries.  Returns (lens, kinds, first segment per chunk)."""
    seg_ends = np.cumsum(seg_len)
    chunk_ends = np.arange(chunk, n + chunk, chunk, dtype=np.int64)
    chunk_ends[-1] = n
    bounds = np.union1d(seg_ends, chunk_ends)
    lens = np.diff(np.concatenate([[0], bounds]))
    kinds = seg_kind[np.searchsorted(seg_ends, bounds, side="left")]
    first = np.searchsorted(bounds, np.concatenate([[0], chunk_ends]), side="right")
    first[0] = 0
    return lens.astype(np.int64), kinds.astype(np.uint8), first


def _chunk_values_v1(vals: np.ndarray, chunk: int) -> Chunked:
    n = vals.size
    blobs, sizes = [], []
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        blobs.append(enc.encode_rle_v1(vals[a:b]))
        sizes.append(8 * (b - a))
    return _pack([RLE_V1] * len(blobs), blobs, sizes)


def _chunk_values_v2(vals, seg_len, seg_kind, chunk: int) -> Chunked:
    n = vals.size
    lens, kinds, first = _split_segments(seg_len, seg_kind, n, chunk)
    blobs, sizes = [], []
    for i, a in enumerate(range(0, n, chunk)):
        b = min(n, a + chunk)
        s0, s1 = int(first[i]), int(first[i + 1])
        blobs.append(enc.encode_rle_v2(vals[a:b], lens[s0:s1], kinds[s0:s1]))
        sizes.append(8 * (b - a))
    return _pack([RLE_V2] * len(blobs), blobs, sizes)


# ---------------------------------------------------------------------------
# Byte generators for Deflate
# ---------------------------------------------------------------------------

class _Vocab:
    def __init__(self, seed: int, size: int = 4096):
        rng = np.random.default_rng([seed, 99])
        lens = rng.integers(3, 11, size)
        letters = rng.integers(97, 123, int(lens.sum()), dtype=np.uint8)
        # each word followed by one space
        self.len1 = (lens + 1).astype(np.int64)
        self.start = np.concatenate([[0], np.cumsum(self.len1)[:-1]]).astype(np.int64)
        flat = np.empty(int(self.len1.sum()), dtype=np.uint8)
        flat[:] = 32
        word_pos = np.repeat(self.start, lens) + (np.arange(lens.sum()) -
                                                 np.repeat(np.cumsum(lens) - lens, lens))
        flat[word_pos] = letters
        self.flat = flat
        p = np.arange(1, size + 1, dtype=np.float64) ** -1.1
        self.cdf = np.cumsum(p / p.sum())


_VOCABS: dict = {}


def _vocab(seed: int) -> _Vocab:
    if seed not in _VOCABS:
        _VOCABS[seed] = _Vocab(seed)
    return _VOCABS[seed]


def zipf_text(size: int, rng: np.random.Generator, vocab: _Vocab) -> bytes:
    ntok = size // 4 + 16
    ids = np.searchsorted(vocab.cdf, rng.random(ntok))
    ids = np.minimum(ids, vocab.cdf.size - 1)
    l1 = vocab.len1[ids]
    ends = np.cumsum(l1)
    k = int(np.searchsorted(ends, size)) + 1
    ids, l1 = ids[:k], l1[:k]
    idx = np.repeat(vocab.start[ids], l1) + (np.arange(int(l1.sum())) -
                                              np.repeat(np.cumsum(l1) - l1, l1))
    return vocab.flat[idx[:size]].tobytes()


def int32_column(size: int, rng: np.random.Generator, run_heavy: bool = False) -> bytes:
    distinct = rng.integers(-(1 << 31), 1 << 31, 64).astype(np.int32)
    n = size // 4 + 1
    if run_heavy:
        nrun = n // 2 + 2
        rl = np.floor(np.exp(rng.uniform(np.log(2), np.log(201), nrun))).astype(np.int64)
        rv = distinct[rng.integers(0, 64, nrun)]
        e = np.repeat(rv, rl)[:n]
        while e.size < n:  # pragma: no cover
            e = np.concatenate([e, e])[:n]
    else:
        e = distinct[rng.integers(0, 64, n)]
    return e.astype("<i4").tobytes()[:size]


def random_bytes(size: int, rng: np.random.Generator) -> bytes:
    return rng.integers(0, 256, size, dtype=np.uint8).tobytes()


def deflate_raw(data: bytes, level: int = 9, fixed: bool = False) -> bytes:
    strategy = zlib.Z_FIXED if fixed else zlib.Z_DEFAULT_STRATEGY
    co = zlib.compressobj(level, zlib.DEFLATED, -15, 8, strategy)
    return co.compress(data) + co.flush()


# Content classes for deflate chunks.
ZIPF, INT32, RANDOM, INT32_RUNS = 0, 1, 2, 3


def lz4_block(data: bytes) -> bytes:
    """One LZ4 block (the reference LZ4 library's compressor, via pyarrow)."""
    import pyarrow as pa
    return pa.Codec("lz4_raw").compress(data, asbytes=True)


def _class_data(seed, wl, j, size, klass):
    rng = np.random.default_rng([seed, wl, j])
    if klass == ZIPF:
        data = zipf_text(size, rng, _vocab(seed))
    elif klass == INT32:
        data = int32_column(size, rng)
    elif klass == INT32_RUNS:
        data = int32_column(size, rng, run_heavy=True)
    else:
        data = random_bytes(size, rng)
    return data, rng


def _deflate_chunk(args):
    seed, wl, j, size, klass, fixed_share = args
    data, rng = _class_data(seed, wl, j, size, klass)
    fixed = klass != RANDOM and rng.random() < fixed_share
    return deflate_raw(data, 9, fixed), fixed


def _lz4_chunk(args):
    seed, wl, j, size, klass = args
    return lz4_block(_class_data(seed, wl, j, size, klass)[0])


def _map(fn, items, nproc=None):
    nproc = nproc or workers()
    if nproc <= 1 or len(items) < 64:
        return [fn(x) for x in items]
    ctx = mp.get_context("fork")
    pool = ctx.Pool(nproc)
    try:
        res = pool.map(fn, items, chunksize=max(1, len(items) // (8 * nproc)))
        pool.close()
    except BaseException:
        pool.terminate()
        raise
    finally:
        # Every worker has exited before the caller goes on.
        pool.join()
    return res


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def rle_v1_workload(seed: int = 0, n_values: int = 1 << 20, chunk_values: int = 16384) -> Chunked:
    vals = rle_v1_values(n_values, np.random.default_rng([seed, WL_RLE_V1]))
    ch = _chunk_values_v1(vals, chunk_values)
    ch.info.update(workload="rle_v1", n_values=n_values, chunk_values=chunk_values, seed=seed)
    return ch


def rle_v2_workload(seed: int = 0, n_values: int = 1 << 25, chunk_values: int = 32768) -> Chunked:
    vals, sl, sk = rle_v2_segments(n_values, np.random.default_rng([seed, WL_RLE_V2]))
    ch = _chunk_values_v2(vals, sl, sk, chunk_values)
    share = {int(k): float(sl[sk == k].sum()) / n_values for k in (1, 2, 3, 4)}
    ch.info.update(workload="rle_v2", n_values=n_values, chunk_values=chunk_values, seed=seed,
                   value_share={"short_repeat": share[1], "direct": share[2],
                                "patched_base": share[3], "delta": share[4]})
    return ch


def deflate_workload(seed: int = 0, total_bytes: int = 1 << 30, chunk_bytes: int = 65536,
                     fixed_share: float = 1 / 3) -> Chunked:
    n = total_bytes // chunk_bytes
    crng = np.random.default_rng([seed, WL_DEFLATE])
    classes = crng.choice(3, size=n, p=[0.5, 0.3, 0.2])
    items = [(seed, WL_DEFLATE, j, chunk_bytes, int(classes[j]), fixed_share) for j in range(n)]
    res = _map(_deflate_chunk, items)
    ch = _pack([DEFLATE] * n, [r[0] for r in res], [chunk_bytes] * n)
    ch.info.update(workload="deflate", total_bytes=n * chunk_bytes, chunk_bytes=chunk_bytes,
                   seed=seed, classes=classes.astype(np.uint8),
                   fixed_chunks=int(sum(r[1] for r in res)))
    return ch


def lz4_workload(seed: int = 0, total_bytes: int = 1 << 30, chunk_bytes: int = 65536) -> Chunked:
    """The Deflate workload's chunks (same content classes, same bytes) as
    LZ4 blocks."""
    n = total_bytes // chunk_bytes
    crng = np.random.default_rng([seed, WL_DEFLATE])
    classes = crng.choice(3, size=n, p=[0.5, 0.3, 0.2])
    items = [(seed, WL_DEFLATE, j, chunk_bytes, int(classes[j])) for j in range(n)]
    blobs = _map(_lz4_chunk, items)
    ch = _pack([LZ4] * n, blobs, [chunk_bytes] * n)
    ch.info.update(workload="lz4", total_bytes=n * chunk_bytes, chunk_bytes=chunk_bytes, seed=seed,
                   classes=classes.astype(np.uint8))
    return ch


def _lognormal_sizes(rng, n, median=65536, sigma=1.0, lo=4096, hi=1 << 20):
    s = np.exp(rng.normal(np.log(median), sigma, n))
    return np.clip(s, lo, hi).astype(np.int64)


def _batched_chunk(args):
    seed, wl, j, codec, size = args
    rng = np.random.default_rng([seed, wl, j])
    if codec == RLE_V1:
        nv = size // 8
        return enc.encode_rle_v1(rle_v1_values(nv, rng)) if nv else b""
    if codec == RLE_V2:
        nv = size // 8
        if nv == 0:
            return b""
        vals, sl, sk = rle_v2_segments(nv, rng)
        return enc.encode_rle_v2(vals, sl, sk)
    klass = int(rng.choice(3, p=[0.5, 0.3, 0.2]))
    return _deflate_chunk((seed, wl * 1000 + 7, j, size, klass, 1 / 3))[0]


def batched_workload(seed: int = 0, n_chunks: int = 20000) -> Chunked:
    """Mixed codecs, log-normal sizes.

    Chunks are indexed RLE v1 first, then RLE v2, then Deflate, so that every
    RLE chunk's output (a multiple of 8 bytes) starts 8-byte aligned in the
    back-to-back output layout.  The order in which chunks are decoded is the
    scheduler's business and independent of this indexing.
    """
    rng = np.random.default_rng([seed, WL_BATCHED])
    codecs = rng.choice(np.array([RLE_V1, RLE_V2, DEFLATE], dtype=np.uint8), size=n_chunks,
                        p=[0.4, 0.3, 0.3])
    sizes = _lognormal_sizes(rng, n_chunks)
    sizes = np.where(codecs == DEFLATE, sizes, sizes // 8 * 8)
    order = np.argsort(codecs, kind="stable")
    codecs, sizes = codecs[order], sizes[order]
    items = [(seed, WL_BATCHED, int(order[j]), int(codecs[j]), int(sizes[j]))
             for j in range(n_chunks)]
    blobs = _map(_batched_chunk, items)
    ch = _pack(codecs, blobs, sizes)
    ch.info.update(workload="batched", n_chunks=n_chunks, seed=seed)
    return ch


def learned_workload(seed: int = 0, n_chunks: int = 20000) -> Chunked:
    """Deflate only, ratios skewed by content: random / Zipf text / run-heavy int32."""
    rng = np.random.default_rng([seed, WL_LEARNED])
    sizes = _lognormal_sizes(rng, n_chunks)
    classes = rng.choice(np.array([RANDOM, ZIPF, INT32_RUNS]), size=n_chunks)
    items = [(seed, WL_LEARNED, j, int(sizes[j]), int(classes[j]), 1 / 3) for j in range(n_chunks)]
    res = _map(_deflate_chunk, items)
    ch = _pack([DEFLATE] * n_chunks, [r[0] for r in res], sizes)
    ch.info.update(workload="learned", n_chunks=n_chunks, seed=seed,
                   classes=classes.astype(np.uint8))
    return ch
