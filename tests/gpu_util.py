"""Helpers for GPU parity tests: move a workload to the device, decode it with
the HIP library, decode it with the oracle, compare."""
from __future__ import annotations

import numpy as np

import oracle


def device_inputs(ch, dev):
    import torch
    comp = torch.from_numpy(ch.comp).to(dev) if ch.comp.size else torch.zeros(16, dtype=torch.uint8, device=dev)
    co = torch.from_numpy(np.ascontiguousarray(ch.chunk_offsets).view(np.int64)).to(dev)
    oo = torch.from_numpy(np.ascontiguousarray(ch.out_offsets).view(np.int64)).to(dev)
    return comp, co, oo


GUARD = 64       # bytes of each guard range (a multiple of 8 keeps RLE outputs aligned)
GUARD_BYTE = 0xA5


def guarded(ch):
    """The same chunks with a guard chunk before the first, between every two
    and after the last: guard k has an empty compressed range and GUARD output
    bytes, so chunk i's output range moves GUARD * (i + 1) bytes up and is
    fenced on both sides by ranges no chunk may write.  (A guard itself fails
    as TRUNCATED before writing anything.)  Returns the new layout and the
    index of every original chunk in it."""
    import workloads
    n = ch.n_chunks
    co = np.repeat(np.asarray(ch.chunk_offsets, dtype=np.uint64), 2)
    oo = np.zeros(2 * n + 2, dtype=np.uint64)
    src = np.asarray(ch.out_offsets, dtype=np.uint64)
    k = np.arange(n + 1, dtype=np.uint64)
    oo[0::2] = src + GUARD * k
    oo[1::2] = src + GUARD * (k + 1)
    # Guards take their neighbour's codec when it is a valid one.
    own = np.asarray(ch.codecs, dtype=np.uint8)
    gc = np.where((own >= 1) & (own <= 5), own, 1).astype(np.uint8)
    codecs = np.ones(2 * n + 1, dtype=np.uint8)
    codecs[1::2] = own
    codecs[0:2 * n:2] = gc
    if n:
        codecs[2 * n] = gc[-1]
    return workloads.Chunked(codecs, ch.comp, co, oo, dict(ch.info)), np.arange(n) * 2 + 1


def check_guards(got, guarded_ch):
    """Every guard range (even chunk index) still holds GUARD_BYTE."""
    oo = guarded_ch.out_offsets
    for g in range(0, guarded_ch.n_chunks, 2):
        a, b = int(oo[g]), int(oo[g + 1])
        seg = got[a:b]
        if not (seg == GUARD_BYTE).all():
            first = int(np.nonzero(seg != GUARD_BYTE)[0][0])
            raise AssertionError(f"guard before chunk {g // 2} written at byte {first}")


def gpu_decode(codec, ch, dev, **kw):
    import torch
    import paper_2307_03760_amd as codag
    comp, co, oo = device_inputs(ch, dev)
    out = torch.full((max(ch.out_bytes, 1),), GUARD_BYTE, dtype=torch.uint8, device=dev)
    st = torch.full((max(ch.n_chunks, 1),), 99, dtype=torch.int32, device=dev)
    codag.decompress(codec, comp, co, out, oo, status=st[:ch.n_chunks], **kw)
    torch.cuda.synchronize()
    return out[:ch.out_bytes].cpu().numpy(), st[:ch.n_chunks].cpu().numpy()


def _guard_status(codec):
    st, _ = oracle.decode_chunk(int(codec), np.zeros(0, np.uint8), GUARD)
    return st


def oracle_decode(codec, ch, threads=8, elem_bytes=0, unsigned_values=False):
    """The oracle's decode of a chunk array, with the RLE element type."""
    if codec == oracle.BYTE_RLE or elem_bytes not in (0, 8) or unsigned_values:
        out, st, _ = oracle.decompress_ex(codec, ch.comp if ch.comp.size else np.zeros(16, np.uint8),
                                          ch.chunk_offsets, ch.out_offsets,
                                          elem_bytes=elem_bytes or 8, unsigned=bool(unsigned_values))
        return out, st
    return oracle.decompress(codec, ch.comp, ch.chunk_offsets, ch.out_offsets, threads=threads)


def assert_parity(codec, ch, dev, threads=8, guards=True, **kw):
    """GPU output and statuses equal the oracle's, chunk by chunk, in the
    workload's own layout; then again with guard ranges around every chunk's
    output, which must come back untouched (no chunk, failing or not, writes
    outside its range)."""
    import paper_2307_03760_amd as codag
    got, got_st = gpu_decode(codec, ch, dev, **kw)
    ref, ref_st = oracle_decode(codec, ch, threads, kw.get("elem_bytes", 0), kw.get("unsigned_values", False))
    compare_chunks(got, got_st, ref, ref_st, ch.out_offsets)
    if guards:
        del got
        codag.get_error()
        gch, idx = guarded(ch)
        g_got, g_st = gpu_decode(codec, gch, dev, **kw)
        check_guards(g_got, gch)
        assert (g_st[0::2] == _guard_status(codec)).all(), "guard status"
        compare_shifted(g_got, g_st[idx], ref, ref_st, ch.out_offsets, gch.out_offsets[idx])
        rc, bad = codag.get_error()
        assert bad == 0 and rc == _guard_status(codec), (rc, bad)
    return got_st


def compare_shifted(got, got_st, ref, ref_st, ref_offsets, got_starts):
    """compare_chunks for outputs that sit at got_starts[i] instead of ref_offsets[i]."""
    bad = np.nonzero(got_st != ref_st)[0]
    assert bad.size == 0, f"status differs at chunks {bad[:10]}: gpu {got_st[bad[:10]]} oracle {ref_st[bad[:10]]}"
    for i in np.nonzero(ref_st == 0)[0]:
        a, b = int(ref_offsets[i]), int(ref_offsets[i + 1])
        g = int(got_starts[i])
        if not np.array_equal(got[g:g + b - a], ref[a:b]):
            first = int(np.nonzero(got[g:g + b - a] != ref[a:b])[0][0])
            raise AssertionError(f"chunk {i} (guarded layout): first differing byte {first} of {b - a}")


def oracle_mixed(codecs, comp, chunk_offsets, out_offsets, threads=8):
    """Oracle decode of a chunk array whose codec varies per chunk: each run
    of equal codecs is decoded as one array."""
    codecs = np.asarray(codecs)
    n = codecs.size
    out = np.zeros(int(out_offsets[-1]) if n else 0, dtype=np.uint8)
    status = np.zeros(n, dtype=np.int32)
    a = 0
    while a < n:
        b = a
        while b < n and codecs[b] == codecs[a]:
            b += 1
        c = int(codecs[a])
        if c in (oracle.RLE_V1, oracle.RLE_V2, oracle.DEFLATE, oracle.LZ4):
            o, s = oracle.decompress(c, comp, chunk_offsets[a:b + 1], out_offsets[a:b + 1],
                                     threads=threads)
            lo, hi = int(out_offsets[a]), int(out_offsets[b])
            out[lo:hi] = o[lo:hi]
            status[a:b] = s
        else:
            status[a:b] = oracle.E_INVALID_ARGUMENT
        a = b
    return out, status


def batch_device_inputs(ch, dev):
    import torch
    comp, co, oo = device_inputs(ch, dev)
    codecs = torch.from_numpy(np.ascontiguousarray(ch.codecs, dtype=np.uint8)).to(dev)
    return codecs, comp, co, oo


def compare_chunks(got, got_st, ref, ref_st, out_offsets, chunks=None):
    """Equal status for every listed chunk and equal bytes for those that decoded."""
    idx = np.arange(len(ref_st)) if chunks is None else np.asarray(chunks)
    bad = idx[got_st[idx] != ref_st[idx]]
    assert bad.size == 0, f"status differs at chunks {bad[:10]}: gpu {got_st[bad[:10]]} oracle {ref_st[bad[:10]]}"
    for i in idx:
        if ref_st[i] != 0:
            continue
        a, b = int(out_offsets[i]), int(out_offsets[i + 1])
        if not np.array_equal(got[a:b], ref[a:b]):
            first = int(np.nonzero(got[a:b] != ref[a:b])[0][0])
            raise AssertionError(f"chunk {i}: first differing byte {first} of {b - a}")
