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


def gpu_decode(codec, ch, dev, **kw):
    import torch
    import paper_2307_03760_amd as codag
    comp, co, oo = device_inputs(ch, dev)
    out = torch.full((max(ch.out_bytes, 1),), 0xA5, dtype=torch.uint8, device=dev)
    st = torch.full((max(ch.n_chunks, 1),), 99, dtype=torch.int32, device=dev)
    codag.decompress(codec, comp, co, out, oo, status=st[:ch.n_chunks], **kw)
    torch.cuda.synchronize()
    return out[:ch.out_bytes].cpu().numpy(), st[:ch.n_chunks].cpu().numpy()


def assert_parity(codec, ch, dev, threads=8, **kw):
    """GPU output and statuses equal the oracle's, chunk by chunk."""
    got, got_st = gpu_decode(codec, ch, dev, **kw)
    ref, ref_st = oracle.decompress(codec, ch.comp, ch.chunk_offsets, ch.out_offsets, threads=threads)
    bad = np.nonzero(got_st != ref_st)[0]
    assert bad.size == 0, f"status differs at chunks {bad[:10]}: gpu {got_st[bad[:10]]} oracle {ref_st[bad[:10]]}"
    for i in np.nonzero(ref_st == 0)[0]:
        a, b = int(ch.out_offsets[i]), int(ch.out_offsets[i + 1])
        if not np.array_equal(got[a:b], ref[a:b]):
            first = a + int(np.nonzero(got[a:b] != ref[a:b])[0][0])
            raise AssertionError(f"chunk {i}: first differing byte {first - a} of {b - a}")
    return got_st


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
        if c in (oracle.RLE_V1, oracle.RLE_V2, oracle.DEFLATE):
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
