"""Pins for the oracle's Deflate decoder (CPU only).

Checked against zlib (an independent implementation, through its public
API) in both directions, hand-derived streams, RFC 1951's printed length and
distance tables (typed into deflate_bits.py), brute force over tiny inputs,
and zlib's accept/reject decisions on crafted and corrupted streams.
"""
import itertools
import json
import os
import zlib

import numpy as np
import pytest

import oracle
import workloads
from deflate_bits import DIST_BASE, DIST_EXTRA, LEN_BASE, LEN_EXTRA, BitWriter, fixed_copy, fixed_litlen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "deflate_hand_streams.json")


def inflate(data: bytes, cap: int):
    return oracle.decode_chunk(oracle.DEFLATE, data, cap)


def zlib_inflate(data: bytes):
    """zlib's verdict: output bytes, or None if it rejects the stream."""
    d = zlib.decompressobj(-15)
    try:
        out = d.decompress(data)
    except zlib.error:
        return None
    return out if d.eof else None


@pytest.mark.parametrize("ex", [e for e in json.load(open(GOLDEN)) if e["hex"]], ids=lambda e: e["name"])
def test_hand_streams(ex):
    want = bytes.fromhex(ex["output_hex"])
    st, out = inflate(bytes.fromhex(ex["hex"]), len(want))
    assert st == oracle.OK and out == want
    assert zlib_inflate(bytes.fromhex(ex["hex"])) == want


def test_overlapping_copy_rfc_example():
    """RFC 1951 3.2.3: after "XY", <length 5, distance 2> gives "XYXYXYX"."""
    w = BitWriter()
    w.put(1, 1)
    w.put(1, 2)
    fixed_litlen(w, ord("X"))
    fixed_litlen(w, ord("Y"))
    fixed_copy(w, 5, 2)
    fixed_litlen(w, 256)
    data = w.getvalue()
    assert zlib_inflate(data) == b"XYXYXYX"
    assert inflate(data, 7) == (oracle.OK, b"XYXYXYX")


@pytest.mark.parametrize("length", list(range(3, 259)))
def test_every_length_code(length):
    """Every copy length, written with RFC 1951's printed table, vs zlib."""
    w = BitWriter()
    w.put(1, 1)
    w.put(1, 2)
    for c in b"abcdefg":
        fixed_litlen(w, c)
    fixed_copy(w, length, 7)
    fixed_litlen(w, 256)
    data = w.getvalue()
    want = zlib_inflate(data)
    assert want is not None and len(want) == 7 + length
    assert inflate(data, len(want)) == (oracle.OK, want)


@pytest.mark.parametrize("sym", range(30))
def test_every_distance_code(sym):
    rng = np.random.default_rng(sym)
    prefix = rng.integers(0, 256, 32768, dtype=np.uint8).tobytes()
    for dist in {DIST_BASE[sym], DIST_BASE[sym] + (1 << DIST_EXTRA[sym]) - 1}:
        w = BitWriter()
        w.put(0, 1)
        w.put(0, 2)          # stored block carrying the prefix
        w.align()
        w.put(len(prefix), 16)
        w.put(~len(prefix) & 0xFFFF, 16)
        for b in prefix:
            w.put(b, 8)
        w.put(1, 1)
        w.put(1, 2)
        fixed_copy(w, 10, dist)
        fixed_litlen(w, 256)
        data = w.getvalue()
        want = zlib_inflate(data)
        assert want is not None
        assert inflate(data, len(want)) == (oracle.OK, want)


def test_length_284_with_31_extra_is_258():
    """Length code 284 with extra bits 31 (RFC range text 227-257) decodes as 258, as zlib does."""
    w = BitWriter()
    w.put(1, 1)
    w.put(1, 2)
    fixed_litlen(w, ord("q"))
    fixed_litlen(w, 284)
    w.put(31, 5)
    w.put_code(0, 5)        # distance 1
    fixed_litlen(w, 256)
    data = w.getvalue()
    assert zlib_inflate(data) == b"q" * 259
    assert inflate(data, 259) == (oracle.OK, b"q" * 259)


STRATEGIES = [zlib.Z_DEFAULT_STRATEGY, zlib.Z_FILTERED, zlib.Z_HUFFMAN_ONLY, zlib.Z_RLE, zlib.Z_FIXED]


def _samples():
    rng = np.random.default_rng(7)
    vocab = workloads._vocab(0)
    return {
        "empty": b"",
        "one": b"z",
        "text": workloads.zipf_text(60000, rng, vocab),
        "int32": workloads.int32_column(50000, rng),
        "runs": workloads.int32_column(40000, rng, run_heavy=True),
        "random": workloads.random_bytes(70000, rng),
        "zeros": bytes(100000),
        "periodic": bytes(range(7)) * 5000,
    }


@pytest.mark.parametrize("level", [0, 1, 6, 9])
@pytest.mark.parametrize("strategy", STRATEGIES)
def test_zlib_streams(level, strategy):
    for name, data in _samples().items():
        co = zlib.compressobj(level, zlib.DEFLATED, -15, 8, strategy)
        comp = co.compress(data) + co.flush()
        assert inflate(comp, len(data)) == (oracle.OK, data), name


def test_brute_force_tiny_strings():
    """All strings over {a, b, c} of length <= 5, through stored, fixed and dynamic blocks."""
    for n in range(6):
        for t in itertools.product(b"abc", repeat=n):
            data = bytes(t)
            for level, strategy in ((0, 0), (9, zlib.Z_FIXED), (9, 0), (1, zlib.Z_HUFFMAN_ONLY)):
                co = zlib.compressobj(level, zlib.DEFLATED, -15, 8, strategy)
                comp = co.compress(data) + co.flush()
                assert inflate(comp, len(data)) == (oracle.OK, data)


def test_output_capacity_readings():
    data = workloads.zipf_text(20000, np.random.default_rng(1), workloads._vocab(0))
    comp = workloads.deflate_raw(data)
    assert inflate(comp, len(data))[0] == oracle.OK
    assert inflate(comp, len(data) - 1)[0] == oracle.E_OVERFLOW
    assert inflate(comp, len(data) + 1)[0] == oracle.E_UNDERFLOW
    # Bytes after the final block are ignored (zlib leaves them unused).
    assert inflate(comp + b"\x12\x34", len(data)) == (oracle.OK, data)
    for cut in (0, 1, len(comp) // 3, len(comp) - 1):
        assert inflate(comp[:cut], len(data))[0] == oracle.E_TRUNCATED


def _dynamic_header(w, hlit, hdist, hclen):
    w.put(1, 1)
    w.put(2, 2)
    w.put(hlit - 257, 5)
    w.put(hdist - 1, 5)
    w.put(hclen - 4, 4)


def test_crafted_rejections_agree_with_zlib():
    cases = {}
    w = BitWriter(); w.put(1, 1); w.put(3, 2); cases["btype3"] = w.getvalue()
    w = BitWriter(); w.put(1, 1); w.put(0, 2); w.align(); w.put(5, 16); w.put(5, 16)
    cases["bad_nlen"] = w.getvalue() + b"abcde"
    w = BitWriter(); w.put(1, 1); w.put(1, 2); fixed_litlen(w, 286); cases["litlen286"] = w.getvalue()
    w = BitWriter(); w.put(1, 1); w.put(1, 2); fixed_litlen(w, 97); fixed_litlen(w, 257)
    w.put_code(30, 5); cases["dist30"] = w.getvalue()
    w = BitWriter(); w.put(1, 1); w.put(1, 2); fixed_litlen(w, 97); fixed_copy(w, 3, 2)
    fixed_litlen(w, 256); cases["too_far"] = w.getvalue()
    w = BitWriter(); _dynamic_header(w, 287, 1, 4); cases["hlit287"] = w.getvalue() + b"\0" * 8
    w = BitWriter(); _dynamic_header(w, 257, 31, 4); cases["hdist31"] = w.getvalue() + b"\0" * 8
    # Code-length code with a single length-1 code (incomplete): rejected.
    w = BitWriter(); _dynamic_header(w, 257, 1, 4); w.put(0, 3); w.put(0, 3); w.put(0, 3); w.put(1, 3)
    cases["cl_incomplete"] = w.getvalue() + b"\0" * 40
    for name, data in cases.items():
        assert zlib_inflate(data) is None, name
        st, _ = inflate(data, 1 << 16)
        assert st in (oracle.E_CORRUPT, oracle.E_TRUNCATED), name
        assert st == oracle.E_CORRUPT, name


def test_corrupted_streams_accept_reject_like_zlib():
    """Random bit flips: the oracle accepts exactly when zlib does, with zlib's output."""
    rng = np.random.default_rng(11)
    samples = _samples()
    base = [workloads.deflate_raw(samples["text"][:3000]),
            workloads.deflate_raw(samples["int32"][:4000], fixed=True),
            workloads.deflate_raw(samples["random"][:500], level=0),
            workloads.deflate_raw(samples["runs"][:5000])]
    agree = 0
    for trial in range(3000):
        comp = bytearray(base[trial % len(base)])
        for _ in range(int(rng.integers(1, 4))):
            i = int(rng.integers(0, len(comp)))
            comp[i] ^= 1 << int(rng.integers(0, 8))
        comp = bytes(comp)
        want = zlib_inflate(comp)
        if want is None:
            st, _ = inflate(comp, 1 << 20)
            assert st in (oracle.E_CORRUPT, oracle.E_TRUNCATED)
        else:
            st, out = inflate(comp, len(want))
            assert (st, out) == (oracle.OK, want)
        agree += 1
    assert agree == 3000


def test_workload_generator_roundtrip_small():
    ch = workloads.deflate_workload(seed=2, total_bytes=64 * 65536)
    out, status = oracle.decompress(oracle.DEFLATE, ch.comp, ch.chunk_offsets, ch.out_offsets)
    assert (status == 0).all()
    for j in range(ch.n_chunks):
        a, b = int(ch.chunk_offsets[j]), int(ch.chunk_offsets[j + 1])
        assert zlib_inflate(ch.comp[a:b].tobytes()) == out[j * 65536:(j + 1) * 65536].tobytes()
    assert ch.info["fixed_chunks"] > 0
