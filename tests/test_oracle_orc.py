"""Oracle pins for the ORC read path around the decoders: compressed-stream
framing (ZLIB codec), byte RLE (byte columns and PRESENT bitmaps), and the
integer encodings with other element types (unsigned streams such as string
lengths, 16- and 32-bit columns).

The files are written by Apache ORC's C++ writer through pyarrow -- an
independent implementation -- and the oracle's decode of each stream must
give back the column pyarrow was handed.  Hand-worked streams cover the
byte-RLE and framing rules on their own.
"""
import json
import os
import zlib

import numpy as np
import pytest

import oracle
from orc_walk import DATA, DIRECT, DIRECT_V2, LENGTH, PRESENT, file_streams

pa = pytest.importorskip("pyarrow")
po = pytest.importorskip("pyarrow.orc")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "byte_rle_hand_streams.json")


def _write(tmp_path, table, **kw):
    path = str(tmp_path / "t.orc")
    po.write_table(table, path, **kw)
    return file_streams(path)


def _stream(f, col, kind, n_bytes_out):
    """Oracle: inflate the stream if the file is compressed."""
    raw = f["stripes"][0]["streams"][(col, kind)]
    if f["compression"] == 0:
        return raw
    st, data = oracle.orc_inflate_stream(raw, f["block_size"], n_bytes_out)
    assert st == oracle.OK
    return data


def _decode(codec, data, out_bytes, **kw):
    comp = np.frombuffer(bytes(data) + b"\0", dtype=np.uint8)  # never empty
    out, st, made = oracle.decompress_ex(codec, comp, np.array([0, len(data)], np.uint64),
                                         np.array([0, out_bytes], np.uint64), **kw)
    return int(st[0]), out


def _columns(n, rng):
    vals = np.cumsum(rng.integers(-50, 100, n))
    big = rng.random(n) < 0.02
    vals[big] = rng.integers(-(1 << 40), 1 << 40, int(big.sum()))
    nulls = rng.random(n) < 0.1
    words = np.array([str(int(v)) for v in rng.integers(0, 10 ** 6, n)])
    return {
        "i64": pa.array(vals, mask=nulls),
        "s": pa.array(words),
        "i8": pa.array((vals % 97).astype(np.int8)),
        "i16": pa.array((vals % 30011).astype(np.int16)),
        "i32": pa.array((vals * 37).astype(np.int32)),
        "b": pa.array(rng.random(n) < 0.3),
    }, vals, nulls, words


@pytest.mark.parametrize("version,block,compression", [("0.12", 65536, "zlib"), ("0.12", 131072, "zlib"),
                                                       ("0.11", 65536, "zlib"), ("0.12", 0, "uncompressed")])
def test_orc_file_columns(tmp_path, version, block, compression):
    rng = np.random.default_rng(7)
    n = 300_000
    cols, vals, nulls, words = _columns(n, rng)
    kw = {"file_version": version, "compression": compression}
    if block:
        kw["compression_block_size"] = block
    f = _write(tmp_path, pa.table(cols), **kw)
    assert len(f["stripes"]) == 1
    enc = f["stripes"][0]["encodings"]
    rle = oracle.RLE_V2 if version == "0.12" else oracle.RLE_V1
    assert enc[1] == (DIRECT_V2 if version == "0.12" else DIRECT)
    big = 1 << 24
    # int64 with nulls: PRESENT (byte RLE over MSB-first bits), then the
    # non-null values (signed integer RLE).
    present = _stream(f, 1, PRESENT, big)
    st, bits = _decode(oracle.BYTE_RLE, present, (n + 7) // 8)
    assert st == oracle.OK
    assert np.array_equal(np.unpackbits(bits)[:n].astype(bool), ~nulls)
    data = _stream(f, 1, DATA, big)
    st, out = _decode(rle, data, 8 * int((~nulls).sum()))
    assert st == oracle.OK and np.array_equal(out.view(np.int64), vals[~nulls])
    # string lengths: unsigned integer RLE
    lengths = _stream(f, 2, LENGTH, big)
    st, out = _decode(rle, lengths, 8 * n, unsigned=True)
    assert st == oracle.OK
    assert np.array_equal(out.view(np.uint64), np.char.str_len(words).astype(np.uint64))
    # The same stream read as signed gives zigzag-decoded values instead.
    st, out_s = _decode(rle, lengths, 8 * n)
    assert st == oracle.OK and not np.array_equal(out_s, out)
    # int8: byte RLE
    st, out = _decode(oracle.BYTE_RLE, _stream(f, 3, DATA, big), n)
    assert st == oracle.OK and np.array_equal(out.view(np.int8), (vals % 97).astype(np.int8))
    # int16 / int32: signed integer RLE, stored at the column's width
    for col, dt, eb in ((4, np.int16, 2), (5, np.int32, 4)):
        st, out = _decode(rle, _stream(f, col, DATA, big), eb * n, elem_bytes=eb)
        expect = (vals % 30011).astype(np.int16) if dt == np.int16 else (vals * 37).astype(np.int32)
        assert st == oracle.OK and np.array_equal(out.view(dt), expect)
    # bool: byte RLE over MSB-first bits
    st, bits = _decode(oracle.BYTE_RLE, _stream(f, 6, DATA, big), (n + 7) // 8)
    assert st == oracle.OK
    assert np.array_equal(np.unpackbits(bits)[:n].astype(bool), cols["b"].to_numpy(zero_copy_only=False))


def test_narrow_element_is_low_bytes():
    """Any element width stores the low bytes of the 64-bit decoded value."""
    rng = np.random.default_rng(3)
    from workloads import enc
    v = rng.integers(-(1 << 62), 1 << 62, 3000)
    for codec, blob in ((oracle.RLE_V1, enc.encode_rle_v1(v)), (oracle.RLE_V2, enc.encode_rle_v2(v))):
        st, full = _decode(codec, blob, 8 * v.size)
        assert st == oracle.OK
        for eb, dt in ((1, np.int8), (2, np.int16), (4, np.int32)):
            st, out = _decode(codec, blob, eb * v.size, elem_bytes=eb)
            assert st == oracle.OK and np.array_equal(out.view(dt), full.view(np.int64).astype(dt))


def test_byte_rle_hand_streams():
    cases = json.load(open(GOLDEN))["cases"]
    for c in cases:
        data = bytes.fromhex(c["stream"])
        st, out = _decode(oracle.BYTE_RLE, data, c["out_bytes"])
        assert st == getattr(oracle, c["status"]), c
        if c["status"] == "OK":
            expect = b"".join(bytes([b]) * k for b, k in c["expect"])
            assert out.tobytes() == expect, c


def _frame(chunks):
    out = bytearray()
    for payload, original in chunks:
        h = (len(payload) << 1) | int(original)
        out += bytes([h & 255, (h >> 8) & 255, h >> 16]) + payload
    return bytes(out)


def test_orc_framing_rules():
    """Chunks are original bytes or raw Deflate; all but the last hold
    exactly the block size; cut-off headers and chunks are TRUNCATED."""
    block = 1000
    rng = np.random.default_rng(5)
    raw = bytes(rng.integers(0, 4, 3500, dtype=np.uint8))
    parts = [raw[i:i + block] for i in range(0, len(raw), block)]

    def deflated(p):
        c = zlib.compressobj(9, zlib.DEFLATED, -15)
        return c.compress(p) + c.flush()

    mixed = _frame([(deflated(parts[0]), False), (parts[1], True), (deflated(parts[2]), False),
                    (parts[3], True)])
    st, out = oracle.orc_inflate_stream(mixed, block, 10_000)
    assert st == oracle.OK and out == raw
    st, _ = oracle.orc_inflate_stream(mixed, block, 3499)
    assert st == oracle.E_OVERFLOW
    st, _ = oracle.orc_inflate_stream(mixed[:-1], block, 10_000)
    assert st == oracle.E_TRUNCATED
    one = _frame([(deflated(parts[0]), False)])
    st, _ = oracle.orc_inflate_stream(one + b"\x05\x00", block, 10_000)  # header cut off
    assert st == oracle.E_TRUNCATED
    # The first failing chunk decides: a short chunk that is no longer last.
    st, _ = oracle.orc_inflate_stream(mixed + b"\x05\x00", block, 10_000)
    assert st == oracle.E_UNDERFLOW
    short = _frame([(deflated(parts[0][:999]), False), (deflated(parts[1]), False)])
    st, _ = oracle.orc_inflate_stream(short, block, 10_000)
    assert st == oracle.E_UNDERFLOW
    long_ = _frame([(deflated(parts[0] + b"x"), False), (deflated(parts[1]), False)])
    st, _ = oracle.orc_inflate_stream(long_, block, 10_000)
    assert st == oracle.E_OVERFLOW
    st, out = oracle.orc_inflate_stream(b"", block, 10)
    assert st == oracle.OK and out == b""
    st, _ = oracle.orc_inflate_stream(_frame([(b"\xff\xff", False)]), block, 10_000)
    assert st != oracle.OK  # not a Deflate stream
