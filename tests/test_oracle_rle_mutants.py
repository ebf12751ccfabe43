"""The oracle's RLE v1 / RLE v2 / byte RLE acceptance rules pinned against an
independent reader: Apache ORC's own (through pyarrow), on DATA streams that
pyarrow wrote and that the test then damages in one to three bytes (for a
ZLIB-compressed file, in the framed bytes, so the oracle's framing and
Deflate decoder are pinned along).

Apache ORC's reader decodes exactly the column's value count and reports
no status codes, so the pin is one-sided:
  * a stream the oracle accepts decodes to the same values in both;
  * a stream Apache ORC rejects, the oracle rejects too;
  * a stream only the oracle rejects fails as OVERFLOW (a run or group that
    passes the column's value count, which Apache ORC cuts short) or CORRUPT
    (input left over once the output is full, which Apache ORC never reads),
    and what the oracle wrote before it stopped equals Apache ORC's values.
One reading differs and is left out, counted: a PATCHED_BASE run whose patch
list has a zero gap after its first entry (no writer makes one).  The oracle
ORs such a patch into the value at the same position; Apache ORC's reader
applies no patch after it.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from orc_walk import V2_WIDTHS, _closest_width, _varint_end, integer_data_streams

pa = pytest.importorskip("pyarrow")
po = pytest.importorskip("pyarrow.orc")


def _values(rng):
    """Repeats (SHORT_REPEAT / RLE v1 runs), a monotone stretch (DELTA) and
    wide random values (DIRECT, PATCHED_BASE when a few are outliers)."""
    reps = np.repeat(rng.integers(-1000, 1000, 50), 10)
    mono = np.cumsum(rng.integers(1, 50, 1500))
    wide = rng.integers(-(1 << 40), 1 << 40, 1000)
    small = rng.integers(0, 1 << 10, 1000)
    small[rng.choice(1000, 20, replace=False)] = rng.integers(1 << 30, 1 << 40, 20)
    return np.concatenate([reps, mono, wide, small]).astype(np.int64)


def _unpack_msb(buf: bytes, width: int, count: int):
    bits = int.from_bytes(buf, "big")
    total = 8 * len(buf)
    return [(bits >> (total - width * (k + 1))) & ((1 << width) - 1) for k in range(count)]


def _pb_zero_gap(stream: bytes) -> bool:
    """True if some PATCHED_BASE run met by walking the run headers from the
    start has a patch entry after its first one with a zero gap.  The walk
    stops where a header or payload would pass the end of the stream."""
    i, n = 0, len(stream)
    while i < n:
        h = stream[i]
        kind = h >> 6
        if kind == 0:
            i += 2 + ((h >> 3) & 7)
            continue
        if i + 2 > n:
            return False
        code = (h >> 1) & 31
        cnt = (((h & 1) << 8) | stream[i + 1]) + 1
        if kind == 1:
            i += 2 + (cnt * V2_WIDTHS[code] + 7) // 8
        elif kind == 2:
            if i + 4 > n:
                return False
            b2, b3 = stream[i + 2], stream[i + 3]
            pw, pgw, pll = V2_WIDTHS[b2 & 31], (b3 >> 5) + 1, b3 & 31
            if pgw + pw > 64:
                return False
            ew = _closest_width(pgw + pw)
            psec = i + 4 + (b2 >> 5) + 1 + (cnt * V2_WIDTHS[code] + 7) // 8
            pbytes = (pll * ew + 7) // 8
            if psec + pbytes > n:
                return False
            entries = _unpack_msb(stream[psec:psec + pbytes], ew, pll)
            if any((e >> pw) == 0 for e in entries[1:]):
                return True
            i = psec + pbytes
        else:
            try:
                j = _varint_end(stream, _varint_end(stream, i + 2))
            except IndexError:
                return False
            i = j + (max(cnt - 2, 0) * (V2_WIDTHS[code] if code else 0) + 7) // 8
    return False


@pytest.mark.parametrize("version", ["0.11", "0.12"])
def test_mutated_streams_against_orc_reader(tmp_path, version):
    rng = np.random.default_rng([2024, 0 if version == "0.11" else 1])
    values = _values(rng)
    n = values.size
    path = str(tmp_path / "t.orc")
    po.write_table(pa.table({"x": pa.array(values, type=pa.int64())}), path,
                   file_version=version, compression="uncompressed")
    kind, streams = integer_data_streams(path)
    assert len(streams) == 1
    codec = oracle.RLE_V1 if kind == 0 else oracle.RLE_V2
    assert codec == (oracle.RLE_V1 if version == "0.11" else oracle.RLE_V2)
    data = open(path, "rb").read()
    s = streams[0]
    assert data.count(s) == 1
    off = data.find(s)
    st, out = oracle.decode_chunk(codec, s, 8 * n)
    assert st == oracle.OK and np.array_equal(np.frombuffer(out, np.int64), values)

    counts = {"same": 0, "both_reject": 0, "oracle_stricter": 0, "pb_zero_gap": 0}
    mpath = str(tmp_path / "m.orc")
    for _ in range(250):
        m = bytearray(data)
        for _ in range(int(rng.integers(1, 4))):
            m[off + int(rng.integers(0, len(s)))] = int(rng.integers(0, 256))
        ms = bytes(m[off:off + len(s)])
        with open(mpath, "wb") as f:
            f.write(m)
        st, out = oracle.decode_chunk(codec, ms, 8 * n)
        ov = np.frombuffer(out, np.int64)
        try:
            got = po.read_table(mpath).column(0).to_numpy()
        except Exception:  # Apache ORC rejected the stream
            assert st != oracle.OK, "the oracle accepts a stream Apache ORC rejects"
            counts["both_reject"] += 1
            continue
        if codec == oracle.RLE_V2 and _pb_zero_gap(ms):
            counts["pb_zero_gap"] += 1
            continue
        assert got.size == n
        if st == oracle.OK:
            np.testing.assert_array_equal(ov, got)
            counts["same"] += 1
        else:
            assert st in (oracle.E_OVERFLOW, oracle.E_CORRUPT), st
            np.testing.assert_array_equal(ov, got[:ov.size])
            counts["oracle_stricter"] += 1
    assert counts["same"] > 0 and counts["both_reject"] > 0
    assert counts["pb_zero_gap"] <= 10, counts


def test_mutated_byte_rle_against_orc_reader(tmp_path):
    """The same one-sided pin for ORC byte RLE (the DATA stream of a byte
    column): runs of repeated bytes and literal stretches."""
    rng = np.random.default_rng([2024, 2])
    values = np.concatenate([np.repeat(rng.integers(-128, 128, 60), rng.integers(1, 40, 60)),
                             rng.integers(-128, 128, 2000)]).astype(np.int8)
    n = values.size
    path = str(tmp_path / "b.orc")
    po.write_table(pa.table({"x": pa.array(values, type=pa.int8())}), path, compression="uncompressed")
    _, streams = integer_data_streams(path)
    assert len(streams) == 1
    data = open(path, "rb").read()
    s = streams[0]
    assert data.count(s) == 1
    off = data.find(s)
    st, out = oracle.decode_chunk(oracle.BYTE_RLE, s, n)
    assert st == oracle.OK and np.array_equal(np.frombuffer(out, np.int8), values)

    counts = {"same": 0, "both_reject": 0, "oracle_stricter": 0}
    mpath = str(tmp_path / "m.orc")
    for _ in range(250):
        m = bytearray(data)
        for _ in range(int(rng.integers(1, 4))):
            m[off + int(rng.integers(0, len(s)))] = int(rng.integers(0, 256))
        with open(mpath, "wb") as f:
            f.write(m)
        st, out = oracle.decode_chunk(oracle.BYTE_RLE, bytes(m[off:off + len(s)]), n)
        ov = np.frombuffer(out, np.int8)
        try:
            got = po.read_table(mpath).column(0).to_numpy()
        except Exception:  # Apache ORC rejected the stream
            assert st != oracle.OK, "the oracle accepts a stream Apache ORC rejects"
            counts["both_reject"] += 1
            continue
        assert got.size == n
        if st == oracle.OK:
            np.testing.assert_array_equal(ov, got)
            counts["same"] += 1
        else:
            assert st in (oracle.E_OVERFLOW, oracle.E_CORRUPT), st
            np.testing.assert_array_equal(ov, got[:ov.size])
            counts["oracle_stricter"] += 1
    assert counts["same"] > 0 and counts["both_reject"] > 0


def test_mutated_zlib_streams_against_orc_reader(tmp_path):
    """The same one-sided pin through ORC's compression framing: an RLE v2
    DATA stream of a ZLIB-compressed file, damaged in its framed bytes
    (chunk headers and raw Deflate), read by the oracle's framing and
    Deflate decoder and then its RLE v2 decoder.  A stream Apache ORC reads
    is one the oracle's framing and Deflate accept."""
    from orc_walk import DATA, file_streams
    rng = np.random.default_rng([2024, 3])
    values = _values(rng)
    n = values.size
    path = str(tmp_path / "z.orc")
    po.write_table(pa.table({"x": pa.array(values, type=pa.int64())}), path, file_version="0.12",
                   compression="zlib", compression_block_size=65536)
    f = file_streams(path)
    assert f["compression"] == 1 and len(f["stripes"]) == 1
    raw, block = f["stripes"][0]["streams"][(1, DATA)], f["block_size"]
    data = open(path, "rb").read()
    assert data.count(raw) == 1
    off = data.find(raw)
    big = 1 << 22

    def oracle_read(framed):
        st, dec = oracle.orc_inflate_stream(framed, block, big)
        if st != oracle.OK:
            return st, None, None
        st, out = oracle.decode_chunk(oracle.RLE_V2, bytes(dec), 8 * n)
        return st, np.frombuffer(out, np.int64), bytes(dec)

    st, ov, _ = oracle_read(raw)
    assert st == oracle.OK and np.array_equal(ov, values)

    counts = {"same": 0, "both_reject": 0, "oracle_stricter": 0, "pb_zero_gap": 0}
    mpath = str(tmp_path / "m.orc")
    for _ in range(250):
        m = bytearray(data)
        for _ in range(int(rng.integers(1, 4))):
            m[off + int(rng.integers(0, len(raw)))] = int(rng.integers(0, 256))
        with open(mpath, "wb") as fh:
            fh.write(m)
        st, ov, dec = oracle_read(bytes(m[off:off + len(raw)]))
        try:
            got = po.read_table(mpath).column(0).to_numpy()
        except Exception:  # Apache ORC rejected the stream
            assert st != oracle.OK, "the oracle accepts a stream Apache ORC rejects"
            counts["both_reject"] += 1
            continue
        assert dec is not None, "Apache ORC reads a stream whose framing or Deflate the oracle rejects"
        if _pb_zero_gap(dec):
            counts["pb_zero_gap"] += 1
            continue
        assert got.size == n
        if st == oracle.OK:
            np.testing.assert_array_equal(ov, got)
            counts["same"] += 1
        else:
            assert st in (oracle.E_OVERFLOW, oracle.E_CORRUPT), st
            np.testing.assert_array_equal(ov, got[:ov.size])
            counts["oracle_stricter"] += 1
    assert counts["same"] > 0 and counts["both_reject"] > 0
    assert counts["pb_zero_gap"] < 125, counts
