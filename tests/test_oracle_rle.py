"""Pins for the oracle's ORC RLE v1/v2 decoders (CPU only).

The oracle is checked against things other than itself:
  * hand-derived streams (tests/golden/rle_hand_streams.json);
  * files written by Apache ORC's C++ writer through pyarrow, an independent
    implementation of both encodings;
  * round trips through this repository's encoders (written separately from
    the oracle) over brute-force tiny inputs and forced sub-encodings;
  * the readings for errors (truncation, overflow, trailing bytes).
"""
import itertools
import json
import os
import tempfile

import numpy as np
import pytest

import oracle
import workloads
from workloads import enc

from orc_walk import integer_data_streams

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rle_hand_streams.json")
I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1


def decode(codec, data, n_values):
    st, out = oracle.decode_chunk(codec, data, 8 * n_values)
    return st, np.frombuffer(out, dtype=np.int64)


@pytest.mark.parametrize("ex", json.load(open(GOLDEN)), ids=lambda e: e["name"])
def test_hand_streams(ex):
    codec = oracle.RLE_V1 if ex["codec"] == "rle_v1" else oracle.RLE_V2
    st, vals = decode(codec, bytes.fromhex(ex["hex"]), len(ex["values"]))
    assert st == oracle.OK
    assert vals.tolist() == ex["values"]


def _orc_roundtrip(values, version):
    pa = pytest.importorskip("pyarrow")
    po = pytest.importorskip("pyarrow.orc")
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "t.orc")
        po.write_table(pa.table({"x": pa.array(values, type=pa.int64())}), path,
                       file_version=version, compression="uncompressed")
        return integer_data_streams(path)


def _orc_cases():
    rng = np.random.default_rng(123)
    cases = {
        "runs": np.concatenate([np.arange(300) * 5 - 7, np.full(200, -3), np.arange(140)[::-1]]),
        "literals": rng.integers(-(1 << 40), 1 << 40, 777),
        "extremes": np.array([I64_MIN, I64_MAX, 0, -1, 1, I64_MIN, I64_MAX, 2, 2, 2, 2] * 7),
        "small_random": rng.integers(-3, 4, 1000),
        "monotone": np.cumsum(rng.integers(1, 1000, 2000)) + (1 << 40),
        "outliers": np.where(rng.random(2048) < 0.02, rng.integers(1 << 12, 1 << 48, 2048),
                             rng.integers(0, 4096, 2048)),
        "sparse_outliers": np.where(np.arange(1500) % 700 == 13, 1 << 45,
                                    rng.integers(0, 4096, 1500)),
        "wide": rng.integers(I64_MIN, I64_MAX, 600, dtype=np.int64),
        "mixed": np.concatenate([np.full(7, 123456789), rng.integers(-100, 100, 50),
                                 np.arange(600) * -17, np.full(3, -1 << 50)]),
    }
    return cases


@pytest.mark.parametrize("version,codec", [("0.11", oracle.RLE_V1), ("0.12", oracle.RLE_V2)])
@pytest.mark.parametrize("case", sorted(_orc_cases()))
def test_against_apache_orc_writer(version, codec, case):
    values = np.asarray(_orc_cases()[case], dtype=np.int64)
    kind, streams = _orc_roundtrip(values, version)
    assert kind == (0 if codec == oracle.RLE_V1 else 2)
    assert len(streams) == 1
    st, vals = decode(codec, streams[0], values.size)
    assert st == oracle.OK
    np.testing.assert_array_equal(vals, values)


def test_orc_writer_emits_every_v2_subencoding():
    """The Apache ORC writer's streams cover all four RLE v2 sub-encodings."""
    rng = np.random.default_rng(5)
    seen = set()
    probes = {
        0: np.full(5, 77),                                    # SHORT_REPEAT
        1: rng.integers(-(1 << 30), 1 << 30, 300),            # DIRECT
        2: np.where(np.arange(512) % 50 == 3, 1 << 40, rng.integers(0, 4096, 512)),  # PATCHED
        3: np.cumsum(rng.integers(1, 9, 300)),                # DELTA
    }
    for want, vals in probes.items():
        _, streams = _orc_roundtrip(np.asarray(vals, dtype=np.int64), "0.12")
        first_type = streams[0][0] >> 6
        seen.add(first_type)
        assert first_type == want
        st, out = decode(oracle.RLE_V2, streams[0], len(vals))
        assert st == oracle.OK and np.array_equal(out, vals)
    assert seen == {0, 1, 2, 3}


def width_code_cases():
    """Columns for which the Apache ORC writer (through pyarrow) emits, over
    all of them, every one of the 32 RLE v2 width codes: random values of
    each zigzag bit width (DIRECT at the byte-aligned widths), monotone
    columns with steps of each width (DELTA), values of each width with 3%
    large outliers (PATCHED_BASE data and patch widths at every code) and
    {0, -1} with outliers (width 1)."""
    rng = np.random.default_rng(2024)
    cols = []
    for b in range(1, 65):
        lo, hi = 1 << (b - 1), (1 << b) - 1
        z = rng.integers(lo, hi, 512, dtype=np.uint64, endpoint=True)
        cols.append(((z >> np.uint64(1)).astype(np.int64)) ^ (-(z & np.uint64(1)).astype(np.int64)))
    for b in range(1, 63):
        steps = rng.integers(1 << (b - 1), (1 << b) - 1, 512, endpoint=True)
        cols.append(np.cumsum(steps // 2 if b > 60 else steps).astype(np.int64))
    for b in range(1, 58):
        for _ in range(3):
            base = rng.integers(0, 1 << b, 512) | (1 << (b - 1))
            top = min(63, b + 1 + int(rng.integers(1, 62 - b + 1)))
            cols.append(np.where(rng.random(512) < 0.03,
                                 rng.integers(1 << (top - 1), (1 << top) - 1, 512), base).astype(np.int64))
    cols.append(np.where(rng.random(512) < 0.03, rng.integers(1 << 20, 1 << 30, 512),
                         -rng.integers(0, 2, 512)).astype(np.int64))
    return cols


def test_every_width_code_from_orc_writer():
    """All 32 RLE v2 width codes occur, as widths, in streams the Apache ORC
    writer produced, and the oracle decodes every one of those streams to the
    column that was written."""
    from orc_walk import rle_v2_width_codes
    seen = set()
    for vals in width_code_cases():
        kind, streams = _orc_roundtrip(vals, "0.12")
        assert kind == 2 and len(streams) == 1
        seen.update(rle_v2_width_codes(streams[0]))
        st, out = decode(oracle.RLE_V2, streams[0], vals.size)
        assert st == oracle.OK
        np.testing.assert_array_equal(out, vals)
    assert seen == set(range(32)), sorted(set(range(32)) - seen)


def test_patched_base_filler_entries_from_orc_writer():
    """Gaps over 255 between outliers are written as (255, 0) filler entries."""
    vals = np.zeros(512, dtype=np.int64) + np.arange(512) % 4000
    vals[[3, 400]] = [1 << 44, 1 << 43]       # gap 397 > 255 between patches
    vals = vals + (np.arange(512) % 7)
    _, streams = _orc_roundtrip(vals, "0.12")
    assert streams[0][0] >> 6 == 2
    st, out = decode(oracle.RLE_V2, streams[0], 512)
    assert st == oracle.OK and np.array_equal(out, vals)


EDGE = [0, 1, -1, 2, -2, 1 << 40, -(1 << 40), I64_MIN, I64_MAX]


@pytest.mark.parametrize("codec", [oracle.RLE_V1, oracle.RLE_V2])
def test_brute_force_tiny_sequences(codec):
    """Every sequence of length <= 3 over the edge values round-trips."""
    for n in range(0, 4):
        for seq in itertools.product(EDGE, repeat=n):
            vals = np.array(seq, dtype=np.int64)
            data = enc.encode_rle_v1(vals) if codec == oracle.RLE_V1 else enc.encode_rle_v2(vals)
            st, out = decode(codec, data, n)
            assert st == oracle.OK, (seq, data.hex())
            assert out.tolist() == list(seq)


@pytest.mark.parametrize("kind", [enc.SHORT_REPEAT, enc.DIRECT, enc.PATCHED_BASE, enc.DELTA])
def test_forced_subencodings_roundtrip(kind):
    rng = np.random.default_rng(kind)
    for trial in range(40):
        n = int(rng.integers(1, 1500))
        if kind == enc.SHORT_REPEAT:
            vals = np.repeat(rng.integers(I64_MIN, I64_MAX, n, dtype=np.int64), rng.integers(1, 12, n))[:n]
        elif kind == enc.DELTA:
            step = rng.integers(0, 1 << int(rng.integers(1, 60)), n)
            vals = np.cumsum(step).astype(np.int64) * (1 if trial % 2 else -1)
        elif kind == enc.PATCHED_BASE:
            base = rng.integers(0, 1 << int(rng.integers(1, 20)), n)
            big = rng.integers(0, 1 << int(rng.integers(20, 60)), n)
            vals = np.where(rng.random(n) < 0.03, big, base) - int(rng.integers(-1000, 1000))
            if trial % 3 == 0:   # long gaps: forces filler entries
                vals = np.where(np.arange(n) % 600 == 1, big, base)
        else:
            bits = int(rng.integers(1, 64))
            vals = rng.integers(-(1 << (bits - 1)), 1 << (bits - 1), n)
        vals = np.asarray(vals, dtype=np.int64)
        data = enc.encode_rle_v2(vals, np.array([n]), np.array([kind], dtype=np.uint8))
        st, out = decode(oracle.RLE_V2, data, n)
        assert st == oracle.OK
        np.testing.assert_array_equal(out, vals)


def test_workload_generators_roundtrip_small():
    for ch in (workloads.rle_v1_workload(seed=3, n_values=50000, chunk_values=4096),
               workloads.rle_v2_workload(seed=3, n_values=70000, chunk_values=8192)):
        codec = int(ch.codecs[0])
        out, status = oracle.decompress(codec, ch.comp, ch.chunk_offsets, ch.out_offsets)
        assert (status == 0).all()
        if ch.info["workload"] == "rle_v1":
            ref = workloads.rle_v1_values(50000, np.random.default_rng([3, workloads.WL_RLE_V1]))
        else:
            ref = workloads.rle_v2_segments(70000, np.random.default_rng([3, workloads.WL_RLE_V2]))[0]
        np.testing.assert_array_equal(out.view(np.int64), ref)


# ---- error readings -------------------------------------------------------

def test_truncation_is_truncated():
    vals = np.random.default_rng(9).integers(-(1 << 40), 1 << 40, 300)
    for codec, data in ((oracle.RLE_V1, enc.encode_rle_v1(vals)), (oracle.RLE_V2, enc.encode_rle_v2(vals))):
        for cut in (1, 2, len(data) // 2, len(data) - 1):
            st, _ = decode(codec, data[:cut], 300)
            assert st == oracle.E_TRUNCATED


def test_capacity_readings():
    vals = np.arange(100, dtype=np.int64) * 3
    for codec, data in ((oracle.RLE_V1, enc.encode_rle_v1(vals)), (oracle.RLE_V2, enc.encode_rle_v2(vals))):
        assert decode(codec, data, 100)[0] == oracle.OK
        assert decode(codec, data, 99)[0] == oracle.E_OVERFLOW   # group does not fit
        assert decode(codec, data, 101)[0] == oracle.E_TRUNCATED  # input ends first
        assert decode(codec, data + b"\x00", 100)[0] == oracle.E_CORRUPT  # trailing byte
        assert oracle.decode_chunk(codec, data, 8 * 100 - 4)[0] == oracle.E_INVALID_ARGUMENT


def test_overlong_varints_are_corrupt():
    # RLE v1 literal list of one varint with 11 bytes / a 10th byte above 1.
    assert decode(oracle.RLE_V1, bytes([0xFF]) + b"\x80" * 10 + b"\x00", 1)[0] == oracle.E_CORRUPT
    assert decode(oracle.RLE_V1, bytes([0xFF]) + b"\xff" * 9 + b"\x02", 1)[0] == oracle.E_CORRUPT
    st, v = decode(oracle.RLE_V1, bytes([0xFF]) + b"\xff" * 9 + b"\x01", 1)
    assert st == oracle.OK and v[0] == I64_MIN  # zigzag of 2^64-1


def test_patched_base_invalid_widths_and_positions():
    # data width 64 with any patch width cannot hold patch << W.
    hdr = bytes([0x80 | (31 << 1), 0x00, 0x00, 0x21])
    assert decode(oracle.RLE_V2, hdr + b"\x00" * 20, 1)[0] == oracle.E_CORRUPT
    # patch position beyond the run: length 2, one entry with gap 3.
    s = bytes([0x82, 0x01, 0x07, 0x21, 0x05, 0x00]) + bytes([0x3 << 6 | 0x3F, 0xC0])
    assert decode(oracle.RLE_V2, s, 2)[0] == oracle.E_CORRUPT


def test_delta_negative_base_and_wrap():
    # DELTA with a negative delta base subtracts the magnitudes.
    vals = np.array([1000, 990, 985, 900, 0, -5], dtype=np.int64)
    data = enc.encode_rle_v2(vals, np.array([6]), np.array([enc.DELTA], dtype=np.uint8))
    assert data[0] >> 6 == 3
    st, out = decode(oracle.RLE_V2, data, 6)
    assert st == oracle.OK and out.tolist() == vals.tolist()
    # Fixed delta wrapping modulo 2^64.
    vals = (np.uint64(I64_MAX - 2) + np.arange(5, dtype=np.uint64)).view(np.int64)
    data = enc.encode_rle_v2(vals, np.array([5]), np.array([enc.DELTA], dtype=np.uint8))
    st, out = decode(oracle.RLE_V2, data, 5)
    assert st == oracle.OK and np.array_equal(out, vals)
