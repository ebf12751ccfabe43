"""Oracle pins for the LZ4 block decoder.

Pinned three ways, none of which reuses the oracle's own code:
  - blocks written by pyarrow's LZ4 (the reference LZ4 library's block
    compressor) over the workload's data classes must decode to the data;
  - blocks written by a small greedy encoder (workloads/lz4enc.py: long
    matches, offsets up to 65535, overlapping copies, literal runs past 15
    and 270) must decode
    through pyarrow's LZ4 to the data, and through the oracle to the same;
  - hand-worked blocks (tests/golden/lz4_hand_streams.json), including the
    error statuses, worked out from the block format by hand.
ORC files written with the LZ4 codec by Apache ORC's C++ writer (through
pyarrow) pin the oracle's ORC stream framing with LZ4 chunks.
"""
import json
import os

import numpy as np
import pytest

import oracle
from orc_walk import DATA, DIRECT_V2, LENGTH, file_streams
from workloads.lz4enc import lz4_greedy

pa = pytest.importorskip("pyarrow")
po = pytest.importorskip("pyarrow.orc")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lz4_hand_streams.json")
STATUS = {"OK": oracle.OK, "TRUNCATED": oracle.E_TRUNCATED, "CORRUPT": oracle.E_CORRUPT,
          "OVERFLOW": oracle.E_OVERFLOW, "UNDERFLOW": oracle.E_UNDERFLOW}


def _decode(blocks, caps, capacity=False):
    sizes = [len(b) for b in blocks]
    comp = np.frombuffer(b"".join(bytes(b) for b in blocks) + b"\0", dtype=np.uint8)
    co = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    oo = np.concatenate([[0], np.cumsum(caps)]).astype(np.uint64)
    out, st, made = oracle.decompress_ex(oracle.LZ4, comp, co, oo, capacity=capacity)
    return out, st, made, oo


def _one(block, cap, capacity=False):
    out, st, made, _ = _decode([block], [cap], capacity)
    return int(st[0]), bytes(out[: int(made[0])])


def _data(kind, n, rng):
    if kind == "zipf":
        return (np.minimum(rng.zipf(1.3, n), 255)).astype(np.uint8).tobytes()
    if kind == "int32":
        return np.cumsum(rng.integers(-3, 50, n // 4)).astype(np.int32).tobytes()
    if kind == "random":
        return rng.integers(0, 256, n, dtype=np.uint8).tobytes()
    if kind == "runs":
        return np.repeat(rng.integers(0, 1 << 20, n // 64), 16).astype(np.int32).tobytes()
    if kind == "text":
        words = [b"alpha", b"beta", b"gamma", b"delta", b"epsilon", b" ", b"\n"]
        return b"".join(words[i] for i in rng.integers(0, len(words), n // 4))[:n]
    return bytes(n)


@pytest.mark.parametrize("kind", ["zipf", "int32", "random", "runs", "text", "zeros"])
@pytest.mark.parametrize("n", [0, 1, 13, 4096, 65536, 300_001])
def test_pyarrow_blocks_decode(kind, n):
    rng = np.random.default_rng([n, len(kind)])
    data = _data(kind, n, rng)
    block = pa.Codec("lz4_raw").compress(data, asbytes=True)
    st, out = _one(block, len(data))
    assert st == oracle.OK
    assert out == data


def _greedy_cases():
    rng = np.random.default_rng(11)
    far = rng.integers(0, 256, 70000, dtype=np.uint8).tobytes()
    return {
        "long_run": b"q" * 100_000 + b"tail-end!",
        "overlap_period_3": b"abc" * 7000 + b"0123456789xyz",
        "far_offsets": far + far[:65000] + far[5000:70000] + b"....tail....",
        "literal_runs": rng.integers(0, 256, 300, dtype=np.uint8).tobytes() * 3 + b"\x00" * 40 + b"end--",
        "mixed": _data("text", 50_000, rng) + _data("int32", 40_000, rng) + b"-" * 20,
    }


@pytest.mark.parametrize("name", sorted(_greedy_cases()))
def test_greedy_blocks_both_decoders(name):
    data = _greedy_cases()[name]
    block = lz4_greedy(data)
    ref = pa.Codec("lz4_raw").decompress(block, decompressed_size=len(data), asbytes=True)
    assert ref == data  # the encoder here writes valid blocks
    st, out = _one(block, len(data))
    assert st == oracle.OK
    assert out == data


def test_hand_streams():
    doc = json.load(open(GOLDEN))
    for case in doc["streams"]:
        block, cap = bytes(case["bytes"]), case["cap"]
        st, out = _one(block, cap)
        assert st == STATUS[case["status"]], case["name"]
        if case["status"] == "OK":
            want = case["out_text"].encode() if "out_text" in case else \
                case["out_repeat"][0].encode() * case["out_repeat"][1] + case["out_tail"].encode()
            assert out == want, case["name"]
            assert len(want) == cap
            # an independent decoder agrees with the worked-out output
            assert pa.Codec("lz4_raw").decompress(block, decompressed_size=cap, asbytes=True) == want
        else:
            assert len(out) == case["produced"], case["name"]


def test_capacity_mode_and_chunk_ranges():
    rng = np.random.default_rng(5)
    datas = [_data(k, n, rng) for k, n in [("text", 5000), ("random", 777), ("runs", 9000), ("zipf", 1)]]
    blocks = [pa.Codec("lz4_raw").compress(d, asbytes=True) for d in datas]
    # exact ranges
    out, st, made, oo = _decode(blocks, [len(d) for d in datas])
    assert (st == oracle.OK).all()
    assert bytes(out) == b"".join(datas)
    # generous ranges in capacity mode: every chunk reports what it made
    caps = [len(d) + 100 for d in datas]
    out, st, made, oo = _decode(blocks, caps, capacity=True)
    assert (st == oracle.OK).all()
    assert made.tolist() == [len(d) for d in datas]
    for d, o in zip(datas, oo[:-1]):
        assert bytes(out[int(o):int(o) + len(d)]) == d
    # the same ranges without capacity mode are underfilled
    _, st, _, _ = _decode(blocks, caps)
    assert (st == oracle.E_UNDERFLOW).all()


def test_every_truncation_is_an_error():
    data = b"abcabcabcabcXYZXYZXYZ" * 30 + b"0123456789"
    block = lz4_greedy(data)
    for cut in range(len(block)):
        st, out = _one(block[:cut], len(data))
        assert st in (oracle.E_TRUNCATED, oracle.E_UNDERFLOW), cut
        assert data.startswith(out)
        # only a cut right after a sequence's literals ends the block early
        if st == oracle.E_UNDERFLOW:
            assert len(out) < len(data)


@pytest.mark.parametrize("block_size", [65536, 262144])
def test_orc_lz4_file_streams(tmp_path, block_size):
    """ORC's LZ4 codec: one LZ4 block per compression chunk."""
    rng = np.random.default_rng(3)
    n = 400_000
    vals = np.cumsum(rng.integers(-50, 100, n))
    words = np.array([str(int(v)) for v in rng.integers(0, 10 ** 6, n)])
    path = str(tmp_path / "t.orc")
    po.write_table(pa.table({"i": pa.array(vals), "s": pa.array(words)}), path, compression="lz4",
                   compression_block_size=block_size)
    f = file_streams(path)
    assert f["compression"] == 4 and f["block_size"] == block_size
    sf = f["stripes"][0]
    assert sf["encodings"][1] == DIRECT_V2
    st, raw = oracle.orc_inflate_stream(sf["streams"][(1, DATA)], block_size, 1 << 24, codec=oracle.LZ4)
    assert st == oracle.OK
    comp = np.frombuffer(raw + b"\0", dtype=np.uint8)
    out, st2, _ = oracle.decompress_ex(oracle.RLE_V2, comp, np.array([0, len(raw)], np.uint64),
                                       np.array([0, 8 * n], np.uint64))
    assert st2[0] == oracle.OK
    assert (out.view(np.int64) == vals).all()
    st, chars = oracle.orc_inflate_stream(sf["streams"][(2, DATA)], block_size, 1 << 24, codec=oracle.LZ4)
    assert st == oracle.OK
    assert chars == "".join(words).encode()
    st, lens = oracle.orc_inflate_stream(sf["streams"][(2, LENGTH)], block_size, 1 << 24, codec=oracle.LZ4)
    assert st == oracle.OK and len(lens) > 0


@pytest.mark.parametrize("kind", ["text", "int32", "runs"])
def test_damaged_blocks_against_reference_library(kind):
    """Blocks written by pyarrow's LZ4 and damaged in one to three bytes,
    decoded by the oracle and by the reference library (pyarrow's
    "lz4_raw" decompress, told the original size).  That library reports no
    status codes and, as pyarrow calls it, does not check that a block fills
    the size it was told, so the pin is one-sided: a block the oracle
    accepts gives the same bytes in both; a block the library rejects, the
    oracle rejects; a block only the oracle rejects is UNDERFLOW (it ends
    before the size) or CORRUPT (a match offset of 0, which the format
    forbids and the library does not check), and what the oracle wrote is
    the start of the library's output."""
    rng = np.random.default_rng([31, len(kind)])
    data = _data(kind, 60000, rng)
    codec = pa.Codec("lz4_raw")
    block = codec.compress(data, asbytes=True)
    n = len(data)
    counts = {"same": 0, "both_reject": 0, "oracle_stricter": 0}
    for _ in range(200):
        b = bytearray(block)
        for _ in range(int(rng.integers(1, 4))):
            b[int(rng.integers(0, len(b)))] = int(rng.integers(0, 256))
        st, out = _one(bytes(b), n)
        try:
            got = codec.decompress(bytes(b), decompressed_size=n, asbytes=True)
        except Exception:  # the reference library rejected the block
            assert st != oracle.OK, "the oracle accepts a block the reference library rejects"
            counts["both_reject"] += 1
            continue
        if st == oracle.OK:
            assert out == got
            counts["same"] += 1
        else:
            assert st in (oracle.E_UNDERFLOW, oracle.E_CORRUPT), st
            assert out == got[:len(out)]
            counts["oracle_stricter"] += 1
    assert counts["same"] > 0 and counts["both_reject"] > 0
