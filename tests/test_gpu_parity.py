"""GPU parity: the HIP path, called through the C ABI, against the oracle.

Bit-exact output and equal per-chunk status on the same seeded inputs, at
small sizes spanning several chunks with a ragged tail, at the full workload
sizes in the benchmark's launch configuration, and on edge and corrupt cases.
"""
import sys
import zlib

import numpy as np
import pytest

import oracle
import workloads
from workloads import enc

from gpu_util import assert_parity, gpu_decode

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2307_03760_amd as codag
    codag.lib()
    return torch.device("cuda:0")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _chunks(codec, blobs, sizes):
    return workloads._pack([codec] * len(blobs), blobs, sizes)


# ---- small workloads: several chunks and a ragged tail ---------------------

@pytest.mark.parametrize("wpb", [1, 2, 4])
def test_rle_v1_small_one_wave(dev, wpb):
    ch = workloads.rle_v1_workload(seed=5, n_values=100_003, chunk_values=16384)
    _say(f"rle_v1 small one wave per chunk wpb={wpb} chunks={ch.n_chunks}")
    assert (assert_parity(oracle.RLE_V1, ch, dev, waves_per_block=wpb, group_parallel=1) == 0).all()


@pytest.mark.parametrize("wpb", [1, 4])
def test_rle_v1_small(dev, wpb):
    ch = workloads.rle_v1_workload(seed=5, n_values=100_003, chunk_values=16384)
    _say(f"rle_v1 small wpb={wpb} chunks={ch.n_chunks}")
    assert (assert_parity(oracle.RLE_V1, ch, dev, waves_per_block=wpb) == 0).all()


@pytest.mark.parametrize("wpb", [1, 2, 4])
def test_rle_v2_small_one_wave(dev, wpb):
    ch = workloads.rle_v2_workload(seed=5, n_values=300_001, chunk_values=32768)
    _say(f"rle_v2 small one wave per chunk wpb={wpb} chunks={ch.n_chunks}")
    assert (assert_parity(oracle.RLE_V2, ch, dev, waves_per_block=wpb, group_parallel=1) == 0).all()


@pytest.mark.parametrize("chunk_values", [32768, 5000, 700])
def test_rle_v2_small_group_parallel(dev, chunk_values):
    """Chunks long and short enough that the ranges hold many runs, a few, or
    none (more ranges than runs)."""
    ch = workloads.rle_v2_workload(seed=5, n_values=300_001, chunk_values=chunk_values)
    _say(f"rle_v2 small group-parallel chunk_values={chunk_values} chunks={ch.n_chunks}")
    assert (assert_parity(oracle.RLE_V2, ch, dev, group_parallel=2) == 0).all()


@pytest.mark.parametrize("tb", [9, 10])
def test_deflate_small(dev, tb):
    ch = workloads.deflate_workload(seed=5, total_bytes=48 * 65536)
    _say(f"deflate small tb={tb} chunks={ch.n_chunks}")
    assert (assert_parity(oracle.DEFLATE, ch, dev, lit_table_bits=tb) == 0).all()


@pytest.mark.parametrize("hist,wpb", [(2, 1), (4, 2), (8, 4), (16, 1), (32, 1)])
def test_deflate_window_sizes(dev, hist, wpb):
    """Every output-window size: back-references beyond the window read the
    already written output from HBM."""
    ch = workloads.deflate_workload(seed=6, total_bytes=40 * 65536 + 777)
    _say(f"deflate window {hist} KiB wpb={wpb} chunks={ch.n_chunks}")
    assert (assert_parity(oracle.DEFLATE, ch, dev, history_kib=hist, waves_per_block=wpb) == 0).all()


def test_rle_v2_each_subencoding(dev):
    rng = np.random.default_rng(21)
    blobs, sizes = [], []
    for kind in (enc.SHORT_REPEAT, enc.DIRECT, enc.PATCHED_BASE, enc.DELTA, enc.AUTO):
        for trial in range(12):
            n = int(rng.integers(1, 3000))
            bits = int(rng.integers(1, 64))
            if kind == enc.SHORT_REPEAT:
                v = np.repeat(rng.integers(-(1 << 62), 1 << 62, n), rng.integers(1, 12, n))[:n]
            elif kind == enc.DELTA:
                v = np.cumsum(rng.integers(0, 1 << min(bits, 40), n)) * (1 if trial % 2 else -1)
            elif kind == enc.PATCHED_BASE:
                v = np.where(rng.random(n) < 0.04, rng.integers(0, 1 << 50, n), rng.integers(0, 1 << 11, n))
                if trial % 3 == 0:
                    v = np.where(np.arange(n) % 611 == 7, 1 << 47, rng.integers(0, 4000, n))
            else:
                v = rng.integers(-(1 << (bits - 1)), 1 << (bits - 1), n)
            v = np.asarray(v, dtype=np.int64)
            blobs.append(enc.encode_rle_v2(v, np.array([n]), np.array([kind], dtype=np.uint8)))
            sizes.append(8 * n)
    ch = _chunks(oracle.RLE_V2, blobs, sizes)
    for gp in (1, 2):
        _say(f"rle_v2 forced sub-encodings chunks={ch.n_chunks} group_parallel={gp}")
        assert (assert_parity(oracle.RLE_V2, ch, dev, group_parallel=gp) == 0).all()


def test_rle_extremes(dev):
    I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1
    vals = [np.array([I64_MIN, I64_MAX, 0, -1, 1] * 40, dtype=np.int64),
            np.arange(1000, dtype=np.int64) * -128,
            (np.uint64(I64_MAX - 200) + np.arange(500, dtype=np.uint64)).view(np.int64),
            np.random.default_rng(3).integers(I64_MIN, I64_MAX, 777, dtype=np.int64),
            # 4,000 groups in one chunk (a run of three and a one-value list, repeated):
            # the group-parallel ranges hold hundreds of short groups each.
            np.column_stack([np.repeat(np.random.default_rng(4).integers(-9999, 9999, 2000), 3).reshape(-1, 3),
                             np.random.default_rng(5).integers(I64_MIN, I64_MAX, 2000)]).reshape(-1)]
    for codec, encode, gp in ((oracle.RLE_V1, enc.encode_rle_v1, 1), (oracle.RLE_V1, enc.encode_rle_v1, 2),
                              (oracle.RLE_V2, enc.encode_rle_v2, 1), (oracle.RLE_V2, enc.encode_rle_v2, 2)):
        ch = _chunks(codec, [encode(v) for v in vals], [8 * v.size for v in vals])
        _say(f"rle extremes codec={codec} group_parallel={gp}")
        assert (assert_parity(codec, ch, dev, group_parallel=gp) == 0).all()


def test_deflate_strategies_and_levels(dev):
    rng = np.random.default_rng(8)
    vocab = workloads._vocab(0)
    datas = [b"", b"x", bytes(70000), bytes(range(7)) * 9000, workloads.zipf_text(90000, rng, vocab),
             workloads.int32_column(65536, rng), workloads.random_bytes(100000, rng),
             workloads.int32_column(65536, rng, run_heavy=True)]
    blobs, sizes = [], []
    for d in datas:
        for level in (0, 1, 6, 9):
            for strategy in (zlib.Z_DEFAULT_STRATEGY, zlib.Z_HUFFMAN_ONLY, zlib.Z_RLE, zlib.Z_FIXED):
                co = zlib.compressobj(level, zlib.DEFLATED, -15, 8, strategy)
                blobs.append(co.compress(d) + co.flush())
                sizes.append(len(d))
    ch = _chunks(oracle.DEFLATE, blobs, sizes)
    _say(f"deflate strategies chunks={ch.n_chunks}")
    assert (assert_parity(oracle.DEFLATE, ch, dev) == 0).all()


def test_unaligned_chunk_layout(dev):
    """Compressed chunks at odd offsets, Deflate outputs at odd offsets."""
    rng = np.random.default_rng(4)
    blobs, sizes = [], []
    for i in range(40):
        d = workloads.zipf_text(int(rng.integers(1, 30000)), rng, workloads._vocab(0))
        blobs.append(workloads.deflate_raw(d, fixed=bool(i % 3 == 0)))
        sizes.append(len(d))
    ch = _chunks(oracle.DEFLATE, blobs, sizes)
    assert (assert_parity(oracle.DEFLATE, ch, dev) == 0).all()


def _stored(payload: bytes, final: bool = True) -> bytes:
    """One stored block (RFC 1951 section 3.2.4): header byte, LEN, NLEN, bytes."""
    n = len(payload)
    return bytes([int(final)]) + n.to_bytes(2, "little") + (n ^ 0xFFFF).to_bytes(2, "little") + payload


def test_deflate_input_fetch_boundaries(dev):
    """Compressed lengths at and around multiples of the decoder's 512-byte
    input fetch (a single stored block is its payload plus 5 bytes), chunk
    starts at many alignments, stored runs read in several pieces, and
    Huffman streams of lengths spread over the residues: bytes past a
    chunk's end must read as zero and each ring half must hold the bytes
    the decoder asks for."""
    rng = np.random.default_rng(21)
    blobs, sizes, boundary = [], [], []
    for k in (1, 2, 3, 4, 8):
        for d in (-17, -16, -5, -1, 0, 1, 5, 16, 17):
            # A small chunk first, so that this one starts at the next of the
            # 16 alignments in turn.
            at = sum(len(b) for b in blobs)
            pad = bytes((len(boundary) - at - 5) % 16)
            blobs.append(_stored(pad))
            sizes.append(len(pad))
            payload = rng.integers(0, 256, 512 * k + d - 5, dtype=np.uint8).tobytes()
            boundary.append(len(blobs))
            blobs.append(_stored(payload))
            sizes.append(len(payload))
    for a, b in ((500, 20), (1, 1030), (255, 257), (4000, 3)):  # two stored blocks back to back
        p, q = (rng.integers(0, 256, n, dtype=np.uint8).tobytes() for n in (a, b))
        blobs.append(_stored(p, final=False) + _stored(q))
        sizes.append(a + b)
    for i in range(24):
        d = workloads.zipf_text(int(rng.integers(600, 9000)), rng, workloads._vocab(0))
        blobs.append(workloads.deflate_raw(d, fixed=bool(i % 2)))
        sizes.append(len(d))
    ch = _chunks(oracle.DEFLATE, blobs, sizes)
    assert len({int(ch.chunk_offsets[i]) % 16 for i in boundary}) == 16
    _say(f"deflate fetch boundaries chunks={ch.n_chunks}")
    assert (assert_parity(oracle.DEFLATE, ch, dev) == 0).all()


# ---- edge cases -------------------------------------------------------------

def test_empty_and_degenerate(dev):
    import paper_2307_03760_amd as codag
    # zero chunks is a no-op
    ch = _chunks(oracle.RLE_V1, [], [])
    out, st = gpu_decode(oracle.RLE_V1, ch, dev)
    assert st.size == 0
    # empty chunks: OK when both sides are empty, CORRUPT for leftover input,
    # TRUNCATED when output is expected from no input
    for codec, one in ((oracle.RLE_V1, enc.encode_rle_v1(np.array([5], dtype=np.int64))),
                       (oracle.RLE_V2, enc.encode_rle_v2(np.array([5], dtype=np.int64)))):
        ch = _chunks(codec, [b"", one, b"", one], [0, 0, 8, 8])
        st = assert_parity(codec, ch, dev)
        assert st.tolist() == [0, oracle.E_CORRUPT, oracle.E_TRUNCATED, 0]
    ch = _chunks(oracle.DEFLATE, [b"", b"\x03\x00", b"\x03\x00", b"\x01\x00\x00\xff\xff"], [0, 0, 5, 0])
    st = assert_parity(oracle.DEFLATE, ch, dev)
    assert st.tolist() == [oracle.E_TRUNCATED, 0, oracle.E_UNDERFLOW, 0]
    codag.get_error()


def test_rle_output_rules(dev):
    import torch
    import paper_2307_03760_amd as codag
    one = enc.encode_rle_v1(np.arange(4, dtype=np.int64))
    ch = _chunks(oracle.RLE_V1, [one, one], [32, 32])
    comp, co, oo = [torch.from_numpy(np.ascontiguousarray(a).view(np.uint8 if a.dtype == np.uint8 else np.int64)).to(dev)
                    for a in (ch.comp, ch.chunk_offsets, ch.out_offsets)]
    out = torch.zeros(80, dtype=torch.uint8, device=dev)
    st = torch.zeros(2, dtype=torch.int32, device=dev)
    # shift the output by 4 bytes: both chunks misaligned
    codag.decompress(oracle.RLE_V1, comp, co, out[4:68], oo, status=st)
    assert st.cpu().tolist() == [oracle.E_INVALID_ARGUMENT] * 2
    assert (out.cpu().numpy() == 0).all()  # nothing written
    rc, bad = codag.get_error()
    assert rc == oracle.E_INVALID_ARGUMENT and bad == 0
    assert codag.get_error() == (0, None)  # cleared


def test_capacity_statuses(dev):
    vals = np.arange(200, dtype=np.int64) * 7
    blobs, sizes = [], []
    for codec, encode, gp in ((oracle.RLE_V1, enc.encode_rle_v1, 1), (oracle.RLE_V1, enc.encode_rle_v1, 2),
                              (oracle.RLE_V2, enc.encode_rle_v2, 1), (oracle.RLE_V2, enc.encode_rle_v2, 2)):
        data = encode(vals)
        ch = _chunks(codec, [data, data, data, data + b"\x00", data[:-1]], [1600, 1592, 1608, 1600, 1600])
        st = assert_parity(codec, ch, dev, group_parallel=gp)
        assert st.tolist() == [0, oracle.E_OVERFLOW, oracle.E_TRUNCATED, oracle.E_CORRUPT, oracle.E_TRUNCATED]
    d = workloads.zipf_text(30000, np.random.default_rng(2), workloads._vocab(0))
    z = workloads.deflate_raw(d)
    ch = _chunks(oracle.DEFLATE, [z, z, z, z[:-3], z + b"junk"], [len(d), len(d) - 1, len(d) + 1, len(d), len(d)])
    st = assert_parity(oracle.DEFLATE, ch, dev)
    assert st.tolist() == [0, oracle.E_OVERFLOW, oracle.E_UNDERFLOW, oracle.E_TRUNCATED, 0]


def test_short_repeat_stretch_ending_at_capacity(dev):
    """A stretch of SHORT_REPEAT runs that fills the output exactly, followed
    by a header whose value is cut off by the end of the input: with the
    output full nothing more is parsed and the leftover byte makes the chunk
    CORRUPT; with room for one more value the cut-off header is an OVERFLOW
    (capacity is checked before the payload), as in the sequential decode."""
    runs = bytes([0x07, 0x0a]) * 3             # three runs of ten 5s (width 1)
    blobs, sizes = [], []
    for tail in (b"\x00", b"\x00\x02", b"\x40", b"\x07"):
        for cap in (30, 31, 40):
            blobs.append(runs + tail)
            sizes.append(8 * cap)
    ch = _chunks(oracle.RLE_V2, blobs, sizes)
    for gp in (1, 2):
        st = assert_parity(oracle.RLE_V2, ch, dev, group_parallel=gp)
        assert st[0] == oracle.E_CORRUPT and st[1] == oracle.E_OVERFLOW


# ---- corrupt inputs: same status class as the oracle -------------------------

def _mutants(blobs, rng, count):
    out = []
    for t in range(count):
        b = bytearray(blobs[t % len(blobs)])
        if t % 4 == 3:
            b = b[: int(rng.integers(0, len(b)))]
        else:
            for _ in range(int(rng.integers(1, 4))):
                if b:
                    i = int(rng.integers(0, len(b)))
                    b[i] ^= 1 << int(rng.integers(0, 8))
        out.append(bytes(b))
    return out


@pytest.mark.parametrize("codec,gp", [(oracle.RLE_V1, 1), (oracle.RLE_V1, 2), (oracle.RLE_V2, 1),
                                      (oracle.RLE_V2, 2), (oracle.DEFLATE, 0)])
def test_corrupt_streams_status_parity(dev, codec, gp):
    rng = np.random.default_rng(100 + codec)
    if codec == oracle.DEFLATE:
        vocab = workloads._vocab(0)
        raw = [workloads.zipf_text(5000, rng, vocab), workloads.int32_column(6000, rng),
               workloads.random_bytes(700, rng)]
        base = [workloads.deflate_raw(raw[0]), workloads.deflate_raw(raw[1], fixed=True),
                workloads.deflate_raw(raw[2], level=0)]
        sizes = [len(r) for r in raw]
    else:
        ch0 = (workloads.rle_v1_workload if codec == oracle.RLE_V1 else workloads.rle_v2_workload)(
            seed=9, n_values=6000, chunk_values=2000)
        base = [ch0.comp[int(ch0.chunk_offsets[i]):int(ch0.chunk_offsets[i + 1])].tobytes() for i in range(3)]
        sizes = [16000] * 3
    muts = _mutants(base, rng, 600)
    ch = _chunks(codec, muts, [sizes[t % len(sizes)] for t in range(len(muts))])
    _say(f"corrupt codec={codec} group_parallel={gp} chunks={ch.n_chunks}")
    st = assert_parity(codec, ch, dev, group_parallel=gp)
    assert (st != 0).sum() > 100



@pytest.mark.parametrize("version,gp", [("0.11", 1), ("0.11", 2), ("0.12", 1), ("0.12", 2)])
def test_orc_writer_streams_damaged(dev, tmp_path, version, gp):
    """Integer DATA streams written by Apache ORC's writer (through pyarrow),
    as written and damaged in one to three bytes: GPU output and statuses
    equal the oracle's on both RLE paths."""
    pa = pytest.importorskip("pyarrow")
    po = pytest.importorskip("pyarrow.orc")
    from orc_walk import integer_data_streams
    from test_oracle_rle_mutants import _values
    rng = np.random.default_rng([77, gp, 0 if version == "0.11" else 1])
    values = _values(rng)
    path = str(tmp_path / "t.orc")
    po.write_table(pa.table({"x": pa.array(values, type=pa.int64())}), path,
                   file_version=version, compression="uncompressed")
    kind, streams = integer_data_streams(path)
    codec = oracle.RLE_V1 if kind == 0 else oracle.RLE_V2
    s = streams[0]
    muts = [s]
    for _ in range(300):
        b = bytearray(s)
        for _ in range(int(rng.integers(1, 4))):
            b[int(rng.integers(0, len(b)))] = int(rng.integers(0, 256))
        muts.append(bytes(b))
    ch = _chunks(codec, muts, [8 * values.size] * len(muts))
    _say(f"orc-written damaged codec={codec} group_parallel={gp} chunks={ch.n_chunks}")
    st = assert_parity(codec, ch, dev, group_parallel=gp)
    assert st[0] == 0 and (st != 0).any()


def test_orc_writer_byte_rle_damaged(dev, tmp_path):
    """The byte RLE DATA stream of a byte column written by Apache ORC's
    writer, as written and damaged in one to three bytes: GPU output and
    statuses equal the oracle's."""
    pa = pytest.importorskip("pyarrow")
    po = pytest.importorskip("pyarrow.orc")
    from orc_walk import integer_data_streams
    rng = np.random.default_rng([78, 4])
    values = np.concatenate([np.repeat(rng.integers(-128, 128, 60), rng.integers(1, 40, 60)),
                             rng.integers(-128, 128, 2000)]).astype(np.int8)
    path = str(tmp_path / "b.orc")
    po.write_table(pa.table({"x": pa.array(values, type=pa.int8())}), path, compression="uncompressed")
    _, streams = integer_data_streams(path)
    s = streams[0]
    muts = [s]
    for _ in range(300):
        b = bytearray(s)
        for _ in range(int(rng.integers(1, 4))):
            b[int(rng.integers(0, len(b)))] = int(rng.integers(0, 256))
        muts.append(bytes(b))
    ch = _chunks(oracle.BYTE_RLE, muts, [values.size] * len(muts))
    _say(f"orc-written damaged byte RLE chunks={ch.n_chunks}")
    st = assert_parity(oracle.BYTE_RLE, ch, dev)
    assert st[0] == 0 and (st != 0).any()

# ---- full workload sizes, benchmark launch configuration ---------------------

@pytest.mark.parametrize("gp", [0, 1])
def test_full_rle_v1(dev, gp):
    ch = workloads.rle_v1_workload(seed=0)
    _say(f"full rle_v1 chunks={ch.n_chunks} group_parallel={gp}")
    assert (assert_parity(oracle.RLE_V1, ch, dev, group_parallel=gp) == 0).all()


@pytest.mark.parametrize("gp", [0, 1])
def test_full_rle_v2(dev, gp):
    ch = workloads.rle_v2_workload(seed=0)
    _say(f"full rle_v2 chunks={ch.n_chunks} group_parallel={gp}")
    assert (assert_parity(oracle.RLE_V2, ch, dev, threads=16, group_parallel=gp) == 0).all()


def test_full_deflate(dev):
    ch = workloads.deflate_workload(seed=0)
    _say(f"full deflate chunks={ch.n_chunks}")
    assert (assert_parity(oracle.DEFLATE, ch, dev, threads=16) == 0).all()
