"""GPU parity of the read path around the decoders: compressed ORC streams
(codag_orc_inflate_stream), byte RLE, and the integer encodings with other
element types -- against the oracle on synthetic streams (with guard ranges
and mutated streams), and end to end on files the Apache ORC writer produces
through pyarrow: every stream of the file inflated on the GPU and decoded on
the GPU gives back the columns pyarrow was handed."""
import sys
import zlib

import numpy as np
import pytest

import oracle
import workloads
from workloads import enc

from gpu_util import assert_parity

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


# ---- element types of the integer encodings -------------------------------

@pytest.mark.parametrize("codec", [oracle.RLE_V1, oracle.RLE_V2])
@pytest.mark.parametrize("eb,uns", [(1, False), (2, False), (4, False), (8, True), (4, True), (1, True)])
def test_element_types(dev, codec, eb, uns):
    rng = np.random.default_rng(31 + eb + 10 * uns)
    make = workloads.rle_v1_workload if codec == oracle.RLE_V1 else workloads.rle_v2_workload
    src = make(seed=7, n_values=60_000, chunk_values=7000)
    blobs = [src.comp[int(src.chunk_offsets[i]):int(src.chunk_offsets[i + 1])].tobytes() for i in range(src.n_chunks)]
    vals = [int(src.out_offsets[i + 1] - src.out_offsets[i]) // 8 for i in range(src.n_chunks)]
    # The workload's streams read at every element width, as signed and as
    # unsigned values: every reading is defined, and the oracle's decode of
    # it is the reference.
    ch = _chunks(codec, blobs, [eb * v for v in vals])
    _say(f"typed codec={codec} elem={eb} unsigned={uns}")
    assert (assert_parity(codec, ch, dev, elem_bytes=eb, unsigned_values=uns) == 0).all()
    muts = _mutants(blobs[:3], rng, 200)
    ch = _chunks(codec, muts, [eb * vals[t % 3] for t in range(len(muts))])
    st = assert_parity(codec, ch, dev, elem_bytes=eb, unsigned_values=uns)
    assert (st != 0).sum() > 20


def test_element_type_argument_checks(dev):
    import paper_2307_03760_amd as codag
    from gpu_util import gpu_decode
    ch = workloads.rle_v1_workload(seed=3, n_values=1000, chunk_values=500)
    for kw in ({"elem_bytes": 3}, {"unsigned_values": 2}, {"elem_bytes": 4, "group_parallel": 2},
               {"elem_bytes": 2, "variant": 1}):
        with pytest.raises(codag.CodagError):
            gpu_decode(oracle.RLE_V1, ch, dev, **kw)
    # An output range that is not a multiple of the element is refused per chunk.
    odd = _chunks(oracle.RLE_V2, [enc.encode_rle_v2(np.arange(10, dtype=np.int64))], [10 * 4 + 2])
    st = assert_parity(oracle.RLE_V2, odd, dev, guards=False, elem_bytes=4)  # guards would be misaligned too
    assert st.tolist() == [oracle.E_INVALID_ARGUMENT]
    codag.get_error()


# ---- byte RLE --------------------------------------------------------------

def test_byte_rle(dev):
    rng = np.random.default_rng(41)
    datas = [b"", bytes(1000), bytes(range(256)) * 3]
    for _ in range(60):
        n = int(rng.integers(1, 40000))
        datas.append(np.repeat(rng.integers(0, 6, n), rng.integers(1, 12, n))[:n].astype(np.uint8).tobytes())
    blobs = [enc.encode_byte_rle(d) for d in datas]
    ch = _chunks(oracle.BYTE_RLE, blobs, [len(d) for d in datas])
    _say(f"byte rle chunks={ch.n_chunks}")
    assert (assert_parity(oracle.BYTE_RLE, ch, dev) == 0).all()
    # capacity and corrupt statuses
    z = enc.encode_byte_rle(datas[5])
    ch = _chunks(oracle.BYTE_RLE, [z, z, z, z + b"\x00", z[:-1]],
                 [len(datas[5]), len(datas[5]) - 1, len(datas[5]) + 1, len(datas[5]), len(datas[5])])
    st = assert_parity(oracle.BYTE_RLE, ch, dev)
    assert st[0] == 0 and (st[1:] != 0).all()
    muts = _mutants(blobs[3:10], rng, 300)
    ch = _chunks(oracle.BYTE_RLE, muts, [len(datas[3 + t % 7]) for t in range(len(muts))])
    st = assert_parity(oracle.BYTE_RLE, ch, dev)
    assert (st != 0).sum() > 50


# ---- compressed ORC streams ------------------------------------------------

def _gpu_inflate(framed: bytes, block: int, out_cap: int, dev):
    import torch
    import paper_2307_03760_amd as codag
    src = torch.from_numpy(np.frombuffer(framed + b"\0" * 16, np.uint8).copy()).to(dev)[:len(framed)]
    out = torch.full((max(out_cap, 1),), 0xA5, dtype=torch.uint8, device=dev)[:out_cap]
    out_len = torch.zeros(1, dtype=torch.int64, device=dev)
    st = torch.full((1,), 99, dtype=torch.int32, device=dev)
    codag.orc_inflate_stream(src, block, out, out_len, st)
    torch.cuda.synchronize()
    n = int(out_len.item())
    return int(st.item()), out[:n].cpu().numpy().tobytes()


def _frame(chunks):
    out = bytearray()
    for payload, original in chunks:
        h = (len(payload) << 1) | int(original)
        out += bytes([h & 255, (h >> 8) & 255, h >> 16]) + payload
    return bytes(out)


def test_orc_framing_rules_match_oracle(dev):
    block = 1000
    rng = np.random.default_rng(5)
    raw = bytes(rng.integers(0, 4, 3500, dtype=np.uint8))
    parts = [raw[i:i + block] for i in range(0, len(raw), block)]

    def deflated(p):
        c = zlib.compressobj(9, zlib.DEFLATED, -15)
        return c.compress(p) + c.flush()

    mixed = _frame([(deflated(parts[0]), False), (parts[1], True), (deflated(parts[2]), False),
                    (parts[3], True)])
    one = _frame([(deflated(parts[0]), False)])
    cases = [(mixed, 10_000), (mixed, 3499), (mixed[:-1], 10_000), (one + b"\x05\x00", 10_000),
             (mixed + b"\x05\x00", 10_000),
             (_frame([(deflated(parts[0][:999]), False), (deflated(parts[1]), False)]), 10_000),
             (_frame([(deflated(parts[0] + b"x"), False), (deflated(parts[1]), False)]), 10_000),
             (b"", 10), (_frame([(b"\xff\xff", False)]), 10_000)]
    for framed, cap in cases:
        ref_st, ref = oracle.orc_inflate_stream(framed, block, cap)
        got_st, got = _gpu_inflate(framed, block, cap, dev)
        assert got_st == ref_st, (len(framed), cap, got_st, ref_st)
        if ref_st == oracle.OK:
            assert got == ref


@pytest.mark.parametrize("version,block,compression", [("0.12", 65536, "zlib"), ("0.11", 65536, "zlib"),
                                                       ("0.12", 131072, "zlib"), ("0.12", 0, "uncompressed")])
def test_orc_file_end_to_end(dev, tmp_path, version, block, compression):
    """Every stream of a pyarrow-written ORC file: inflated on the GPU (if
    compressed) and decoded on the GPU, equal to the oracle's result and to
    the columns written."""
    import torch
    import paper_2307_03760_amd as codag
    pa = pytest.importorskip("pyarrow")
    po = pytest.importorskip("pyarrow.orc")
    from orc_walk import DATA, LENGTH, PRESENT, file_streams
    rng = np.random.default_rng(17)
    n = 400_000
    vals = np.cumsum(rng.integers(-50, 100, n))
    big = rng.random(n) < 0.02
    vals[big] = rng.integers(-(1 << 40), 1 << 40, int(big.sum()))
    nulls = rng.random(n) < 0.1
    words = np.array([str(int(v)) for v in rng.integers(0, 10 ** 6, n)])
    table = pa.table({"i64": pa.array(vals, mask=nulls), "s": pa.array(words),
                      "i8": pa.array((vals % 97).astype(np.int8)),
                      "i32": pa.array((vals * 37).astype(np.int32))})
    path = str(tmp_path / "t.orc")
    kw = {"file_version": version, "compression": compression}
    if block:
        kw["compression_block_size"] = block
    po.write_table(table, path, **kw)
    f = file_streams(path)
    assert len(f["stripes"]) == 1
    streams = f["stripes"][0]["streams"]
    rle = oracle.RLE_V2 if version == "0.12" else oracle.RLE_V1
    nn = int((~nulls).sum())
    plan = [  # (column, stream kind, codec, output bytes, elem_bytes, unsigned, expected bytes)
        (1, PRESENT, oracle.BYTE_RLE, (n + 7) // 8, 0, False, np.packbits(~nulls).tobytes()),
        (1, DATA, rle, 8 * nn, 0, False, vals[~nulls].astype(np.int64).tobytes()),
        (2, LENGTH, rle, 8 * n, 0, True, np.char.str_len(words).astype(np.uint64).tobytes()),
        (3, DATA, oracle.BYTE_RLE, n, 0, False, (vals % 97).astype(np.int8).tobytes()),
        (4, DATA, rle, 4 * n, 4, False, (vals * 37).astype(np.int32).tobytes()),
    ]
    for col, kind, codec, out_bytes, eb, uns, expect in plan:
        framed = streams[(col, kind)]
        if f["compression"]:
            ref_st, stream = oracle.orc_inflate_stream(framed, f["block_size"], 1 << 26)
            got_st, got = _gpu_inflate(framed, f["block_size"], 1 << 26, dev)
            assert ref_st == oracle.OK and got_st == oracle.OK and got == stream, (col, kind)
        else:
            stream = framed
        _say(f"orc {version} {compression} column {col} stream {kind}: {len(framed)} -> {len(stream)} bytes")
        # GPU decode of the stream as one chunk (straight from the bytes the GPU inflated).
        comp = torch.from_numpy(np.frombuffer(stream + b"\0" * 16, np.uint8).copy()).to(dev)
        co = torch.tensor([0, len(stream)], dtype=torch.int64, device=dev)
        oo = torch.tensor([0, out_bytes], dtype=torch.int64, device=dev)
        out = torch.full((out_bytes,), 0xA5, dtype=torch.uint8, device=dev)
        st = torch.full((1,), 99, dtype=torch.int32, device=dev)
        codag.decompress(codec, comp, co, out, oo, status=st, elem_bytes=eb, unsigned_values=uns)
        torch.cuda.synchronize()
        assert int(st.item()) == 0, (col, kind, int(st.item()))
        got = out.cpu().numpy().tobytes()
        if kind == PRESENT:
            assert np.array_equal(np.unpackbits(np.frombuffer(got, np.uint8))[:n],
                                  np.unpackbits(np.frombuffer(expect, np.uint8))[:n])
        else:
            assert got == expect, (col, kind)


def test_orc_zlib_stream_damaged(dev, tmp_path):
    """The framed DATA stream of a ZLIB-compressed file written by Apache
    ORC's writer, as written and damaged in one to three bytes: the GPU's
    framing and Deflate decode gives the oracle's status and bytes, and the
    streams that inflate decode on the GPU like the oracle's RLE v2."""
    pa = pytest.importorskip("pyarrow")
    po = pytest.importorskip("pyarrow.orc")
    from orc_walk import DATA, file_streams
    from test_oracle_rle_mutants import _values
    rng = np.random.default_rng([79, 1])
    values = _values(rng)
    path = str(tmp_path / "z.orc")
    po.write_table(pa.table({"x": pa.array(values, type=pa.int64())}), path, file_version="0.12",
                   compression="zlib", compression_block_size=65536)
    f = file_streams(path)
    raw, block = f["stripes"][0]["streams"][(1, DATA)], f["block_size"]
    cap = 1 << 20
    inflated = []
    n_bad = 0
    for k in range(121):
        b = bytearray(raw)
        if k:
            for _ in range(int(rng.integers(1, 4))):
                b[int(rng.integers(0, len(b)))] = int(rng.integers(0, 256))
        ref_st, ref = oracle.orc_inflate_stream(bytes(b), block, cap)
        got_st, got = _gpu_inflate(bytes(b), block, cap, dev)
        assert got_st == ref_st, (k, got_st, ref_st)
        if ref_st == oracle.OK:
            assert got == ref, k
            inflated.append(ref)
        else:
            n_bad += 1
    assert n_bad > 0 and len(inflated) > 10
    _say(f"orc zlib damaged: {n_bad} streams rejected by the framing or Deflate, {len(inflated)} decoded")
    ch = workloads._pack([oracle.RLE_V2] * len(inflated), inflated, [8 * values.size] * len(inflated))
    for gp in (1, 2):
        st = assert_parity(oracle.RLE_V2, ch, dev, group_parallel=gp)
        assert st[0] == 0
