"""GPU parity of the LZ4 block decoder (codec CODAG_LZ4) with the oracle:
blocks from the reference LZ4 compressor and from the greedy encoder (far
offsets, long matches and literal runs), every window size and workgroup
shape, unaligned layouts, hand-worked error streams, mutated and cut
streams, capacity statuses, the batched launch with LZ4 chunks among the
other codecs, ORC streams with LZ4 chunks, and the full-size workload.
Each comparison also reruns the chunks with guard ranges around every
output range."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import workloads
from workloads.lz4enc import lz4_greedy

from gpu_util import assert_parity, batch_device_inputs, check_guards, compare_chunks, gpu_decode, \
    oracle_mixed

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "lz4_hand_streams.json")


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


def _chunks(blobs, sizes, codec=oracle.LZ4):
    return workloads._pack([codec] * len(blobs), blobs, sizes)


def _far_data(rng, n):
    """Data whose repeats sit 40..65 KiB back, so matches reach past any
    LDS window into the output already written."""
    base = rng.integers(0, 256, 66000, dtype=np.uint8).tobytes()
    parts, size = [], 0
    while size < n:
        a = int(rng.integers(0, 60000))
        piece = base[a:a + int(rng.integers(20, 3000))]
        parts.append(piece)
        size += len(piece)
    return (base + b"".join(parts))[:n]


def _mixed_blobs(rng, count, greedy_every=3):
    blobs, sizes = [], []
    kinds = [workloads.ZIPF, workloads.INT32, workloads.RANDOM, workloads.INT32_RUNS]
    for i in range(count):
        n = int(rng.integers(0, 90_000)) if i % 7 else int(rng.integers(0, 40))
        if i % 11 == 5:
            data = _far_data(rng, n)
        else:
            data, _ = workloads._class_data(5, 99, i, n, kinds[i % 4])
        blob = lz4_greedy(data) if i % greedy_every == 0 else workloads.lz4_block(data)
        blobs.append(blob)
        sizes.append(len(data))
    return blobs, sizes


@pytest.mark.parametrize("hist,wpb", [(4, 0), (2, 1), (4, 2), (8, 4), (16, 1), (32, 1)])
def test_lz4_small(dev, hist, wpb):
    rng = np.random.default_rng(hist * 10 + wpb)
    blobs, sizes = _mixed_blobs(rng, 90)
    ch = _chunks(blobs, sizes)
    _say(f"lz4 small hist={hist} wpb={wpb} chunks={ch.n_chunks}")
    assert (assert_parity(oracle.LZ4, ch, dev, history_kib=hist, waves_per_block=wpb) == 0).all()


def test_lz4_workload_small(dev):
    ch = workloads.lz4_workload(seed=3, total_bytes=1 << 23)
    _say(f"lz4 workload chunks={ch.n_chunks}")
    assert (assert_parity(oracle.LZ4, ch, dev) == 0).all()


def test_lz4_long_fields(dev):
    """Literal and match runs at the nibble and continuation-byte edges, and
    runs far longer than a window."""
    cases = []
    for lit in (0, 1, 14, 15, 16, 269, 270, 271, 524, 525, 5000, 70000):
        for m in (4, 18, 19, 20, 273, 274, 275, 528, 529, 100_000):
            cases.append((lit, m))
    rng = np.random.default_rng(1)
    blobs, sizes = [], []
    for lit, m in cases:
        lits = rng.integers(0, 256, lit + 1, dtype=np.uint8).tobytes()
        # token, literals, offset 1, match, then the 12 trailing literals
        tail = b"0123456789AB"
        tok = (min(lit + 1, 15) << 4) | min(m - 4, 15)
        b = bytearray([tok])
        if lit + 1 >= 15:
            v = lit + 1 - 15
            while v >= 255:
                b.append(255)
                v -= 255
            b.append(v)
        b += lits + (1).to_bytes(2, "little")
        if m - 4 >= 15:
            v = m - 4 - 15
            while v >= 255:
                b.append(255)
                v -= 255
            b.append(v)
        b += bytes([12 << 4]) + tail
        blobs.append(bytes(b))
        sizes.append(lit + 1 + m + 12)
    ch = _chunks(blobs, sizes)
    assert (assert_parity(oracle.LZ4, ch, dev) == 0).all()


def _literal_block(data: bytes) -> bytes:
    """An LZ4 block of one literal-only sequence."""
    n = len(data)
    b = bytearray([min(n, 15) << 4])
    if n >= 15:
        v = n - 15
        while v >= 255:
            b.append(255)
            v -= 255
        b.append(v)
    return bytes(b) + data


def test_lz4_input_fetch_boundaries(dev):
    """Blocks whose compressed length falls at and around multiples of the
    decoder's 512-byte input fetch, at many start alignments, with literal
    runs read in several pieces; and greedy blocks of nearby lengths."""
    rng = np.random.default_rng(22)
    blobs, sizes, boundary = [], [], []
    for k in (1, 2, 3, 4, 8):
        for d in (-17, -16, -5, -1, 0, 1, 5, 16, 17):
            # A small block first, so that this one starts at the next of the
            # 16 alignments in turn.
            at = sum(len(b) for b in blobs)
            pad = bytes((len(boundary) - at - 1) % 16)
            blobs.append(_literal_block(pad))
            sizes.append(len(pad))
            boundary.append(len(blobs))
            target = 512 * k + d
            n = next(n for n in range(target, 0, -1) if len(_literal_block(bytes(n))) <= target)
            data = rng.integers(0, 256, n, dtype=np.uint8).tobytes()
            blobs.append(_literal_block(data))
            sizes.append(n)
    for i in range(24):
        data = workloads.zipf_text(int(rng.integers(600, 9000)), rng, workloads._vocab(0))
        blobs.append(lz4_greedy(data) if i % 2 else workloads.lz4_block(data))
        sizes.append(len(data))
    ch = _chunks(blobs, sizes)
    assert len({int(ch.chunk_offsets[i]) % 16 for i in boundary}) == 16
    _say(f"lz4 fetch boundaries chunks={ch.n_chunks}")
    assert (assert_parity(oracle.LZ4, ch, dev) == 0).all()


def test_lz4_unaligned_layout(dev):
    """Compressed chunks and output ranges at odd offsets."""
    rng = np.random.default_rng(8)
    blobs, sizes = [], []
    for i in range(60):
        data = workloads.zipf_text(int(rng.integers(1, 20000)), rng, workloads._vocab(0))
        blobs.append(workloads.lz4_block(data) if i % 2 else lz4_greedy(data))
        sizes.append(len(data))
    ch = _chunks(blobs, sizes)
    assert int(ch.out_offsets[1]) % 16 != 0
    assert (assert_parity(oracle.LZ4, ch, dev) == 0).all()


def test_lz4_hand_streams(dev):
    doc = json.load(open(GOLDEN))
    blobs = [bytes(c["bytes"]) for c in doc["streams"]]
    sizes = [c["cap"] for c in doc["streams"]]
    ch = _chunks(blobs, sizes)
    st = assert_parity(oracle.LZ4, ch, dev)
    names = {"OK": 0, "TRUNCATED": oracle.E_TRUNCATED, "CORRUPT": oracle.E_CORRUPT,
             "OVERFLOW": oracle.E_OVERFLOW, "UNDERFLOW": oracle.E_UNDERFLOW}
    assert st.tolist() == [names[c["status"]] for c in doc["streams"]]


def test_lz4_mutants_and_capacities(dev):
    rng = np.random.default_rng(12)
    base, sizes = _mixed_blobs(rng, 12, greedy_every=2)
    blobs, caps = [], []
    for t in range(600):
        k = t % len(base)
        b = bytearray(base[k])
        cap = sizes[k]
        r = t % 6
        if r == 0 and b:
            b = b[: int(rng.integers(0, len(b)))]
        elif r in (1, 2):
            for _ in range(int(rng.integers(1, 4))):
                if b:
                    b[int(rng.integers(0, len(b)))] ^= 1 << int(rng.integers(0, 8))
        elif r == 3:
            cap = int(rng.integers(0, cap + 1))  # overflow
        elif r == 4:
            cap += int(rng.integers(1, 300))  # underflow
        blobs.append(bytes(b))
        caps.append(cap)
    ch = _chunks(blobs, caps)
    _say("lz4 mutants")
    st = assert_parity(oracle.LZ4, ch, dev)
    for code in (oracle.E_TRUNCATED, oracle.E_CORRUPT, oracle.E_OVERFLOW, oracle.E_UNDERFLOW, 0):
        assert (st == code).sum() > 10, code


def test_lz4_batched_mixed(dev):
    import torch
    import paper_2307_03760_amd as codag
    rng = np.random.default_rng(21)
    lz, lz_sizes = _mixed_blobs(rng, 40)
    rl = workloads.rle_v2_workload(seed=2, n_values=200_000, chunk_values=9000)
    df = workloads.deflate_workload(seed=2, total_bytes=1 << 21, chunk_bytes=65536)
    # RLE chunks first: their output ranges must stay 8-byte aligned, and
    # the byte codecs' ranges after them may have any length.
    blobs, sizes, codecs = [], [], []
    for src, c in ((rl, oracle.RLE_V2), (df, oracle.DEFLATE)):
        for i in range(40):
            if c == oracle.DEFLATE:
                blobs.append(lz[i])
                sizes.append(lz_sizes[i])
                codecs.append(oracle.LZ4)
            j = i % src.n_chunks
            blobs.append(src.comp[int(src.chunk_offsets[j]):int(src.chunk_offsets[j + 1])].tobytes())
            sizes.append(int(src.out_offsets[j + 1] - src.out_offsets[j]))
            codecs.append(c)
    ch = workloads._pack(codecs, blobs, sizes)
    ref, ref_st = oracle_mixed(ch.codecs, ch.comp, ch.chunk_offsets, ch.out_offsets)
    cd, comp, co, oo = batch_device_inputs(ch, dev)
    for order in (codag.ORDER_INDEX, codag.ORDER_LEARNED):
        plan = codag.Plan(order=order)
        out = torch.full((ch.out_bytes,), 0xA5, dtype=torch.uint8, device=dev)
        st = torch.full((ch.n_chunks,), 99, dtype=torch.int32, device=dev)
        plan.decompress(cd, comp, co, out, oo, status=st)
        torch.cuda.synchronize()
        compare_chunks(out.cpu().numpy(), st.cpu().numpy(), ref, ref_st, ch.out_offsets)
        plan.close()
    assert (ref_st == 0).all()


def _frame(blocks_raw, block, rng, codec_fn):
    """An ORC stream: each block_size piece compressed with codec_fn, or
    stored original when that is not shorter."""
    out = bytearray()
    for piece in blocks_raw:
        c = codec_fn(piece)
        if len(c) < len(piece) and rng.random() < 0.9:
            out += ((len(c) << 1)).to_bytes(3, "little") + c
        else:
            out += ((len(piece) << 1) | 1).to_bytes(3, "little") + piece
    return bytes(out)


def test_orc_lz4_streams_match_oracle(dev):
    import torch
    import paper_2307_03760_amd as codag
    rng = np.random.default_rng(40)
    block = 4096
    cases = []
    for t in range(12):
        n = int(rng.integers(0, 60_000))
        data = workloads.zipf_text(n, rng, workloads._vocab(1)) if t % 2 else _far_data(rng, n)
        pieces = [data[i:i + block] for i in range(0, len(data), block)]
        framed = _frame(pieces, block, rng, lz4_greedy if t % 3 == 0 else workloads.lz4_block)
        cap = len(data) + (0 if t % 4 else int(rng.integers(-500, 500)))
        cases.append((framed, max(cap, 0)))
    # a chunk that decodes short of block_size before the last, and a cut header
    short = _frame([b"x" * 100, b"y" * 100], block, rng, workloads.lz4_block)
    cases += [(short, 1000), (cases[1][0] + b"\x05", 1 << 17)]
    for framed, cap in cases:
        ref_st, ref = oracle.orc_inflate_stream(framed, block, cap, codec=oracle.LZ4)
        src = torch.from_numpy(np.frombuffer(framed + b"\0", dtype=np.uint8).copy()).to(dev)[: len(framed)]
        out = torch.full((max(cap, 1),), 0xA5, dtype=torch.uint8, device=dev)[:cap]
        out_len = torch.zeros(1, dtype=torch.int64, device=dev)
        st = torch.full((1,), 99, dtype=torch.int32, device=dev)
        codag.orc_decompress_stream(codag.LZ4, src, block, out, out_len, st)
        torch.cuda.synchronize()
        assert int(st.item()) == ref_st
        if ref_st == 0:
            assert int(out_len.item()) == len(ref)
            assert out[: len(ref)].cpu().numpy().tobytes() == ref


def test_orc_lz4_file_end_to_end(dev, tmp_path):
    import torch
    import paper_2307_03760_amd as codag
    pa = pytest.importorskip("pyarrow")
    po = pytest.importorskip("pyarrow.orc")
    from orc_walk import DATA, LENGTH, file_streams
    rng = np.random.default_rng(9)
    n = 500_000
    vals = np.cumsum(rng.integers(-50, 100, n))
    words = np.array([str(int(v)) for v in rng.integers(0, 10 ** 6, n)])
    path = str(tmp_path / "t.orc")
    po.write_table(pa.table({"i": pa.array(vals), "s": pa.array(words)}), path, compression="lz4",
                   compression_block_size=65536)
    f = file_streams(path)
    sf = f["stripes"][0]

    def inflate(framed, cap):
        src = torch.from_numpy(np.frombuffer(framed, dtype=np.uint8).copy()).to(dev)
        out = torch.zeros(cap, dtype=torch.uint8, device=dev)
        out_len = torch.zeros(1, dtype=torch.int64, device=dev)
        st = torch.full((1,), 99, dtype=torch.int32, device=dev)
        codag.orc_decompress_stream(codag.LZ4, src, f["block_size"], out, out_len, st)
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        return out[: int(out_len.item())]

    data = inflate(sf["streams"][(1, DATA)], 1 << 24)
    vals_out = torch.empty(n, dtype=torch.int64, device=dev)
    co = torch.tensor([0, data.numel()], dtype=torch.int64, device=dev)
    oo = torch.tensor([0, 8 * n], dtype=torch.int64, device=dev)
    st = torch.full((1,), 99, dtype=torch.int32, device=dev)
    codag.decompress(codag.RLE_V2, data, co, vals_out.view(torch.uint8), oo, status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert (vals_out.cpu().numpy() == vals).all()
    chars = inflate(sf["streams"][(2, DATA)], 1 << 24)
    assert chars.cpu().numpy().tobytes() == "".join(words).encode()
    lens = inflate(sf["streams"][(2, LENGTH)], 1 << 22)
    assert lens.numel() > 0


def test_lz4_full_workload(dev):
    ch = workloads.lz4_workload(seed=0)
    _say(f"full lz4 chunks={ch.n_chunks}")
    assert (assert_parity(oracle.LZ4, ch, dev, threads=16) == 0).all()
