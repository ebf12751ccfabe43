"""GPU parity of the decoding-unit ablations (codag_opts.variant): the
leader-lane decoders (one lane parses, the wave writes), the prefetch wave
in front of the main decoders, and the block-per-chunk leader (RLE v1) give
the oracle's output and statuses on the same cases as the main decoders --
small workloads with ragged tails, extremes, capacity errors, mutated
streams and the full workloads -- with guard ranges around every chunk."""
import sys
import zlib

import numpy as np
import pytest

import oracle
import workloads
from workloads import enc

from gpu_util import assert_parity

pytestmark = pytest.mark.gpu

LEADER, PREFETCH, BLOCK = 1, 2, 3
RLE_V1_VARIANTS = [LEADER, PREFETCH, BLOCK]
DEFLATE_VARIANTS = [LEADER, PREFETCH]


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


@pytest.mark.parametrize("variant", RLE_V1_VARIANTS)
def test_rle_v1_variants(dev, variant):
    ch = workloads.rle_v1_workload(seed=5, n_values=100_003, chunk_values=16384)
    _say(f"rle_v1 variant {variant} small")
    assert (assert_parity(oracle.RLE_V1, ch, dev, variant=variant) == 0).all()
    I64_MIN, I64_MAX = -(1 << 63), (1 << 63) - 1
    vals = [np.array([I64_MIN, I64_MAX, 0, -1, 1] * 40, dtype=np.int64),
            np.arange(1000, dtype=np.int64) * -128,
            np.random.default_rng(3).integers(I64_MIN, I64_MAX, 777, dtype=np.int64)]
    ch = _chunks(oracle.RLE_V1, [enc.encode_rle_v1(v) for v in vals], [8 * v.size for v in vals])
    _say(f"rle_v1 variant {variant} extremes")
    assert (assert_parity(oracle.RLE_V1, ch, dev, variant=variant) == 0).all()
    data = enc.encode_rle_v1(np.arange(200, dtype=np.int64) * 7)
    ch = _chunks(oracle.RLE_V1, [data, data, data, data + b"\x00", data[:-1], b"", data],
                 [1600, 1592, 1608, 1600, 1600, 8, 0])
    st = assert_parity(oracle.RLE_V1, ch, dev, variant=variant)
    assert st.tolist()[:5] == [0, oracle.E_OVERFLOW, oracle.E_TRUNCATED, oracle.E_CORRUPT,
                               oracle.E_TRUNCATED]


@pytest.mark.parametrize("variant", RLE_V1_VARIANTS)
def test_rle_v1_variants_corrupt(dev, variant):
    rng = np.random.default_rng(201)
    ch0 = workloads.rle_v1_workload(seed=9, n_values=6000, chunk_values=2000)
    base = [ch0.comp[int(ch0.chunk_offsets[i]):int(ch0.chunk_offsets[i + 1])].tobytes() for i in range(3)]
    muts = _mutants(base, rng, 300)
    ch = _chunks(oracle.RLE_V1, muts, [16000] * len(muts))
    _say(f"rle_v1 variant {variant} corrupt")
    st = assert_parity(oracle.RLE_V1, ch, dev, variant=variant)
    assert (st != 0).sum() > 50


@pytest.mark.parametrize("variant", RLE_V1_VARIANTS)
def test_rle_v1_variants_full(dev, variant):
    ch = workloads.rle_v1_workload(seed=0)
    _say(f"rle_v1 variant {variant} full")
    assert (assert_parity(oracle.RLE_V1, ch, dev, variant=variant) == 0).all()


@pytest.mark.parametrize("variant", DEFLATE_VARIANTS)
def test_deflate_variants(dev, variant):
    ch = workloads.deflate_workload(seed=5, total_bytes=48 * 65536 + 999)
    _say(f"deflate variant {variant} small")
    assert (assert_parity(oracle.DEFLATE, ch, dev, variant=variant) == 0).all()
    rng = np.random.default_rng(8)
    vocab = workloads._vocab(0)
    datas = [b"", b"x", bytes(70000), bytes(range(7)) * 9000, workloads.zipf_text(90000, rng, vocab),
             workloads.int32_column(65536, rng), workloads.random_bytes(100000, rng)]
    blobs, sizes = [], []
    for d in datas:
        for level in (0, 1, 9):
            for strategy in (zlib.Z_DEFAULT_STRATEGY, zlib.Z_HUFFMAN_ONLY, zlib.Z_RLE, zlib.Z_FIXED):
                co = zlib.compressobj(level, zlib.DEFLATED, -15, 8, strategy)
                blobs.append(co.compress(d) + co.flush())
                sizes.append(len(d))
    ch = _chunks(oracle.DEFLATE, blobs, sizes)
    _say(f"deflate variant {variant} strategies")
    assert (assert_parity(oracle.DEFLATE, ch, dev, variant=variant) == 0).all()
    d = workloads.zipf_text(30000, np.random.default_rng(2), vocab)
    z = workloads.deflate_raw(d)
    ch = _chunks(oracle.DEFLATE, [z, z, z, z[:-3], z + b"junk"],
                 [len(d), len(d) - 1, len(d) + 1, len(d), len(d)])
    st = assert_parity(oracle.DEFLATE, ch, dev, variant=variant)
    assert st.tolist() == [0, oracle.E_OVERFLOW, oracle.E_UNDERFLOW, oracle.E_TRUNCATED, 0]


@pytest.mark.parametrize("variant", DEFLATE_VARIANTS)
def test_deflate_variants_corrupt(dev, variant):
    rng = np.random.default_rng(203)
    vocab = workloads._vocab(0)
    raw = [workloads.zipf_text(5000, rng, vocab), workloads.int32_column(6000, rng),
           workloads.random_bytes(700, rng)]
    base = [workloads.deflate_raw(raw[0]), workloads.deflate_raw(raw[1], fixed=True),
            workloads.deflate_raw(raw[2], level=0)]
    muts = _mutants(base, rng, 300)
    ch = _chunks(oracle.DEFLATE, muts, [len(raw[t % 3]) for t in range(len(muts))])
    _say(f"deflate variant {variant} corrupt")
    st = assert_parity(oracle.DEFLATE, ch, dev, variant=variant)
    assert (st != 0).sum() > 50


@pytest.mark.parametrize("variant", DEFLATE_VARIANTS)
def test_deflate_variants_full(dev, variant):
    ch = workloads.deflate_workload(seed=0)
    _say(f"deflate variant {variant} full")
    assert (assert_parity(oracle.DEFLATE, ch, dev, threads=16, variant=variant) == 0).all()


def test_variant_argument_checks(dev):
    import torch
    import paper_2307_03760_amd as codag
    ch = workloads.rle_v2_workload(seed=3, n_values=1000, chunk_values=500)
    from gpu_util import gpu_decode
    for codec, variant in ((oracle.RLE_V2, LEADER), (oracle.DEFLATE, BLOCK), (oracle.RLE_V1, 4),
                           (oracle.RLE_V1, -1)):
        with pytest.raises(codag.CodagError) as e:
            gpu_decode(codec, ch, dev, variant=variant)
        assert e.value.status == codag.E_INVALID_ARGUMENT
    ticks = torch.zeros(ch.n_chunks, dtype=torch.int64, device=dev)
    with pytest.raises(codag.CodagError):
        gpu_decode(oracle.RLE_V1, ch, dev, variant=LEADER, chunk_ticks=ticks)
