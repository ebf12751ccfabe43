"""GPU test of codag_decompress_noalloc: through the C ABI, the no-allocation
variant gives the same output and per-chunk statuses as codag_decompress_ex
on two calls in a row (the second with a smaller input, so what the first
left in the shared scratch array must not leak into it), and rejects a
launch whose workspace would not fit the scratch array."""
import sys

import numpy as np
import pytest

import oracle
import workloads

from gpu_util import device_inputs

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


def _decode(fn, codec, ch, dev, **kw):
    import torch
    comp, co, oo = device_inputs(ch, dev)
    out = torch.full((max(ch.out_bytes, 1),), 0xA5, dtype=torch.uint8, device=dev)
    st = torch.full((max(ch.n_chunks, 1),), 99, dtype=torch.int32, device=dev)
    fn(codec, comp, co, out, oo, status=st[:ch.n_chunks], **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy(), st[:ch.n_chunks].cpu().numpy()


def _mutated(ch, seed, count):
    comp = ch.comp.copy()
    rng = np.random.default_rng(seed)
    for i in rng.choice(ch.n_chunks, count, replace=False):
        a, b = int(ch.chunk_offsets[i]), int(ch.chunk_offsets[i + 1])
        comp[a + int(rng.integers(0, b - a))] ^= 0x5A
    return workloads.Chunked(ch.codecs, comp, ch.chunk_offsets, ch.out_offsets)


CASES = [
    # (codec, first call, second call (smaller), options)
    (oracle.RLE_V1,
     lambda: workloads.rle_v1_workload(seed=0),                                  # 64 chunks
     lambda: _mutated(workloads.rle_v1_workload(seed=3, n_values=90_000, chunk_values=4000), 1, 5),
     {}),
    (oracle.RLE_V1,
     lambda: workloads.rle_v1_workload(seed=4, n_values=256 * 2000, chunk_values=2000),  # 256 chunks
     lambda: workloads.rle_v1_workload(seed=5, n_values=30_001, chunk_values=16384),
     {"group_parallel": 2}),
    (oracle.RLE_V2,
     lambda: workloads.rle_v2_workload(seed=6, n_values=400_000, chunk_values=32768),
     lambda: workloads.rle_v2_workload(seed=7, n_values=50_000, chunk_values=32768),
     {}),
    (oracle.RLE_V2,
     lambda: workloads.rle_v2_workload(seed=12, n_values=2048 * 300, chunk_values=300),  # 2048 chunks
     lambda: _mutated(workloads.rle_v2_workload(seed=13, n_values=90_000, chunk_values=3000), 2, 6),
     {"group_parallel": 2}),
    (oracle.DEFLATE,
     lambda: workloads.deflate_workload(seed=8, total_bytes=40 * 65536),
     lambda: workloads.deflate_workload(seed=9, total_bytes=5 * 65536 + 1000),
     {}),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_noalloc_matches_ex(dev, case):
    import paper_2307_03760_amd as codag
    codec, first, second, kw = CASES[case]
    for call, make in enumerate((first, second)):
        ch = make()
        _say(f"noalloc case {case} call {call}: codec {codec}, {ch.n_chunks} chunks, {kw}")
        ref, ref_st = _decode(codag.decompress, codec, ch, dev, **kw)
        got, got_st = _decode(codag.decompress_noalloc, codec, ch, dev, **kw)
        assert np.array_equal(got_st, ref_st)
        assert np.array_equal(got, ref)
        codag.get_error()


@pytest.mark.parametrize("codec,over", [(oracle.RLE_V1, 373), (oracle.RLE_V2, 2049)])
def test_noalloc_rejects_workspace_beyond_scratch(dev, codec, over):
    """Forced group-parallel launches whose workspace exceeds the scratch
    array (RLE v1: 528 bytes per chunk, RLE v2: 96, of 196,608) are refused;
    the allocating entry point takes them, and with the default path choice
    the no-allocation entry point decodes them one wave per chunk."""
    import paper_2307_03760_amd as codag
    make = workloads.rle_v1_workload if codec == oracle.RLE_V1 else workloads.rle_v2_workload
    ch = make(seed=10, n_values=over * 64, chunk_values=64)
    assert ch.n_chunks == over
    _say(f"noalloc limit codec {codec}: {over} chunks")
    with pytest.raises(codag.CodagError) as e:
        _decode(codag.decompress_noalloc, codec, ch, dev, group_parallel=2)
    assert e.value.status == codag.E_INVALID_ARGUMENT
    _, st = _decode(codag.decompress, codec, ch, dev, group_parallel=2)
    assert (st == 0).all()
    ref, ref_st = _decode(codag.decompress, codec, ch, dev)
    got, got_st = _decode(codag.decompress_noalloc, codec, ch, dev)
    assert np.array_equal(got_st, ref_st) and np.array_equal(got, ref)
    # One below the limit fits.
    sub = make(seed=11, n_values=(over - 1) * 64, chunk_values=64)
    ref, ref_st = _decode(codag.decompress, codec, sub, dev, group_parallel=2)
    got, got_st = _decode(codag.decompress_noalloc, codec, sub, dev, group_parallel=2)
    assert np.array_equal(got_st, ref_st) and np.array_equal(got, ref) and (got_st == 0).all()
