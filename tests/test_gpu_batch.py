"""GPU parity of the batched persistent launch (codag_decompress_batch):
mixed-codec chunk arrays decode bit-exactly like the oracle under every
queue order, launch shape and window size, eagerly and through captured
graphs replayed several times, and report the same per-chunk status."""
import sys

import numpy as np
import pytest

import oracle
import workloads

from gpu_util import (GUARD_BYTE, batch_device_inputs, check_guards, compare_chunks, compare_shifted,
                      guarded, oracle_mixed)

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


@pytest.fixture(scope="module")
def small():
    ch = workloads.batched_workload(seed=11, n_chunks=240)
    ref, ref_st = oracle_mixed(ch.codecs, ch.comp, ch.chunk_offsets, ch.out_offsets)
    assert (ref_st == 0).all()
    return ch, ref, ref_st


def _guarded_order(order, n):
    """A queue order for the guarded layout: chunk i becomes 2i + 1 (entries
    out of range stay out of range), then the guards."""
    order = np.asarray(order, dtype=np.int64)
    mapped = np.where(order < n, 2 * order + 1, 2 * n + 1 + order)
    return np.concatenate([mapped, np.arange(0, 2 * n + 1, 2)]).astype(np.int32)


def _run(plan, ch, dev, order=None, ticks=False, reps=1, between=None, guards=True):
    """Decodes ch with the plan `reps` times and returns [(out, status)] per
    rep (and the ticks).  With guards, the same plan first decodes the
    guarded layout (every chunk fenced by ranges no chunk may write): the
    guards must come back untouched and each chunk must decode exactly as in
    the plain layout.  The error word is cleared after that run, so what the
    caller reads afterwards is the plain runs' alone."""
    import torch
    import paper_2307_03760_amd as codag
    g_res = None
    if guards:
        gch, idx = guarded(ch)
        codecs, comp, co, oo = batch_device_inputs(gch, dev)
        out = torch.full((max(gch.out_bytes, 1),), GUARD_BYTE, dtype=torch.uint8, device=dev)
        st = torch.full((gch.n_chunks,), 99, dtype=torch.int32, device=dev)
        order_t = None if order is None else \
            torch.from_numpy(_guarded_order(order, ch.n_chunks)).to(dev)
        plan.decompress(codecs, comp, co, out, oo, status=st, order=order_t)
        torch.cuda.synchronize()
        g_out, g_st = out[:gch.out_bytes].cpu().numpy(), st.cpu().numpy()
        check_guards(g_out, gch)
        assert (g_st[0::2] == oracle.E_TRUNCATED).all(), "guard status"
        g_res = (g_out, g_st[idx], gch.out_offsets[idx])
        del out
        codag.get_error()
    codecs, comp, co, oo = batch_device_inputs(ch, dev)
    out = torch.full((max(ch.out_bytes, 1),), GUARD_BYTE, dtype=torch.uint8, device=dev)
    st = torch.full((max(ch.n_chunks, 1),), 99, dtype=torch.int32, device=dev)
    tk = torch.zeros(max(ch.n_chunks, 1), dtype=torch.int64, device=dev) if ticks else None
    order_t = None if order is None else torch.from_numpy(np.asarray(order, np.int32)).to(dev)
    results = []
    for r in range(reps):
        if r and between is not None:
            between(out, st)
        plan.decompress(codecs, comp, co, out, oo, status=st[:ch.n_chunks], order=order_t,
                        chunk_ticks=None if tk is None else tk[:ch.n_chunks])
        torch.cuda.synchronize()
        results.append((out[:ch.out_bytes].cpu().numpy(), st[:ch.n_chunks].cpu().numpy()))
    if g_res is not None:
        got, got_st = results[0]
        compare_shifted(g_res[0], g_res[1], got, got_st, ch.out_offsets, g_res[2])
    return results, (None if tk is None else tk[:ch.n_chunks].cpu().numpy())


@pytest.mark.parametrize("wpb,hist", [(1, 8), (2, 8), (4, 8), (2, 16), (1, 16)])
def test_batch_index_order(dev, small, wpb, hist):
    import paper_2307_03760_amd as codag
    ch, ref, ref_st = small
    _say(f"batch index wpb={wpb} hist={hist} chunks={ch.n_chunks}")
    plan = codag.Plan(waves_per_block=wpb, history_kib=hist)
    (res,), ticks = _run(plan, ch, dev, ticks=True)
    compare_chunks(*res, ref, ref_st, ch.out_offsets)
    assert (ticks > 0).all()
    plan.close()


@pytest.mark.parametrize("kind", ["reverse", "random", "codec_interleaved"])
def test_batch_given_orders(dev, small, kind):
    import paper_2307_03760_amd as codag
    ch, ref, ref_st = small
    n = ch.n_chunks
    if kind == "reverse":
        order = np.arange(n)[::-1]
    elif kind == "random":
        order = np.random.default_rng(3).permutation(n)
    else:
        order = np.argsort(np.arange(n) % 3, kind="stable")
    _say(f"batch given order {kind}")
    plan = codag.Plan(order=codag.ORDER_GIVEN, waves_per_cu=4)
    (res,), _ = _run(plan, ch, dev, order=order)
    compare_chunks(*res, ref, ref_st, ch.out_offsets)


def _interleaved_layout(ch):
    """The same chunks re-indexed so that the codecs alternate in the chunk
    array itself (round robin over RLE v1, RLE v2, Deflate), with a pad chunk
    (empty input, 1-7 output bytes, so it fails as TRUNCATED before writing)
    wherever an RLE chunk's output would otherwise start unaligned.  Returns
    the layout and, per chunk of it, the original chunk index (-1 for pads)."""
    codecs = np.asarray(ch.codecs)
    by_codec = [list(np.nonzero(codecs == c)[0]) for c in (oracle.RLE_V1, oracle.RLE_V2, oracle.DEFLATE)]
    seq = []
    while any(by_codec):
        for q in by_codec:
            if q:
                seq.append(int(q.pop(0)))
    out_codecs, blobs, sizes, src = [], [], [], []
    at = 0
    for i in seq:
        c = int(codecs[i])
        if c != oracle.DEFLATE and at % 8:
            out_codecs.append(oracle.DEFLATE)
            blobs.append(np.zeros(0, np.uint8))
            sizes.append(8 - at % 8)
            src.append(-1)
            at += 8 - at % 8
        a, b = int(ch.chunk_offsets[i]), int(ch.chunk_offsets[i + 1])
        n_out = int(ch.out_offsets[i + 1] - ch.out_offsets[i])
        out_codecs.append(c)
        blobs.append(np.asarray(ch.comp[a:b]))
        sizes.append(n_out)
        src.append(i)
        at += n_out
    return workloads._pack(out_codecs, blobs, sizes), np.array(src)


@pytest.mark.parametrize("order", ["index", "codec"])
def test_batch_codec_interleaved_layout(dev, small, order):
    """Chunks whose codecs alternate in the chunk array (not only in the queue
    order) decode bit-exactly, pads between them stay unwritten, and the
    codec-grouped queue order gives the same result on that layout."""
    import paper_2307_03760_amd as codag
    ch, _, _ = small
    lay, src = _interleaved_layout(ch)
    assert (np.diff(lay.codecs.astype(np.int64)) != 0).mean() > 0.5
    ref, ref_st = oracle_mixed(lay.codecs, lay.comp, lay.chunk_offsets, lay.out_offsets)
    assert (ref_st[src >= 0] == 0).all() and (ref_st[src < 0] == oracle.E_TRUNCATED).all()
    _say(f"batch interleaved layout order={order} chunks={lay.n_chunks}")
    plan = codag.Plan(order=codag.ORDER_CODEC if order == "codec" else codag.ORDER_INDEX)
    (res,), _ = _run(plan, lay, dev)
    got, got_st = res
    compare_chunks(got, got_st, ref, ref_st, lay.out_offsets)
    for k in np.nonzero(src < 0)[0]:
        a, b = int(lay.out_offsets[k]), int(lay.out_offsets[k + 1])
        assert (got[a:b] == GUARD_BYTE).all(), f"pad chunk {k} written"
    plan.close()


def test_batch_graph_replays(dev, small):
    """A captured graph replayed three times, with eager work between the
    replays (clearing the output and status), gives the full result each time."""
    import paper_2307_03760_amd as codag
    ch, ref, ref_st = small
    _say("batch graph replays")
    plan = codag.Plan(use_graph=True, order=codag.ORDER_GIVEN)
    order = np.random.default_rng(4).permutation(ch.n_chunks)

    def clear(out, st):
        out.fill_(0x5A)
        st.fill_(77)
        (out[:1024].to(dev).float() * 2).sum().item()

    results, _ = _run(plan, ch, dev, order=order, reps=3, between=clear)
    for res in results:
        compare_chunks(*res, ref, ref_st, ch.out_offsets)


def test_batch_bad_codec_corrupt_and_bad_order(dev):
    """Per-chunk status like the oracle for an unknown codec byte, corrupt
    and truncated chunks inside a batch; an order entry out of range is
    skipped and reported."""
    import torch
    import paper_2307_03760_amd as codag
    ch = workloads.batched_workload(seed=12, n_chunks=60)
    comp = ch.comp.copy()
    codecs = ch.codecs.copy()
    rng = np.random.default_rng(5)
    for i in rng.choice(ch.n_chunks, 12, replace=False):
        a, b = int(ch.chunk_offsets[i]), int(ch.chunk_offsets[i + 1])
        comp[a + int(rng.integers(0, b - a))] ^= 0xFF
    codecs[7] = 9
    bad = workloads.Chunked(codecs, comp, ch.chunk_offsets, ch.out_offsets)
    ref, ref_st = oracle_mixed(bad.codecs, bad.comp, bad.chunk_offsets, bad.out_offsets)
    assert ref_st[7] == oracle.E_INVALID_ARGUMENT and (ref_st != 0).sum() >= 2
    _say("batch corrupt")
    codag.get_error()  # clear what earlier launches left
    plan = codag.Plan()
    (res,), _ = _run(plan, bad, dev)
    compare_chunks(*res, ref, ref_st, bad.out_offsets)
    rc, first = codag.get_error()
    assert rc == int(ref_st[np.nonzero(ref_st)[0][0]]) and first == int(np.nonzero(ref_st)[0][0])
    # An order naming a chunk that does not exist.
    gplan = codag.Plan(order=codag.ORDER_GIVEN)
    order = np.arange(ch.n_chunks)
    order[5] = ch.n_chunks + 3
    good = workloads.Chunked(ch.codecs, ch.comp, ch.chunk_offsets, ch.out_offsets)
    (res,), _ = _run(gplan, good, dev, order=order)
    got, got_st = res
    assert got_st[5] == 99 and (np.delete(got_st, 5) == 0).all()
    rc, first = codag.get_error()
    assert rc == codag.E_INVALID_ARGUMENT and first == 5
    torch.cuda.synchronize()


def test_batch_empty_and_argument_checks(dev):
    import torch
    import paper_2307_03760_amd as codag
    plan = codag.Plan()
    z = torch.zeros(1, dtype=torch.int64, device=dev)
    u8 = torch.zeros(16, dtype=torch.uint8, device=dev)
    plan.decompress(u8[:0], u8, z, u8, z)            # zero chunks: nothing to do
    torch.cuda.synchronize()
    with pytest.raises(codag.CodagError):
        codag.Plan(waves_per_block=3)
    with pytest.raises(codag.CodagError):
        codag.Plan(history_kib=32)
    gplan = codag.Plan(order=codag.ORDER_GIVEN)
    ch = workloads.batched_workload(seed=13, n_chunks=4)
    codecs, comp, co, oo = batch_device_inputs(ch, dev)
    out = torch.empty(ch.out_bytes, dtype=torch.uint8, device=dev)
    with pytest.raises(codag.CodagError):
        gplan.decompress(codecs, comp, co, out, oo)   # given order without an order


def test_autotune_keeps_a_valid_fast_config(dev, small):
    import torch
    import paper_2307_03760_amd as codag
    ch, ref, ref_st = small
    _say("autotune")
    plan = codag.Plan()
    codecs, comp, co, oo = batch_device_inputs(ch, dev)
    out = torch.empty(ch.out_bytes, dtype=torch.uint8, device=dev)
    best = plan.autotune(codecs, comp, co, out, oo, reps=2)
    assert best > 0
    o = plan.opts
    assert o["waves_per_block"] in (1, 2, 4) and o["history_kib"] in (4, 8, 16) and o["waves_per_cu"] >= 1
    (res,), _ = _run(plan, ch, dev)
    compare_chunks(*res, ref, ref_st, ch.out_offsets)


@pytest.mark.parametrize("tb,claim,order", [(10, 1, 0), (9, 2, 0), (10, 4, 3), (9, 1, 3), (10, 3, 2)])
def test_batch_table_bits_claims_codec_order(dev, small, tb, claim, order):
    """Deflate table bits 10, several chunks per queue claim, and the
    codec-grouped order (sorted on the device) decode like the oracle."""
    import paper_2307_03760_amd as codag
    ch, ref, ref_st = small
    _say(f"batch tb={tb} claim={claim} order={order}")
    plan = codag.Plan(lit_table_bits=tb, chunks_per_claim=claim, order=order, use_graph=True)
    assert plan.opts["lit_table_bits"] == tb and plan.opts["chunks_per_claim"] == claim
    (res, res2), _ = _run(plan, ch, dev, reps=2)
    compare_chunks(*res, ref, ref_st, ch.out_offsets)
    compare_chunks(*res2, ref, ref_st, ch.out_offsets)
    plan.close()


def test_autotune_cache_hit_and_text(dev, small):
    """A second autotune of the same chunk array is served from the cache
    (same configuration and time, no timing); the cache survives a text round
    trip through clear and load; the cached configuration decodes correctly."""
    import time
    import torch
    import paper_2307_03760_amd as codag
    ch, ref, ref_st = small
    codag.autotune_cache_clear()
    codecs, comp, co, oo = batch_device_inputs(ch, dev)
    out = torch.empty(ch.out_bytes, dtype=torch.uint8, device=dev)
    p1 = codag.Plan()
    best1 = p1.autotune(codecs, comp, co, out, oo, reps=2)
    text = codag.autotune_cache_save()
    assert text.count("\n") == 1 and text.split("|")[0].startswith("gfx")
    p2 = codag.Plan()
    t = time.perf_counter()
    best2 = p2.autotune(codecs, comp, co, out, oo, reps=2)
    cached_s = time.perf_counter() - t
    assert best2 == pytest.approx(best1, rel=1e-5)
    keys = ("history_kib", "lit_table_bits", "waves_per_block", "chunks_per_claim", "waves_per_cu", "order")
    assert all(p1.opts[k] == p2.opts[k] for k in keys)
    codag.autotune_cache_clear()
    codag.autotune_cache_load(text)
    assert codag.autotune_cache_save() == text
    p3 = codag.Plan()
    assert p3.autotune(codecs, comp, co, out, oo, reps=2) == pytest.approx(best1, rel=1e-5)
    assert all(p1.opts[k] == p3.opts[k] for k in keys)
    (res,), _ = _run(p3, ch, dev)
    compare_chunks(*res, ref, ref_st, ch.out_offsets)
    _say(f"autotune cached in {cached_s * 1e3:.1f} ms; opts {p3.opts}")
    for p in (p1, p2, p3):
        p.close()
    codag.autotune_cache_clear()


def test_batch_full_size(dev):
    """20,000 mixed chunks (about 2 GiB out) in the benchmark's launch
    (persistent, graph-captured): every chunk equals the oracle's decode
    byte for byte, and with guard ranges around every chunk none is written."""
    import paper_2307_03760_amd as codag
    ch = workloads.batched_workload(seed=0, n_chunks=20000)
    _say(f"batch full size: {ch.n_chunks} chunks, {ch.out_bytes / 2**30:.2f} GiB out")
    ref, ref_st = oracle_mixed(ch.codecs, ch.comp, ch.chunk_offsets, ch.out_offsets, threads=16)
    assert (ref_st == 0).all()
    plan = codag.Plan(use_graph=True)
    (res,), _ = _run(plan, ch, dev)
    compare_chunks(*res, ref, ref_st, ch.out_offsets)
    plan.close()
