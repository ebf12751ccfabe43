"""GPU parity of the learned scheduler: header features, the cost model's
forward pass, gradient and Adam step against the float64 oracle, training on
decode times the decoder measures, the learned queue order, and the gain
test (makespan of the learned order against the plain queue)."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from oracle import mlp

from gpu_util import batch_device_inputs, compare_chunks, oracle_mixed

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


def _oracle_features(ch):
    rows = []
    for i in range(ch.n_chunks):
        a, b = int(ch.chunk_offsets[i]), int(ch.chunk_offsets[i + 1])
        rows.append(mlp.features(int(ch.codecs[i]), ch.comp[a:b].tobytes(),
                                 int(ch.out_offsets[i + 1] - ch.out_offsets[i])))
    return np.array(rows)


def _random_model(seed, n):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, mlp.N_PARAMS).astype(np.float32)
    norm = np.concatenate([rng.normal(0, 1, 16), rng.uniform(0.5, 2, 16), [14.0, 2.0]]).astype(np.float32)
    feat = rng.normal(0, 1.5, (n, 16)).astype(np.float32)
    target = rng.normal(14, 2, n).astype(np.float32)
    return p, norm, feat, target


# Tolerances.  Every quantity is a sum of at most a few thousand FP32
# products of O(1) terms, so the GPU's rounding error relative to the largest
# magnitude involved stays well below 1e-4; the bounds leave a margin.
FEAT_TOL = 1e-5
PRED_TOL = 1e-4          # relative to max |prediction - target mean| + 1
GRAD_TOL = 1e-3          # relative to max |gradient|


@pytest.mark.parametrize("wl", ["batched", "learned"])
def test_features_match_oracle(dev, wl):
    import paper_2307_03760_amd as codag
    ch = (workloads.batched_workload(seed=21, n_chunks=200) if wl == "batched"
          else workloads.learned_workload(seed=21, n_chunks=200))
    _say(f"features {wl}")
    plan = codag.Plan()
    codecs, comp, co, oo = batch_device_inputs(ch, dev)
    got = plan.features(codecs, comp, co, oo).cpu().numpy()
    ref = _oracle_features(ch)
    np.testing.assert_allclose(got, ref, rtol=0, atol=FEAT_TOL)
    if wl == "learned":
        assert ref[:, 8].sum() > 50 and ref[:, 9].max() > 0   # dynamic blocks were parsed


def test_forward_and_gradient_match_oracle(dev):
    import torch
    import paper_2307_03760_amd as codag
    _say("gradient")
    for n in (1, 37, 3001):
        p, norm, feat, target = _random_model(n, n)
        plan = codag.Plan()
        plan.set_params(p, norm)
        q, qn = plan.get_params()
        assert np.array_equal(q, p) and np.array_equal(qn, norm)
        f_d, t_d = torch.from_numpy(feat).to(dev), torch.from_numpy(target).to(dev)
        pred = plan.predict(f_d).cpu().numpy()
        ref_pred = mlp.forward(p, norm, feat)
        scale = np.abs(ref_pred - norm[32]).max() + 1
        assert np.abs(pred - ref_pred).max() <= PRED_TOL * scale
        loss, g = plan.grad(f_d, t_d)
        ref_loss, ref_g = mlp.loss_and_grad(p, norm, feat, target)
        assert loss == pytest.approx(ref_loss, rel=1e-4)
        err = np.abs(g - ref_g).max() / np.abs(ref_g).max()
        assert err <= GRAD_TOL, (n, err)


def test_adam_steps_match_oracle(dev):
    import torch
    import paper_2307_03760_amd as codag
    _say("adam")
    p, norm, feat, target = _random_model(9, 500)
    plan = codag.Plan()
    plan.set_params(p, norm)
    f_d, t_d = torch.from_numpy(feat).to(dev), torch.from_numpy(target).to(dev)
    lr = 1e-3
    losses = plan.train(f_d, t_d, steps=1, lr=lr, seed=0)
    q, _ = plan.get_params()
    ref_loss, g = mlp.loss_and_grad(p, norm, feat, target)
    ref_q, _, _ = mlp.adam_step(p, g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    assert losses[0] == pytest.approx(ref_loss, rel=1e-4)
    # A first Adam step moves every parameter by about lr * sign(g); where |g|
    # is at the level of FP32 noise the sign itself is not determined.
    clear = np.abs(g) > 1e-3 * np.abs(g).max()
    assert np.abs(q - ref_q)[clear].max() <= 1e-3 * lr + 1e-7
    assert np.abs(q - ref_q).max() <= 2 * lr + 1e-7


ADAM_STEPS = 5


def _oracle_trajectory(p, norm, feat, target, lr, steps, b1=0.9, b2=0.999):
    """The oracle's own training: each step's gradient at its own parameters."""
    m, v = np.zeros_like(p, dtype=np.float64), np.zeros_like(p, dtype=np.float64)
    q = p.astype(np.float64)
    losses, grads = [], []
    for t in range(1, steps + 1):
        L, g = mlp.loss_and_grad(q, norm, feat, target)
        losses.append(L)
        grads.append(g)
        q, m, v = mlp.adam_step(q, g, m, v, t, lr, b1=b1, b2=b2)
    return q, np.array(losses), grads


def test_adam_several_steps_match_oracle(dev):
    """Five full-batch Adam steps on the GPU against the oracle stepping on
    its own gradients.  The learning rate is large enough that the gradient
    changes from step to step (so the two moment averages, their decay rates
    and the bias corrections at steps 2-5 all matter: the same trajectory
    with the decay rates swapped ends far outside the tolerance)."""
    import torch
    import paper_2307_03760_amd as codag
    _say("adam several steps")
    p, norm, feat, target = _random_model(19, 400)
    lr = 2e-2
    plan = codag.Plan()
    plan.set_params(p, norm)
    f_d, t_d = torch.from_numpy(feat).to(dev), torch.from_numpy(target).to(dev)
    losses = plan.train(f_d, t_d, steps=ADAM_STEPS, lr=lr, seed=0)
    q, qn = plan.get_params()
    assert np.array_equal(qn, norm)      # seed 0 keeps the normalization
    ref_q, ref_losses, grads = _oracle_trajectory(p, norm, feat, target, lr, ADAM_STEPS)
    np.testing.assert_allclose(losses, ref_losses, rtol=2e-4)
    # The gradient really changes between steps.
    g0, g4 = grads[0], grads[-1]
    assert np.linalg.norm(g4 - g0) > 0.2 * np.linalg.norm(g0)
    # Parameters whose first gradient is clear of FP32 noise follow the
    # oracle to a small fraction of one step; the rest (sign of the first
    # step undetermined) within two steps' worth.
    clear = np.abs(g0) > 1e-3 * np.abs(g0).max()
    err = np.abs(q - ref_q)
    tol = 2e-2 * lr
    assert err[clear].max() <= tol, err[clear].max() / lr
    assert err.max() <= 2 * lr + tol
    # What a swap of the decay rates would give.
    swapped, _, _ = _oracle_trajectory(p, norm, feat, target, lr, ADAM_STEPS, b1=0.999, b2=0.9)
    assert np.abs(swapped - ref_q)[clear].max() > 10 * tol


def test_training_is_deterministic_and_reduces_loss(dev):
    import torch
    import paper_2307_03760_amd as codag
    _say("train")
    rng = np.random.default_rng(3)
    feat = rng.normal(0, 1, (4000, 16)).astype(np.float32)
    w = rng.normal(0, 1, 16)
    target = (14 + feat @ w * 0.5 + 0.3 * np.tanh(feat[:, 0] * feat[:, 1])).astype(np.float32)
    f_d, t_d = torch.from_numpy(feat).to(dev), torch.from_numpy(target).to(dev)
    runs = []
    for _ in range(2):
        plan = codag.Plan()
        losses = plan.train(f_d, t_d, steps=300, lr=3e-3, seed=7)
        runs.append((losses, plan.get_params()[0]))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    losses = runs[0][0]
    assert losses[-1] < 0.05 * losses[0], (losses[0], losses[-1])


def test_model_save_load_round_trip(dev):
    """codag_sched_save writes the documented layout; codag_sched_load into a
    fresh plan gives back the same parameters and the same predictions; a
    damaged, truncated or foreign blob is rejected and leaves the model as it
    was."""
    import struct
    import torch
    import paper_2307_03760_amd as codag
    p, norm, feat, target = _random_model(12, 500)
    a = codag.Plan()
    with pytest.raises(codag.CodagError):
        a.save_model()  # no model yet
    a.set_params(p, norm)
    blob = a.save_model()
    assert len(blob) == codag.SCHED_BLOB_BYTES == 8 + 16 + 4 * (mlp.N_PARAMS + 34) + 8
    assert blob[:8] == b"CODAGMLP" and struct.unpack("<4I", blob[8:24]) == (1, 16, mlp.N_PARAMS, 34)
    assert np.array_equal(np.frombuffer(blob[24:24 + 4 * mlp.N_PARAMS], "<f4"), p)
    assert np.array_equal(np.frombuffer(blob[24 + 4 * mlp.N_PARAMS:-8], "<f4"), norm)
    h = 0xcbf29ce484222325
    for byte in blob[:-8]:
        h = ((h ^ byte) * 0x100000001b3) & (2 ** 64 - 1)
    assert struct.unpack("<Q", blob[-8:])[0] == h
    b = codag.Plan()
    b.load_model(blob)
    pb, nb = b.get_params()
    assert np.array_equal(pb, p) and np.array_equal(nb, norm)
    f_d = torch.from_numpy(feat).to(dev)
    assert torch.equal(a.predict(f_d), b.predict(f_d))
    other = codag.Plan()
    other.set_params(p * 0.5, norm)
    keep = other.get_params()
    damaged = bytearray(blob)
    damaged[100] ^= 1
    nan = bytearray(blob)
    nan[24:28] = struct.pack("<f", float("nan"))
    h = 0xcbf29ce484222325
    for byte in nan[:-8]:
        h = ((h ^ byte) * 0x100000001b3) & (2 ** 64 - 1)
    nan[-8:] = struct.pack("<Q", h)
    for bad in (bytes(damaged), blob[:-1], b"X" + blob[1:], bytes(nan)):
        with pytest.raises(codag.CodagError):
            other.load_model(bad)
        got = other.get_params()
        assert np.array_equal(got[0], keep[0]) and np.array_equal(got[1], keep[1])
    for pl in (a, b, other):
        pl.close()


def _spearman(a, b):
    ra, rb = np.argsort(np.argsort(a)), np.argsort(np.argsort(b))
    return float(np.corrcoef(ra, rb)[0, 1])


def test_learned_order_and_gain(dev):
    """Train on measured decode times of one workload, then use the model on
    a second, full-size one (20,000 Deflate chunks, about 2 GiB out): the
    predictions rank chunks like their measured times, the learned queue is a
    permutation sorted by predicted time, its simulated makespan (measured
    times, as many workers as resident waves) beats the plain index-order
    queue, and the batched launch under it is faster and decodes the same
    bytes."""
    import torch
    import paper_2307_03760_amd as codag
    train_ch = workloads.learned_workload(seed=31, n_chunks=6000)
    test_ch = workloads.learned_workload(seed=32, n_chunks=20000)
    _say("learned: measure")
    plan = codag.Plan()

    def measure(ch):
        codecs, comp, co, oo = batch_device_inputs(ch, dev)
        out = torch.empty(ch.out_bytes, dtype=torch.uint8, device=dev)
        tk = torch.zeros(ch.n_chunks, dtype=torch.int64, device=dev)
        plan.decompress(codecs, comp, co, out, oo, chunk_ticks=tk)
        plan.decompress(codecs, comp, co, out, oo, chunk_ticks=tk)   # warm caches and clocks
        torch.cuda.synchronize()
        return tk.cpu().numpy().astype(np.float64), (codecs, comp, co, oo)

    ticks_tr, dtr = measure(train_ch)
    ticks_te, dte = measure(test_ch)
    feat_tr = plan.features(*dtr)
    target = torch.from_numpy(np.log2(ticks_tr).astype(np.float32)).to(dev)
    _say("learned: train")
    losses = plan.train(feat_tr, target, steps=600, lr=3e-3, seed=1)
    assert losses[-1] < 0.5 * losses[0]
    pred = plan.predict(plan.features(*dte)).cpu().numpy()
    rho = _spearman(pred, ticks_te)
    _say(f"learned: spearman {rho:.3f}")
    assert rho > 0.7
    order = plan.order(*dte).cpu().numpy()
    assert np.array_equal(np.sort(order), np.arange(test_ch.n_chunks))
    # Sorted by predicted time, up to the 4096-bucket quantization.
    _, norm = plan.get_params()
    lo, hi = norm[32] - 4 * norm[33], norm[32] + 4 * norm[33]
    clipped = np.clip(pred[order], lo, hi)
    assert (np.diff(clipped) <= (hi - lo) / 4095 + 1e-4).all()
    # Makespan on as many workers as the persistent grid has waves.
    props = torch.cuda.get_device_properties(dev)
    workers = props.multi_processor_count * plan.opts["waves_per_cu"]
    rng = np.random.default_rng(2)
    spans = {
        "index": mlp.makespan(ticks_te, range(test_ch.n_chunks), workers),
        "random": mlp.makespan(ticks_te, rng.permutation(test_ch.n_chunks), workers),
        "lpt_mlp": mlp.makespan(ticks_te, order, workers),
        "lpt_measured": mlp.makespan(ticks_te, np.argsort(-ticks_te, kind="stable"), workers),
    }
    _say(f"learned: makespans {spans} max chunk {ticks_te.max():.0f} "
         f"mean load {ticks_te.sum() / workers:.0f}")
    assert spans["lpt_measured"] <= spans["index"]
    assert spans["lpt_mlp"] < spans["index"]
    # Measured: the batched launch in index order and in the learned order
    # (features, inference and sort included), each captured in a graph.
    codecs, comp, co, oo = dte
    out = torch.full((test_ch.out_bytes,), 0xA5, dtype=torch.uint8, device=dev)
    st = torch.full((test_ch.n_chunks,), 99, dtype=torch.int32, device=dev)
    ref, ref_st = oracle.decompress(oracle.DEFLATE, test_ch.comp, test_ch.chunk_offsets,
                                    test_ch.out_offsets, threads=16)
    assert (ref_st == 0).all()
    times = {}
    for name, o in (("index", codag.ORDER_INDEX), ("learned", codag.ORDER_LEARNED)):
        plan.set_opts(order=o, use_graph=True)
        ms = []
        for _ in range(3):
            out.fill_(0)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.decompress(codecs, comp, co, out, oo, status=st)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
            st_h = st.cpu().numpy()
            assert (st_h == 0).all()
        times[name] = sorted(ms)[1]
        # Every chunk, byte for byte, under both orders.
        compare_chunks(out.cpu().numpy(), st.cpu().numpy(), ref, ref_st, test_ch.out_offsets)
    _say(f"learned: launch ms {times}")
    assert times["learned"] < times["index"]


def test_untrained_learned_order_falls_back_to_index(dev):
    import torch
    import paper_2307_03760_amd as codag
    ch = workloads.batched_workload(seed=41, n_chunks=50)
    plan = codag.Plan(order=codag.ORDER_LEARNED)
    codecs, comp, co, oo = batch_device_inputs(ch, dev)
    out = torch.empty(ch.out_bytes, dtype=torch.uint8, device=dev)
    st = torch.full((ch.n_chunks,), 99, dtype=torch.int32, device=dev)
    plan.decompress(codecs, comp, co, out, oo, status=st)
    torch.cuda.synchronize()
    ref, ref_st = oracle_mixed(ch.codecs, ch.comp, ch.chunk_offsets, ch.out_offsets)
    compare_chunks(out.cpu().numpy(), st.cpu().numpy(), ref, ref_st, ch.out_offsets)
    with pytest.raises(codag.CodagError):
        plan.get_params()
    with pytest.raises(codag.CodagError):
        plan.order(codecs, comp, co, oo)
