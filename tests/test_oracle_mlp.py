"""Pins for the cost-model oracle (oracle/mlp.py) against facts that do not
come from the oracle itself: central finite differences, closed forms of
special networks, hand-computed forwards, the closed form of Adam's first
steps, hand-built Deflate headers and brute-force schedules."""
from __future__ import annotations

import itertools
import math

import numpy as np
import pytest

from deflate_bits import BitWriter
from oracle import mlp

F, H = mlp.N_FEATURES, mlp.N_HIDDEN


def _random_model(seed, n=9):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.4, mlp.N_PARAMS)
    norm = np.concatenate([rng.normal(0, 1, F), rng.uniform(0.5, 2, F), [12.0, 3.0]])
    feat = rng.normal(0, 1.5, (n, F))
    target = rng.normal(12, 3, n)
    return p, norm, feat, target


def test_layout_sizes():
    assert mlp.N_PARAMS == 5313 and mlp.N_NORM == 34
    assert (mlp.OFF_B1, mlp.OFF_W2, mlp.OFF_B2, mlp.OFF_W3, mlp.OFF_B3) == (1024, 1088, 5184, 5248, 5312)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gradient_matches_central_differences(seed):
    p, norm, feat, target = _random_model(seed)
    _, g = mlp.loss_and_grad(p, norm, feat, target)
    rng = np.random.default_rng(seed + 100)
    # A few indices from every parameter block.
    blocks = [(mlp.OFF_W1, mlp.OFF_B1), (mlp.OFF_B1, mlp.OFF_W2), (mlp.OFF_W2, mlp.OFF_B2),
              (mlp.OFF_B2, mlp.OFF_W3), (mlp.OFF_W3, mlp.OFF_B3), (mlp.OFF_B3, mlp.N_PARAMS)]
    idx = [int(k) for lo, hi in blocks for k in rng.integers(lo, hi, size=min(12, hi - lo))]
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (mlp.loss(pp, norm, feat, target) - mlp.loss(pm, norm, feat, target)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_zero_first_layer_closed_form():
    """W1 = 0, b1 = 0: h1 = 0, h2 = relu(b2), y = w3.relu(b2) + b3 for every
    sample, so only b2 (where positive), w3 and b3 get gradient."""
    rng = np.random.default_rng(5)
    W1, b1 = np.zeros((H, F)), np.zeros(H)
    W2 = rng.normal(0, 1, (H, H))
    b2 = rng.normal(0, 1, H)
    w3 = rng.normal(0, 1, H)
    b3 = 0.25
    p = mlp.pack(W1, b1, W2, b2, w3, b3)
    norm = np.concatenate([np.zeros(F), np.ones(F), [0.0, 1.0]])
    feat = rng.normal(0, 1, (6, F))
    target = rng.normal(0, 1, 6)
    L, g = mlp.loss_and_grad(p, norm, feat, target)
    hpos = np.maximum(b2, 0)
    y = float(w3 @ hpos + b3)
    r = 2 * np.mean(y - target)                      # dL/dy summed over samples
    assert L == pytest.approx(np.mean((y - target) ** 2), rel=1e-12)
    W1g, b1g, W2g, b2g, w3g, b3g = mlp.unpack(g)
    assert np.all(W1g == 0) and np.all(b1g == 0) and np.all(W2g == 0)
    np.testing.assert_allclose(b2g, r * w3 * (b2 > 0), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(w3g, r * hpos, rtol=1e-12, atol=1e-15)
    assert b3g == pytest.approx(r, rel=1e-12)


def test_forward_hand_computed():
    W1, b1, W2, b2, w3 = np.zeros((H, F)), np.zeros(H), np.zeros((H, H)), np.zeros(H), np.zeros(H)
    W1[0, 0], W2[0, 0], w3[0], b3 = 1.0, 2.0, 3.0, 0.5
    p = mlp.pack(W1, b1, W2, b2, w3, b3)
    norm = np.concatenate([np.zeros(F), np.ones(F), [10.0, 2.0]])
    feat = np.zeros((3, F))
    feat[:, 0] = [1.5, -1.0, 0.0]
    # x0 = 1.5: z1 = 1.5, z2 = 3, y = 9.5;  x0 <= 0: y = 0.5.  pred = 2y + 10.
    np.testing.assert_allclose(mlp.forward(p, norm, feat), [29.0, 11.0, 11.0], rtol=0, atol=1e-12)
    # Normalization: x' = (x - mu) * s.
    norm2 = norm.copy()
    norm2[0], norm2[F] = 0.5, 3.0       # x' = (1.5 - 0.5) * 3 = 3 -> y = 18.5
    assert mlp.forward(p, norm2, feat[:1])[0] == pytest.approx(2 * 18.5 + 10, abs=1e-12)


def test_adam_first_steps_closed_form():
    """With bias correction, a constant gradient g gives m_hat = g and
    v_hat = g^2 at every step, so each step moves by lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p, m, v = np.ones(4), np.zeros(4), np.zeros(4)
    lr, eps = 0.01, 1e-8
    for t in (1, 2, 3):
        q, m, v = mlp.adam_step(p, g, m, v, t, lr, eps=eps)
        np.testing.assert_allclose(q, p - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-12)
        p = q


def test_adam_varying_gradient_weighted_averages():
    """Unrolling Adam's moment recursions (Kingma and Ba, Section 3) gives
    m_t = (1 - b1) * sum_i b1^(t-i) g_i, whose weights sum to 1 - b1^t, so
    the bias-corrected m_hat_t is the weighted average of g_1..g_t with
    weights b1^(t-i); v_hat_t likewise averages g_i^2 with weights b2^(t-i).
    With b1 = 1/2 and b2 = 3/4 and gradients that change every step, the
    parameters after each step are checked against those averages; swapping
    the two decay rates moves them far away."""
    b1, b2, lr, eps = 0.5, 0.75, 0.1, 1e-8
    gs = [np.array([1.0, -2.0, 0.5]), np.array([-1.0, 1.0, 0.5]),
          np.array([3.0, 0.0, -0.25]), np.array([0.5, 4.0, 1.0])]
    p0 = np.array([0.3, -0.7, 2.0])

    def by_averages(dec1, dec2):
        p = p0.copy()
        out = []
        for t in range(1, len(gs) + 1):
            w1 = np.array([dec1 ** (t - i) for i in range(1, t + 1)])
            w2 = np.array([dec2 ** (t - i) for i in range(1, t + 1)])
            G = np.array(gs[:t])
            m_hat = (w1[:, None] * G).sum(0) / w1.sum()
            v_hat = (w2[:, None] * G * G).sum(0) / w2.sum()
            p = p - lr * m_hat / (np.sqrt(v_hat) + eps)
            out.append(p)
        return out

    expect = by_averages(b1, b2)
    # Step 2 by hand for the first parameter: m_hat = (0.5 * 1 - 1) / 1.5 = -1/3,
    # v_hat = (0.75 * 1 + 1) / 1.75 = 1, so it moves up by lr / 3.
    assert expect[1][0] == pytest.approx(expect[0][0] + lr / 3, abs=1e-9)
    p, m, v = p0.copy(), np.zeros(3), np.zeros(3)
    for t, g in enumerate(gs, start=1):
        p, m, v = mlp.adam_step(p, g, m, v, t, lr, b1=b1, b2=b2, eps=eps)
        np.testing.assert_allclose(p, expect[t - 1], rtol=0, atol=1e-12)
    swapped = by_averages(b2, b1)
    assert np.abs(swapped[-1] - expect[-1]).max() > 1e-2


def test_adam_without_momentum_is_rms_scaled():
    """b1 = 0 leaves m_hat_t = g_t: each step is lr * g_t / (sqrt(v_hat_t) + eps)
    with v_hat_t the b2-weighted average of the squared gradients."""
    b2, lr = 0.6, 0.05
    gs = [np.array([2.0, -1.0]), np.array([-1.0, 3.0]), np.array([0.5, 0.5])]
    p, m, v = np.zeros(2), np.zeros(2), np.zeros(2)
    sq = []
    for t, g in enumerate(gs, start=1):
        q, m, v = mlp.adam_step(p, g, m, v, t, lr, b1=0.0, b2=b2, eps=0.0)
        sq.append(g * g)
        w = np.array([b2 ** (t - i) for i in range(1, t + 1)])
        v_hat = (w[:, None] * np.array(sq)).sum(0) / w.sum()
        np.testing.assert_allclose(q - p, -lr * g / np.sqrt(v_hat), rtol=1e-12, atol=0)
        p = q


def _dynamic_stream(lit_lengths, dist_lengths, hclen=19):
    """A dynamic-block header written by hand: a complete code-length code
    (13 symbols of 4 bits, 6 of 5 bits), then every length sent literally."""
    order = (16, 17, 18, 0, 8, 7, 9, 6, 10, 5, 11, 4, 12, 3, 13, 2, 14, 1, 15)
    cl = [0] * 19
    sent = order[:hclen]
    for k, sym in enumerate(sent):
        cl[sym] = 4 if k < 13 else 5
    # Canonical codes for the code-length alphabet (RFC 1951, 3.2.2).
    codes, code = {}, 0
    for L in (4, 5):
        for sym in range(19):
            if cl[sym] == L:
                codes[sym] = (code, L)
                code += 1
        code <<= 1
    w = BitWriter()
    w.put(1, 1)
    w.put(2, 2)
    w.put(len(lit_lengths) - 257, 5)
    w.put(len(dist_lengths) - 1, 5)
    w.put(hclen - 4, 4)
    for sym in sent:
        w.put(cl[sym], 3)
    for L in list(lit_lengths) + list(dist_lengths):
        c, n = codes[L]
        w.put_code(c, n)
    return w.getvalue() + b"\0" * 8


def test_features_dynamic_header_pins():
    lit = [8] * 255 + [9, 9]                 # complete: 255/256 + 2/512
    comp = _dynamic_stream(lit, [1, 1])
    f = mlp.features(mlp.DEFLATE, comp, 1000)
    assert f[0] == pytest.approx(math.log2(1 + len(comp)))
    assert f[1] == pytest.approx(math.log2(1001))
    assert list(f[3:9]) == [0, 0, 1, 0, 0, 1]
    assert f[9] == pytest.approx(257 / 286) and f[10] == pytest.approx(2 / 30)
    assert f[11] == pytest.approx(19 / 19)
    np.testing.assert_allclose(f[12:16], [0, 255 / 257, 2 / 257, 0])
    # Lengths in every bin, with zeros (unused symbols) left out of the shares.
    lit = [0] * 10 + [3] * 4 + [7] * 20 + [10] * 30 + [12] * 40 + [0] * 160
    comp = _dynamic_stream(lit, [2] * 30)
    f = mlp.features(mlp.DEFLATE, comp, 5)
    assert f[9] == pytest.approx(264 / 286) and f[10] == pytest.approx(1.0)
    np.testing.assert_allclose(f[12:16], np.array([4, 20, 30, 40]) / 94)


def test_features_incomplete_code_length_code_reads_as_absent():
    comp = bytearray(_dynamic_stream([8] * 256 + [8], [1]))
    w = BitWriter()
    w.put(1, 1); w.put(2, 2); w.put(0, 5); w.put(0, 5); w.put(0, 4)
    for _ in range(4):
        w.put(1, 3)                           # four codes of length 1: Kraft sum 2
    f = mlp.features(mlp.DEFLATE, w.getvalue() + b"\0" * 4, 10)
    assert f[8] == 1 and np.all(f[9:] == 0)
    # Cut inside the lengths: also absent.
    f = mlp.features(mlp.DEFLATE, bytes(comp[:20]), 10)
    assert f[8] == 1 and np.all(f[9:] == 0)


def test_features_other_blocks_and_codecs():
    w = BitWriter(); w.put(1, 1); w.put(0, 2); w.align(); w.put(3, 16); w.put(0xFFFC, 16)
    f = mlp.features(mlp.DEFLATE, w.getvalue() + b"abc", 3)
    assert list(f[5:12]) == [1, 1, 0, 0, 0, 0, 0]
    w = BitWriter(); w.put(1, 1); w.put(1, 2)
    f = mlp.features(mlp.DEFLATE, w.getvalue(), 0)
    assert list(f[6:9]) == [0, 1, 0] and f[1] == 0
    w = BitWriter(); w.put(1, 1); w.put(3, 2)
    assert np.all(mlp.features(mlp.DEFLATE, w.getvalue(), 8)[6:] == 0)
    assert np.all(mlp.features(mlp.DEFLATE, b"", 8)[6:] == 0)
    f = mlp.features(mlp.RLE_V2, b"\x00" * 31, 64)
    assert f[0] == 5 and f[1] == pytest.approx(math.log2(65)) and list(f[3:]) == [0, 1, 0] + [0] * 10


def _opt_makespan(d, m):
    best = math.inf
    for assign in itertools.product(range(m), repeat=len(d)):
        loads = [0] * m
        for c, w in enumerate(assign):
            loads[w] += d[c]
        best = min(best, max(loads))
    return best


def test_makespan_hand_and_lpt_bound():
    d = [3, 3, 2, 2, 2]
    assert mlp.makespan(d, range(5), 2) == 7      # 3|3, 2->5, 2->5, 2->7
    assert mlp.makespan(d, [2, 3, 4, 0, 1], 2) == 7
    assert mlp.makespan(d, range(5), 5) == 3
    rng = np.random.default_rng(7)
    for _ in range(30):
        n, m = int(rng.integers(2, 8)), int(rng.integers(2, 4))
        d = [int(x) for x in rng.integers(1, 20, n)]
        opt = _opt_makespan(d, m)
        lpt = mlp.makespan(d, sorted(range(n), key=lambda c: -d[c]), m)
        assert opt <= lpt <= (4 / 3 - 1 / (3 * m)) * opt + 1e-9   # Graham's LPT bound
        assert opt <= mlp.makespan(d, range(n), m) <= (2 - 1 / m) * opt + 1e-9
