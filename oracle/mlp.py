"""Oracle for the learned scheduler: TEST INFRASTRUCTURE ONLY.

Plain float64 NumPy versions of what the cost model computes, written out
step by step so they can be checked by eye:

* ``features`` -- the 16 header-only features of one chunk.  The Deflate
  fields (BTYPE, HLIT, HDIST, HCLEN, the code-length code and the run-length
  coded code lengths) follow RFC 1951, section 3.2.3 and section 3.2.7.
* ``forward`` / ``loss_and_grad`` -- the 16-64-64-1 ReLU network with mean
  squared error on the normalized target, and its gradient by the chain rule
  (the derivative of ReLU is taken as 0 at 0).
* ``adam_step`` -- one Adam update (Kingma and Ba, "Adam: A Method for
  Stochastic Optimization", ICLR 2015, Algorithm 1) with bias correction.
* ``makespan`` -- greedy list scheduling of a queue onto identical workers
  (Graham 1969): each chunk goes, in queue order, to the worker that becomes
  free first.

Parameter layout (packed float vector of 5313): W1[64][16], b1[64],
W2[64][64], b2[64], w3[64], b3 (row-major, W[out][in]).  Normalization
vector of 34: feature means mu[16], feature scales s[16] (x' = (x - mu) * s),
target mean my, target scale sy (prediction = y * sy + my).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may use this module.
"""
from __future__ import annotations

import heapq
import math

import numpy as np

N_FEATURES, N_HIDDEN = 16, 64
OFF_W1 = 0
OFF_B1 = OFF_W1 + N_HIDDEN * N_FEATURES
OFF_W2 = OFF_B1 + N_HIDDEN
OFF_B2 = OFF_W2 + N_HIDDEN * N_HIDDEN
OFF_W3 = OFF_B2 + N_HIDDEN
OFF_B3 = OFF_W3 + N_HIDDEN
N_PARAMS = OFF_B3 + 1
N_NORM = 2 * N_FEATURES + 2

RLE_V1, RLE_V2, DEFLATE = 1, 2, 3


# ---------------------------------------------------------------------------
# Features
# ---------------------------------------------------------------------------

class _Bits:
    """LSB-first bit reader over a byte string (RFC 1951, section 3.1.1)."""

    def __init__(self, data: bytes):
        self.data = data
        self.pos = 0  # in bits

    def get(self, n: int) -> int:
        v = 0
        for k in range(n):
            byte = self.pos >> 3
            if byte >= len(self.data):
                raise EOFError
            v |= ((self.data[byte] >> (self.pos & 7)) & 1) << k
            self.pos += 1
        return v


def _canonical_decoder(lengths):
    """{(length, code): symbol} for a canonical Huffman code (RFC 1951, 3.2.2)."""
    max_len = max(lengths) if lengths else 0
    bl_count = [0] * (max_len + 1)
    for L in lengths:
        if L:
            bl_count[L] += 1
    code, next_code = 0, [0] * (max_len + 1)
    for bits in range(1, max_len + 1):
        code = (code + bl_count[bits - 1]) << 1
        next_code[bits] = code
    table = {}
    for sym, L in enumerate(lengths):
        if L:
            table[(L, next_code[L])] = sym
            next_code[L] += 1
    return table, max_len


def _read_symbol(bits: _Bits, table, max_len):
    """Huffman codes are packed starting with the most significant code bit."""
    code = 0
    for L in range(1, max_len + 1):
        code = (code << 1) | bits.get(1)
        if (L, code) in table:
            return table[(L, code)]
    raise ValueError("invalid code")


_CL_ORDER = (16, 17, 18, 0, 8, 7, 9, 6, 10, 5, 11, 4, 12, 3, 13, 2, 14, 1, 15)


def _dynamic_lengths(bits: _Bits):
    """HLIT, HDIST, HCLEN and the literal/length + distance code lengths of a
    dynamic block header, or None if the header is not a valid one.

    A code-length code is accepted only if it is complete (Kraft sum 1); a
    repeat of the previous length with no previous length, or a repeat that
    runs past HLIT + HDIST lengths, is invalid.
    """
    hlit = bits.get(5) + 257
    hdist = bits.get(5) + 1
    hclen = bits.get(4) + 4
    cl = [0] * 19
    for k in range(hclen):
        cl[_CL_ORDER[k]] = bits.get(3)
    if sum(2.0 ** -L for L in cl if L) != 1.0:
        return None
    table, max_len = _canonical_decoder(cl)
    lengths = []
    while len(lengths) < hlit + hdist:
        sym = _read_symbol(bits, table, max_len)
        if sym < 16:
            lengths.append(sym)
            continue
        if sym == 16:
            if not lengths:
                return None
            value, count = lengths[-1], 3 + bits.get(2)
        elif sym == 17:
            value, count = 0, 3 + bits.get(3)
        else:
            value, count = 0, 11 + bits.get(7)
        if len(lengths) + count > hlit + hdist:
            return None
        lengths.extend([value] * count)
    return hlit, hdist, hclen, lengths[:hlit]


def features(codec: int, comp: bytes, out_len: int) -> np.ndarray:
    """The 16 features of one chunk, read from its sizes and (Deflate) the
    header of its first block; zero where a field is absent or unreadable."""
    f = np.zeros(N_FEATURES)
    f[0] = math.log2(1 + len(comp))
    f[1] = math.log2(1 + out_len)
    f[2] = f[1] - f[0]
    if codec in (RLE_V1, RLE_V2, DEFLATE):
        f[2 + codec] = 1.0
    if codec != DEFLATE or not comp:
        return f
    bits = _Bits(comp)
    try:
        bits.get(1)  # BFINAL
        btype = bits.get(2)
    except EOFError:
        return f
    if btype == 3:
        return f
    f[6 + btype] = 1.0
    if btype != 2:
        return f
    try:
        parsed = _dynamic_lengths(bits)
    except (EOFError, ValueError):
        parsed = None
    if parsed is None:
        return f
    hlit, hdist, hclen, lit = parsed
    f[9], f[10], f[11] = hlit / 286, hdist / 30, hclen / 19
    used = [L for L in lit if L]
    if used:
        for L in used:
            f[12 + (0 if L <= 6 else 1 if L <= 8 else 2 if L <= 10 else 3)] += 1
        f[12:16] /= len(used)
    return f


# ---------------------------------------------------------------------------
# Network
# ---------------------------------------------------------------------------

def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    W1 = p[OFF_W1:OFF_B1].reshape(N_HIDDEN, N_FEATURES)
    b1 = p[OFF_B1:OFF_W2]
    W2 = p[OFF_W2:OFF_B2].reshape(N_HIDDEN, N_HIDDEN)
    b2 = p[OFF_B2:OFF_W3]
    w3 = p[OFF_W3:OFF_B3]
    b3 = p[OFF_B3]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]]).astype(np.float64)


def _inputs(norm, feat):
    norm = np.asarray(norm, dtype=np.float64)
    mu, s = norm[:N_FEATURES], norm[N_FEATURES:2 * N_FEATURES]
    return (np.asarray(feat, dtype=np.float64) - mu) * s


def _layers(p, norm, feat):
    W1, b1, W2, b2, w3, b3 = unpack(p)
    x = _inputs(norm, feat)      # n x 16
    z1 = x @ W1.T + b1           # n x 64
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2          # n x 64
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3             # n
    return x, z1, h1, z2, h2, y


def forward(p, norm, feat) -> np.ndarray:
    """Predicted log2 decode cycles for each row of feat."""
    norm = np.asarray(norm, dtype=np.float64)
    y = _layers(p, norm, feat)[-1]
    return y * norm[2 * N_FEATURES + 1] + norm[2 * N_FEATURES]


def loss(p, norm, feat, target) -> float:
    norm = np.asarray(norm, dtype=np.float64)
    y = _layers(p, norm, feat)[-1]
    t = (np.asarray(target, dtype=np.float64) - norm[2 * N_FEATURES]) / norm[2 * N_FEATURES + 1]
    return float(np.mean((y - t) ** 2))


def loss_and_grad(p, norm, feat, target):
    """Mean squared error on the normalized target and its gradient with
    respect to the packed parameters."""
    norm = np.asarray(norm, dtype=np.float64)
    W1, b1, W2, b2, w3, b3 = unpack(p)
    x, z1, h1, z2, h2, y = _layers(p, norm, feat)
    t = (np.asarray(target, dtype=np.float64) - norm[2 * N_FEATURES]) / norm[2 * N_FEATURES + 1]
    n = len(y)
    L = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / n                  # dL/dy
    g_w3 = h2.T @ dy
    g_b3 = dy.sum()
    dz2 = np.outer(dy, w3) * (z2 > 0)      # dL/dz2
    g_W2 = dz2.T @ h1
    g_b2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)             # dL/dz1
    g_W1 = dz1.T @ x
    g_b1 = dz1.sum(axis=0)
    return L, pack(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3)


def adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """Parameters and moments after Adam step t (t counts from 1)."""
    m = b1 * np.asarray(m, dtype=np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1 - b2) * g * g
    m_hat = m / (1 - b1 ** t)
    v_hat = v / (1 - b2 ** t)
    return np.asarray(p, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


# ---------------------------------------------------------------------------
# Scheduling
# ---------------------------------------------------------------------------

def makespan(durations, order, workers: int) -> float:
    """Finish time of the last chunk when `workers` identical workers take
    chunks in queue order, each as soon as it is free."""
    free = [0.0] * workers
    heapq.heapify(free)
    end = 0.0
    for c in order:
        t = heapq.heappop(free) + float(durations[c])
        end = max(end, t)
        heapq.heappush(free, t)
    return end
