"""Tiny raw-deflate bit writer for crafting test streams (test helper).

Writes fixed-Huffman and stored blocks by hand so tests can build streams
that zlib's compressor would never emit (edge lengths, distances, corrupt
codes), then compare the oracle with zlib's decompressor on them.
"""
from __future__ import annotations


class BitWriter:
    def __init__(self):
        self.bits = []

    def put(self, value: int, n: int):
        """n bits of value, least significant first (header fields, extra bits)."""
        for i in range(n):
            self.bits.append((value >> i) & 1)

    def put_code(self, code: int, n: int):
        """A Huffman code, most significant bit first."""
        for i in range(n - 1, -1, -1):
            self.bits.append((code >> i) & 1)

    def align(self):
        while len(self.bits) % 8:
            self.bits.append(0)

    def getvalue(self) -> bytes:
        bits = self.bits + [0] * (-len(self.bits) % 8)
        out = bytearray()
        for i in range(0, len(bits), 8):
            out.append(sum(b << k for k, b in enumerate(bits[i:i + 8])))
        return bytes(out)


def fixed_litlen(w: BitWriter, sym: int):
    if sym < 144:
        w.put_code(0x30 + sym, 8)
    elif sym < 256:
        w.put_code(0x190 + sym - 144, 9)
    elif sym < 280:
        w.put_code(sym - 256, 7)
    else:
        w.put_code(0xC0 + sym - 280, 8)


LEN_BASE = [3, 4, 5, 6, 7, 8, 9, 10, 11, 13, 15, 17, 19, 23, 27, 31, 35, 43, 51, 59, 67, 83, 99,
            115, 131, 163, 195, 227, 258]
LEN_EXTRA = [0] * 8 + [1] * 4 + [2] * 4 + [3] * 4 + [4] * 4 + [5] * 4 + [0]
DIST_BASE = [1, 2, 3, 4, 5, 7, 9, 13, 17, 25, 33, 49, 65, 97, 129, 193, 257, 385, 513, 769, 1025,
             1537, 2049, 3073, 4097, 6145, 8193, 12289, 16385, 24577]
DIST_EXTRA = [0, 0, 0, 0, 1, 1, 2, 2, 3, 3, 4, 4, 5, 5, 6, 6, 7, 7, 8, 8, 9, 9, 10, 10, 11, 11,
              12, 12, 13, 13]


def fixed_copy(w: BitWriter, length: int, dist: int):
    """A (length, distance) pair in a fixed block, from RFC 1951's printed tables."""
    li = max(i for i in range(29) if LEN_BASE[i] <= length and (i < 28 or length == 258))
    if length == 258:
        li = 28
    fixed_litlen(w, 257 + li)
    w.put(length - LEN_BASE[li], LEN_EXTRA[li])
    di = max(i for i in range(30) if DIST_BASE[i] <= dist)
    w.put_code(di, 5)
    w.put(dist - DIST_BASE[di], DIST_EXTRA[di])
