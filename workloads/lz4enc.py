"""A small LZ4 block encoder (input production only).

Greedy matching through a hash of the next four bytes, matches extended
forward.  It writes what the reference compressor rarely does -- offsets
up to the format's 65535, very long matches and literal runs, overlapping
copies -- so tests can reach those paths.  Its blocks keep the format's end
rules (the last five bytes are literals, no match starts in the last
twelve), so every LZ4 decoder accepts them.
"""
from __future__ import annotations


def lz4_greedy(data: bytes, max_off: int = 65535, min_tail: int = 5) -> bytes:
    n, out, table = len(data), bytearray(), {}
    anchor = i = 0
    limit = n - 12

    def length_bytes(v):
        while v >= 255:
            out.append(255)
            v -= 255
        out.append(v)

    while i < limit:
        key = data[i:i + 4]
        j = table.get(key)
        table[key] = i
        if j is None or i - j > max_off:
            i += 1
            continue
        m = 4
        while i + m < n - min_tail and data[j + m] == data[i + m]:
            m += 1
        lit = i - anchor
        out.append((min(lit, 15) << 4) | min(m - 4, 15))
        if lit >= 15:
            length_bytes(lit - 15)
        out += data[anchor:i]
        out += (i - j).to_bytes(2, "little")
        if m - 4 >= 15:
            length_bytes(m - 4 - 15)
        i += m
        anchor = i
    lit = n - anchor
    out.append(min(lit, 15) << 4)
    if lit >= 15:
        length_bytes(lit - 15)
    out += data[anchor:]
    return bytes(out)
