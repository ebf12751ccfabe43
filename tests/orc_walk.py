"""Minimal ORC file walker (test helper).

Extracts the raw DATA stream of an integer column from an uncompressed ORC
file written by pyarrow (Apache ORC's C++ writer), so the oracle's RLE
decoders can be checked against an independent implementation.  Only the
protobuf fields needed to find the stream are read: postscript -> footer ->
stripe information -> stripe footer -> stream list.
"""
from __future__ import annotations


def _varint(buf: bytes, i: int):
    shift = result = 0
    while True:
        b = buf[i]
        i += 1
        result |= (b & 0x7F) << shift
        if b < 0x80:
            return result, i
        shift += 7


def _fields(buf: bytes):
    """Yield (field number, wire type, value) of a protobuf message."""
    i = 0
    while i < len(buf):
        key, i = _varint(buf, i)
        num, wt = key >> 3, key & 7
        if wt == 0:
            v, i = _varint(buf, i)
        elif wt == 1:
            v, i = buf[i:i + 8], i + 8
        elif wt == 2:
            n, i = _varint(buf, i)
            v, i = buf[i:i + n], i + n
        elif wt == 5:
            v, i = buf[i:i + 4], i + 4
        else:
            raise ValueError(f"unsupported wire type {wt}")
        yield num, wt, v


def integer_data_streams(path: str, column: int = 1):
    """Return (encoding kind, [DATA stream bytes per stripe]) for a column.

    Encoding kind is ORC's ColumnEncoding kind: 0 = DIRECT (RLE v1),
    2 = DIRECT_V2 (RLE v2).
    """
    data = open(path, "rb").read()
    ps_len = data[-1]
    ps = data[-1 - ps_len:-1]
    footer_len = compression = None
    for num, _, v in _fields(ps):
        if num == 1:
            footer_len = v
        elif num == 2:
            compression = v
    if compression not in (None, 0):
        raise ValueError("only uncompressed ORC files are supported")
    footer = data[-1 - ps_len - footer_len:-1 - ps_len]
    stripes = []
    for num, _, v in _fields(footer):
        if num == 3:
            info = {n: val for n, _, val in _fields(v)}
            stripes.append(info)
    out, kinds = [], set()
    for st in stripes:
        offset, index_len, data_len, sf_len = st[1], st.get(2, 0), st[3], st[4]
        sf = data[offset + index_len + data_len: offset + index_len + data_len + sf_len]
        streams, encodings = [], []
        for num, _, v in _fields(sf):
            if num == 1:
                streams.append({n: val for n, _, val in _fields(v)})
            elif num == 2:
                encodings.append({n: val for n, _, val in _fields(v)})
        pos = offset
        found = None
        for s in streams:
            kind, col, length = s.get(1, 0), s.get(2, 0), s.get(3, 0)
            if col == column and kind == 0:
                raise ValueError("column has a PRESENT stream (nulls); not supported")
            if col == column and kind == 1:
                found = data[pos:pos + length]
            pos += length
        if found is None:
            raise ValueError("no DATA stream for the column")
        kinds.add(encodings[column].get(1, 0))
        out.append(found)
    if len(kinds) != 1:
        raise ValueError("mixed encodings across stripes")
    return kinds.pop(), out


# ORC RLE v2 width codes (5-bit code -> bits), as the format defines them.
V2_WIDTHS = [c + 1 for c in range(24)] + [26, 28, 30, 32, 40, 48, 56, 64]


def _closest_width(n: int) -> int:
    return next(w for w in V2_WIDTHS if w >= n)


def _varint_end(buf: bytes, i: int) -> int:
    while buf[i] & 0x80:
        i += 1
    return i + 1


def rle_v2_width_codes(stream: bytes):
    """Walk the run headers of an RLE v2 stream (skipping payloads) and
    return the width codes it uses as widths: DIRECT and PATCHED_BASE data
    widths, PATCHED_BASE patch widths, and DELTA widths other than the fixed
    code 0.  Raises if the runs do not end exactly at the end of the stream."""
    codes, i = [], 0
    while i < len(stream):
        h = stream[i]
        kind = h >> 6
        if kind == 0:
            i += 2 + ((h >> 3) & 7)
            continue
        code = (h >> 1) & 31
        n = (((h & 1) << 8) | stream[i + 1]) + 1
        if kind == 1:
            codes.append(code)
            i += 2 + (n * V2_WIDTHS[code] + 7) // 8
        elif kind == 2:
            b2, b3 = stream[i + 2], stream[i + 3]
            pw, pgw, pll = V2_WIDTHS[b2 & 31], (b3 >> 5) + 1, b3 & 31
            codes += [code, b2 & 31]
            i += 4 + (b2 >> 5) + 1 + (n * V2_WIDTHS[code] + 7) // 8 + (pll * _closest_width(pgw + pw) + 7) // 8
        else:
            if code:
                codes.append(code)
            j = _varint_end(stream, _varint_end(stream, i + 2))
            i = j + (max(n - 2, 0) * (V2_WIDTHS[code] if code else 0) + 7) // 8
    if i != len(stream):
        raise ValueError("runs do not end at the end of the stream")
    return codes


def _lz4_block(chunk: bytes, cap: int) -> bytes:
    """An LZ4 block through the oracle's decoder in capacity mode (its LZ4
    decoder is pinned against pyarrow's on its own)."""
    import numpy as np

    import oracle
    comp = np.frombuffer(bytes(chunk) + b"\0", dtype=np.uint8)
    out, st, made = oracle.decompress_ex(oracle.LZ4, comp, np.array([0, len(chunk)], np.uint64),
                                         np.array([0, cap], np.uint64), capacity=True)
    if st[0] != oracle.OK:
        raise ValueError("bad LZ4 metadata chunk")
    return bytes(out[: int(made[0])])


def _unframe_meta(buf: bytes, compression: int, block: int) -> bytes:
    """Metadata sections (footer, stripe footers) of a compressed file: the
    compression chunks inflated with Python's zlib (ZLIB) or expanded as LZ4
    blocks (LZ4).  Test plumbing only (the data streams go through the
    oracle and the GPU path)."""
    if compression == 0:
        return buf
    import zlib
    out, pos = bytearray(), 0
    while pos < len(buf):
        h = buf[pos] | buf[pos + 1] << 8 | buf[pos + 2] << 16
        pos += 3
        n = h >> 1
        chunk = buf[pos:pos + n]
        pos += n
        if h & 1:
            out += chunk
        elif compression == ZLIB:
            out += zlib.decompress(chunk, -15)
        else:
            out += _lz4_block(chunk, block)
    return bytes(out)


# ORC compression kinds handled here (CompressionKind).
NONE, ZLIB, LZ4 = 0, 1, 4


# ORC stream kinds (Stream.Kind) and column encodings (ColumnEncoding.Kind).
PRESENT, DATA, LENGTH = 0, 1, 2
DIRECT, DIRECT_V2 = 0, 2


def file_streams(path: str):
    """The raw (still framed, if compressed) streams of every stripe:
    {"compression": 0 none / 1 zlib / 4 lz4, "block_size": int, "stripes": [
    {"rows": n, "streams": {(column, kind): bytes}, "encodings": [kind per column]}]}."""
    data = open(path, "rb").read()
    ps_len = data[-1]
    ps = dict((num, v) for num, _, v in _fields(data[-1 - ps_len:-1]))
    footer_len, compression, block = ps[1], ps.get(2, 0), ps.get(3, 256 * 1024)
    if compression not in (NONE, ZLIB, LZ4):
        raise ValueError("only uncompressed, ZLIB and LZ4 files")
    footer = _unframe_meta(data[-1 - ps_len - footer_len:-1 - ps_len], compression, block)
    stripes = []
    for num, _, v in _fields(footer):
        if num != 3:
            continue
        info = {n: val for n, _, val in _fields(v)}
        offset, index_len, data_len, sf_len, rows = info[1], info.get(2, 0), info[3], info[4], info.get(5, 0)
        sf = _unframe_meta(data[offset + index_len + data_len:offset + index_len + data_len + sf_len],
                           compression, block)
        streams, encodings, pos = {}, [], offset
        for n2, _, v2 in _fields(sf):
            if n2 == 1:
                s = {n: val for n, _, val in _fields(v2)}
                kind, col, length = s.get(1, 0), s.get(2, 0), s.get(3, 0)
                if pos >= offset + index_len:
                    streams[(col, kind)] = data[pos:pos + length]
                pos += length
            elif n2 == 2:
                encodings.append({n: val for n, _, val in _fields(v2)}.get(1, 0))
        stripes.append({"rows": rows, "streams": streams, "encodings": encodings})
    return {"compression": compression, "block_size": block, "stripes": stripes}
