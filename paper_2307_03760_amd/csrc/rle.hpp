// ORC integer RLE v1 and v2 decoding by one wavefront (CODAG Section IV-A,
// IV-D: every lane runs the serial decode; Section IV-F: "write_run" has
// each lane compute its own element of a run).
//
// The serial part (headers, varints, widths) is wave-uniform scalar code fed
// by the LDS ring; the wide parts are lane-parallel: literal lists are split
// with ballots over terminator bytes, bit-packed values are unpacked one per
// lane, DELTA runs use a wave prefix sum, and every store writes 64
// consecutive int64 values with one instruction.
#pragma once

#include "../../include/codag.h"
#include "stream.hpp"

namespace codag {

// Seven-bit groups of up to eight varint bytes (little-endian, already
// masked to the varint's bytes) packed into one integer.
__device__ __forceinline__ uint64_t pack7(uint64_t x) {
    x &= 0x7f7f7f7f7f7f7f7full;
    x = (x & 0x007f007f007f007full) | ((x & 0x7f007f007f007f00ull) >> 1);
    x = (x & 0x00003fff00003fffull) | ((x & 0x3fff00003fff0000ull) >> 2);
    x = (x & 0x000000000fffffffull) | ((x & 0x0fffffff00000000ull) >> 4);
    return x;
}

__device__ __forceinline__ uint64_t low_bytes(uint64_t x, uint32_t nb) {
    return nb >= 8 ? x : x & ((1ull << (8 * nb)) - 1);
}

// Unsigned base-128 varint at byte position pos (wave-uniform).  Bytes past
// the end of the chunk read as zero, i.e. as terminators, so a varint cut off
// by the end is seen ending past `end` and reported TRUNCATED.
__device__ __forceinline__ int read_varint(InRing &in, uint32_t &pos, uint32_t end, uint64_t &z) {
    in.ensure(pos + 24);
    uint64_t x = in.peek8(pos);
    uint64_t t = ~x & 0x8080808080808080ull;
    uint32_t nb;
    uint64_t v;
    if (t) {
        nb = (uint32_t)(__builtin_ctzll(t) >> 3) + 1;
        v = pack7(low_bytes(x, nb));
    } else {
        uint64_t y = in.peek8(pos + 8);
        uint32_t b8 = (uint32_t)(y & 0xff), b9 = (uint32_t)((y >> 8) & 0xff);
        if (b8 & 0x80) {
            if (b9 > 1) {
                return CODAG_E_CORRUPT;  // bits above bit 63, or an 11th byte
            }
            nb = 10;
        } else {
            nb = 9;
        }
        v = pack7(x) | ((uint64_t)(b8 & 0x7f) << 56) | (nb == 10 ? (uint64_t)b9 << 63 : 0);
    }
    if (pos + nb > end) return CODAG_E_TRUNCATED;
    pos += nb;
    z = v;
    return CODAG_OK;
}

// A literal list of `count` zigzag varints starting at pos, lane-parallel.
// Each pass looks at a 256-byte window (4 bytes per lane): terminator bytes
// (bit 7 clear) are counted per lane, an exclusive scan built from three
// ballots numbers them, their positions go to LDS, and then lane k decodes
// varint k from the bytes between terminators k-1 and k.
__device__ __forceinline__ int rle_literal_list(InRing &in, uint32_t &pos, uint32_t end,
                                                uint32_t count, uint64_t *out, uint32_t *ends) {
    uint32_t done = 0;
    while (done < count) {
        uint32_t p0 = pos & ~3u;
        in.ensure(p0 + 272);
        uint32_t w = in.word((p0 >> 2) + lane());
        uint32_t at = p0 + 4 * lane();
        uint32_t tm = 0;
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (!((w >> (8 * k + 7)) & 1) && at + k >= pos) tm |= 1u << k;
        uint32_t cnt = __builtin_popcount(tm);
        uint64_t b0 = ballot(cnt & 1), b1 = ballot(cnt & 2), b2 = ballot(cnt & 4);
        uint32_t idx = count_below(b0) + 2 * count_below(b1) + 4 * count_below(b2);
        uint32_t total = (uint32_t)(__builtin_popcountll(b0) + 2 * __builtin_popcountll(b1) +
                                    4 * __builtin_popcountll(b2));
        if (total == 0) return CODAG_E_CORRUPT;  // >= 253 continuation bytes
        uint32_t use = min(total, count - done);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            if ((tm >> k) & 1) {
                if (idx < use) ends[idx] = at + k;
                idx++;
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int it = 0; it < 2; it++) {
            uint32_t k = lane() + 64 * it;
            int st = CODAG_OK;
            if (k < use) {
                uint32_t s = k ? ends[k - 1] + 1 : pos;
                uint32_t e = ends[k];
                uint32_t nb = e - s + 1;
                uint64_t lo, hi;
                ring_read16(in, s, lo, hi);
                uint32_t b9 = (uint32_t)((hi >> 8) & 0xff);
                if (nb > 10)
                    st = CODAG_E_CORRUPT;
                else if (e >= end)
                    st = CODAG_E_TRUNCATED;
                else if (nb == 10 && b9 > 1)
                    st = CODAG_E_CORRUPT;
                uint64_t z = pack7(low_bytes(lo, nb));
                if (nb > 8) z |= (hi & 0x7f) << 56;
                if (nb > 9) z |= (uint64_t)(b9 & 1) << 63;
                if (st == CODAG_OK) out[done + k] = unzigzag(z);
            }
            uint64_t bad = ballot(st != CODAG_OK);
            if (bad) return (int)uni((uint32_t)readlane((uint32_t)st, (uint32_t)__builtin_ctzll(bad)));
        }
        pos = uni(ends[use - 1]) + 1;
        done += use;
    }
    return CODAG_OK;
}

// ---- RLE v1 ------------------------------------------------------------

// Runs: header 0..127 = length - 3, a signed delta byte, a zigzag varint base.
// Literal lists: header -1..-128 = -count, then count zigzag varints.
__device__ __forceinline__ int decode_rle_v1(InRing &in, uint64_t *out, uint32_t cap, uint32_t *ends) {
    uint32_t pos = in.skip, end = in.gend;
    uint32_t n = 0;
    while (n < cap) {
        if (pos >= end) return CODAG_E_TRUNCATED;
        in.ensure(pos + 16);
        uint64_t x = in.peek8(pos);
        int32_t h = (int8_t)(x & 0xff);
        if (h >= 0) {
            uint32_t len = (uint32_t)h + 3;
            if (pos + 2 > end) return CODAG_E_TRUNCATED;
            int32_t delta = (int8_t)((x >> 8) & 0xff);
            pos += 2;
            uint64_t z;
            int st = read_varint(in, pos, end, z);
            if (st) return st;
            if (n + len > cap) return CODAG_E_OVERFLOW;
            uint64_t base = unzigzag(z);
            for (uint32_t i = lane(); i < len; i += kWave)
                out[n + i] = base + (uint64_t)(int64_t)((int32_t)i * delta);
            n += len;
        } else {
            uint32_t len = (uint32_t)(-h);
            pos += 1;
            if (n + len > cap) return CODAG_E_OVERFLOW;
            int st = rle_literal_list(in, pos, end, len, out + n, ends);
            if (st) return st;
            n += len;
        }
    }
    return pos == end ? CODAG_OK : CODAG_E_CORRUPT;
}

// ---- RLE v2 ------------------------------------------------------------

__device__ __forceinline__ uint32_t orc_width(uint32_t code) {
    if (code < 24) return code + 1;
    switch (code) {
        case 24: return 26;
        case 25: return 28;
        case 26: return 30;
        case 27: return 32;
        case 28: return 40;
        case 29: return 48;
        case 30: return 56;
        default: return 64;
    }
}

// Smallest codable width holding n bits; 0 when n > 64.
__device__ __forceinline__ uint32_t orc_fit_width(uint32_t n) {
    if (n <= 24) return n;
    if (n <= 32) return (n + 1) & ~1u;
    if (n <= 64) return (n + 7) & ~7u;
    return 0;
}

__device__ __forceinline__ uint64_t bytes_be(uint64_t le8, uint32_t nbytes) {
    return __builtin_bswap64(le8) >> (64 - 8 * nbytes);
}

// Unpacks value `i` (lane-parallel) of a section of `w`-bit values starting
// at byte `sec`; callers ensure the bytes are in the ring.
__device__ __forceinline__ uint64_t packed_value(const InRing &in, uint32_t sec, uint32_t i, uint32_t w) {
    return ring_bits_msb(in, 8ull * sec + (uint64_t)i * w, w);
}

__device__ __forceinline__ void ensure_packed_batch(InRing &in, uint32_t sec, uint32_t i0, uint32_t w) {
    uint64_t last_bit = (uint64_t)(i0 + kWave) * w;  // one past the batch's last bit
    in.ensure(sec + (uint32_t)((last_bit + 7) >> 3) + 12);
}

// A stretch of SHORT_REPEAT runs starting at pos.  Every lane decodes the
// 64-byte window as if a SHORT_REPEAT header started at its own byte (width,
// count and value from the following bytes); the wave then walks the chain of
// runs from lane 0, pulling each run's fields out with readlane instead of a
// round trip to LDS per run.  Stops at the first header that is not a
// SHORT_REPEAT, past the window, at the end of input or when the output is
// full, leaving pos at the next unread header.
__device__ __forceinline__ int rle_v2_short_repeats(InRing &in, uint32_t &pos, uint32_t end,
                                                    uint64_t *out, uint32_t &n, uint32_t cap) {
    in.ensure(pos + 80);
    uint64_t lo, hi;
    ring_read16(in, pos + lane(), lo, hi);
    uint32_t h = (uint32_t)(lo & 0xff);
    uint32_t w = ((h >> 3) & 7) + 1;
    uint64_t vbytes = (lo >> 8) | (hi << 56);
    uint64_t v = unzigzag(__builtin_bswap64(vbytes) >> (64 - 8 * w));
    uint32_t s = 0;
    int st = CODAG_OK;
    while (s < 64 && pos + s < end) {
        uint32_t hs = readlane(h, s);
        if (hs >> 6) break;  // not a SHORT_REPEAT header
        uint32_t ws = ((hs >> 3) & 7) + 1, cs = (hs & 7) + 3;
        if (n + cs > cap) {
            st = CODAG_E_OVERFLOW;
            break;
        }
        if (pos + s + 1 + ws > end) {
            st = CODAG_E_TRUNCATED;
            break;
        }
        uint64_t vs = readlane64(v, s);
        if (lane() < cs) out[n + lane()] = vs;
        n += cs;
        s += 1 + ws;
        if (n >= cap) break;
    }
    pos += s;
    return st;
}

__device__ __forceinline__ int decode_rle_v2(InRing &in, uint64_t *out, uint32_t cap) {
    uint32_t pos = in.skip, end = in.gend;
    uint32_t n = 0;
    const uint32_t l = lane();
    while (n < cap) {
        if (pos >= end) return CODAG_E_TRUNCATED;
        in.ensure(pos + 24);
        uint64_t x = in.peek8(pos);
        uint32_t b0 = (uint32_t)(x & 0xff), type = b0 >> 6;
        if (type == 0) {
            // SHORT_REPEAT: byte width and count in the header, then the value.
            int st = rle_v2_short_repeats(in, pos, end, out, n, cap);
            if (st) return st;
            continue;
        }
        if (pos + 2 > end) return CODAG_E_TRUNCATED;
        uint32_t b1 = (uint32_t)((x >> 8) & 0xff);
        uint32_t len = (((b0 & 1) << 8) | b1) + 1;
        if (type == 1) {
            // DIRECT: len zigzag values packed at width w.
            uint32_t w = orc_width((b0 >> 1) & 31);
            if (n + len > cap) return CODAG_E_OVERFLOW;
            uint32_t sec = pos + 2, nbytes = (len * w + 7) >> 3;
            if (sec + nbytes > end) return CODAG_E_TRUNCATED;
            for (uint32_t i0 = 0; i0 < len; i0 += kWave) {
                ensure_packed_batch(in, sec, i0, w);
                uint32_t i = i0 + l;
                if (i < len) out[n + i] = unzigzag(packed_value(in, sec, i, w));
            }
            pos = sec + nbytes;
            n += len;
        } else if (type == 2) {
            // PATCHED_BASE.
            if (pos + 4 > end) return CODAG_E_TRUNCATED;
            uint32_t b2 = (uint32_t)((x >> 16) & 0xff), b3 = (uint32_t)((x >> 24) & 0xff);
            uint32_t w = orc_width((b0 >> 1) & 31);
            uint32_t bw = (b2 >> 5) + 1, pw = orc_width(b2 & 31);
            uint32_t pgw = (b3 >> 5) + 1, pll = b3 & 31;
            uint32_t ew = orc_fit_width(pgw + pw);
            if (w + pw > 64 || ew == 0) return CODAG_E_CORRUPT;
            if (n + len > cap) return CODAG_E_OVERFLOW;
            uint32_t bsec = pos + 4;
            if (bsec + bw > end) return CODAG_E_TRUNCATED;
            uint64_t braw = bytes_be(in.peek8(bsec), bw);
            uint64_t sign = 1ull << (8 * bw - 1);
            uint64_t base = (braw & sign) ? 0 - (braw & ~sign) : braw;
            uint32_t dsec = bsec + bw, dbytes = (len * w + 7) >> 3;
            if (dsec + dbytes > end) return CODAG_E_TRUNCATED;
            uint32_t psec = dsec + dbytes, pbytes = (pll * ew + 7) >> 3;
            if (psec + pbytes > end) return CODAG_E_TRUNCATED;
            // Patch list: entry j on lane j, read straight from global memory.
            uint64_t gap = 0, patch = 0;
            if (l < pll) {
                uint64_t bit = 8ull * psec + (uint64_t)l * ew;
                uint32_t byte = (uint32_t)(bit >> 3), wi = byte >> 2;
                uint32_t o = 8 * (byte & 3) + (uint32_t)(bit & 7);
                const uint32_t *g = reinterpret_cast<const uint32_t *>(in.gbase);
                uint32_t a = g[wi];
                uint32_t b = 4 * (wi + 1) < end ? g[wi + 1] : 0;
                uint32_t c = 4 * (wi + 2) < end ? g[wi + 2] : 0;
                uint64_t hi = ((uint64_t)bswap32(a) << 32) | bswap32(b);
                uint64_t top = o ? (hi << o) | ((uint64_t)bswap32(c) >> (32 - o)) : hi;
                uint64_t e = ew >= 64 ? top : top >> (64 - ew);
                gap = e >> pw;
                patch = pw >= 64 ? e : e & ((1ull << pw) - 1);
            }
            bool filler = gap == 255 && patch == 0;
            uint64_t cursor = wave_inclusive_sum(gap);
            if (ballot(l < pll && !filler && cursor >= len)) return CODAG_E_CORRUPT;
            uint32_t jp = 0;
            for (uint32_t i0 = 0; i0 < len; i0 += kWave) {
                ensure_packed_batch(in, dsec, i0, w);
                uint32_t i = i0 + l;
                uint64_t v = i < len ? packed_value(in, dsec, i, w) : 0;
                while (jp < pll) {
                    uint32_t pj = (uint32_t)readlane64(cursor, jp);
                    if (pj >= i0 + kWave) break;
                    if (!(readlane64(gap, jp) == 255 && readlane64(patch, jp) == 0)) {
                        uint64_t pt = readlane64(patch, jp);
                        if (i == pj) v |= pt << w;
                    }
                    jp++;
                }
                if (i < len) out[n + i] = base + v;
            }
            pos = psec + pbytes;
            n += len;
        } else {
            // DELTA: width code 0 = fixed delta; zigzag base and delta base.
            uint32_t code = (b0 >> 1) & 31;
            uint32_t w = code ? orc_width(code) : 0;
            uint32_t p = pos + 2;
            uint64_t zb, zd;
            int st = read_varint(in, p, end, zb);
            if (st) return st;
            st = read_varint(in, p, end, zd);
            if (st) return st;
            if (n + len > cap) return CODAG_E_OVERFLOW;
            uint64_t base = unzigzag(zb), dbase = unzigzag(zd);
            if (w == 0) {
                for (uint32_t i = l; i < len; i += kWave) out[n + i] = base + (uint64_t)i * dbase;
                pos = p;
            } else {
                if (l == 0) out[n] = base;
                if (l == 1 && len >= 2) out[n + 1] = base + dbase;
                uint32_t nd = len >= 2 ? len - 2 : 0, nbytes = (nd * w + 7) >> 3;
                if (p + nbytes > end) return CODAG_E_TRUNCATED;
                bool neg = (uint32_t)(dbase >> 63) != 0;
                uint64_t prev = base + dbase;
                for (uint32_t i0 = 0; i0 < nd; i0 += kWave) {
                    ensure_packed_batch(in, p, i0, w);
                    uint32_t i = i0 + l;
                    uint64_t d = i < nd ? packed_value(in, p, i, w) : 0;
                    uint64_t s = wave_inclusive_sum(d);
                    uint64_t v = neg ? prev - s : prev + s;
                    if (i < nd) out[n + 2 + i] = v;
                    prev = uni64(readlane64(v, kWave - 1));
                }
                pos = p + nbytes;
            }
            n += len;
        }
    }
    return pos == end ? CODAG_OK : CODAG_E_CORRUPT;
}

}  // namespace codag
