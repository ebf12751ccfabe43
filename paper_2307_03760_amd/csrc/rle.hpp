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

#include <type_traits>

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

// Element type of an integer column: B-byte little-endian values (the low
// bytes of each decoded 64-bit value, which is how a narrower column holds
// it) and SIGNED values zigzag-coded, unsigned ones not (ORC writes
// unsigned streams, such as string lengths, without zigzag).
template <int B, bool SIGNED>
struct Elem {
    static constexpr int kBytes = B;
    static constexpr bool kSigned = SIGNED;
    using T = typename std::conditional<
        B == 1, uint8_t,
        typename std::conditional<B == 2, uint16_t,
                                  typename std::conditional<B == 4, uint32_t, uint64_t>::type>::type>::type;
    __device__ static __forceinline__ uint64_t val(uint64_t z) { return SIGNED ? unzigzag(z) : z; }
};
using I64 = Elem<8, true>;

// An unsigned base-128 varint from its bytes: x = the first eight, y = the
// next two (little-endian).  Returns its length in bytes (9 or 10 for the
// long forms), or 0 if it is longer than ten bytes or has bits above bit 63.
// Bytes past the end of the chunk read as zero, i.e. as terminators, so a
// varint cut off by the end is seen ending past `end` (the caller reports
// TRUNCATED).
__device__ __forceinline__ uint32_t varint_bytes(uint64_t x, uint32_t y, uint64_t &z) {
    uint64_t t = ~x & 0x8080808080808080ull;
    if (t) {
        uint32_t nb = (uint32_t)(__builtin_ctzll(t) >> 3) + 1;
        z = pack7(low_bytes(x, nb));
        return nb;
    }
    uint32_t b8 = y & 0xff, b9 = (y >> 8) & 0xff;
    if ((b8 & 0x80) && b9 > 1) return 0;  // bits above bit 63, or an 11th byte
    uint32_t nb = (b8 & 0x80) ? 10 : 9;
    z = pack7(x) | ((uint64_t)(b8 & 0x7f) << 56) | (nb == 10 ? (uint64_t)b9 << 63 : 0);
    return nb;
}

// Unsigned base-128 varint at byte position pos (wave-uniform).
template <class Ring>
__device__ __forceinline__ int read_varint(Ring &in, uint32_t &pos, uint32_t end, uint64_t &z) {
    in.ensure(pos + 24);
    uint64_t lo, hi;
    ring_read16(in, pos, lo, hi);
    uint32_t nb = uni(varint_bytes(uni64(lo), uni((uint32_t)hi), z));
    if (nb == 0) return CODAG_E_CORRUPT;
    if (pos + nb > end) return CODAG_E_TRUNCATED;
    pos += nb;
    return CODAG_OK;
}

// Terminator bytes (bit 7 clear) of a little-endian word, one bit per byte.
__device__ __forceinline__ uint32_t terminators4(uint32_t w) {
    uint32_t t = (~w & 0x80808080u) >> 7;  // bits 0, 8, 16, 24
    return (t | (t >> 7) | (t >> 14) | (t >> 21)) & 15;
}

// A literal list of `count` zigzag varints starting at pos, 512 bytes per
// pass: lane l holds bytes [p0 + 8l, p0 + 8l + 8) and the 16 before them.
// Each lane counts the terminator bytes (bit 7 clear) in its 8; a wave
// prefix sum numbers them, a wave running maximum gives the position after
// the last terminator of the lanes below, and then every lane decodes, from
// its registers, the varints whose terminators it holds and stores them at
// their index -- no compaction through LDS.
template <class E = I64, class Ring>
__device__ __forceinline__ int rle_literal_list(Ring &in, uint32_t &pos, uint32_t end,
                                                uint32_t count, typename E::T *out) {
    const uint32_t l = lane();
    uint32_t done = 0;
    while (done < count) {
        const uint32_t p0 = pos & ~7u;
        in.ensure(p0 + 528);
        const uint32_t at = p0 + 8 * l, wb = at >> 2;
        uint32_t wd[6];
#pragma unroll
        for (uint32_t j = 0; j < 6; j++) wd[j] = in.word(wb - 4 + j);  // bytes [at - 16, at + 8)
        uint32_t tm = terminators4(wd[4]) | (terminators4(wd[5]) << 4);
        if (at < pos) tm &= pos - at >= 8 ? 0u : (0xffu << (pos - at)) & 0xffu;
        const uint32_t cnt = __builtin_popcount(tm);
        const uint32_t incl = wave_inclusive_sum32(cnt);
        const uint32_t total = readlane(incl, kWave - 1);
        if (total == 0) return CODAG_E_CORRUPT;  // >= 505 continuation bytes
        const uint32_t use = min(total, count - done);
        // One past the last terminator of the lanes below (0: none).
        const uint32_t after = tm ? at + (31 - __builtin_clz(tm)) + 1 : 0;
        const uint32_t prev = wave_shift_up1(wave_inclusive_max32(after));
        uint32_t s = max(prev, pos), g = incl - cnt, rem = tm, stop = 0;
        int st = CODAG_OK;
        while (ballot(rem != 0 && g < use)) {
            if (rem != 0 && g < use) {
                const uint32_t e = at + (uint32_t)__builtin_ctz(rem);  // terminator position
                rem &= rem - 1;
                const uint32_t nb = e - s + 1;
                if (nb > 10) {
                    if (st == CODAG_OK) st = CODAG_E_CORRUPT;
                } else {
                    // Bytes [s, e] from the register window: offset o in 7..23.
                    const uint32_t o = s + 16 - at, wi = o >> 2, sh = o & 3;
                    uint32_t v[4];
#pragma unroll
                    for (uint32_t t = 0; t < 4; t++) {
                        uint32_t k = wi + t, r = 0;
#pragma unroll
                        for (uint32_t j = 1; j < 6; j++) r = k == j ? wd[j] : r;
                        v[t] = r;
                    }
                    const uint64_t x = ((uint64_t)__builtin_amdgcn_alignbyte(v[2], v[1], sh) << 32) |
                                       __builtin_amdgcn_alignbyte(v[1], v[0], sh);
                    const uint32_t y = __builtin_amdgcn_alignbyte(v[3], v[2], sh);
                    const uint32_t b9 = (y >> 8) & 0xff;
                    if (st == CODAG_OK) {
                        if (e >= end) st = CODAG_E_TRUNCATED;
                        else if (nb == 10 && b9 > 1) st = CODAG_E_CORRUPT;
                    }
                    uint64_t z = pack7(low_bytes(x, nb));
                    if (nb > 8) z |= (uint64_t)(y & 0x7f) << 56;
                    if (nb > 9) z |= (uint64_t)(b9 & 1) << 63;
                    if (st == CODAG_OK) out[done + g] = (typename E::T)E::val(z);
                }
                if (g == use - 1) stop = e + 1;
                s = e + 1;
                g++;
            }
        }
        // The first failing varint in list order: lanes hold increasing
        // indices, and each lane keeps its first failure.
        const uint64_t bad = ballot(st != CODAG_OK);
        if (bad) return (int)uni((uint32_t)readlane((uint32_t)st, (uint32_t)__builtin_ctzll(bad)));
        pos = uni(readlane(stop, (uint32_t)__builtin_ctzll(ballot(stop != 0))));
        done += use;
    }
    return CODAG_OK;
}

// ---- RLE v1 ------------------------------------------------------------

// One group at pos, whose first value is value n of the chunk.  Runs: header
// 0..127 = length - 3, a signed delta byte, a zigzag varint base.  Literal
// lists: header -1..-128 = -count, then count zigzag varints.  One 16-byte
// read gives a run's header, delta and base together.  Advances pos and n.
template <class E = I64, class Ring>
__device__ __forceinline__ int rle_v1_group(Ring &in, uint32_t &pos, uint32_t end, typename E::T *out,
                                            uint32_t &n, uint32_t cap) {
    if (pos >= end) return CODAG_E_TRUNCATED;
    in.ensure(pos + 24);
    uint64_t lo, hi;
    ring_read16(in, pos, lo, hi);
    lo = uni64(lo);
    int32_t h = (int8_t)(lo & 0xff);
    if (h >= 0) {
        uint32_t len = (uint32_t)h + 3;
        if (pos + 2 > end) return CODAG_E_TRUNCATED;
        int32_t delta = (int8_t)((lo >> 8) & 0xff);
        hi = uni64(hi);
        uint64_t z;
        uint32_t nb = varint_bytes((lo >> 16) | (hi << 48), (uint32_t)(hi >> 16), z);
        if (nb == 0) return CODAG_E_CORRUPT;
        if (pos + 2 + nb > end) return CODAG_E_TRUNCATED;
        pos += 2 + nb;
        if (n + len > cap) return CODAG_E_OVERFLOW;
        uint64_t base = E::val(z);
        for (uint32_t i = lane(); i < len; i += kWave)
            out[n + i] = (typename E::T)(base + (uint64_t)(int64_t)((int32_t)i * delta));
        n += len;
        return CODAG_OK;
    }
    uint32_t len = (uint32_t)(-h);
    pos += 1;
    if (n + len > cap) return CODAG_E_OVERFLOW;
    int st = rle_literal_list<E>(in, pos, end, len, out + n);
    if (st) return st;
    n += len;
    return CODAG_OK;
}

template <class E = I64, class Ring>
__device__ __forceinline__ int decode_rle_v1(Ring &in, typename E::T *out, uint32_t cap) {
    uint32_t pos = in.skip, end = in.gend;
    uint32_t n = 0;
    while (n < cap) {
        int st = rle_v1_group<E>(in, pos, end, out, n, cap);
        if (st) return st;
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

// The same for widths of at most 32 bits: two ring words always hold the
// value (its first bit is at most 31 bits into the first word).
__device__ __forceinline__ uint32_t packed_value32(const InRing &in, uint32_t sec, uint32_t i, uint32_t w) {
    const uint32_t bit = 8 * sec + i * w, wi = bit >> 5;
    const uint64_t x = ((uint64_t)bswap32(in.word_at(wi, 0)) << 32) | bswap32(in.word_at(wi, 1));
    return (uint32_t)((x << (bit & 31)) >> (64 - w));
}

// A packed section this long (plus a few bytes of lookahead) is readable in
// the ring at once.
constexpr uint32_t kWholeSection = kFetchBytes - 32;

__device__ __forceinline__ void ensure_packed_batch(InRing &in, uint32_t sec, uint32_t i0, uint32_t w) {
    uint64_t last_bit = (uint64_t)(i0 + kWave) * w;  // one past the batch's last bit
    in.ensure(sec + (uint32_t)((last_bit + 7) >> 3) + 12);
}

// A stretch of SHORT_REPEAT runs starting at pos, 64 bytes at a time.
// Every lane decodes the window as if a SHORT_REPEAT header started at its
// own byte (width, count and value from the following bytes) and links it
// to where the next header would start.  The wave then walks the chain of
// runs from lane 0 with one lane read per run, marking the lanes where runs
// start, and every marked lane writes its run at the position a wave prefix
// sum of the run lengths gives it; a chain that runs past the window goes
// on in the next one.  Stops at the first header that is not a
// SHORT_REPEAT, at the end of input or when the output is full, leaving pos
// at the next unread header; when that header lies in the window, its first
// eight bytes are returned in x (next = true).
template <class E = I64>
__device__ __forceinline__ int rle_v2_short_repeats(InRing &in, uint32_t &pos, uint32_t end,
                                                    typename E::T *out, uint32_t &n, uint32_t cap,
                                                    uint64_t &x, bool &next) {
    const uint32_t l = lane();
    for (;;) {
        in.ensure(pos + 84);
        uint64_t lo, hi;
        ring_read16(in, pos + l, lo, hi);
        const uint32_t h = (uint32_t)(lo & 0xff);
        const uint32_t w = ((h >> 3) & 7) + 1;
        const uint64_t vbytes = (lo >> 8) | (hi << 56);
        const uint64_t v = E::val(__builtin_bswap64(vbytes) >> (64 - 8 * w));
        // Each lane's run, if one starts there: where the next would start
        // (below 128), or 128 + lane where the chain must stop (not a
        // SHORT_REPEAT header, or the value past the end of the input).  The
        // walk's only dependent step is the lane read; a stop lane it marked
        // is unmarked afterwards.
        const uint32_t cs = (h & 7) + 3;
        const uint32_t nxt = (h >> 6) == 0 && pos + l + 1 + w <= end ? l + 1 + w : 128 + l;
        uint32_t s = 0;
        uint64_t starts = 0;
        for (;;) {  // two runs per loop trip: one taken branch per two runs
            starts |= 1ull << s;
            s = readlane(nxt, s);
            if (s >= kWave) break;
            starts |= 1ull << s;
            s = readlane(nxt, s);
            if (s >= kWave) break;
        }
        if (s >= 128) {
            s -= 128;
            starts &= ~(1ull << s);
        }
        // Output positions of the runs in order.  A run that starts once
        // the output is full ends the walk there; one that would pass it is
        // an overflow; neither is stored.
        const bool mine = (starts >> l) & 1;
        const uint32_t c = mine ? cs : 0;
        const uint32_t at = n + wave_inclusive_sum32(c) - c;
        const uint32_t n1 = uni(readlane(at + c, kWave - 1));
        uint32_t ff = kWave, fo = kWave;
        if (n1 > cap) {  // the output fills inside this window
            const uint64_t full = ballot(mine && at >= cap), over = ballot(mine && at < cap && at + c > cap);
            ff = full ? (uint32_t)__builtin_ctzll(full) : kWave;
            fo = over ? (uint32_t)__builtin_ctzll(over) : kWave;
        }
        const uint32_t lim = min(ff, fo);
        if (mine && l < lim) {
            // Two values per store (8-byte aligned 16-byte stores), the odd
            // last one alone.
            if constexpr (E::kBytes == 8) {
                typedef uint64_t u64x2 __attribute__((ext_vector_type(2), aligned(8)));
                const u64x2 vv = {v, v};
                for (uint32_t j = 0; j < 10; j += 2)
                    if (j + 1 < c) *reinterpret_cast<u64x2 *>(out + at + j) = vv;
                if (c & 1) out[at + c - 1] = v;
            } else {
                for (uint32_t j = 0; j < c; j++) out[at + j] = (typename E::T)v;
            }
        }
        if (fo < ff) {
            n = uni(readlane(at, fo));
            return CODAG_E_OVERFLOW;
        }
        if (ff < kWave) {
            n = cap;
            pos += ff;
            return CODAG_OK;
        }
        n = n1;
        if (s < kWave) {
            // Stopped at a lane that does not continue the chain: a
            // SHORT_REPEAT header inside the input there has its value cut
            // off; any other header is handed back.  With the output already
            // full nothing more is parsed: the caller reports the bytes left
            // over.
            int st = CODAG_OK;
            if (pos + s < end && n < cap) {
                const uint32_t hs = readlane(h, s);
                if ((hs >> 6) == 0)
                    st = n + (hs & 7) + 3 > cap ? CODAG_E_OVERFLOW : CODAG_E_TRUNCATED;
                x = uni64(readlane64(lo, s));
                next = true;
            }
            pos += s;
            return st;
        }
        pos += s;
        if (n >= cap || pos >= end) return CODAG_OK;
    }
}

// Runs from byte position pos, their first value being value n of the
// chunk, until value cap.  On an error, n is the first value of the run that
// failed.
template <class E = I64>
__device__ __forceinline__ int decode_rle_v2_runs(InRing &in, uint32_t &pos, uint32_t end,
                                                  typename E::T *out, uint32_t &n, uint32_t cap) {
    using T = typename E::T;
    const uint32_t l = lane();
    uint64_t x = 0;     // the header's first eight bytes
    bool have = false;  // x already read (handed back by a SHORT_REPEAT stretch)
    while (n < cap) {
        if (pos >= end) return CODAG_E_TRUNCATED;
        in.ensure(pos + 24);
        if (!have) x = in.peek8(pos);
        have = false;
        uint32_t b0 = (uint32_t)(x & 0xff), type = b0 >> 6;
        if (type == 0) {
            // SHORT_REPEAT: byte width and count in the header, then the value.
            int st = rle_v2_short_repeats<E>(in, pos, end, out, n, cap, x, have);
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
            if (nbytes <= kWholeSection) {
                // The whole section is readable at once: eight unrolled
                // batches, so their LDS reads overlap.
                in.ensure(sec + nbytes + 12);
                if (w <= 32) {
#pragma unroll
                    for (uint32_t b = 0; b < 8; b++) {
                        uint32_t i = kWave * b + l;
                        if (i < len) out[n + i] = (T)E::val(packed_value32(in, sec, i, w));
                    }
                } else {
#pragma unroll
                    for (uint32_t b = 0; b < 8; b++) {
                        uint32_t i = kWave * b + l;
                        if (i < len) out[n + i] = (T)E::val(packed_value(in, sec, i, w));
                    }
                }
            } else if (w <= 32) {
                // Two batches per ring check (at most 512 bytes together).
                for (uint32_t i0 = 0; i0 < len; i0 += 2 * kWave) {
                    ensure_packed_batch(in, sec, i0 + kWave, w);
                    const uint32_t i = i0 + l, j = i + kWave;
                    const uint32_t a = i < len ? packed_value32(in, sec, i, w) : 0;
                    const uint32_t b = j < len ? packed_value32(in, sec, j, w) : 0;
                    if (i < len) out[n + i] = (T)E::val(a);
                    if (j < len) out[n + j] = (T)E::val(b);
                }
            } else if (w <= 56) {
                // Two batches per ring check (at most 896 bytes together).
                for (uint32_t i0 = 0; i0 < len; i0 += 2 * kWave) {
                    ensure_packed_batch(in, sec, i0 + kWave, w);
                    const uint32_t i = i0 + l, j = i + kWave;
                    const uint64_t a = i < len ? packed_value(in, sec, i, w) : 0;
                    const uint64_t b = j < len ? packed_value(in, sec, j, w) : 0;
                    if (i < len) out[n + i] = (T)E::val(a);
                    if (j < len) out[n + j] = (T)E::val(b);
                }
            } else {
                for (uint32_t i0 = 0; i0 < len; i0 += kWave) {
                    ensure_packed_batch(in, sec, i0, w);
                    uint32_t i = i0 + l;
                    if (i < len) out[n + i] = (T)E::val(packed_value(in, sec, i, w));
                }
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
            if (ew == 0) return CODAG_E_CORRUPT;  // gap + patch entries over 64 bits
            if (n + len > cap) return CODAG_E_OVERFLOW;
            uint32_t bsec = pos + 4;
            if (bsec + bw > end) return CODAG_E_TRUNCATED;
            // The base's bytes follow the 4-byte header: up to four of them
            // are already in x.
            uint64_t braw = bytes_be(bw <= 4 ? x >> 32 : in.peek8(bsec), bw);
            uint64_t sign = 1ull << (8 * bw - 1);
            uint64_t base = (braw & sign) ? 0 - (braw & ~sign) : braw;
            uint32_t dsec = bsec + bw, dbytes = (len * w + 7) >> 3;
            if (dsec + dbytes > end) return CODAG_E_TRUNCATED;
            uint32_t psec = dsec + dbytes, pbytes = (pll * ew + 7) >> 3;
            if (psec + pbytes > end) return CODAG_E_TRUNCATED;
            // Patch list: entry j on lane j, from the ring when the data and
            // the list fit in it together (no global load, whose wait would
            // also wait for every store in flight), else from global memory.
            uint64_t gap = 0, patch = 0;
            const bool whole = psec + pbytes - dsec <= kWholeSection;
            if (whole) in.ensure(psec + pbytes + 12);
            if (l < pll) {
                uint64_t e;
                if (whole) {
                    e = ring_bits_msb(in, 8ull * psec + (uint64_t)l * ew, ew);
                } else {
                    uint64_t bit = 8ull * psec + (uint64_t)l * ew;
                    uint32_t byte = (uint32_t)(bit >> 3), wi = byte >> 2;
                    uint32_t o = 8 * (byte & 3) + (uint32_t)(bit & 7);
                    const uint32_t *g = reinterpret_cast<const uint32_t *>(in.gbase);
                    uint32_t a = g[wi];
                    uint32_t b = 4 * (wi + 1) < end ? g[wi + 1] : 0;
                    uint32_t c = 4 * (wi + 2) < end ? g[wi + 2] : 0;
                    uint64_t hi = ((uint64_t)bswap32(a) << 32) | bswap32(b);
                    uint64_t top = o ? (hi << o) | ((uint64_t)bswap32(c) >> (32 - o)) : hi;
                    e = ew >= 64 ? top : top >> (64 - ew);
                }
                gap = e >> pw;
                patch = pw >= 64 ? e : e & ((1ull << pw) - 1);
            }
            bool filler = gap == 255 && patch == 0;
            uint64_t cursor = wave_inclusive_sum(gap);
            if (ballot(l < pll && !filler && cursor >= len)) return CODAG_E_CORRUPT;
            // Patch j lands on value cursor[j] (below 2^13: at most 31
            // gaps below 2^8).  A filler entry's patch is zero, so OR-ing it
            // in changes nothing and needs no test.
            // Patch bits shifted past bit 63 are dropped (the data width
            // plus the patch width may exceed 64; with a 64-bit data width
            // a patch changes nothing).
            if (w >= 64) patch = 0;
            else patch <<= w;
            const uint32_t cur = (uint32_t)cursor, plo = (uint32_t)patch, phi = (uint32_t)(patch >> 32);
            uint32_t jp = 0;
            if (whole && w <= 32) {
                // All eight batches' values first, so their LDS reads
                // overlap; then the patches and the stores.
                uint32_t vb[8];
#pragma unroll
                for (uint32_t b = 0; b < 8; b++) {
                    const uint32_t i = kWave * b + l;
                    vb[b] = i < len ? packed_value32(in, dsec, i, w) : 0;
                }
#pragma unroll
                for (uint32_t b = 0; b < 8; b++) {
                    const uint32_t i0 = kWave * b, i = i0 + l;
                    if (i0 >= len) break;
                    uint64_t v = vb[b];
                    while (jp < pll) {
                        const uint32_t pj = readlane(cur, jp);
                        if (pj >= i0 + kWave) break;
                        const uint64_t pt = ((uint64_t)readlane(phi, jp) << 32) | readlane(plo, jp);
                        if (i == pj) v |= pt;
                        jp++;
                    }
                    if (i < len) out[n + i] = (T)(base + v);
                }
                pos = psec + pbytes;
                n += len;
                continue;
            }
            for (uint32_t i0 = 0; i0 < len; i0 += kWave) {
                if (!whole) ensure_packed_batch(in, dsec, i0, w);
                uint32_t i = i0 + l;
                uint64_t v = i >= len ? 0 : w <= 32 ? packed_value32(in, dsec, i, w) : packed_value(in, dsec, i, w);
                while (jp < pll) {
                    const uint32_t pj = readlane(cur, jp);
                    if (pj >= i0 + kWave) break;
                    const uint64_t pt = ((uint64_t)readlane(phi, jp) << 32) | readlane(plo, jp);
                    if (i == pj) v |= pt;
                    jp++;
                }
                if (i < len) out[n + i] = (T)(base + v);
            }
            pos = psec + pbytes;
            n += len;
        } else {
            // DELTA: width code 0 = fixed delta; zigzag base and delta base.
            uint32_t code = (b0 >> 1) & 31;
            uint32_t w = code ? orc_width(code) : 0;
            uint32_t p = pos + 2;
            uint64_t zb, zd;
            {
                // Both varints from one 32-byte read.
                in.ensure(p + 36);
                uint64_t a0, a1, a2, a3;
                ring_read16(in, p, a0, a1);
                ring_read16(in, p + 16, a2, a3);
                a0 = uni64(a0);
                a1 = uni64(a1);
                a2 = uni64(a2);
                uint32_t nb = varint_bytes(a0, (uint32_t)a1, zb);
                if (nb == 0) return CODAG_E_CORRUPT;
                if (p + nb > end) return CODAG_E_TRUNCATED;
                // The second varint's bytes: ten from offset nb (1..10) of
                // a0..a2, by byte alignment of the words around it.
                const uint32_t d0 = (uint32_t)a0, d1 = (uint32_t)(a0 >> 32), d2 = (uint32_t)a1,
                               d3 = (uint32_t)(a1 >> 32), d4 = (uint32_t)a2, d5 = (uint32_t)(a2 >> 32);
                const uint32_t wi = nb >> 2, sb = nb & 3;
                const uint32_t e0 = wi == 0 ? d0 : wi == 1 ? d1 : d2;
                const uint32_t e1 = wi == 0 ? d1 : wi == 1 ? d2 : d3;
                const uint32_t e2 = wi == 0 ? d2 : wi == 1 ? d3 : d4;
                const uint32_t e3 = wi == 0 ? d3 : wi == 1 ? d4 : d5;
                const uint64_t x = ((uint64_t)uni(__builtin_amdgcn_alignbyte(e2, e1, sb)) << 32) |
                                   uni(__builtin_amdgcn_alignbyte(e1, e0, sb));
                const uint32_t y = uni(__builtin_amdgcn_alignbyte(e3, e2, sb));
                p += nb;
                uint32_t nb2 = varint_bytes(x, y, zd);
                if (nb2 == 0) return CODAG_E_CORRUPT;
                if (p + nb2 > end) return CODAG_E_TRUNCATED;
                p += nb2;
            }
            if (n + len > cap) return CODAG_E_OVERFLOW;
            uint64_t base = E::val(zb), dbase = unzigzag(zd);  // the delta base is always signed
            if (w == 0) {
                for (uint32_t i = l; i < len; i += kWave) out[n + i] = (T)(base + (uint64_t)i * dbase);
                pos = p;
            } else {
                if (l == 0) out[n] = (T)base;
                if (l == 1 && len >= 2) out[n + 1] = (T)(base + dbase);
                uint32_t nd = len >= 2 ? len - 2 : 0, nbytes = (nd * w + 7) >> 3;
                if (p + nbytes > end) return CODAG_E_TRUNCATED;
                bool neg = (uint32_t)(dbase >> 63) != 0;
                uint64_t prev = base + dbase;
                const bool whole = nbytes <= kWholeSection;
                if (whole) in.ensure(p + nbytes + 12);
                if (whole && w <= 24) {
                    // Narrow deltas: a batch's sums fit 32 bits (64 x 2^24),
                    // and the batches only share the running value, so
                    // their reads and scans overlap.
#pragma unroll
                    for (uint32_t b = 0; b < 8; b++) {
                        const uint32_t i = kWave * b + l;
                        const uint32_t d = i < nd ? packed_value32(in, p, i, w) : 0;
                        const uint32_t s = wave_inclusive_sum32(d);
                        const uint64_t v = neg ? prev - s : prev + s;
                        if (i < nd) out[n + 2 + i] = (T)v;
                        const uint32_t t = uni(readlane(s, kWave - 1));
                        prev = neg ? prev - t : prev + t;
                    }
                } else {
                    for (uint32_t i0 = 0; i0 < nd; i0 += kWave) {
                        if (!whole) ensure_packed_batch(in, p, i0, w);
                        uint32_t i = i0 + l;
                        uint64_t d = i < nd ? packed_value(in, p, i, w) : 0;
                        uint64_t s = wave_inclusive_sum(d);
                        uint64_t v = neg ? prev - s : prev + s;
                        if (i < nd) out[n + 2 + i] = (T)v;
                        prev = uni64(readlane64(v, kWave - 1));
                    }
                }
                pos = p + nbytes;
            }
            n += len;
        }
    }
    return CODAG_OK;
}

template <class E = I64>
__device__ __forceinline__ int decode_rle_v2(InRing &in, typename E::T *out, uint32_t cap) {
    uint32_t pos = in.skip, n = 0;
    const int st = decode_rle_v2_runs<E>(in, pos, in.gend, out, n, cap);
    if (st) return st;
    return pos == in.gend ? CODAG_OK : CODAG_E_CORRUPT;
}

// ---- ORC byte RLE -------------------------------------------------------

// Byte columns and PRESENT bitmaps: a header 0..127 is a run of header + 3
// copies of the next byte, -1..-128 is followed by -header literal bytes.
// Runs are written one byte per lane; literal bytes are copied from the
// ring one per lane.  Checks in the order header, run byte, capacity, then
// the literal bytes.
template <class Ring>
__device__ __forceinline__ int decode_byte_rle(Ring &in, uint8_t *out, uint32_t cap) {
    uint32_t pos = in.skip, end = in.gend, n = 0;
    const uint32_t l = lane();
    while (n < cap) {
        if (pos >= end) return CODAG_E_TRUNCATED;
        in.ensure(pos + 136);
        const uint64_t x = in.peek8(pos);
        const uint32_t h = (uint32_t)(x & 0xff);
        if (h < 128) {
            const uint32_t len = h + 3;
            if (pos + 2 > end) return CODAG_E_TRUNCATED;
            if (n + len > cap) return CODAG_E_OVERFLOW;
            const uint8_t b = (uint8_t)(x >> 8);
            for (uint32_t i = l; i < len; i += kWave) out[n + i] = b;
            pos += 2;
            n += len;
        } else {
            const uint32_t len = 256 - h;
            pos += 1;
            if (n + len > cap) return CODAG_E_OVERFLOW;
            if (pos + len > end) return CODAG_E_TRUNCATED;
            for (uint32_t i = l; i < len; i += kWave) {
                const uint32_t q = pos + i;
                out[n + i] = (uint8_t)(in.word(q >> 2) >> (8 * (q & 3)));
            }
            pos += len;
            n += len;
        }
    }
    return pos == end ? CODAG_OK : CODAG_E_CORRUPT;
}

}  // namespace codag
