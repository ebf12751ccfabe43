// Deflate (RFC 1951) decoding by one wavefront.
//
// CODAG (Section II-A, III) locates Deflate's cost in Huffman decoding and
// dictionary copies.  Here:
//   * The symbol chain is wave-uniform scalar code: a 64-bit bit buffer in
//     scalar registers, refilled one 32-bit word at a time from the LDS input
//     ring, and one lookup per symbol in LDS tables that the whole wave builds
//     in parallel for each block.
//   * Output goes first to a per-wave history window in LDS (the last H bytes
//     of output) and reaches HBM behind the decoder, 1 KiB at a time, as one
//     16-byte store per lane of an aligned kilobyte ("coalesced on-demand
//     writing", Section IV-F).  Literals ("write_byte") are one LDS byte write
//     each; back-references ("memcpy", Section IV-F) are copied by all lanes
//     at once from the window, including the overlapping case where the
//     length exceeds the distance.  Only a reference reaching further back
//     than the window reads HBM.  Reading just-written output from HBM would
//     make each copy wait for all outstanding stores of the wave.
#pragma once

#include "../../include/codag.h"
#include "stream.hpp"

namespace codag {

// Table entry (16 bits): bits 0-3 code length, 4-12 symbol, 13-15 kind.
enum : uint32_t {
    kLit = 0,      // literal byte (symbol 0..255)
    kBase = 1,     // length symbol 257..285, or distance symbol 0..29
    kEob = 2,      // end of block
    kSlow = 3,     // code longer than the table: canonical decode
    kInvalid = 4,  // no code starts with these bits
    kBadSym = 5,   // a code for a symbol that may not appear (286, 287; 30, 31)
    kSym = 6,      // code-length alphabet symbol
};

__device__ __forceinline__ uint32_t entry16(uint32_t kind, uint32_t len, uint32_t sym) {
    return len | (sym << 4) | (kind << 13);
}

enum TableUse { kLitLen = 0, kDist = 1, kCodeLen = 2 };

__device__ __forceinline__ uint32_t symbol_kind(int use, uint32_t s) {
    if (use == kCodeLen) return kSym;
    if (use == kLitLen) return s < 256 ? kLit : s == 256 ? kEob : s <= 285 ? kBase : kBadSym;
    return s <= 29 ? kBase : kBadSym;
}

// Base value and extra-bit count of length symbols 257..285 (lane k holds
// symbol 257 + k) and distance symbols 0..29 (lane k holds symbol k), packed
// as base | extra << 16 (RFC 1951 section 3.2.5).
__device__ __forceinline__ uint32_t length_lane_table() {
    uint32_t k = lane();
    if (k >= 29) return 0;
    if (k == 28) return 258;
    if (k < 8) return k + 3;
    uint32_t e = (k >> 2) - 1;
    return (((4 + (k & 3)) << e) + 3) | (e << 16);
}
__device__ __forceinline__ uint32_t distance_lane_table() {
    uint32_t k = lane();
    if (k >= 30) return 0;
    if (k < 4) return k + 1;
    uint32_t e = (k >> 1) - 1;
    return (((2 + (k & 1)) << e) + 1) | (e << 16);
}

// Per-code metadata for the slow path: count, first code and offset into
// `sorted` for each code length 1..15.
struct CodeMeta {
    uint32_t count[16];
    uint32_t first[16];
    uint32_t offs[16];
};

struct BuildResult {
    int32_t left;    // unused codes scaled to 2^15 (< 0: over-subscribed)
    uint32_t total;  // number of symbols with a code
    uint32_t ones;   // number of codes of length 1
};

// Builds the lookup table (2^tb entries) of the canonical code whose lengths
// are lens[0..n) (n <= 320), lane-parallel: per-length counts and each
// symbol's rank come from ballots, then every symbol fills its table slots.
__device__ __forceinline__ BuildResult build_table(const uint8_t *lens, uint32_t n, uint32_t tb,
                                                   int use, uint16_t *tab, uint16_t *sorted,
                                                   CodeMeta *meta) {
    const uint32_t l = lane();
    uint32_t cnt[16];
#pragma unroll
    for (int k = 0; k < 16; k++) cnt[k] = 0;
    uint32_t rank[5];
#pragma unroll
    for (int p = 0; p < 5; p++) {
        uint32_t s = 64 * p + l;
        uint32_t m = s < n ? lens[s] : 0;
        rank[p] = 0;
#pragma unroll
        for (int len = 1; len < 16; len++) {
            uint64_t b = ballot(m == (uint32_t)len);
            if (m == (uint32_t)len) rank[p] = cnt[len] + count_below(b);
            cnt[len] += (uint32_t)__builtin_popcountll(b);
        }
    }
    BuildResult r;
    int32_t left = 1;
    uint32_t total = 0;
#pragma unroll
    for (int len = 1; len < 16; len++) {
        left = 2 * left - (int32_t)cnt[len];
        total += cnt[len];
        if (left < 0) break;
    }
    r.left = left;
    r.total = total;
    r.ones = cnt[1];
    if (left < 0) return r;
    if (l < 16) {
        uint32_t code = 0, off = 0, c = 0, f = 0, o = 0;
#pragma unroll
        for (int len = 1; len < 16; len++) {
            if ((uint32_t)len == l) {
                c = cnt[len];
                f = code;
                o = off;
            }
            off += cnt[len];
            code = (code + cnt[len]) << 1;
        }
        meta->count[l] = c;
        meta->first[l] = f;
        meta->offs[l] = o;
    }
    if (left > 0) {  // incomplete: codes not in the set are invalid
        for (uint32_t i = l; i < (1u << tb); i += kWave) tab[i] = (uint16_t)entry16(kInvalid, 0, 0);
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int p = 0; p < 5; p++) {
        uint32_t s = 64 * p + l;
        uint32_t m = s < n ? lens[s] : 0;
        if (m != 0) {
            uint32_t code = meta->first[m] + rank[p];
            sorted[meta->offs[m] + rank[p]] = (uint16_t)s;
            if (m <= tb) {
                uint32_t rev = __builtin_bitreverse32(code) >> (32 - m);
                uint16_t e = (uint16_t)entry16(symbol_kind(use, s), m, s);
                for (uint32_t k = 0; k < (1u << (tb - m)); k++) tab[rev | (k << m)] = e;
            } else {
                uint32_t prefix = code >> (m - tb);
                tab[__builtin_bitreverse32(prefix) >> (32 - tb)] = (uint16_t)entry16(kSlow, 0, 0);
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    return r;
}

constexpr uint32_t kDistBits = 8;
constexpr uint32_t kCodeLenBits = 7;

// Order in which the code-length code's lengths are sent (RFC 1951 3.2.7).
__constant__ const uint8_t kCodeLenOrder[19] = {16, 17, 18, 0, 8,  7, 9,  6, 10, 5,
                                                11, 4,  12, 3, 13, 2, 14, 1, 15};

// What one wave keeps in LDS while inflating, besides the input ring: the
// Huffman tables and the output history window.
template <int TB, uint32_t H>
struct DeflateLds {
    uint8_t window[H];  // output byte at absolute address a lives at window[a % H]
    uint16_t lit[1u << TB];
    uint16_t dist[1u << kDistBits];  // also the code-length table (7 bits)
    CodeMeta lit_meta, dist_meta;
    uint16_t lit_sorted[288];
    uint16_t dist_sorted[32];
    uint8_t lens[320];
};

// Wave-uniform LSB-first bit reader over the ring.
struct BitIn {
    uint64_t buf;    // valid bits are the low `cnt`
    uint32_t cnt;
    uint32_t next;   // byte position of the next (aligned) word to load
    int32_t remain;  // input bits not yet consumed (negative: past the end);
                     // 32 bits because there is no scalar 64-bit ordered
                     // compare (chunks are below 256 MiB)

    template <class Ring>
    __device__ __forceinline__ void seek(Ring &in, uint32_t pos) {
        if (pos >= in.loaded + Ring::kFetch) in.restart(pos);
        uint32_t a = pos & ~3u;
        in.ensure(a + 4);
        uint32_t w = uni(in.word(a >> 2));
        uint32_t sh = 8 * (pos & 3);
        buf = w >> sh;
        cnt = 32 - sh;
        next = a + 4;
        remain = 8 * ((int32_t)in.gend - (int32_t)pos);
    }
    template <class Ring>
    __device__ __forceinline__ void refill(Ring &in) {
        if (cnt <= 32) {
            if (in.loaded < next + 4) in.ensure(next + 4);
            uint32_t w = uni(in.word(next >> 2));
            buf |= (uint64_t)w << cnt;
            cnt += 32;
            next += 4;
        }
    }
    // Consume n bits (n <= cnt); false if that runs past the end of input.
    __device__ __forceinline__ bool drop(uint32_t n) {
        buf >>= n;
        cnt -= n;
        remain -= (int32_t)n;
        return remain >= 0;
    }
    // Consume n bits without the end-of-input test.  Bits past the end read
    // as zero; `remain` only decreases, so a decoder that tests it wherever
    // it stops (an error, the end of a block) reports running past the end
    // exactly where a bit-by-bit reader would have.
    __device__ __forceinline__ void skip(uint32_t n) {
        buf >>= n;
        cnt -= n;
        remain -= (int32_t)n;
    }
    // Refill with at most one ring advance (the reader moves 4 bytes at a
    // time, the ring 1 KiB), keeping the hot loop free of inner loops.
    template <class Ring>
    __device__ __forceinline__ void refill1(Ring &in) {
        if (cnt <= 32) {
            if (in.loaded < next + 4) in.commit();
            uint32_t w = uni(in.word(next >> 2));
            buf |= (uint64_t)w << cnt;
            cnt += 32;
            next += 4;
        }
    }
    __device__ __forceinline__ uint32_t peek(uint32_t n) const {
        return (uint32_t)(buf & ((1ull << n) - 1));
    }
    // Byte position of the next unconsumed bit (on a byte boundary).
    __device__ __forceinline__ uint32_t byte_pos() const { return next - cnt / 8; }
};

// Canonical decode of a code longer than the table (CODAG's "Huffman tree
// traversal"): extends the code one bit at a time through lengths 1..15.
__device__ __forceinline__ uint32_t slow_symbol(const BitIn &bi, const CodeMeta *meta,
                                                const uint16_t *sorted, int use) {
    uint32_t code = 0, bits = (uint32_t)bi.buf;
    for (uint32_t len = 1; len < 16; len++) {
        code = (code << 1) | ((bits >> (len - 1)) & 1);
        uint32_t c = uni(meta->count[len]), f = uni(meta->first[len]);
        if (code - f < c) {
            uint32_t s = uni((uint32_t)sorted[uni(meta->offs[len]) + code - f]);
            return entry16(symbol_kind(use, s), len, s);
        }
    }
    return entry16(kInvalid, 0, 0);
}

// Single-byte LDS writes in the decode loops are issued by all lanes with
// the same address and value rather than by one lane: a one-lane branch
// inside a loop that also has early exits makes the compiler treat the loop
// exit as divergent, which moves the whole bit reader out of scalar
// registers.

// Output through the LDS history window.  Positions are 32-bit offsets from
// `base`, the chunk's output address rounded down to 1 KiB (uniform values
// stay in scalar registers; there are no scalar 64-bit ordered compares).
// Bytes below `fa` are in HBM; bytes in [fa, o0 + pos) only in the window,
// where the byte at offset x lives at window[(base + x) % H].
// `room` = fa + H - (o0 + pos): bytes that can be appended before the oldest
// unflushed kilobyte must go out.
template <uint32_t H>
struct WindowOut {
    uint8_t *base;  // 1 KiB aligned
    uint8_t *win;   // the wave's window (H bytes, LDS)
    uint32_t o0;    // the chunk's first output byte, relative to base (0..1023)
    uint32_t fa;    // relative, multiple of 1 KiB
    uint32_t cap, pos, room;

    __device__ __forceinline__ void init(uint8_t *out, uint32_t capacity, uint8_t *window) {
        // Pointer arithmetic keeps `base` a global pointer: flat stores
        // would also count against the LDS wait counter.
        o0 = (uint32_t)(reinterpret_cast<uintptr_t>(out) & 1023);
        base = out - o0;
        win = window;
        fa = 0;
        cap = capacity;
        pos = 0;
        room = H - o0;
    }
    // base is 1 KiB aligned and H a power of two >= 1 KiB, so the slot of an
    // offset does not depend on base.
    __device__ __forceinline__ uint32_t slot(uint32_t x) const { return x & (H - 1); }

    // Writes the kilobyte [fa, fa + 1024) to HBM, restricted to the bytes of
    // the chunk's range below `limit` (relative).
    __device__ __forceinline__ void flush_block(uint32_t limit) {
        uint32_t a = fa + 16 * lane();
        uint32_t sl = slot(a);
        if (a >= o0 && a + 16 <= limit) {
            *reinterpret_cast<uint4 *>(base + a) = *reinterpret_cast<const uint4 *>(win + sl);
        } else if (a + 16 > o0 && a < limit) {
            for (uint32_t k = 0; k < 16; k++)
                if (a + k >= o0 && a + k < limit) base[a + k] = win[sl + k];
        }
        fa += 1024;
    }
    __device__ __forceinline__ void make_room(uint32_t len) {
        while (room < len) {
            flush_block(o0 + cap);
            room += 1024;
        }
    }
    // As make_room for len <= 258: one flush always suffices.
    __device__ __forceinline__ void make_room1(uint32_t len) {
        if (room < len) {
            flush_block(o0 + cap);
            room += 1024;
        }
    }
    __device__ __forceinline__ void put_literal(uint32_t b) {
        make_room1(1);
        win[slot(o0 + pos)] = (uint8_t)b;  // same byte from every lane
        pos++;
        room--;
    }
    // Back-reference: len bytes from dist bytes back (dist <= pos).  With
    // len > dist the bytes repeat with period dist.
    __device__ __forceinline__ void copy(uint32_t dist, uint32_t len) {
        make_room1(len);
        uint32_t dst = o0 + pos;
        if (dist + len <= H) {
            // Every source byte is still in the window and this copy's own
            // writes only replace bytes older than dist.
            if (dist >= len) {
                for (uint32_t i = lane(); i < len; i += kWave) win[slot(dst + i)] = win[slot(dst - dist + i)];
            } else {
                uint32_t r = lane() % dist, step = kWave % dist;
                for (uint32_t i = lane(); i < len; i += kWave) {
                    win[slot(dst + i)] = win[slot(dst - dist + r)];
                    r += step;
                    if (r >= dist) r -= dist;
                }
            }
        } else {
            // Far reference (dist > H - len >= len): bytes below dst + len - H
            // may be overwritten in the window but are already in HBM.
            int32_t lds_from = (int32_t)(dst + len) - (int32_t)H;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            for (uint32_t i = lane(); i < len; i += kWave) {
                uint32_t q = dst - dist + i;
                // Separate loads keep each access in its own address space (a
                // select between the two pointers would become a flat load).
                uint8_t g = 0;
                if ((int32_t)q < lds_from) g = base[q];
                uint8_t w = win[slot(q)];
                win[slot(dst + i)] = (int32_t)q >= lds_from ? w : g;
            }
        }
        pos += len;
        room -= len;
    }
    // Writes every byte produced so far to HBM.
    __device__ __forceinline__ void finish() {
        uint32_t end = o0 + pos;
        while (fa < end) flush_block(end);
    }
};

// Reads a dynamic block's header up to its code lengths (RFC 1951 3.2.7):
// HLIT, HDIST, HCLEN, the code-length code (built into cltab, 7-bit
// table), then the HLIT + HDIST lengths into lens.  Returns a status.
template <class Ring>
__device__ __forceinline__ int read_code_lengths(Ring &in, BitIn &bi, uint16_t *cltab,
                                                 CodeMeta *meta, uint16_t *sorted, uint8_t *lens,
                                                 uint32_t &hlit, uint32_t &hdist, uint32_t &hclen) {
    const uint32_t l = lane();
    bi.refill(in);
    hlit = bi.peek(5) + 257;
    hdist = ((uint32_t)(bi.buf >> 5) & 31) + 1;
    hclen = ((uint32_t)(bi.buf >> 10) & 15) + 4;
    if (!bi.drop(14)) return CODAG_E_TRUNCATED;
    if (hlit > 286 || hdist > 30) return CODAG_E_CORRUPT;
    if (l < 19) lens[l] = 0;
    __builtin_amdgcn_wave_barrier();
    for (uint32_t i = 0; i < hclen; i++) {
        bi.refill(in);
        uint32_t v = bi.peek(3);
        if (!bi.drop(3)) return CODAG_E_TRUNCATED;
        lens[kCodeLenOrder[i]] = (uint8_t)v;  // same byte from every lane
    }
    __builtin_amdgcn_wave_barrier();
    BuildResult cl = build_table(lens, 19, kCodeLenBits, kCodeLen, cltab, sorted, meta);
    if (cl.left != 0) return CODAG_E_CORRUPT;
    uint32_t idx = 0, total = hlit + hdist, prev = 0;
    while (idx < total) {
        bi.refill(in);
        uint32_t e = uni((uint32_t)cltab[bi.peek(kCodeLenBits)]);
        uint32_t sym = (e >> 4) & 511;
        if (!bi.drop(e & 15)) return CODAG_E_TRUNCATED;
        if (sym < 16) {
            lens[idx] = (uint8_t)sym;  // same byte from every lane
            prev = sym;
            idx++;
            continue;
        }
        uint32_t rep, val;
        if (sym == 16) {
            if (idx == 0) return CODAG_E_CORRUPT;
            rep = 3 + bi.peek(2);
            if (!bi.drop(2)) return CODAG_E_TRUNCATED;
            val = prev;
        } else if (sym == 17) {
            rep = 3 + bi.peek(3);
            if (!bi.drop(3)) return CODAG_E_TRUNCATED;
            val = 0;
        } else {
            rep = 11 + bi.peek(7);
            if (!bi.drop(7)) return CODAG_E_TRUNCATED;
            val = 0;
        }
        if (idx + rep > total) return CODAG_E_CORRUPT;
        for (uint32_t k = l; k < rep; k += kWave) lens[idx + k] = (uint8_t)val;
        prev = val;
        idx += rep;
    }
    __builtin_amdgcn_wave_barrier();
    return CODAG_OK;
}

// Returned by the one-symbol form of inflate_symbols after a literal or a
// copy (not a status).
constexpr int kMore = 1;

// Symbols of one Huffman block, up to and including end-of-block.  Returns
// CODAG_OK at the end of the block or an error status; running past the end
// of input anywhere before that point is reported as CODAG_E_TRUNCATED.
// The loop is kept small and with few exits: literals first, then
// length/distance pairs; everything rare leaves the loop.  With ONE, it
// returns kMore after the first literal or copy.
template <int TB, uint32_t H, bool ONE = false, class Ring>
__device__ __forceinline__ int inflate_symbols(Ring &in, BitIn &bi, WindowOut<H> &o,
                                               DeflateLds<TB, H> *lds, bool have_dist,
                                               uint32_t len_tab, uint32_t dist_tab) {
    int st;
    for (;;) {
        bi.refill1(in);
        uint32_t e = uni((uint32_t)lds->lit[bi.peek(TB)]);
        if (e < (kBase << 13)) {  // literal
            bi.skip(e & 15);
            if (o.pos == o.cap) {
                st = CODAG_E_OVERFLOW;
                break;
            }
            o.put_literal(e >> 4);
            if (ONE) return kMore;
            continue;
        }
        if ((e >> 13) == kSlow) e = slow_symbol(bi, &lds->lit_meta, lds->lit_sorted, kLitLen);
        uint32_t kind = e >> 13;
        if (kind == kLit) {
            bi.skip(e & 15);
            if (o.pos == o.cap) {
                st = CODAG_E_OVERFLOW;
                break;
            }
            o.put_literal((e >> 4) & 255);
            if (ONE) return kMore;
            continue;
        }
        if (kind != kBase) {  // end of block, or an invalid code
            if (kind != kInvalid) bi.skip(e & 15);
            st = kind == kEob ? CODAG_OK : CODAG_E_CORRUPT;
            break;
        }
        // Length, then distance.
        bi.skip(e & 15);
        uint32_t lb = readlane(len_tab, ((e >> 4) & 511) - 257);
        uint32_t ex = lb >> 16;
        uint32_t len = (lb & 0xffff) + bi.peek(ex);
        bi.skip(ex);
        bi.refill1(in);
        uint32_t d = uni((uint32_t)lds->dist[bi.peek(kDistBits)]);
        if ((d >> 13) == kSlow) d = slow_symbol(bi, &lds->dist_meta, lds->dist_sorted, kDist);
        if ((d >> 13) != kBase || !have_dist) {
            if ((d >> 13) == kBadSym && have_dist) bi.skip(d & 15);
            st = CODAG_E_CORRUPT;
            break;
        }
        bi.skip(d & 15);
        uint32_t db = readlane(dist_tab, (d >> 4) & 31);
        uint32_t dex = db >> 16;
        uint32_t dist = (db & 0xffff) + bi.peek(dex);
        bi.skip(dex);
        if (dist > o.pos) {
            st = CODAG_E_CORRUPT;
            break;
        }
        if (o.pos + len > o.cap) {
            st = CODAG_E_OVERFLOW;
            break;
        }
        o.copy(dist, len);
        if (ONE) return kMore;
    }
    return bi.remain < 0 ? CODAG_E_TRUNCATED : st;
}

// ---------------------------------------------------------------------------
// Batched symbol decoding.
//
// The serial dependency of Huffman decoding is the position of the next
// code.  Here every lane decodes, from its own bit offset b + lane, the whole
// token that would start there -- a literal, or a length code with its extra
// bits and the distance code with its extra bits -- with two table lookups
// issued by all lanes at once.  A wave-uniform walk then follows the real
// token starts through those 64 candidates with one lane read per token, and
// collects up to 64 tokens (at most kBatchOut output bytes) in registers.
// The batch is then written out: literals by one store per lane, copies
// whose source lies before the batch lane-parallel (one lane per copy), and
// the few copies that read bytes of the batch itself one after another.
// Anything unusual (codes longer than the tables, invalid codes, an output
// overflow, a distance reaching before the chunk) ends the batch and goes
// through one step of the symbol-at-a-time loop above, so the statuses are
// exactly that loop's.
// ---------------------------------------------------------------------------

constexpr uint32_t kBatchOut = 1024;

// Length and distance bases and extra-bit counts (RFC 1951 section 3.2.5)
// in closed form.
__device__ __forceinline__ uint32_t length_extra(uint32_t k) {  // k = symbol - 257
    return (k < 8 || k == 28) ? 0 : (k >> 2) - 1;
}
__device__ __forceinline__ uint32_t length_base(uint32_t k) {
    return k < 8 ? k + 3 : k == 28 ? 258 : ((4 + (k & 3)) << ((k >> 2) - 1)) + 3;
}
__device__ __forceinline__ uint32_t dist_extra(uint32_t d) { return d < 4 ? 0 : (d >> 1) - 1; }
__device__ __forceinline__ uint32_t dist_base(uint32_t d) {
    return d < 4 ? d + 1 : ((2 + (d & 1)) << ((d >> 1) - 1)) + 1;
}

// Token words: a literal is 1 << 16 | byte, a copy is length << 16 | 0x8000;
// bits 8-13 hold the bits the token takes in the input; 0x4000 marks a
// token the batch cannot take (0x4000: end of block, 0xc000: anything that
// needs the symbol-at-a-time path).
constexpr uint32_t kTokCopy = 0x8000u, kTokStop = 0x4000u, kTokOther = 0xc000u;

// The token starting at bit b + lane (b + 63 at most), as a token word, and
// a copy's distance (0 otherwise).  The lane's 64 input bits come from the
// wave-uniform words s0..s4 (input words b/32 .. b/32 + 4); a length code
// with its extra bits, the distance code and its extra bits take at most 36
// bits.
template <int TB, uint32_t H, bool ALIGNED = false>
__device__ __forceinline__ void lane_token(uint32_t s0, uint32_t s1, uint32_t s2, uint32_t s3,
                                           uint32_t s4, uint32_t b, const DeflateLds<TB, H> *lds,
                                           bool have_dist, uint32_t &info, uint32_t &dist) {
    // ALIGNED: b is a multiple of 32, so lane l starts in word l / 32 and
    // s4 is not needed.
    const uint32_t a = (ALIGNED ? 0u : (b & 31)) + lane();
    const uint32_t k = a >> 5, sh = a & 31;
    const uint32_t wa = ALIGNED ? (k ? s1 : s0) : k == 0 ? s0 : k == 1 ? s1 : s2;
    const uint32_t wb = ALIGNED ? (k ? s2 : s1) : k == 0 ? s1 : k == 1 ? s2 : s3;
    const uint32_t wc = ALIGNED ? (k ? s3 : s2) : k == 0 ? s2 : k == 1 ? s3 : s4;
    const uint64_t x = ((uint64_t)__builtin_amdgcn_alignbit(wc, wb, sh) << 32) |
                       __builtin_amdgcn_alignbit(wb, wa, sh);
    const uint32_t xl = (uint32_t)x;
    const uint32_t e = lds->lit[xl & ((1u << TB) - 1)];
    const uint32_t kind = e >> 13, cl = e & 15, sym = (e >> 4) & 511;
    // Every lane also decodes a length/distance pair from its bits (the
    // distance lookup reads the table whatever the entry was) and the kind
    // picks the result: no branches, so no scalar mask bookkeeping.  The
    // length code and its extra bits end by bit 20, the distance code's
    // index by bit 28, its extra bits by bit 50.
    // The choices are all-ones/zero masks rather than conditionals, which
    // the compiler would turn back into branches.
    const uint32_t kk = (sym - 257) & 31;  // length symbol 257 + kk
    const uint32_t lsmall = 0u - (uint32_t)(kk < 8), l258 = 0u - (uint32_t)(kk == 28);
    const uint32_t ex = ((kk >> 2) - 1) & ~(lsmall | l258);
    const uint32_t lbig = ((4 + (kk & 3)) << (((kk >> 2) - 1) & 31)) + 3;
    const uint32_t lbase = (((kk + 3) & lsmall) | (lbig & ~lsmall) | l258) & (258u | ~l258);
    const uint32_t len = lbase + ((xl >> cl) & ((1u << ex) - 1));
    const uint32_t p2 = cl + ex;
    const uint32_t d = lds->dist[(xl >> p2) & ((1u << kDistBits) - 1)];
    const uint32_t dcl = d & 15, ds = (d >> 4) & 31, q = p2 + dcl;  // distance symbol ds
    const uint32_t dsmall = 0u - (uint32_t)(ds < 4);
    const uint32_t dex = ((ds >> 1) - 1) & ~dsmall;
    const uint32_t dbase = ((ds + 1) & dsmall) | ((((2 + (ds & 1)) << dex) + 1) & ~dsmall);
    const uint32_t dv = dbase + ((uint32_t)(x >> q) & ((1u << dex) - 1));
    const uint32_t m_lit = 0u - (uint32_t)(kind == kLit), m_eob = 0u - (uint32_t)(kind == kEob);
    const uint32_t m_copy = 0u - (uint32_t)(kind == kBase && have_dist && (d >> 13) == kBase);
    info = (((1u << 16) | (cl << 8) | sym) & m_lit) | ((kTokStop | (cl << 8)) & m_eob) |
           (((len << 16) | kTokCopy | ((q + dex) << 8)) & m_copy) | (kTokOther & ~(m_lit | m_eob | m_copy));
    dist = dv & m_copy;
}

// A copy's distance packed into its token word: distance - 1 (15 bits) in
// bits 0-7 and 25-31, which a copy does not otherwise use.
__device__ __forceinline__ uint32_t pack_token(uint32_t info, uint32_t dist) {
    const uint32_t d = dist - 1;
    return (info & kTokCopy) ? info | (d & 0xff) | ((d >> 8) << 25) : info;
}
__device__ __forceinline__ uint32_t token_dist(uint32_t w) { return ((w & 0xff) | ((w >> 25) << 8)) + 1; }
__device__ __forceinline__ uint32_t token_len(uint32_t w) { return (w >> 16) & 511; }

// The walk's view of a candidate: its bits plus, from bit 8, its output
// length plus 12, so one add advances both the bit position within the
// window (bits 0-7) and the batch budget (from bit 8); bit 31 marks a token
// the batch cannot take.  The budget starts at kBudget0 and the batch is
// full once it reaches 1024 (bit 18): at most 60 tokens, and at most 766
// output bytes before the last token, so at most kBatchOut in all.
constexpr uint32_t kWalkStop = 1u << 31, kBudget0 = 257, kBudgetFull = 1u << 18;
constexpr uint32_t kWindowEnd = 1u << 6;  // bit position 64 or beyond
__device__ __forceinline__ uint32_t walk_word(uint32_t info) {
    return (info & kTokStop) ? kWalkStop : ((info >> 8) & 63) + ((((info >> 16) & 511) + 12) << 8);
}

template <int TB, uint32_t H, class Ring>
__device__ __forceinline__ int inflate_batched(Ring &in, BitIn &bi, WindowOut<H> &o,
                                               DeflateLds<TB, H> *lds, bool have_dist,
                                               uint32_t len_tab, uint32_t dist_tab) {
    const uint32_t l = lane();
    // Candidates are decoded for fixed 64-bit windows of the input (lane l:
    // the token at bit 64 w + l).  The walk's tokens are staged, as packed
    // token words, in the code-length scratch (free while symbols decode),
    // one word per token of the batch.
    uint32_t *stage = reinterpret_cast<uint32_t *>(lds->lens);
    constexpr uint32_t kStageSpare = 64;  // 16 words no batch uses (at most 60 tokens)
    static_assert(sizeof(lds->lens) >= 4 * (kStageSpare + 16), "staging space");
    uint32_t p = 8 * bi.next - bi.cnt;  // bit position of the next code
    // Input words [cend - 64, cend), one per lane, read from the ring once
    // per 240 bytes or so; a window takes its four words out with readlane.
    uint32_t cache = 0, cend = 0;
    uint32_t wk = p >> 6;      // the window being walked (64-bit units)
    uint32_t cur = 0, walk = 0;  // packed token and walk word of this lane's candidate in window wk
    bool have = false;
    for (;;) {
        o.make_room(kBatchOut);
        // ---- collect a batch of tokens
        uint32_t ntok = 0;
        uint32_t stop = 0;  // 1 full, 2 end of block, 3 one symbol the slow way
        const uint32_t total0 = o.pos, p0 = p;
        uint32_t budget = kBudget0;
        // Candidates of window wk: every lane's packed token and walk word.
        auto candidates = [&]() {
            const uint32_t wi = 2 * wk;
            if (wi + 4 > cend || wi + 64 < cend) {
                in.ensure(4 * (wi + 64) + 4);
                cache = in.word(wi + l);
                cend = wi + 64;
            }
            const uint32_t c0 = wi + 64 - cend;
            uint32_t info, dist;
            lane_token<TB, H, true>(readlane(cache, c0), readlane(cache, c0 + 1), readlane(cache, c0 + 2),
                                    readlane(cache, c0 + 3), 0u, 64 * wk, lds, have_dist, info, dist);
            cur = pack_token(info, dist);
            walk = walk_word(info);
        };
        if (!have) candidates();
        for (;;) {
            // The walk follows token starts only, one lane read and one add
            // per token, until a token the batch cannot take, the end of the
            // window or a full batch (output bounds are checked lane-parallel
            // once the batch is complete).
            uint32_t T = (p - 64 * wk) | (budget << 8);
            uint32_t w = readlane(walk, T & 63);
            uint64_t mark = 0;
            while (!((w | T) & (kWalkStop | kWindowEnd | kBudgetFull))) {
                // One scalar instruction sets the bit (bit T mod 64).
                asm volatile("s_bitset1_b64 %0, %1" : "+s"(mark) : "s"(T));
                T += w;
                w = readlane(walk, T & 63);
            }
            // Stage this window's tokens in walk order.  Lanes without one
            // write a spare staging word past the batch's 60, so the store
            // needs no lane mask.
            const bool staged = (mark >> l) & 1;
            stage[staged ? ntok + count_below(mark) : kStageSpare + (l & 15)] = cur;
            ntok += (uint32_t)__builtin_popcountll(mark);
            budget = T >> 8;
            const uint32_t t = T & 255;
            p = 64 * wk + t;
            if (t < 64) {  // the batch ends in this window; its candidates stay
                if (budget >= 1024) {
                    stop = 1;  // batch full
                } else {
                    const uint32_t inf = readlane(cur, t);
                    if (inf == (kTokStop | (inf & 0x3f00))) {  // end of block
                        p += (inf >> 8) & 63;
                        stop = 2;
                    } else {
                        stop = 3;
                    }
                }
                have = true;
                break;
            }
            wk++;  // into the next window (a token ends at most 48 bits past this one)
            candidates();
        }
        uint32_t bout = budget - kBudget0 - 12 * ntok;
        __builtin_amdgcn_wave_barrier();
        // Every lane reads a staging word (all in bounds); lanes past the
        // batch drop it.
        const uint32_t staged = stage[l];
        const uint32_t tok = l < ntok ? staged : 0u;
        uint8_t *const trash = reinterpret_cast<uint8_t *>(stage) + 4 * l;
        const uint32_t tdist = (tok & kTokCopy) ? token_dist(tok) : 0u;
        // Each token's output length and offset in the chunk (one prefix sum
        // for the bounds and the writes).
        const uint32_t vlen = token_len(tok);
        const uint32_t before = total0 + wave_inclusive_sum32(vlen) - vlen;
        // Output bounds, lane-parallel: the first token whose distance
        // reaches before the chunk or whose output would pass the end ends
        // the batch, and goes through the symbol-at-a-time path.
        if (ntok) {
            const uint64_t badm = ballot(l < ntok && (tdist > before || before + vlen > o.cap));
            if (badm) {
                const uint32_t j = (uint32_t)__builtin_ctzll(badm);
                const uint32_t bits = l < j ? (tok >> 8) & 63 : 0u;
                ntok = j;
                bout = readlane(before, j) - total0;
                p = p0 + readlane(wave_inclusive_sum32(bits), 63);
                stop = 3;
            }
        }

        // ---- write the batch
        if (ntok) {
            const bool valid = l < ntok;
            const uint32_t len = valid ? vlen : 0;
            const bool is_copy = valid && (tok & kTokCopy);
            const uint32_t start = o.o0 + total0;  // first byte of the batch (window coordinates)
            const uint32_t dst = o.o0 + before;    // this token's first byte
            uint8_t *const lit_to = valid && !is_copy ? o.win + o.slot(dst) : trash;
            *lit_to = (uint8_t)tok;
            const uint32_t src = dst - tdist;
            const bool before = is_copy && src + len <= start;  // source entirely before the batch
            // Bytes below lds_from may be overwritten in the window by this
            // batch; they were flushed to HBM before it started.
            const int32_t lds_from = (int32_t)(start + bout) - (int32_t)H;
            const bool far = ballot(before && (int32_t)src < lds_from) != 0;
            if (!far) {
                // Every source byte is in the window: no global loads, so
                // nothing waits for the flushes still in flight.
                for (uint32_t r = 0; ballot(before && r < len); r += 16) {
                    if (before && r < len) {
                        const uint32_t n = min(len - r, 16u), q0 = src + r;
                        const uint32_t a0 = q0 & ~3u, sh = q0 & 3;
                        uint32_t w[5];
#pragma unroll
                        for (uint32_t j = 0; j < 5; j++)
                            w[j] = *reinterpret_cast<const uint32_t *>(o.win + o.slot(a0 + 4 * j));
#pragma unroll
                        for (uint32_t j = 0; j < 4; j++) {
                            const uint32_t v = __builtin_amdgcn_alignbyte(w[j + 1], w[j], sh);
#pragma unroll
                            for (uint32_t b = 0; b < 4; b++) {
                                // Bytes past the copy go to this lane's slot
                                // of the (already read) token staging words,
                                // so the sixteen stores need no lane masks.
                                uint8_t *to = 4 * j + b < n ? o.win + o.slot(dst + r + 4 * j + b) : trash;
                                *to = (uint8_t)(v >> (8 * b));
                            }
                        }
                    }
                }
            } else {
                // Some source bytes were flushed: read them from HBM.
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                for (uint32_t r = 0; ballot(before && r < len); r += 16) {
                    if (before && r < len) {
                        // Sixteen source bytes as five aligned words (from the
                        // window, and from HBM where they fall below lds_from),
                        // all loads issued before any is used; then byte stores.
                        // HBM words may take up to three bytes either side of the
                        // copy's range: the same aligned word, so the same
                        // allocation; those bytes are discarded.
                        const uint32_t n = min(len - r, 16u), q0 = src + r;
                        const uint32_t a0 = q0 & ~3u, sh = q0 & 3;
                        uint32_t w[5], g[5] = {0, 0, 0, 0, 0};
#pragma unroll
                        for (uint32_t j = 0; j < 5; j++)
                            w[j] = *reinterpret_cast<const uint32_t *>(o.win + o.slot(a0 + 4 * j));
                        const int32_t nglob = lds_from - (int32_t)q0;  // leading bytes taken from HBM
                        if (nglob > 0) {
                            const uint32_t *gp = reinterpret_cast<const uint32_t *>(o.base + a0);
#pragma unroll
                            for (uint32_t j = 0; j < 5; j++) g[j] = gp[j];
                        }
                        // Every loaded word is used here (masked), so no load
                        // is left in flight past this loop: the wait for it
                        // would also wait for every flush store.
#pragma unroll
                        for (uint32_t j = 0; j < 4; j++) {
                            uint32_t v = __builtin_amdgcn_alignbyte(w[j + 1], w[j], sh);
                            const uint32_t gv = __builtin_amdgcn_alignbyte(g[j + 1], g[j], sh);
                            const int32_t kb = nglob - 4 * (int32_t)j;  // bytes of this word from HBM
                            const uint32_t m = kb >= 4 ? 0xffffffffu : kb <= 0 ? 0u : (1u << (8 * kb)) - 1;
                            v = (gv & m) | (v & ~m);
#pragma unroll
                            for (uint32_t b = 0; b < 4; b++) {
                                uint8_t *to = 4 * j + b < n ? o.win + o.slot(dst + r + 4 * j + b) : trash;
                                *to = (uint8_t)(v >> (8 * b));
                            }
                        }
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            // Copies that read bytes of this batch, in order (their sources
            // are recent, so always in the window).
            uint64_t m = ballot(is_copy && !before);
            while (m) {
                uint32_t k = (uint32_t)__builtin_ctzll(m);
                m &= m - 1;
                uint32_t cd = readlane(dst, k), cs = readlane(tdist, k), cl = readlane(len, k);
                if (cs >= cl) {
                    for (uint32_t i = l; i < cl; i += kWave) o.win[o.slot(cd + i)] = o.win[o.slot(cd - cs + i)];
                } else {
                    uint32_t rr = l % cs, step = kWave % cs;
                    for (uint32_t i = l; i < cl; i += kWave) {
                        o.win[o.slot(cd + i)] = o.win[o.slot(cd - cs + rr)];
                        rr += step;
                        if (rr >= cs) rr -= cs;
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
            o.pos += bout;
            o.room -= bout;
        }
        if (stop == 1) continue;
        bi.seek(in, p >> 3);
        bi.skip(p & 7);
        if (stop == 2) return bi.remain < 0 ? CODAG_E_TRUNCATED : CODAG_OK;
        int st = inflate_symbols<TB, H, true>(in, bi, o, lds, have_dist, len_tab, dist_tab);
        if (st != kMore) return st;
        p = 8 * bi.next - bi.cnt;
        // A window's candidates depend only on its input bits: if the next
        // token is still in window wk, they stay.
        have = have && (p >> 6) == wk;
        wk = p >> 6;
    }
}

// Leader-lane symbol loop: lane 0 decodes the token at the current bit
// position (the same per-lane token decoder the batched path runs on every
// lane), writes it to an LDS slot, and the wave reads it back and writes the
// literal or copy.  Every token takes one decode by one lane and one LDS
// round trip.  Anything but a plain literal or an in-range copy goes through
// one step of the symbol-at-a-time loop, so statuses are that loop's.
template <int TB, uint32_t H, class Ring>
__device__ __forceinline__ int inflate_leader(Ring &in, BitIn &bi, WindowOut<H> &o,
                                              DeflateLds<TB, H> *lds, bool have_dist,
                                              uint32_t len_tab, uint32_t dist_tab) {
    uint32_t p = 8 * bi.next - bi.cnt;  // bit position of the next code
    uint32_t *slot = reinterpret_cast<uint32_t *>(lds->lens);  // free while symbols decode
    for (;;) {
        const uint32_t wi = p >> 5;
        in.ensure(4 * (wi + 5) + 4);
        if (lane() == 0) {
            uint32_t info, dist;
            lane_token<TB, H>(in.word(wi), in.word(wi + 1), in.word(wi + 2), in.word(wi + 3),
                              in.word(wi + 4), p, lds, have_dist, info, dist);
            slot[0] = info;
            slot[1] = dist;
        }
        __builtin_amdgcn_wave_barrier();
        const uint32_t info = uni(slot[0]), dist = uni(slot[1]);
        __builtin_amdgcn_wave_barrier();
        const uint32_t bits = (info >> 8) & 63;
        if (!(info & kTokStop)) {
            if (!(info & kTokCopy)) {
                if (o.pos < o.cap) {
                    o.put_literal(info & 0xff);
                    p += bits;
                    continue;
                }
            } else {
                const uint32_t len = info >> 16;
                if (dist <= o.pos && o.pos + len <= o.cap) {
                    o.copy(dist, len);
                    p += bits;
                    continue;
                }
            }
        }
        bi.seek(in, p >> 3);
        bi.skip(p & 7);
        int st = inflate_symbols<TB, H, true>(in, bi, o, lds, have_dist, len_tab, dist_tab);
        if (st != kMore) return st;
        p = 8 * bi.next - bi.cnt;
    }
}

// MODE kAllLanes: the batched token decoder above (every lane decodes a
// candidate token); kLeaderLane: lane 0 alone decodes each token and hands
// it to the wave through LDS (the single-thread decoding CODAG compares
// against, Section V-E).
enum : int { kAllLanes = 0, kLeaderLane = 1 };

// With `made` non-null the output range is a capacity: a final block that
// ends inside it is OK and *made receives the bytes produced.
template <int TB, uint32_t H, int MODE = kAllLanes, class Ring>
__device__ __forceinline__ int decode_deflate(Ring &in, uint8_t *out, uint32_t cap,
                                              DeflateLds<TB, H> *lds, uint32_t *made = nullptr) {
    const uint32_t l = lane();
    BitIn bi;
    bi.seek(in, in.skip);
    WindowOut<H> o;
    o.init(out, cap, lds->window);
    const uint32_t len_tab = length_lane_table(), dist_tab = distance_lane_table();
    bool fixed_ready = false;
    bool have_dist = true;
    int st = CODAG_OK;

    for (;;) {
        bi.refill(in);
        uint32_t hdr = bi.peek(3);
        if (!bi.drop(3)) { st = CODAG_E_TRUNCATED; break; }
        uint32_t btype = hdr >> 1;
        bool last = hdr & 1;
        if (btype == 0) {
            // Stored block: byte-align, LEN, NLEN = ~LEN, then LEN raw bytes.
            bi.drop(bi.cnt & 7);
            bi.refill(in);
            uint32_t len = bi.peek(16), nlen = (uint32_t)(bi.buf >> 16) & 0xffff;
            if (!bi.drop(32)) { st = CODAG_E_TRUNCATED; break; }
            if (nlen != (~len & 0xffff)) { st = CODAG_E_CORRUPT; break; }
            if (o.pos + len > cap) { st = CODAG_E_OVERFLOW; break; }
            uint32_t p = bi.byte_pos();
            if (p + len > in.gend) { st = CODAG_E_TRUNCATED; break; }
            for (uint32_t done = 0; done < len;) {
                uint32_t piece = min(len - done, Ring::kFetch / 2);
                o.make_room(piece);
                in.ensure(p + done + piece + 4);
                uint32_t dst = o.o0 + o.pos;
                for (uint32_t i = l; i < piece; i += kWave) {
                    uint32_t q = p + done + i;
                    o.win[o.slot(dst + i)] = (uint8_t)(in.word(q >> 2) >> (8 * (q & 3)));
                }
                o.pos += piece;
                o.room -= piece;
                done += piece;
            }
            bi.seek(in, p + len);
        } else if (btype == 3) {
            st = CODAG_E_CORRUPT;
            break;
        } else {
            if (btype == 1) {
                if (!fixed_ready) {
                    for (uint32_t s = l; s < 288 + 32; s += kWave) {
                        uint32_t v = s < 144 ? 8 : s < 256 ? 9 : s < 280 ? 7 : s < 288 ? 8 : 5;
                        lds->lens[s] = (uint8_t)v;
                    }
                    __builtin_amdgcn_wave_barrier();
                    build_table(lds->lens, 288, TB, kLitLen, lds->lit, lds->lit_sorted, &lds->lit_meta);
                    build_table(lds->lens + 288, 32, kDistBits, kDist, lds->dist, lds->dist_sorted,
                                &lds->dist_meta);
                    fixed_ready = true;
                }
                have_dist = true;
            } else {
                // Dynamic block header (RFC 1951 section 3.2.7).
                fixed_ready = false;
                uint32_t hlit, hdist, hclen;
                st = read_code_lengths(in, bi, lds->dist, &lds->dist_meta, lds->dist_sorted,
                                       lds->lens, hlit, hdist, hclen);
                if (st) break;
                __builtin_amdgcn_wave_barrier();
                if (uni((uint32_t)lds->lens[256]) == 0) { st = CODAG_E_CORRUPT; break; }
                BuildResult lr = build_table(lds->lens, hlit, TB, kLitLen, lds->lit, lds->lit_sorted,
                                             &lds->lit_meta);
                if (lr.left < 0 || (lr.left > 0 && !(lr.total == 1 && lr.ones == 1))) {
                    st = CODAG_E_CORRUPT;
                    break;
                }
                BuildResult dr = build_table(lds->lens + hlit, hdist, kDistBits, kDist, lds->dist,
                                             lds->dist_sorted, &lds->dist_meta);
                if (dr.left < 0 || (dr.left > 0 && dr.total != 0 && !(dr.total == 1 && dr.ones == 1))) {
                    st = CODAG_E_CORRUPT;
                    break;
                }
                have_dist = dr.total != 0;
            }
            if constexpr (MODE == kLeaderLane)
                st = inflate_leader<TB, H>(in, bi, o, lds, have_dist, len_tab, dist_tab);
            else
                st = inflate_batched<TB, H>(in, bi, o, lds, have_dist, len_tab, dist_tab);
            if (st) break;
        }
        if (last) break;
    }
    o.finish();
    if (st) return st;
    if (made) {
        *made = o.pos;
        return CODAG_OK;
    }
    return o.pos == cap ? CODAG_OK : CODAG_E_UNDERFLOW;
}

}  // namespace codag
