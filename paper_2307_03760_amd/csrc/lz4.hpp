// LZ4 block decode, one wavefront per chunk, on the same two primitives as
// Deflate: the LDS input ring (input_stream) and the LDS history window with
// kilobyte flushes to HBM (output_stream).  CODAG presents new codecs as
// device functions written against these two streams (Section III, Section
// IV-E); LZ4 is the byte-aligned member of the LZ77 family, so the whole
// decode is the wave-uniform sequence parse plus lane-parallel copies.
//
// A block is a list of sequences: a token byte (literal count in the high
// nibble, match length minus 4 in the low one; a nibble of 15 continues in
// bytes that add to it until one below 255), the literals, a 2-byte
// little-endian offset and the match length's continuation bytes.  The
// block ends right after some sequence's literals.
//
// Status order, field by field as they are read: a field cut off by the end
// of the chunk is TRUNCATED; a literal run longer than the output range left
// is OVERFLOW (before its bytes are looked at, as for a stored Deflate
// block); offset 0 or one past the bytes produced is CORRUPT (no dictionary)
// once the sequence's match length is read; a match past the range is
// OVERFLOW; a block that ends before the range is full is UNDERFLOW unless
// the range is a capacity.
#pragma once

#include "../../include/codag.h"
#include "deflate.hpp"
#include "stream.hpp"

namespace codag {

template <uint32_t H>
struct Lz4Lds {
    uint8_t window[H];  // output byte at absolute address a lives at window[a % H]
};

// One byte at position q, the same on every lane (needs ensure(q + 4)).
template <class Ring>
__device__ __forceinline__ uint32_t lz4_byte(const Ring &in, uint32_t q) {
    return (uni(in.word(q >> 2)) >> (8 * (q & 3))) & 255;
}

// Adds continuation bytes from position q on to len (a nibble was 15):
// returns the position after the last one, or 0 if the chunk ends first.
template <class Ring>
__device__ __forceinline__ uint32_t lz4_more(Ring &in, uint32_t q, uint32_t end, uint32_t &len) {
    for (;;) {
        if (q >= end) return 0;
        in.ensure(q + 4);
        uint32_t b = lz4_byte(in, q++);
        // A run over 2^32 cannot fit any output range; saturate instead of
        // wrapping so the range check still fails.
        len = len + b < len ? 0xffffffffu : len + b;
        if (b != 255) return q;
    }
}

// One sequence the slow, general way (any field length, the last sequence,
// every status): returns kLz4More to go on, else the block's status (OK when
// this was its last sequence).
enum : int { kLz4More = 1 };

template <uint32_t H, class Ring>
__device__ __forceinline__ int lz4_sequence(Ring &in, WindowOut<H> &o, uint32_t &p, uint32_t end,
                                            uint32_t cap) {
    const uint32_t l = lane();
    // The sequence head: 17 bytes from the token on, enough for a token,
    // up to 14 literals and the offset.
    in.ensure(p + 20);
    const uint32_t w = p >> 2, sh = 8 * (p & 3);
    const uint32_t a = in.word_at(w, 0), b = in.word_at(w, 1), c = in.word_at(w, 2),
                   d = in.word_at(w, 3), e = in.word_at(w, 4);
    const uint32_t h0 = uni(__builtin_amdgcn_alignbit(b, a, sh));
    const uint32_t h1 = __builtin_amdgcn_alignbit(c, b, sh);
    const uint32_t h2 = __builtin_amdgcn_alignbit(d, c, sh);
    const uint32_t h3 = __builtin_amdgcn_alignbit(e, d, sh);
    const uint32_t h4 = e >> sh;
    const uint32_t tok = h0 & 255;
    uint32_t lit = tok >> 4, q = p + 1;
    if (lit == 15) {
        q = lz4_more(in, q, end, lit);
        if (!q) return CODAG_E_TRUNCATED;
    }
    if (lit > cap - o.pos) return CODAG_E_OVERFLOW;
    if (lit > end - q) return CODAG_E_TRUNCATED;
    if (lit < 15) {
        // Literals straight from the head: byte 1 + i for lane i.
        o.make_room1(lit);
        const uint32_t j = 1 + l;
        const uint32_t v = j < 4 ? h0 : j < 8 ? h1 : j < 12 ? h2 : h3;
        if (l < lit) o.win[o.slot(o.o0 + o.pos + l)] = (uint8_t)(v >> (8 * (j & 3)));
        o.pos += lit;
        o.room -= lit;
    } else {
        for (uint32_t k = 0; k < lit;) {
            const uint32_t piece = min(lit - k, Ring::kFetch / 2);
            o.make_room(piece);
            in.ensure(q + k + piece + 4);
            const uint32_t dst = o.o0 + o.pos;
            for (uint32_t i = l; i < piece; i += kWave) {
                uint32_t x = q + k + i;
                o.win[o.slot(dst + i)] = (uint8_t)(in.word(x >> 2) >> (8 * (x & 3)));
            }
            o.pos += piece;
            o.room -= piece;
            k += piece;
        }
    }
    q += lit;
    if (q == end) return CODAG_OK;  // the last sequence carries no match
    if (end - q < 2) return CODAG_E_TRUNCATED;
    uint32_t off;
    if (q + 2 <= p + 17) {
        const uint32_t k = q - p;  // 1..15: the offset is still in the head
        const uint32_t lo = k < 4 ? h0 : k < 8 ? h1 : k < 12 ? h2 : h3;
        const uint32_t hi = k < 3 ? h0 : k < 7 ? h1 : k < 11 ? h2 : k < 15 ? h3 : h4;
        off = uni(((lo >> (8 * (k & 3))) & 255) | (((hi >> (8 * ((k + 1) & 3))) & 255) << 8));
    } else {
        in.ensure(q + 6);
        off = lz4_byte(in, q) | lz4_byte(in, q + 1) << 8;
    }
    q += 2;
    uint32_t mlen = tok & 15;
    if (mlen == 15) {
        q = lz4_more(in, q, end, mlen);
        if (!q) return CODAG_E_TRUNCATED;
    }
    mlen = mlen + 4 < mlen ? 0xffffffffu : mlen + 4;
    if (off == 0 || off > o.pos) return CODAG_E_CORRUPT;
    if (mlen > cap - o.pos) return CODAG_E_OVERFLOW;
    // Pieces of at most 256 bytes keep every copy within one flush and well
    // under half the window; each piece repeats the bytes `off` back, so
    // splitting a match does not change what it writes.
    for (uint32_t k = 0; k < mlen;) {
        const uint32_t piece = min(mlen - k, 256u);
        o.copy(off, piece);
        k += piece;
    }
    p = q;
    return kLz4More;
}

__device__ __forceinline__ uint64_t lz4_bit(uint32_t x) { return x < 64 ? 1ull << x : 0ull; }

// Batches of short sequences.  Every lane parses the sequence that would
// start at its own byte of a 64-byte input window (only short fields: at
// most 14 literals, a match of at most 18 bytes).  The real sequence starts
// are the chain of next-start links from the window's first byte; each lane
// gathers, by lane permutes, where its links lead over eight steps and which
// lanes they pass, so a wave-uniform walk covers eight sequences with two
// lane reads.  The batch is the chain's prefix up to anything the general
// step must judge: a long field, the block's last sequence, a cut-off
// stream, output past the range, an offset reaching before the chunk's
// output (the last two found with a prefix sum over the chain).  It holds at
// most 21 sequences and 672 output bytes and is written with the lanes of
// its sequences: all literals first, then every match whose source lies
// before the batch (from the LDS window, or from output already flushed to
// HBM), then the matches that read the batch's own output, in rounds: each
// round copies every pending match whose source ends before the lowest
// pending match's output, the bytes before that being final.
template <uint32_t H, class Ring>
__device__ __forceinline__ int decode_lz4(Ring &in, uint8_t *out, uint32_t cap, Lz4Lds<H> *lds,
                                          uint32_t *made = nullptr) {
    static_assert(H >= 2048, "a batch and its flush must fit the window");
    const uint32_t l = lane();
    WindowOut<H> o;
    o.init(out, cap, lds->window);
    const uint32_t end = in.gend;
    uint32_t p = in.skip;
    int st = CODAG_OK;
    for (;;) {
        if (p >= end) { st = CODAG_E_TRUNCATED; break; }
        in.ensure(p + kWave + 20);
        // This lane's candidate: 17 bytes from p + l.
        const uint32_t x = p + l, wx = x >> 2, sx = 8 * (x & 3);
        const uint32_t a = in.word_at(wx, 0), b = in.word_at(wx, 1), c = in.word_at(wx, 2),
                       d = in.word_at(wx, 3), e = in.word_at(wx, 4);
        const uint32_t g0 = __builtin_amdgcn_alignbit(b, a, sx), g1 = __builtin_amdgcn_alignbit(c, b, sx),
                       g2 = __builtin_amdgcn_alignbit(d, c, sx), g3 = __builtin_amdgcn_alignbit(e, d, sx),
                       g4 = e >> sx;
        const uint32_t tok = g0 & 255, lit = tok >> 4, ml = tok & 15;
        const uint32_t k = 1 + lit;  // the offset's first byte, 1..15 when lit < 15
        const uint32_t lo = k < 4 ? g0 : k < 8 ? g1 : k < 12 ? g2 : g3;
        const uint32_t hi = k < 3 ? g0 : k < 7 ? g1 : k < 11 ? g2 : k < 15 ? g3 : g4;
        const uint32_t off = ((lo >> (8 * (k & 3))) & 255) | (((hi >> (8 * ((k + 1) & 3))) & 255) << 8);
        const uint32_t inl = 3 + lit, outl = lit + ml + 4, mlen = ml + 4;
        // What a sequence needs on its own: short fields, a nonzero offset,
        // its bytes inside the chunk and followed by more (the last sequence
        // has no offset).
        const bool ok = lit < 15 && ml < 15 && off != 0 && x + inl <= end;
        // Links: the next start (64 = none in this window, or stop here).
        const uint32_t n1 = ok ? min(l + inl, 64u) : 64u;
        const uint32_t n2 = lane_follow(n1, n1);
        const uint32_t n3 = lane_follow(n1, n2);
        const uint32_t n4 = lane_follow(n1, n3);
        const uint64_t m4 = lz4_bit(l) | lz4_bit(n1) | lz4_bit(n2) | lz4_bit(n3);
        const uint32_t n8 = lane_follow(n4, n4);
        const uint32_t m8h = lane_pull((uint32_t)(m4 >> 32), n4), m8l = lane_pull((uint32_t)m4, n4);
        const uint64_t m8 = m4 | (n4 < 64 ? (uint64_t)m8h << 32 | m8l : 0ull);
        // Links only lead forward, so eight steps of eight cover the window;
        // the bound is a second guard.
        uint64_t chain = 0;
        for (uint32_t t = 0, step = 0; t < 64 && step < 8; step++) {
            chain |= readlane64(m8, t);
            t = readlane(n8, t);
        }
        // The chain runs through sequences that are fine on their own and
        // ends at (and includes) the first that is not, if any.
        uint64_t exe = chain & ballot(ok);
        const bool on = (exe >> l) & 1;
        const uint32_t my_out = on ? outl : 0u;
        const uint32_t incl = wave_inclusive_sum32(my_out), before = incl - my_out;
        const uint64_t fm = ballot(on && (incl > cap - o.pos || (off > lit && off - lit > o.pos + before)));
        if (fm) exe &= (fm & (0 - fm)) - 1;
        if (!exe) {
            st = lz4_sequence(in, o, p, end, cap);
            if (st != kLz4More) break;
            st = CODAG_OK;
            continue;
        }
        const uint32_t last = 63 - (uint32_t)__builtin_clzll(exe);
        const uint32_t orel = readlane(incl, last);
        const uint32_t s_end = last + 3 + (readlane(tok, last) >> 4);

        const bool mine = (exe >> l) & 1;
        o.make_room(orel);
        const uint32_t bo = o.o0 + o.pos;  // the batch's first output byte
        const uint32_t dl = bo + before;   // this sequence's literals
        const uint32_t dm = dl + lit, src = dm - off;
        // Literals (byte 1 + i of the candidate is literal i).
        for (uint32_t i = 0; i < 14; i++) {
            if (!ballot(mine && i < lit)) break;
            const uint32_t j = 1 + i;
            const uint32_t v = j < 4 ? g0 : j < 8 ? g1 : j < 12 ? g2 : g3;
            if (mine && i < lit) o.win[o.slot(dl + i)] = (uint8_t)(v >> (8 * (j & 3)));
        }
        // Matches whose source lies wholly before the batch: bytes from
        // lds_from on are still in the window, older ones are in HBM.
        const bool indep = mine && src + mlen <= bo;
        const int32_t lds_from = (int32_t)(bo + orel) - (int32_t)H;
        if (ballot(indep && (int32_t)src < lds_from))
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        for (uint32_t i = 0; i < 18; i += 6) {
            if (!ballot(indep && i < mlen)) break;
            uint8_t v[6];
#pragma unroll
            for (uint32_t t = 0; t < 6; t++) {
                const uint32_t q = src + i + t;
                uint8_t g = 0, w = 0;
                if (indep && i + t < mlen) {
                    if ((int32_t)q < lds_from) g = o.base[q];
                    w = o.win[o.slot(q)];
                }
                v[t] = (int32_t)q < lds_from ? g : w;
            }
#pragma unroll
            for (uint32_t t = 0; t < 6; t++)
                if (indep && i + t < mlen) o.win[o.slot(dm + i + t)] = v[t];
        }
        // Matches that read the batch (their sources are all in the window).
        uint64_t pend = ballot(mine && !indep);
        while (pend) {
            const uint32_t t = (uint32_t)__builtin_ctzll(pend);
            const uint32_t front = readlane(dm, t);
            const bool ready = ((pend >> l) & 1) && src + mlen <= front;
            const uint64_t rm = ballot(ready);
            if (!rm) {
                // The lowest pending match overlaps its own output: it
                // repeats its first `off` bytes, one period at a time.
                const uint32_t mo = readlane(off, t), mn = readlane(mlen, t), ms = front - mo;
                for (uint32_t i = 0; i < mn; i += mo) {
                    const uint32_t n = min(mo, mn - i);
                    uint8_t v = 0;
                    if (l < n) v = o.win[o.slot(ms + i + l)];
                    if (l < n) o.win[o.slot(front + i + l)] = v;
                }
                pend &= pend - 1;
                continue;
            }
            for (uint32_t i = 0; i < 18; i += 6) {
                if (!ballot(ready && i < mlen)) break;
                uint8_t v[6];
#pragma unroll
                for (uint32_t t2 = 0; t2 < 6; t2++)
                    v[t2] = ready && i + t2 < mlen ? o.win[o.slot(src + i + t2)] : 0;
#pragma unroll
                for (uint32_t t2 = 0; t2 < 6; t2++)
                    if (ready && i + t2 < mlen) o.win[o.slot(dm + i + t2)] = v[t2];
            }
            pend &= ~rm;
        }
        o.pos += orel;
        o.room -= orel;
        p += s_end;
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
