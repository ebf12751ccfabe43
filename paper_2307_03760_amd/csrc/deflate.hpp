// Deflate (RFC 1951) decoding by one wavefront.
//
// CODAG (Section II-A, III) locates Deflate's cost in Huffman decoding and
// dictionary copies.  Here the symbol chain is wave-uniform scalar code: a
// 64-bit bit buffer in scalar registers, refilled one 32-bit word at a time
// from the LDS input ring, and a lookup per symbol in LDS tables that the
// whole wave builds in parallel for each block.  Literals are staged in a
// vector register (one byte slot per lane byte, 256 bytes per wave) and
// written out together ("write_byte" in Section IV-B); back-references are
// copied by all lanes at once ("memcpy", Section IV-F), including the
// overlapping case where the length exceeds the distance.
#pragma once

#include "../../include/codag.h"
#include "stream.hpp"

namespace codag {

// Table entry: bits 0-3 code length, 4-7 extra bits, 8-10 kind, 16-31 value.
enum : uint32_t {
    kLit = 0,     // literal byte
    kBase = 1,    // length or distance: value = base, plus `extra` bits
    kEob = 2,     // end of block
    kSlow = 3,    // code longer than the table: canonical decode
    kInvalid = 4, // no code starts with these bits
    kBadSym = 5,  // a code for a symbol that may not appear (286, 287; 30, 31)
    kSym = 6,     // code-length alphabet symbol
};

__device__ __forceinline__ uint32_t entry(uint32_t kind, uint32_t len, uint32_t extra, uint32_t value) {
    return len | (extra << 4) | (kind << 8) | (value << 16);
}

enum TableUse { kLitLen = 0, kDist = 1, kCodeLen = 2 };

// The symbol's meaning, from RFC 1951 section 3.2.5.
__device__ __forceinline__ uint32_t symbol_entry(int use, uint32_t s, uint32_t len) {
    if (use == kCodeLen) return entry(kSym, len, 0, s);
    if (use == kLitLen) {
        if (s < 256) return entry(kLit, len, 0, s);
        if (s == 256) return entry(kEob, len, 0, 0);
        if (s > 285) return entry(kBadSym, len, 0, 0);
        if (s == 285) return entry(kBase, len, 0, 258);
        uint32_t k = s - 257;
        if (k < 8) return entry(kBase, len, 0, k + 3);
        uint32_t e = (k >> 2) - 1;
        return entry(kBase, len, e, ((4 + (k & 3)) << e) + 3);
    }
    if (s > 29) return entry(kBadSym, len, 0, 0);
    if (s < 4) return entry(kBase, len, 0, s + 1);
    uint32_t e = (s >> 1) - 1;
    return entry(kBase, len, e, ((2 + (s & 1)) << e) + 1);
}

// Per-code metadata kept for the slow path: count, first code and offset
// into `sorted` for each code length 1..15.
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

// Builds the lookup table (2^tb entries) for the canonical code whose
// lengths are lens[0..n) (n <= 320), lane-parallel.
__device__ __forceinline__ BuildResult build_table(const uint8_t *lens, uint32_t n, uint32_t tb, int use,
                                   uint32_t *tab, uint16_t *sorted, CodeMeta *meta) {
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
        for (uint32_t i = l; i < (1u << tb); i += kWave) tab[i] = entry(kInvalid, 0, 0, 0);
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
                uint32_t e = symbol_entry(use, s, m);
                for (uint32_t k = 0; k < (1u << (tb - m)); k++) tab[rev | (k << m)] = e;
            } else {
                uint32_t prefix = code >> (m - tb);
                tab[__builtin_bitreverse32(prefix) >> (32 - tb)] = entry(kSlow, 0, 0, 0);
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    return r;
}

// The Huffman tables one wave keeps in LDS while inflating.
template <int TB>
struct DeflateLds {
    uint32_t lit[1u << TB];
    uint32_t dist[256];  // 8-bit distance table; also the code-length table (7 bits)
    CodeMeta lit_meta, dist_meta;
    uint16_t lit_sorted[288];
    uint16_t dist_sorted[32];
    uint8_t lens[320];
};
constexpr uint32_t kDistBits = 8;

// Order in which the code-length code's lengths are sent (RFC 1951 3.2.7).
__constant__ const uint8_t kCodeLenOrder[19] = {16, 17, 18, 0, 8,  7, 9,  6, 10, 5,
                                                11, 4,  12, 3, 13, 2, 14, 1, 15};
constexpr uint32_t kCodeLenBits = 7;

// Wave-uniform LSB-first bit reader over the ring.
struct BitIn {
    uint64_t buf;     // valid bits are the low `cnt`
    uint32_t cnt;
    uint32_t next;    // byte position of the next (aligned) word to load
    int64_t remain;   // input bits not yet consumed (negative: past the end)

    __device__ __forceinline__ void seek(InRing &in, uint32_t pos) {
        if (pos >= in.loaded + kFetchBytes) in.restart(pos);
        uint32_t a = pos & ~3u;
        in.ensure(a + 4);
        uint32_t w = uni(in.word(a >> 2));
        uint32_t sh = 8 * (pos & 3);
        buf = w >> sh;
        cnt = 32 - sh;
        next = a + 4;
        remain = 8ll * ((int64_t)in.gend - (int64_t)pos);
    }
    __device__ __forceinline__ void refill(InRing &in) {
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
        remain -= n;
        return remain >= 0;
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
            return symbol_entry(use, s, len);
        }
    }
    return entry(kInvalid, 0, 0, 0);
}

// Output side: staged literals plus direct byte-range writes.
struct ByteOut {
    uint8_t *base;    // the chunk's output range
    uint32_t cap;
    uint32_t pos;     // bytes produced (staged ones included)
    uint32_t spos;    // position of the first staged byte
    uint32_t stage;   // this lane's 4 staged bytes (slot = pos - spos)

    __device__ __forceinline__ void flush() {
        uint32_t n = pos - spos;
        if (n == 0) return;
        uint32_t j = 4 * lane();
        if (j < n) store_bytes(base + spos + j, stage, min(4u, n - j));
        spos = pos;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    }
    __device__ __forceinline__ void put_literal(uint32_t b) {
        uint32_t slot = pos - spos;
        uint32_t sh = 8 * (slot & 3);
        if (lane() == (slot >> 2)) stage = (stage & ~(0xffu << sh)) | (b << sh);
        pos++;
        if (pos - spos == 4 * kWave) flush();
    }
    // Back-reference: len bytes from dist bytes back (dist <= pos).  Bytes
    // repeat with period dist when len > dist.
    __device__ __forceinline__ void copy(uint32_t dist, uint32_t len) {
        flush();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        uint8_t *dst = base + pos;
        const uint8_t *src = base + pos - dist;
        if (dist >= len) {
            for (uint32_t i = lane(); i < len; i += kWave) dst[i] = src[i];
        } else {
            uint32_t r = lane() % dist, step = kWave % dist;
            for (uint32_t i = lane(); i < len; i += kWave) {
                dst[i] = src[r];
                r += step;
                if (r >= dist) r -= dist;
            }
        }
        pos += len;
        spos = pos;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    }
};

// Copies len bytes from global input to the output (stored blocks).
__device__ __forceinline__ void copy_stored(uint8_t *dst, const uint8_t *src, uint32_t len) {
    const uint32_t l = lane();
    // Head: bring the destination to a 4-byte boundary.
    uint32_t head = (uint32_t)((4 - ((uintptr_t)dst & 3)) & 3);
    if (head > len) head = len;
    if (l < head) dst[l] = src[l];
    dst += head;
    src += head;
    len -= head;
    uint32_t words = len >> 2;
    uint32_t a = (uint32_t)((uintptr_t)src & 3);
    const uint32_t *s4 = reinterpret_cast<const uint32_t *>(src - a);
    uint32_t *d4 = reinterpret_cast<uint32_t *>(dst);
    for (uint32_t k0 = 0; k0 < words; k0 += 4 * kWave) {
        uint32_t v[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            uint32_t k = k0 + j * kWave + l;
            if (k < words) {
                uint32_t lo = s4[k];
                uint32_t hi = a ? s4[k + 1] : 0;
                v[j] = a ? __builtin_amdgcn_alignbyte(hi, lo, a) : lo;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
            uint32_t k = k0 + j * kWave + l;
            if (k < words) d4[k] = v[j];
        }
    }
    uint32_t tail = len & 3, t0 = words * 4;
    if (l < tail) dst[t0 + l] = src[t0 + l];
}

template <int TB>
__device__ __forceinline__ int decode_deflate(InRing &in, uint8_t *out, uint32_t cap, DeflateLds<TB> *lds) {
    const uint32_t l = lane();
    BitIn bi;
    bi.seek(in, in.skip);
    ByteOut o;
    o.base = out;
    o.cap = cap;
    o.pos = 0;
    o.spos = 0;
    o.stage = 0;
    bool fixed_ready = false;
    uint32_t lmask = (1u << TB) - 1, dmask = (1u << kDistBits) - 1;
    bool have_dist = true;

    for (;;) {
        bi.refill(in);
        uint32_t hdr = bi.peek(3);
        if (!bi.drop(3)) return CODAG_E_TRUNCATED;
        uint32_t btype = hdr >> 1;
        bool last = hdr & 1;
        if (btype == 0) {
            // Stored block: byte-align, LEN, NLEN = ~LEN, then LEN raw bytes.
            uint32_t pad = bi.cnt & 7;
            bi.drop(pad);
            bi.refill(in);
            uint32_t len = bi.peek(16), nlen = (uint32_t)(bi.buf >> 16) & 0xffff;
            if (!bi.drop(32)) return CODAG_E_TRUNCATED;
            if (nlen != (~len & 0xffff)) return CODAG_E_CORRUPT;
            if (o.pos + len > cap) return CODAG_E_OVERFLOW;
            uint32_t p = bi.byte_pos();
            if (p + len > in.gend) return CODAG_E_TRUNCATED;
            o.flush();
            copy_stored(o.base + o.pos, in.gbase + p, len);
            o.pos += len;
            o.spos = o.pos;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            bi.seek(in, p + len);
        } else if (btype == 3) {
            return CODAG_E_CORRUPT;
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
                bi.refill(in);
                uint32_t hlit = bi.peek(5) + 257;
                uint32_t hdist = ((uint32_t)(bi.buf >> 5) & 31) + 1;
                uint32_t hclen = ((uint32_t)(bi.buf >> 10) & 15) + 4;
                if (!bi.drop(14)) return CODAG_E_TRUNCATED;
                if (hlit > 286 || hdist > 30) return CODAG_E_CORRUPT;
                if (l < 19) lds->lens[l] = 0;
                __builtin_amdgcn_wave_barrier();
                for (uint32_t i = 0; i < hclen; i++) {
                    bi.refill(in);
                    uint32_t v = bi.peek(3);
                    if (!bi.drop(3)) return CODAG_E_TRUNCATED;
                    if (l == 0) lds->lens[kCodeLenOrder[i]] = (uint8_t)v;
                }
                __builtin_amdgcn_wave_barrier();
                BuildResult cl = build_table(lds->lens, 19, kCodeLenBits, kCodeLen, lds->dist,
                                             lds->dist_sorted, &lds->dist_meta);
                if (cl.left != 0) return CODAG_E_CORRUPT;
                uint32_t idx = 0, total = hlit + hdist, prev = 0;
                while (idx < total) {
                    bi.refill(in);
                    uint32_t e = uni(lds->dist[bi.peek(kCodeLenBits)]);
                    uint32_t sym = e >> 16;
                    if (!bi.drop(e & 15)) return CODAG_E_TRUNCATED;
                    if (sym < 16) {
                        if (l == 0) lds->lens[idx] = (uint8_t)sym;
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
                    for (uint32_t k = l; k < rep; k += kWave) lds->lens[idx + k] = (uint8_t)val;
                    prev = val;
                    idx += rep;
                }
                __builtin_amdgcn_wave_barrier();
                if (uni((uint32_t)lds->lens[256]) == 0) return CODAG_E_CORRUPT;
                BuildResult lr = build_table(lds->lens, hlit, TB, kLitLen, lds->lit, lds->lit_sorted,
                                             &lds->lit_meta);
                if (lr.left < 0 || (lr.left > 0 && !(lr.total == 1 && lr.ones == 1)))
                    return CODAG_E_CORRUPT;
                BuildResult dr = build_table(lds->lens + hlit, hdist, kDistBits, kDist, lds->dist,
                                             lds->dist_sorted, &lds->dist_meta);
                if (dr.left < 0 || (dr.left > 0 && dr.total != 0 && !(dr.total == 1 && dr.ones == 1)))
                    return CODAG_E_CORRUPT;
                have_dist = dr.total != 0;
            }
            // Symbols until end of block.
            for (;;) {
                bi.refill(in);
                uint32_t e = uni(lds->lit[bi.peek(TB)]);
                uint32_t kind = (e >> 8) & 7;
                if (kind == kSlow) {
                    e = slow_symbol(bi, &lds->lit_meta, lds->lit_sorted, kLitLen);
                    kind = (e >> 8) & 7;
                }
                if (kind == kInvalid) return CODAG_E_CORRUPT;
                if (!bi.drop(e & 15)) return CODAG_E_TRUNCATED;
                if (kind == kLit) {
                    if (o.pos >= cap) return CODAG_E_OVERFLOW;
                    o.put_literal(e >> 16);
                    continue;
                }
                if (kind == kEob) break;
                if (kind == kBadSym) return CODAG_E_CORRUPT;
                // Length, then distance.
                uint32_t ex = (e >> 4) & 15;
                uint32_t len = (e >> 16) + bi.peek(ex);
                if (!bi.drop(ex)) return CODAG_E_TRUNCATED;
                if (!have_dist) return CODAG_E_CORRUPT;
                bi.refill(in);
                uint32_t d = uni(lds->dist[bi.peek(kDistBits)]);
                uint32_t dk = (d >> 8) & 7;
                if (dk == kSlow) {
                    d = slow_symbol(bi, &lds->dist_meta, lds->dist_sorted, kDist);
                    dk = (d >> 8) & 7;
                }
                if (dk == kInvalid) return CODAG_E_CORRUPT;
                if (!bi.drop(d & 15)) return CODAG_E_TRUNCATED;
                if (dk == kBadSym) return CODAG_E_CORRUPT;
                uint32_t dex = (d >> 4) & 15;
                uint32_t dist = (d >> 16) + bi.peek(dex);
                if (!bi.drop(dex)) return CODAG_E_TRUNCATED;
                if (dist > o.pos) return CODAG_E_CORRUPT;
                if (o.pos + len > cap) return CODAG_E_OVERFLOW;
                o.copy(dist, len);
            }
        }
        if (last) break;
    }
    o.flush();
    return o.pos == cap ? CODAG_OK : CODAG_E_UNDERFLOW;
}

}  // namespace codag
