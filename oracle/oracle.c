/*
 * Oracle decoders: TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain sequential decoders, one byte or one bit at a time, written from
 * the format definitions.  CODAG (Section II-B) keeps the method's result
 * identical to this sequential decode: every chunk is decoded from its
 * first byte, in order, and only the assignment of chunks to workers
 * changes.  Nothing here is blocked, fused or reordered.
 *
 * Formats (the paper names them in Section II-A and Section V-A; the bits
 * come from the Apache ORC integer run-length encodings and RFC 1951):
 *   - ORC integer RLE v1, signed: runs (base, delta, length) and literal
 *     lists of zigzag base-128 varints.
 *   - ORC integer RLE v2, signed: SHORT_REPEAT, DIRECT, PATCHED_BASE and
 *     DELTA sub-encodings.
 *   - Deflate (raw RFC 1951 stream per chunk): stored, fixed-Huffman and
 *     dynamic-Huffman blocks with LZ77 back-references.
 *   - ORC byte RLE, and the LZ4 block format (a further LZ77 codec with
 *     byte-aligned sequences and no entropy stage).
 *
 * Readings taken where the sources are silent (each is listed in the
 * design notes):
 *   - Output ends exactly at the chunk's output capacity.  RLE decodes
 *     groups until the capacity is reached; a group that does not fit is
 *     OVERFLOW; input that ends first is TRUNCATED; input bytes left over
 *     after the last value are CORRUPT.
 *   - Deflate stops at the end of the final block; fewer bytes than the
 *     capacity is UNDERFLOW, more is OVERFLOW; bytes after the final block
 *     are ignored.
 *   - Within a group the fixed header fields are parsed first, then the
 *     validity checks, then the capacity check, then the payload.
 *   - Integer arithmetic wraps modulo 2^64.
 *   - Varints longer than 10 bytes, or carrying bits above bit 63, are
 *     CORRUPT.
 *   - Huffman codes are peeked with zero bits past the end of input; a
 *     bit pattern matching no code is CORRUPT, a matching code that runs
 *     past the end is TRUNCATED.
 *   - A PATCHED_BASE patch entry after the first with a zero gap ORs its
 *     patch into the value the entry before it patched.
 *
 * Which status a rejected stream gets (TRUNCATED, CORRUPT, OVERFLOW, ...)
 * beyond the hand-worked cases is parity unpinned: no independent decoder
 * reports these statuses.  Whether an RLE stream is accepted, and what it
 * decodes to, is pinned one-sidedly against Apache ORC's reader.
 */
#include "oracle.h"

#include <stddef.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* ORC byte reader                                                      */
/* ------------------------------------------------------------------ */

typedef struct {
    const uint8_t *buf;
    uint64_t len;
    uint64_t pos;
} byte_reader;

static int br_byte(byte_reader *r, uint8_t *b) {
    if (r->pos >= r->len) return ORACLE_E_TRUNCATED;
    *b = r->buf[r->pos++];
    return ORACLE_OK;
}

/* Base-128 varint, least significant group first; bit 7 of a byte means
 * "another byte follows".  At most 64 bits of value. */
static int br_uvarint(byte_reader *r, uint64_t *v) {
    uint64_t result = 0;
    int i;
    for (i = 0; i < 10; i++) {
        uint8_t b;
        int st = br_byte(r, &b);
        if (st) return st;
        if (i == 9 && b > 1) return ORACLE_E_CORRUPT; /* bits past bit 63 */
        result |= (uint64_t)(b & 0x7f) << (7 * i);
        if ((b & 0x80) == 0) {
            *v = result;
            return ORACLE_OK;
        }
    }
    return ORACLE_E_CORRUPT; /* unreachable: i == 9 with b >= 0x80 returns above */
}

/* Zigzag: 0, -1, 1, -2, 2, ... are coded as 0, 1, 2, 3, 4, ... */
static int64_t unzigzag(uint64_t z) {
    uint64_t mag = z >> 1;
    return (z & 1) ? (int64_t)(~mag) : (int64_t)mag;
}

static int br_svarint(byte_reader *r, int64_t *v) {
    uint64_t z;
    int st = br_uvarint(r, &z);
    if (st) return st;
    *v = unzigzag(z);
    return ORACLE_OK;
}

/* Big-endian unsigned integer of nbytes bytes. */
static int br_be(byte_reader *r, int nbytes, uint64_t *v) {
    uint64_t x = 0;
    int i;
    for (i = 0; i < nbytes; i++) {
        uint8_t b;
        int st = br_byte(r, &b);
        if (st) return st;
        x = (x << 8) | b;
    }
    *v = x;
    return ORACLE_OK;
}

/* Value `index` of a column of eb-byte little-endian integers: the low eb
 * bytes of the decoded 64-bit value (a narrower column holds values that
 * fit its type; storing the low bytes is the cast to it). */
static void put_elem(uint8_t *out, uint64_t index, uint64_t value, int eb) {
    int k;
    for (k = 0; k < eb; k++) out[index * eb + k] = (uint8_t)(value >> (8 * k));
}

/* A value varint: zigzag for signed columns, plain for unsigned ones (ORC
 * writes unsigned streams, such as string lengths, without zigzag). */
static int br_value_varint(byte_reader *r, int uns, uint64_t *v) {
    uint64_t z;
    int st = br_uvarint(r, &z);
    if (st) return st;
    *v = uns ? z : (uint64_t)unzigzag(z);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------ */
/* ORC integer RLE v1 (signed)                                          */
/* ------------------------------------------------------------------ */
/*
 * A group starts with a signed header byte h.
 *   h in [0, 127]:   a run of h + 3 values; a signed delta byte follows,
 *                    then the zigzag varint base; value k is base + k*delta.
 *   h in [-128, -1]: a literal list of -h zigzag varints.
 * (CODAG Section II-A describes RLE v1 runs as a literal plus a length.)
 */
static int decode_rle_v1(const uint8_t *in, uint64_t in_len, uint8_t *out,
                         uint64_t cap_values, uint64_t *n_out, int eb, int uns) {
    byte_reader r = {in, in_len, 0};
    uint64_t n = 0;
    int st = ORACLE_OK;
    while (n < cap_values) {
        uint8_t hb;
        int8_t h;
        st = br_byte(&r, &hb);
        if (st) goto done;
        h = (int8_t)hb;
        if (h >= 0) {
            uint64_t len = (uint64_t)h + 3, k, base;
            uint8_t db;
            int64_t delta;
            st = br_byte(&r, &db);
            if (st) goto done;
            delta = (int8_t)db;
            st = br_value_varint(&r, uns, &base);
            if (st) goto done;
            if (n + len > cap_values) { st = ORACLE_E_OVERFLOW; goto done; }
            for (k = 0; k < len; k++)
                put_elem(out, n + k, base + k * (uint64_t)delta, eb);
            n += len;
        } else {
            uint64_t len = (uint64_t)(-(int)h), k;
            if (n + len > cap_values) { st = ORACLE_E_OVERFLOW; goto done; }
            for (k = 0; k < len; k++) {
                uint64_t v;
                st = br_value_varint(&r, uns, &v);
                if (st) goto done;
                put_elem(out, n, v, eb);
                n++;
            }
        }
    }
    if (r.pos != r.len) st = ORACLE_E_CORRUPT; /* bytes after the last value */
done:
    *n_out = n;
    return st;
}

/* ------------------------------------------------------------------ */
/* ORC integer RLE v2 (signed)                                          */
/* ------------------------------------------------------------------ */

/* The 5-bit width code: codes 0..23 are widths 1..24; codes 24..31 are
 * widths 26, 28, 30, 32, 40, 48, 56, 64. */
static int orc_decode_width(int code) {
    if (code <= 23) return code + 1;
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

/* Smallest codable width that holds n bits (n >= 1); 0 if n > 64. */
static int orc_closest_width(int n) {
    int code;
    for (code = 0; code < 32; code++)
        if (orc_decode_width(code) >= n) return orc_decode_width(code);
    return 0;
}

/*
 * A packed section: count values of w bits each, big-endian and most
 * significant bit first, starting at a byte boundary and padded to one.
 */
static int read_packed(byte_reader *r, uint64_t count, int w, uint64_t *vals) {
    uint64_t nbytes = (count * (uint64_t)w + 7) / 8, i;
    const uint8_t *p;
    uint64_t bit = 0;
    if (r->len - r->pos < nbytes) return ORACLE_E_TRUNCATED;
    p = r->buf + r->pos;
    for (i = 0; i < count; i++) {
        uint64_t v = 0;
        int j;
        for (j = 0; j < w; j++, bit++) {
            int b = (p[bit >> 3] >> (7 - (bit & 7))) & 1;
            v = (v << 1) | (uint64_t)b;
        }
        vals[i] = v;
    }
    r->pos += nbytes;
    return ORACLE_OK;
}

static int decode_rle_v2(const uint8_t *in, uint64_t in_len, uint8_t *out,
                         uint64_t cap_values, uint64_t *n_out, int eb, int uns) {
    byte_reader r = {in, in_len, 0};
    uint64_t n = 0;
    uint64_t vals[512], patches[32];
    int st = ORACLE_OK;
    while (n < cap_values) {
        uint8_t b0, b1, b2, b3;
        int type;
        st = br_byte(&r, &b0);
        if (st) goto done;
        type = b0 >> 6;
        if (type == 0) {
            /* SHORT_REPEAT: bits 5..3 = byte width - 1, bits 2..0 = count - 3;
             * then the zigzag value, big-endian. */
            int w = ((b0 >> 3) & 7) + 1;
            uint64_t len = (uint64_t)(b0 & 7) + 3, k, z;
            if (n + len > cap_values) { st = ORACLE_E_OVERFLOW; goto done; }
            st = br_be(&r, w, &z);
            if (st) goto done;
            for (k = 0; k < len; k++) put_elem(out, n + k, uns ? z : (uint64_t)unzigzag(z), eb);
            n += len;
        } else if (type == 1) {
            /* DIRECT: width code in bits 5..1, 9-bit (length - 1); then the
             * zigzag values packed at that width. */
            int w;
            uint64_t len, k;
            st = br_byte(&r, &b1);
            if (st) goto done;
            w = orc_decode_width((b0 >> 1) & 31);
            len = ((uint64_t)(b0 & 1) << 8 | b1) + 1;
            if (n + len > cap_values) { st = ORACLE_E_OVERFLOW; goto done; }
            st = read_packed(&r, len, w, vals);
            if (st) goto done;
            for (k = 0; k < len; k++)
                put_elem(out, n + k, uns ? vals[k] : (uint64_t)unzigzag(vals[k]), eb);
            n += len;
        } else if (type == 2) {
            /* PATCHED_BASE: data width code and 9-bit (length - 1) as in
             * DIRECT; byte 2 = (base bytes - 1) << 5 | patch width code;
             * byte 3 = (gap bits - 1) << 5 | patch count.  Then the
             * sign-magnitude base, the data values, and the patch list of
             * (gap << pw | patch) entries at the closest width to gap+patch
             * bits.  A (255, 0) entry only advances the position. */
            int w, bw, pw, pgw, pll, ew;
            uint64_t len, k, base_raw, cursor;
            int64_t base;
            st = br_byte(&r, &b1);
            if (st) goto done;
            st = br_byte(&r, &b2);
            if (st) goto done;
            st = br_byte(&r, &b3);
            if (st) goto done;
            w = orc_decode_width((b0 >> 1) & 31);
            len = ((uint64_t)(b0 & 1) << 8 | b1) + 1;
            bw = (b2 >> 5) + 1;
            pw = orc_decode_width(b2 & 31);
            pgw = (b3 >> 5) + 1;
            pll = b3 & 31;
            ew = orc_closest_width(pgw + pw);
            if (ew == 0) { st = ORACLE_E_CORRUPT; goto done; } /* gap + patch over 64 bits */
            if (n + len > cap_values) { st = ORACLE_E_OVERFLOW; goto done; }
            st = br_be(&r, bw, &base_raw);
            if (st) goto done;
            {
                uint64_t sign = (uint64_t)1 << (8 * bw - 1);
                if (base_raw & sign)
                    base = -(int64_t)(base_raw & ~sign);
                else
                    base = (int64_t)base_raw;
            }
            st = read_packed(&r, len, w, vals);
            if (st) goto done;
            st = read_packed(&r, (uint64_t)pll, ew, patches);
            if (st) goto done;
            cursor = 0;
            for (k = 0; k < (uint64_t)pll; k++) {
                uint64_t gap = patches[k] >> pw;
                uint64_t patch = pw == 64 ? patches[k] : (patches[k] & (((uint64_t)1 << pw) - 1));
                cursor += gap;
                if (gap == 255 && patch == 0) continue; /* filler entry */
                if (cursor >= len) { st = ORACLE_E_CORRUPT; goto done; }
                if (w < 64) vals[cursor] |= patch << w; /* bits past 63 are dropped */
            }
            for (k = 0; k < len; k++) put_elem(out, n + k, (uint64_t)base + vals[k], eb);
            n += len;
        } else {
            /* DELTA: width code in bits 5..1 where code 0 means a fixed
             * delta; 9-bit (length - 1); zigzag base varint; zigzag delta
             * base varint; then length - 2 delta magnitudes whose sign is
             * the delta base's. */
            int code, w;
            uint64_t len, k, cur, base;
            int64_t dbase;
            st = br_byte(&r, &b1);
            if (st) goto done;
            code = (b0 >> 1) & 31;
            w = code == 0 ? 0 : orc_decode_width(code);
            len = ((uint64_t)(b0 & 1) << 8 | b1) + 1;
            st = br_value_varint(&r, uns, &base); /* the delta base is always signed */
            if (st) goto done;
            st = br_svarint(&r, &dbase);
            if (st) goto done;
            if (n + len > cap_values) { st = ORACLE_E_OVERFLOW; goto done; }
            if (w == 0) {
                for (k = 0; k < len; k++)
                    put_elem(out, n + k, base + k * (uint64_t)dbase, eb);
            } else {
                put_elem(out, n, base, eb);
                if (len >= 2) {
                    cur = base + (uint64_t)dbase;
                    put_elem(out, n + 1, cur, eb);
                    st = read_packed(&r, len - 2, w, vals);
                    if (st) goto done;
                    for (k = 2; k < len; k++) {
                        if (dbase >= 0)
                            cur += vals[k - 2];
                        else
                            cur -= vals[k - 2];
                        put_elem(out, n + k, cur, eb);
                    }
                }
            }
            n += len;
        }
    }
    if (r.pos != r.len) st = ORACLE_E_CORRUPT;
done:
    *n_out = n;
    return st;
}

/* ------------------------------------------------------------------ */
/* Deflate (RFC 1951)                                                   */
/* ------------------------------------------------------------------ */

typedef struct {
    const uint8_t *buf;
    uint64_t nbits;  /* 8 * input length */
    uint64_t bitpos; /* next bit to consume; bits are taken LSB-first */
} bit_reader;

/* Bit i of the stream, zero past the end. */
static int bit_at(const bit_reader *r, uint64_t i) {
    if (i >= r->nbits) return 0;
    return (r->buf[i >> 3] >> (i & 7)) & 1;
}

/* A value of n bits, least significant bit first. */
static int bits(bit_reader *r, int n, uint32_t *v) {
    uint32_t x = 0;
    int i;
    if (r->bitpos + (uint64_t)n > r->nbits) return ORACLE_E_TRUNCATED;
    for (i = 0; i < n; i++) x |= (uint32_t)bit_at(r, r->bitpos + i) << i;
    r->bitpos += n;
    *v = x;
    return ORACLE_OK;
}

/* Huffman codes as RFC 1951 section 3.2.2 defines them from the code length
 * of every symbol: codes of one length are consecutive integers taken in
 * increasing symbol order, and the first code of a length is the code after
 * the last one of the previous length, doubled.  A code is read from the
 * stream most significant bit first, so after L bits the bits read form an
 * L-bit integer; the pair (L, that integer) is looked up in a table keyed by
 * 2^L + integer, a key that differs for every pair (L <= 15, so keys are
 * below 2^16).  A code's table is reused by the blocks of a decode; only the
 * keys the previous code set are cleared again. */
#define HUFF_KEYS (1 << 16)
typedef struct {
    int16_t *symbol_of;   /* HUFF_KEYS entries: symbol for key 2^L + code, or -1 */
    uint32_t keys[320];   /* the keys this code set */
    int nkeys;
    long kraft;           /* sum over coded symbols of 2^(15 - L) */
    int ones;             /* codes of length 1 */
} huffman;

/* Assigns codes to lengths[0..n) (RFC 1951 section 3.2.2, steps 1 to 3).
 * Over-subscribed sets (Kraft sum above 1) get no codes. */
static void huff_build(huffman *h, const int *lengths, int n) {
    int length_count[16], next_code[16], len, sym, code;
    while (h->nkeys > 0) h->symbol_of[h->keys[--h->nkeys]] = -1;
    for (len = 0; len < 16; len++) length_count[len] = 0;
    for (sym = 0; sym < n; sym++) length_count[lengths[sym]]++;
    h->kraft = 0;
    for (len = 1; len < 16; len++) h->kraft += (long)length_count[len] << (15 - len);
    h->ones = length_count[1];
    if (h->kraft > (1L << 15)) return;
    code = 0;
    length_count[0] = 0;
    for (len = 1; len < 16; len++) {
        code = (code + length_count[len - 1]) << 1;
        next_code[len] = code;
    }
    for (sym = 0; sym < n; sym++) {
        len = lengths[sym];
        if (len != 0) {
            uint32_t key = (1u << len) | (uint32_t)next_code[len]++;
            h->symbol_of[key] = (int16_t)sym;
            h->keys[h->nkeys++] = key;
        }
    }
}

/* Whether the code can be used (RFC 1951 section 3.2.7 and the readings
 * above): not over-subscribed, and complete, except that a single code of
 * length 1 is allowed and, where allow_empty, no codes at all. */
static int huff_usable(const huffman *h, int allow_empty) {
    if (h->kraft > (1L << 15)) return 0;
    if (h->nkeys == 0) return allow_empty;
    if (h->kraft == (1L << 15)) return 1;
    return h->nkeys == 1 && h->ones == 1;
}

/* Decode one symbol: take code bits one at a time, most significant first,
 * until the bits read so far are a code. */
static int huff_decode(bit_reader *r, const huffman *h, int *sym) {
    uint32_t key = 1;
    int len;
    for (len = 1; len < 16; len++) {
        key = (key << 1) | (uint32_t)bit_at(r, r->bitpos + len - 1);
        if (h->symbol_of[key] >= 0) {
            if (r->bitpos + (uint64_t)len > r->nbits) return ORACLE_E_TRUNCATED;
            r->bitpos += len;
            *sym = h->symbol_of[key];
            return ORACLE_OK;
        }
    }
    return ORACLE_E_CORRUPT; /* matches no code */
}

/* Length symbols 257..285: base length and extra-bit count. */
static void length_code(int sym, int *base, int *extra) {
    int k = sym - 257;
    if (sym == 285) { *base = 258; *extra = 0; return; }
    if (k < 8) { *base = k + 3; *extra = 0; return; }
    *extra = (k >> 2) - 1;
    *base = ((4 + (k & 3)) << *extra) + 3;
}

/* Distance symbols 0..29: base distance and extra-bit count. */
static void distance_code(int sym, int *base, int *extra) {
    if (sym < 4) { *base = sym + 1; *extra = 0; return; }
    *extra = (sym >> 1) - 1;
    *base = ((2 + (sym & 1)) << *extra) + 1;
}

typedef struct {
    uint8_t *out;
    uint64_t cap;
    uint64_t n;
} out_window;

/* The literal/length and distance codes of one block (RFC 1951 section
 * 3.2.5): literals are copied out, 256 ends the block, 257..285 start a
 * <length, backward distance> pair whose bytes are copied from the output
 * already produced. */
static int inflate_block_codes(bit_reader *r, out_window *o, const huffman *lit,
                               const huffman *dist) {
    for (;;) {
        int sym, st;
        st = huff_decode(r, lit, &sym);
        if (st) return st;
        if (sym < 256) {
            if (o->n >= o->cap) return ORACLE_E_OVERFLOW;
            o->out[o->n++] = (uint8_t)sym;
        } else if (sym == 256) {
            return ORACLE_OK;
        } else {
            int lbase, lextra, dsym, dbase, dextra;
            uint32_t x;
            uint64_t length, distance, k;
            if (sym > 285) return ORACLE_E_CORRUPT;
            length_code(sym, &lbase, &lextra);
            st = bits(r, lextra, &x);
            if (st) return st;
            length = (uint64_t)lbase + x;
            if (dist->nkeys == 0) return ORACLE_E_CORRUPT; /* no distance codes */
            st = huff_decode(r, dist, &dsym);
            if (st) return st;
            if (dsym > 29) return ORACLE_E_CORRUPT;
            distance_code(dsym, &dbase, &dextra);
            st = bits(r, dextra, &x);
            if (st) return st;
            distance = (uint64_t)dbase + x;
            if (distance > o->n) return ORACLE_E_CORRUPT;     /* before the chunk */
            if (o->n + length > o->cap) return ORACLE_E_OVERFLOW;
            for (k = 0; k < length; k++) { /* byte by byte: overlap repeats */
                o->out[o->n] = o->out[o->n - distance];
                o->n++;
            }
        }
    }
}

/* A stored block (RFC 1951 section 3.2.4): skip to a byte boundary, LEN and
 * its one's complement NLEN, then LEN literal bytes. */
static int inflate_stored(bit_reader *r, out_window *o) {
    uint32_t len, nlen;
    uint64_t k;
    int st;
    r->bitpos = (r->bitpos + 7) & ~(uint64_t)7;
    st = bits(r, 16, &len);
    if (st) return st;
    st = bits(r, 16, &nlen);
    if (st) return st;
    if (nlen != (~len & 0xffff)) return ORACLE_E_CORRUPT;
    if (o->n + len > o->cap) return ORACLE_E_OVERFLOW;
    if (r->bitpos + 8 * (uint64_t)len > r->nbits) return ORACLE_E_TRUNCATED;
    for (k = 0; k < len; k++) o->out[o->n++] = r->buf[(r->bitpos >> 3) + k];
    r->bitpos += 8 * (uint64_t)len;
    return ORACLE_OK;
}

/* The three codes a decode needs, each with its own key table. */
typedef struct {
    huffman lit, dist, clen;
} code_set;

/* A block with the fixed codes of RFC 1951 section 3.2.6. */
static int inflate_fixed(bit_reader *r, out_window *o, code_set *c) {
    int lengths[288], sym;
    for (sym = 0; sym < 288; sym++)
        lengths[sym] = sym < 144 ? 8 : sym < 256 ? 9 : sym < 280 ? 7 : 8;
    huff_build(&c->lit, lengths, 288);
    for (sym = 0; sym < 30; sym++) lengths[sym] = 5;
    lengths[30] = lengths[31] = 5;
    huff_build(&c->dist, lengths, 32);
    return inflate_block_codes(r, o, &c->lit, &c->dist);
}

/* A block with dynamic codes (RFC 1951 section 3.2.7): HLIT, HDIST and
 * HCLEN, the code lengths of the code-length alphabet in its fixed order,
 * then the HLIT + HDIST literal/length and distance code lengths as one
 * sequence coded with that alphabet (16 repeats the previous length 3-6
 * times, 17 and 18 give runs of 3-10 and 11-138 zeros). */
static int inflate_dynamic(bit_reader *r, out_window *o, code_set *c) {
    static const int clen_order[19] = {16, 17, 18, 0, 8, 7, 9, 6, 10, 5,
                                       11, 4, 12, 3, 13, 2, 14, 1, 15};
    int clen_lengths[19], lengths[286 + 30], hlit, hdist, hclen, filled, i, st;
    uint32_t x;

    st = bits(r, 5, &x);
    if (st) return st;
    hlit = (int)x + 257;
    st = bits(r, 5, &x);
    if (st) return st;
    hdist = (int)x + 1;
    st = bits(r, 4, &x);
    if (st) return st;
    hclen = (int)x + 4;
    if (hlit > 286 || hdist > 30) return ORACLE_E_CORRUPT;

    for (i = 0; i < 19; i++) clen_lengths[i] = 0;
    for (i = 0; i < hclen; i++) {
        st = bits(r, 3, &x);
        if (st) return st;
        clen_lengths[clen_order[i]] = (int)x;
    }
    huff_build(&c->clen, clen_lengths, 19);
    /* The code-length code must be complete. */
    if (c->clen.kraft != (1L << 15)) return ORACLE_E_CORRUPT;

    filled = 0;
    while (filled < hlit + hdist) {
        int sym, value, repeat;
        st = huff_decode(r, &c->clen, &sym);
        if (st) return st;
        if (sym <= 15) {
            lengths[filled++] = sym;
            continue;
        }
        if (sym == 16) {
            if (filled == 0) return ORACLE_E_CORRUPT; /* nothing to repeat */
            value = lengths[filled - 1];
            st = bits(r, 2, &x);
            repeat = 3 + (int)x;
        } else if (sym == 17) {
            value = 0;
            st = bits(r, 3, &x);
            repeat = 3 + (int)x;
        } else {
            value = 0;
            st = bits(r, 7, &x);
            repeat = 11 + (int)x;
        }
        if (st) return st;
        if (filled + repeat > hlit + hdist) return ORACLE_E_CORRUPT;
        for (i = 0; i < repeat; i++) lengths[filled++] = value;
    }
    if (lengths[256] == 0) return ORACLE_E_CORRUPT; /* no end-of-block code */

    huff_build(&c->lit, lengths, hlit);
    if (!huff_usable(&c->lit, 0)) return ORACLE_E_CORRUPT;
    huff_build(&c->dist, lengths + hlit, hdist);
    if (!huff_usable(&c->dist, 1)) return ORACLE_E_CORRUPT;
    return inflate_block_codes(r, o, &c->lit, &c->dist);
}

/* The blocks of one raw Deflate stream (RFC 1951 section 3.2.3): BFINAL,
 * BTYPE, the block; after the final block the output must be full. */
static int decode_deflate(const uint8_t *in, uint64_t in_len, uint8_t *out,
                          uint64_t cap, uint64_t *n_out, code_set *c, int capacity_mode) {
    bit_reader r = {in, 8 * in_len, 0};
    out_window o = {out, cap, 0};
    int st = ORACLE_OK;
    for (;;) {
        uint32_t last, type;
        st = bits(&r, 1, &last);
        if (st) break;
        st = bits(&r, 2, &type);
        if (st) break;
        if (type == 0)
            st = inflate_stored(&r, &o);
        else if (type == 1)
            st = inflate_fixed(&r, &o, c);
        else if (type == 2)
            st = inflate_dynamic(&r, &o, c);
        else
            st = ORACLE_E_CORRUPT;
        if (st) break;
        if (last) {
            /* With capacity_mode the output range is only an upper bound. */
            if (o.n != o.cap && !capacity_mode) st = ORACLE_E_UNDERFLOW;
            break;
        }
    }
    *n_out = o.n;
    return st;
}

/* A key table per code for a decode call, all entries -1. */
static int code_set_init(code_set *c) {
    int16_t *t = (int16_t *)malloc(3 * sizeof(int16_t) * HUFF_KEYS);
    if (!t) return -1;
    memset(t, 0xff, 3 * sizeof(int16_t) * HUFF_KEYS);
    memset(c, 0, sizeof(*c));
    c->lit.symbol_of = t;
    c->dist.symbol_of = t + HUFF_KEYS;
    c->clen.symbol_of = t + 2 * HUFF_KEYS;
    return 0;
}

static void code_set_free(code_set *c) { free(c->lit.symbol_of); }

/* ------------------------------------------------------------------ */
/* ORC byte RLE                                                          */
/* ------------------------------------------------------------------ */
/*
 * A group starts with a signed header byte h.
 *   h in [0, 127]:   a run of h + 3 copies of the next byte.
 *   h in [-128, -1]: -h literal bytes follow.
 * Used by ORC for byte columns and, over bit-packed booleans, for
 * PRESENT streams.  End conditions as for the integer encodings: decode
 * until the output is full; a run that does not fit is OVERFLOW (after its
 * byte is read), a literal list that does not fit is OVERFLOW (before its
 * bytes are read), input ending first is TRUNCATED, input left over is
 * CORRUPT.
 */
static int decode_byte_rle(const uint8_t *in, uint64_t in_len, uint8_t *out,
                           uint64_t cap, uint64_t *n_out) {
    byte_reader r = {in, in_len, 0};
    uint64_t n = 0, k;
    int st = ORACLE_OK;
    while (n < cap) {
        uint8_t hb, b;
        int8_t h;
        st = br_byte(&r, &hb);
        if (st) goto done;
        h = (int8_t)hb;
        if (h >= 0) {
            uint64_t len = (uint64_t)h + 3;
            st = br_byte(&r, &b);
            if (st) goto done;
            if (n + len > cap) { st = ORACLE_E_OVERFLOW; goto done; }
            for (k = 0; k < len; k++) out[n++] = b;
        } else {
            uint64_t len = (uint64_t)(-(int)h);
            if (n + len > cap) { st = ORACLE_E_OVERFLOW; goto done; }
            for (k = 0; k < len; k++) {
                st = br_byte(&r, &b);
                if (st) goto done;
                out[n++] = b;
            }
        }
    }
    if (r.pos != r.len) st = ORACLE_E_CORRUPT;
done:
    *n_out = n;
    return st;
}

/* ------------------------------------------------------------------ */
/* LZ4 block format                                                      */
/* ------------------------------------------------------------------ */
/*
 * A block is a sequence of sequences, each: a token byte (high nibble: the
 * literal count, low nibble: the match length minus 4; a nibble of 15 is
 * continued by bytes added to it until one below 255), the literals, then a
 * 2-byte little-endian offset (1..65535, back from the current output end)
 * and the match length's continuation bytes.  The block ends right after a
 * sequence's literals.  Matches copy byte by byte, so one longer than its
 * offset repeats the last `offset` bytes.  Checks in the order the fields
 * are read: a field cut off by the end of input is TRUNCATED, offset 0 or
 * an offset past the output produced so far is CORRUPT once the whole
 * sequence header is read (there is no dictionary), output past the range
 * is OVERFLOW (checked before the literals are read, as for a stored
 * Deflate block), and the output must fill the range (UNDERFLOW otherwise)
 * unless capacity_mode.
 */
static int lz4_length(byte_reader *r, uint64_t *len) {
    uint8_t b;
    do {
        int st = br_byte(r, &b);
        if (st) return st;
        *len += b;
    } while (b == 255);
    return ORACLE_OK;
}

static int decode_lz4(const uint8_t *in, uint64_t in_len, uint8_t *out, uint64_t cap,
                      uint64_t *n_out, int capacity_mode) {
    byte_reader r = {in, in_len, 0};
    uint64_t n = 0, k;
    int st = ORACLE_OK;
    for (;;) {
        uint8_t tok, lo, hi;
        uint64_t lit, mlen, off;
        st = br_byte(&r, &tok);
        if (st) goto done;
        lit = tok >> 4;
        if (lit == 15) {
            st = lz4_length(&r, &lit);
            if (st) goto done;
        }
        if (lit > cap - n) { st = ORACLE_E_OVERFLOW; goto done; }
        if (r.len - r.pos < lit) { st = ORACLE_E_TRUNCATED; goto done; }
        for (k = 0; k < lit; k++) out[n++] = r.buf[r.pos++];
        if (r.pos == r.len) break; /* the last sequence has no match */
        st = br_byte(&r, &lo);
        if (st) goto done;
        st = br_byte(&r, &hi);
        if (st) goto done;
        off = (uint64_t)lo | (uint64_t)hi << 8;
        mlen = tok & 15;
        if (mlen == 15) {
            st = lz4_length(&r, &mlen);
            if (st) goto done;
        }
        mlen += 4;
        if (off == 0 || off > n) { st = ORACLE_E_CORRUPT; goto done; }
        if (mlen > cap - n) { st = ORACLE_E_OVERFLOW; goto done; }
        for (k = 0; k < mlen; k++, n++) out[n] = out[n - off];
    }
    if (n != cap && !capacity_mode) st = ORACLE_E_UNDERFLOW;
done:
    *n_out = n;
    return st;
}

/* ------------------------------------------------------------------ */
/* Entry points                                                         */
/* ------------------------------------------------------------------ */

/* One chunk; c holds the Huffman key table for Deflate (NULL otherwise). */
static int decode_one_chunk(int codec, const uint8_t *in, uint64_t in_len, uint8_t *out,
                            uint64_t out_cap, uint64_t *produced, code_set *c, int eb, int uns,
                            int capacity_mode) {
    uint64_t n = 0;
    int st;
    *produced = 0;
    if (codec == ORACLE_RLE_V1 || codec == ORACLE_RLE_V2) {
        /* Values are whole little-endian integers of eb bytes, aligned. */
        if (out_cap % (uint64_t)eb != 0 || ((uintptr_t)out % (uintptr_t)eb) != 0)
            return ORACLE_E_INVALID_ARGUMENT;
        if (codec == ORACLE_RLE_V1)
            st = decode_rle_v1(in, in_len, out, out_cap / eb, &n, eb, uns);
        else
            st = decode_rle_v2(in, in_len, out, out_cap / eb, &n, eb, uns);
        *produced = n * eb;
        return st;
    }
    if (codec == ORACLE_BYTE_RLE) {
        st = decode_byte_rle(in, in_len, out, out_cap, &n);
        *produced = n;
        return st;
    }
    if (codec == ORACLE_DEFLATE && c) {
        st = decode_deflate(in, in_len, out, out_cap, &n, c, capacity_mode);
        *produced = n;
        return st;
    }
    if (codec == ORACLE_LZ4) {
        st = decode_lz4(in, in_len, out, out_cap, &n, capacity_mode);
        *produced = n;
        return st;
    }
    return ORACLE_E_INVALID_ARGUMENT;
}

static int valid_elem(int eb) { return eb == 1 || eb == 2 || eb == 4 || eb == 8; }

int oracle_decode_chunk(int codec, const uint8_t *in, uint64_t in_len,
                        uint8_t *out, uint64_t out_cap, uint64_t *produced) {
    return oracle_decode_chunk_ex(codec, 8, 0, 0, in, in_len, out, out_cap, produced);
}

int oracle_decode_chunk_ex(int codec, int elem_bytes, int is_unsigned, int capacity_mode,
                           const uint8_t *in, uint64_t in_len, uint8_t *out, uint64_t out_cap,
                           uint64_t *produced) {
    code_set c;
    int st;
    *produced = 0;
    if (!valid_elem(elem_bytes)) return ORACLE_E_INVALID_ARGUMENT;
    if (codec != ORACLE_DEFLATE)
        return decode_one_chunk(codec, in, in_len, out, out_cap, produced, NULL, elem_bytes,
                                is_unsigned, capacity_mode);
    if (code_set_init(&c)) return ORACLE_E_INVALID_ARGUMENT;
    st = decode_one_chunk(codec, in, in_len, out, out_cap, produced, &c, elem_bytes, is_unsigned,
                          capacity_mode);
    code_set_free(&c);
    return st;
}

int oracle_decompress(int codec, const uint8_t *comp,
                      const uint64_t *chunk_offsets, uint8_t *out,
                      const uint64_t *out_offsets, uint64_t n_chunks,
                      int32_t *status) {
    return oracle_decompress_ex(codec, 8, 0, 0, comp, chunk_offsets, out, out_offsets, n_chunks,
                                status, NULL);
}

int oracle_decompress_ex(int codec, int elem_bytes, int is_unsigned, int capacity_mode,
                         const uint8_t *comp, const uint64_t *chunk_offsets, uint8_t *out,
                         const uint64_t *out_offsets, uint64_t n_chunks, int32_t *status,
                         uint64_t *produced) {
    uint64_t i;
    code_set c;
    if (codec < ORACLE_RLE_V1 || codec > ORACLE_LZ4 || !valid_elem(elem_bytes)) return -1;
    if (n_chunks && (!comp || !chunk_offsets || !out || !out_offsets)) return -1;
    if (codec == ORACLE_DEFLATE && code_set_init(&c)) return -1;
    for (i = 0; i < n_chunks; i++) {
        uint64_t made = 0;
        int st;
        if (chunk_offsets[i + 1] < chunk_offsets[i] || out_offsets[i + 1] < out_offsets[i])
            st = ORACLE_E_INVALID_ARGUMENT;
        else
            st = decode_one_chunk(codec, comp + chunk_offsets[i],
                                  chunk_offsets[i + 1] - chunk_offsets[i],
                                  out + out_offsets[i],
                                  out_offsets[i + 1] - out_offsets[i], &made,
                                  codec == ORACLE_DEFLATE ? &c : NULL, elem_bytes, is_unsigned,
                                  capacity_mode);
        if (status) status[i] = st;
        if (produced) produced[i] = made;
    }
    if (codec == ORACLE_DEFLATE) code_set_free(&c);
    return 0;
}

/* ------------------------------------------------------------------ */
/* ORC compressed streams                                               */
/* ------------------------------------------------------------------ */
/*
 * A compressed ORC stream is a sequence of compression chunks, each a
 * 3-byte little-endian header (length << 1 | original) and `length` bytes:
 * the bytes themselves if `original` is set, else the chunk compressed on
 * its own -- for the ZLIB codec a raw Deflate stream, for the LZ4 codec an
 * LZ4 block.  Readings (the format
 * leaves them open): every chunk but the last of a stream holds exactly
 * block_size uncompressed bytes, as Apache ORC's writers produce them (a
 * shorter one is UNDERFLOW, a longer one OVERFLOW); the last holds at most
 * block_size; a header or chunk cut off by the end of the stream is
 * TRUNCATED; more output than out_cap is OVERFLOW.  The statuses are those
 * of the first chunk that fails.
 */
int oracle_orc_inflate_stream(const uint8_t *in, uint64_t in_len, uint64_t block_size,
                              uint8_t *out, uint64_t out_cap, uint64_t *out_len) {
    return oracle_orc_decompress_stream(ORACLE_DEFLATE, in, in_len, block_size, out, out_cap, out_len);
}

int oracle_orc_decompress_stream(int codec, const uint8_t *in, uint64_t in_len, uint64_t block_size,
                                 uint8_t *out, uint64_t out_cap, uint64_t *out_len) {
    uint64_t pos = 0, n = 0;
    code_set c;
    int st = ORACLE_OK;
    *out_len = 0;
    if (block_size == 0 || block_size >= (1u << 23)) return ORACLE_E_INVALID_ARGUMENT;
    if (codec != ORACLE_DEFLATE && codec != ORACLE_LZ4) return ORACLE_E_INVALID_ARGUMENT;
    if (code_set_init(&c)) return ORACLE_E_INVALID_ARGUMENT;
    while (pos < in_len) {
        uint64_t h, len, room, made = 0;
        int last;
        if (in_len - pos < 3) { st = ORACLE_E_TRUNCATED; break; }
        h = (uint64_t)in[pos] | (uint64_t)in[pos + 1] << 8 | (uint64_t)in[pos + 2] << 16;
        pos += 3;
        len = h >> 1;
        if (in_len - pos < len) { st = ORACLE_E_TRUNCATED; break; }
        last = pos + len == in_len;
        room = out_cap - n < block_size ? out_cap - n : block_size;
        if (h & 1) {
            /* original bytes */
            if (len > room) { st = ORACLE_E_OVERFLOW; break; }
            memcpy(out + n, in + pos, len);
            made = len;
        } else {
            st = codec == ORACLE_DEFLATE ? decode_deflate(in + pos, len, out + n, room, &made, &c, 1)
                                         : decode_lz4(in + pos, len, out + n, room, &made, 1);
            if (st) break;
        }
        if (!last && made != block_size) {
            st = made < block_size ? ORACLE_E_UNDERFLOW : ORACLE_E_OVERFLOW;
            break;
        }
        n += made;
        pos += len;
    }
    code_set_free(&c);
    *out_len = n;
    return st;
}
