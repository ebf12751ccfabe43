/*
 * CPU encoders that produce the compressed inputs for tests and benchmarks.
 *
 * These write ORC integer RLE v1 and RLE v2 streams (signed int64 columns)
 * from value arrays.  They hold encoding logic only: neither the oracle nor
 * the GPU library includes or links this file.  Deflate inputs come from
 * zlib through Python.
 *
 * Formats: the Apache ORC integer run-length encodings (CODAG, Section V-A
 * evaluates RLE v1 and RLE v2 streams from the ORC tools).
 */
#include <stddef.h>
#include <stdint.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Shared writing helpers (encoder side)                                */
/* ------------------------------------------------------------------ */

typedef struct {
    uint8_t *p;
    size_t n;
} sink;

static void put(sink *s, uint8_t b) { s->p[s->n++] = b; }

static uint64_t zz(int64_t v) { return ((uint64_t)v << 1) ^ (uint64_t)(v >> 63); }

static void put_uvarint(sink *s, uint64_t v) {
    while (v >= 0x80) {
        put(s, (uint8_t)(v | 0x80));
        v >>= 7;
    }
    put(s, (uint8_t)v);
}

static int bit_len(uint64_t v) { /* bits needed, at least 1 */
    int b = 1;
    while (b < 64 && (v >> b) != 0) b++;
    return b;
}

/* ------------------------------------------------------------------ */
/* RLE v1: greedy runs of >= 3 values with a constant delta in         */
/* [-128, 127] (at most 130 values), literal lists of <= 128 otherwise.  */
/* ------------------------------------------------------------------ */

static void v1_literals(sink *s, const int64_t *v, size_t n) {
    while (n > 0) {
        size_t k = n > 128 ? 128 : n, i;
        put(s, (uint8_t)(int8_t)(-(int)k));
        for (i = 0; i < k; i++) put_uvarint(s, zz(v[i]));
        v += k;
        n -= k;
    }
}

size_t enc_rle_v1(const int64_t *v, size_t n, uint8_t *out) {
    sink s = {out, 0};
    size_t i = 0, lit = 0;
    while (i < n) {
        if (i + 2 < n) {
            int64_t d = (int64_t)((uint64_t)v[i + 1] - (uint64_t)v[i]);
            if (d >= -128 && d <= 127 &&
                (int64_t)((uint64_t)v[i + 2] - (uint64_t)v[i + 1]) == d) {
                size_t len = 3;
                while (i + len < n && len < 130 &&
                       (int64_t)((uint64_t)v[i + len] - (uint64_t)v[i + len - 1]) == d)
                    len++;
                v1_literals(&s, v + lit, i - lit);
                put(&s, (uint8_t)(len - 3));
                put(&s, (uint8_t)(int8_t)d);
                put_uvarint(&s, zz(v[i]));
                i += len;
                lit = i;
                continue;
            }
        }
        i++;
    }
    v1_literals(&s, v + lit, n - lit);
    return s.n;
}

/* ------------------------------------------------------------------ */
/* RLE v2                                                               */
/* ------------------------------------------------------------------ */

static const int kWidths[32] = {1,  2,  3,  4,  5,  6,  7,  8,  9,  10, 11,
                                12, 13, 14, 15, 16, 17, 18, 19, 20, 21, 22,
                                23, 24, 26, 28, 30, 32, 40, 48, 56, 64};

static int width_code(int w) { /* w must be a codable width */
    int c;
    for (c = 0; c < 32; c++)
        if (kWidths[c] == w) return c;
    return 31;
}

static int closest(int bits) { /* smallest codable width >= bits; 0 if none */
    int c;
    for (c = 0; c < 32; c++)
        if (kWidths[c] >= bits) return kWidths[c];
    return 0;
}

/* MSB-first bit packing, padded to a byte boundary. */
static void put_packed(sink *s, const uint64_t *vals, size_t count, int w) {
    uint64_t acc = 0;
    int nacc = 0;
    size_t i;
    for (i = 0; i < count; i++) {
        int left = w;
        while (left > 0) {
            int take = left > 8 - nacc ? 8 - nacc : left;
            uint64_t bits = (vals[i] >> (left - take)) & ((1u << take) - 1);
            acc = (acc << take) | bits;
            nacc += take;
            left -= take;
            if (nacc == 8) {
                put(s, (uint8_t)acc);
                acc = 0;
                nacc = 0;
            }
        }
    }
    if (nacc) put(s, (uint8_t)(acc << (8 - nacc)));
}

static void v2_short_repeat(sink *s, int64_t value, int count) {
    uint64_t z = zz(value);
    int nbytes = (bit_len(z) + 7) / 8, i;
    put(s, (uint8_t)(((nbytes - 1) << 3) | (count - 3)));
    for (i = nbytes - 1; i >= 0; i--) put(s, (uint8_t)(z >> (8 * i)));
}

static void v2_header2(sink *s, int type, int code, size_t len) {
    put(s, (uint8_t)((type << 6) | (code << 1) | (int)((len - 1) >> 8)));
    put(s, (uint8_t)((len - 1) & 0xff));
}

static void v2_direct(sink *s, const int64_t *v, size_t n) {
    uint64_t z[512], mx = 0;
    size_t i;
    int w;
    for (i = 0; i < n; i++) {
        z[i] = zz(v[i]);
        if (z[i] > mx) mx = z[i];
    }
    w = closest(bit_len(mx));
    v2_header2(s, 1, width_code(w), n);
    put_packed(s, z, n, w);
}

/* DELTA needs all deltas after the first to share the first delta's sign
 * (a zero first delta reads as non-negative).  Emits nothing and returns 0
 * when the values do not suit the encoding. */
static int v2_delta(sink *s, const int64_t *v, size_t n) {
    int64_t d0;
    uint64_t mags[512], mx = 0;
    size_t i;
    int fixed = 1, w;
    if (n < 2) return 0;
    d0 = (int64_t)((uint64_t)v[1] - (uint64_t)v[0]);
    for (i = 2; i < n; i++)
        if ((int64_t)((uint64_t)v[i] - (uint64_t)v[i - 1]) != d0) fixed = 0;
    if (fixed) {
        v2_header2(s, 3, 0, n);
        put_uvarint(s, zz(v[0]));
        put_uvarint(s, zz(d0));
        return 1;
    }
    for (i = 2; i < n; i++) {
        int64_t d = (int64_t)((uint64_t)v[i] - (uint64_t)v[i - 1]);
        if (d0 >= 0 ? d < 0 : d > 0) return 0;
        mags[i - 2] = d0 >= 0 ? (uint64_t)d : (uint64_t)0 - (uint64_t)d;
        if (mags[i - 2] > mx) mx = mags[i - 2];
    }
    w = closest(bit_len(mx));
    if (w == 1) w = 2; /* width code 0 would read as a fixed delta */
    v2_header2(s, 3, width_code(w), n);
    put_uvarint(s, zz(v[0]));
    put_uvarint(s, zz(d0));
    put_packed(s, mags, n - 2, w);
    return 1;
}

/* PATCHED_BASE.  Returns the number of values encoded (it may take fewer
 * than n when the patch list would exceed 31 entries), or 0 if the values
 * do not suit the encoding. */
static size_t v2_patched(sink *s, const int64_t *v, size_t n) {
    int64_t mn = v[0];
    uint64_t data[512], hist[65], absbase, mxpatch = 0;
    size_t i, cum, take, prev, npatch;
    int w = 1, pw, pgw, ew, bw, b, entries;
    uint64_t entry[64];
    for (i = 1; i < n; i++)
        if (v[i] < mn) mn = v[i];
    if (mn == INT64_MIN) return 0;
    for (b = 0; b <= 64; b++) hist[b] = 0;
    for (i = 0; i < n; i++) {
        data[i] = (uint64_t)v[i] - (uint64_t)mn;
        hist[bit_len(data[i])]++;
    }
    /* Data width: the narrowest codable width holding 90% of the values. */
    cum = 0;
    for (b = 1; b <= 64; b++) {
        cum += hist[b];
        if (cum * 10 >= n * 9) { w = closest(b); break; }
    }
    if (w >= 64) return 0;
    /* Take values while the patch list (with filler entries) fits 31. */
    entries = 0;
    prev = 0;
    npatch = 0;
    take = n;
    for (i = 0; i < n; i++) {
        if (data[i] >> w) {
            size_t gap = i - prev, need = 1 + (gap > 255 ? (gap - 1) / 255 : 0);
            if (entries + (int)need > 31) { take = i; break; }
            entries += (int)need;
            prev = i;
            npatch++;
            if ((data[i] >> w) > mxpatch) mxpatch = data[i] >> w;
        }
    }
    if (take == 0 || npatch == 0) return 0;
    pw = closest(bit_len(mxpatch));
    if (w + pw > 64) return 0;
    /* Gap width: bits of the largest gap entry. */
    {
        uint64_t mxgap = 0;
        prev = 0;
        for (i = 0; i < take; i++) {
            if (data[i] >> w) {
                size_t gap = i - prev;
                while (gap > 255) { mxgap = 255; gap -= 255; }
                if (gap > mxgap) mxgap = gap;
                prev = i;
            }
        }
        pgw = bit_len(mxgap);
    }
    ew = closest(pgw + pw);
    if (ew == 0) return 0;
    absbase = mn < 0 ? (uint64_t)0 - (uint64_t)mn : (uint64_t)mn;
    bw = (bit_len(absbase) + 1 + 7) / 8; /* room for the sign bit */
    if (bw > 8) return 0;
    /* Build the patch list. */
    entries = 0;
    prev = 0;
    for (i = 0; i < take; i++) {
        if (data[i] >> w) {
            size_t gap = i - prev;
            while (gap > 255) {
                entry[entries++] = (uint64_t)255 << pw;
                gap -= 255;
            }
            entry[entries++] = ((uint64_t)gap << pw) | (data[i] >> w);
            prev = i;
            data[i] &= (((uint64_t)1 << w) - 1);
        }
    }
    put(s, (uint8_t)((2 << 6) | (width_code(w) << 1) | (int)((take - 1) >> 8)));
    put(s, (uint8_t)((take - 1) & 0xff));
    put(s, (uint8_t)(((bw - 1) << 5) | width_code(pw)));
    put(s, (uint8_t)(((pgw - 1) << 5) | entries));
    {
        uint64_t field = absbase | (mn < 0 ? (uint64_t)1 << (8 * bw - 1) : 0);
        for (b = bw - 1; b >= 0; b--) put(s, (uint8_t)(field >> (8 * b)));
    }
    put_packed(s, data, take, w);
    put_packed(s, entry, (size_t)entries, ew);
    return take;
}

enum { K_AUTO = 0, K_SHORT_REPEAT = 1, K_DIRECT = 2, K_PATCHED = 3, K_DELTA = 4 };

static size_t equal_run(const int64_t *v, size_t n, size_t cap) {
    size_t k = 1;
    while (k < n && k < cap && v[k] == v[0]) k++;
    return k;
}

static size_t const_delta_run(const int64_t *v, size_t n, size_t cap) {
    size_t k;
    if (n < 2) return n;
    for (k = 2; k < n && k < cap; k++)
        if ((uint64_t)v[k] - (uint64_t)v[k - 1] != (uint64_t)v[1] - (uint64_t)v[0]) break;
    return k;
}

/* Encode v[0..n) with one sub-encoding forced where it applies. */
static void v2_forced(sink *s, const int64_t *v, size_t n, int kind) {
    while (n > 0) {
        size_t k = n > 512 ? 512 : n;
        if (kind == K_SHORT_REPEAT) {
            size_t r = equal_run(v, n, 10);
            if (r >= 3) {
                v2_short_repeat(s, v[0], (int)r);
                v += r;
                n -= r;
                continue;
            }
            /* fewer than 3 equal values left: fall through to DIRECT */
            k = r;
        } else if (kind == K_DELTA) {
            if (k >= 2 && v2_delta(s, v, k)) {
                v += k;
                n -= k;
                continue;
            }
        } else if (kind == K_PATCHED) {
            size_t took = v2_patched(s, v, k);
            if (took) {
                v += took;
                n -= took;
                continue;
            }
        }
        v2_direct(s, v, k);
        v += k;
        n -= k;
    }
}

/* A simple general-purpose choice: repeats, fixed-delta runs, monotone
 * blocks as DELTA, everything else DIRECT. */
static void v2_auto(sink *s, const int64_t *v, size_t n) {
    size_t i = 0;
    while (i < n) {
        size_t r = equal_run(v + i, n - i, 10), j;
        if (r >= 3) {
            v2_short_repeat(s, v[i], (int)r);
            i += r;
            continue;
        }
        r = const_delta_run(v + i, n - i, 512);
        if (r >= 4) {
            v2_delta(s, v + i, r);
            i += r;
            continue;
        }
        j = i + 1;
        while (j < n && j - i < 512) {
            if (equal_run(v + j, n - j, 3) >= 3 || const_delta_run(v + j, n - j, 4) >= 4) break;
            j++;
        }
        if (j - i < 2 || !v2_delta(s, v + i, j - i)) v2_direct(s, v + i, j - i);
        i = j;
    }
}

/*
 * Encode segments: segment t covers seg_len[t] values of v (consecutive)
 * with sub-encoding seg_kind[t] (0 = automatic choice).
 */
size_t enc_rle_v2(const int64_t *v, const int64_t *seg_len, const uint8_t *seg_kind,
                  size_t nseg, uint8_t *out) {
    sink s = {out, 0};
    size_t t;
    for (t = 0; t < nseg; t++) {
        size_t n = (size_t)seg_len[t];
        if (seg_kind[t] == K_AUTO)
            v2_auto(&s, v, n);
        else
            v2_forced(&s, v, n, seg_kind[t]);
        v += n;
    }
    return s.n;
}

/* Worst-case encoded size for n values (either codec). */
size_t enc_bound(size_t n) { return 12 * n + 64; }
