// input_stream for one wavefront (CODAG Section IV-B, IV-E).
//
// The chunk's compressed bytes reach the wave through a ring in LDS of twice
// the fetch size, refilled one fetch at a time (the "conditional A" refill
// of Section IV-A); the decoders use 1 KiB fetches, the group-parallel RLE
// v1 passes 4 and 8 KiB.  Each kilobyte is fetched by one 16-byte
// direct-to-LDS load per lane into a separate landing buffer while the
// previous fetch is being decoded, and moved into the ring when decoding
// crosses into it.  Keeping the in-flight
// data out of vector registers matters on this architecture: one counter
// tracks both loads and stores, so waiting on an in-flight register load
// would also wait for every output store issued since.  The landing buffer
// is only read when the ring advances, so the hot loop never waits on it.
//
// Bytes past the end of the chunk read as zero.  Readers see 32-bit words;
// the ring carries a copy of its first 16 bytes after its end so any run of
// four consecutive words is contiguous.  Positions are byte offsets from
// `gbase`, the chunk start rounded down to 16 bytes, and fit in 32 bits
// (chunks are below 2 GiB).
#pragma once

#include "wave.hpp"

namespace codag {

#ifndef CODAG_FETCH_KIB
#define CODAG_FETCH_KIB 1
#endif
constexpr uint32_t kFetchBytes = 1024 * CODAG_FETCH_KIB;  // one or more 64 lanes x 16 bytes
constexpr uint32_t kRingBytes = 2 * kFetchBytes;
constexpr uint32_t kRingWords = kRingBytes / 4;
constexpr uint32_t kRingLdsWords = kRingWords + 4;  // + mirror of the first 16 bytes
constexpr uint32_t kLandWords = kFetchBytes / 4;

typedef __attribute__((address_space(3))) void lds_void;

// Wait until every vector memory operation of this wave has completed
// (s_waitcnt vmcnt(0); the expcnt and lgkmcnt fields are left at their
// maxima).  Direct-to-LDS fetches are not tracked by the compiler, so reads of
// the landing buffer are preceded by this explicitly.
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0f70); }

// F is the fetch size (a multiple of 1 KiB); the ring holds 2F bytes.
template <uint32_t F>
struct InRingT {
    static constexpr uint32_t kFetch = F, kBytes = 2 * F, kWords = kBytes / 4;
    static constexpr uint32_t kLdsWords = kWords + 4, kLand = F / 4;  // allocation sizes in words

    const uint8_t *gbase;  // 16-byte aligned
    uint32_t skip;         // chunk start relative to gbase (0..15)
    uint32_t gend;         // one past the chunk's last byte, relative to gbase
    uint32_t loaded;       // bytes [loaded - kBytes, loaded) are in the ring
    uint32_t *ring;        // this wave's ring (kLdsWords words)
    uint32_t *land;        // this wave's landing buffer (kLand words)

    // Start fetching [loaded, loaded + kFetch) into the landing buffer.
    __device__ __forceinline__ void issue() {
#pragma unroll
        for (uint32_t k = 0; k < kFetch / 1024; k++) {
            uint32_t at = loaded + 1024 * k + 16 * lane();
            if (at < gend)
                __builtin_amdgcn_global_load_lds(gbase + at, (lds_void *)(land + 256 * k), 16, 0, 0);
        }
    }

    __device__ __forceinline__ void init(const uint8_t *chunk, uint32_t len, uint32_t *ring_lds,
                                         uint32_t *land_lds) {
        // Pointer arithmetic (not an integer round trip) keeps the pointer
        // in the global address space, so loads are global, not flat.
        skip = (uint32_t)(reinterpret_cast<uintptr_t>(chunk) & 15);
        gbase = chunk - skip;
        gend = skip + len;
        loaded = 0;
        ring = ring_lds;
        land = land_lds;
        issue();
    }

    // As init, but decoding starts at byte position pos (relative to the
    // chunk start rounded down to 16 bytes), so the first fetch covers it.
    __device__ __forceinline__ void init_at(const uint8_t *chunk, uint32_t len, uint32_t *ring_lds,
                                            uint32_t *land_lds, uint32_t pos) {
        skip = (uint32_t)(reinterpret_cast<uintptr_t>(chunk) & 15);
        gbase = chunk - skip;
        gend = skip + len;
        loaded = pos & ~(kFetch - 1);
        ring = ring_lds;
        land = land_lds;
        issue();
    }

    // Move the landed bytes into the ring and start fetching the next.
    __device__ __forceinline__ void commit() {
        wait_vm();
        const uint32_t half = (loaded / kFetch) & 1;
#pragma unroll
        for (uint32_t k = 0; k < kFetch / 1024; k++) {
            uint32_t at = loaded + 1024 * k + 16 * lane();
            uint4 v = reinterpret_cast<const uint4 *>(land)[64 * k + lane()];
            if (at + 16 > gend) {  // zero the bytes past the end of the chunk
                uint32_t valid = at < gend ? gend - at : 0;
                uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    int keep = (int)valid - 4 * j;
                    uint32_t m = keep >= 4 ? 0xffffffffu : keep <= 0 ? 0u : ((1u << (8 * keep)) - 1);
                    w[j] &= m;
                }
                v = make_uint4(w[0], w[1], w[2], w[3]);
            }
            reinterpret_cast<uint4 *>(ring)[half * (kFetch / 16) + 64 * k + lane()] = v;
            if (half == 0 && k == 0 && lane() == 0) reinterpret_cast<uint4 *>(ring)[kBytes / 16] = v;
        }
        loaded += kFetch;
        issue();
    }

    // Make bytes [end - kFetch, end) readable.
    __device__ __forceinline__ void ensure(uint32_t end) {
        while (loaded < end) commit();
    }

    // Restart the ring at byte position pos (after a long jump ahead).
    __device__ __forceinline__ void restart(uint32_t pos) {
        loaded = pos & ~(kFetch - 1);
        issue();
    }

    __device__ __forceinline__ uint32_t word(uint32_t w) const { return ring[w & (kWords - 1)]; }
    // Words w and w+1 (w+1 may be the mirror).
    __device__ __forceinline__ uint32_t word_next(uint32_t w) const {
        return ring[(w & (kWords - 1)) + 1];
    }
    __device__ __forceinline__ uint32_t word_at(uint32_t w, uint32_t k) const {
        return ring[(w & (kWords - 1)) + k];
    }

    // Eight bytes starting at byte position pos, little-endian, identical on
    // all lanes (needs ensure(pos + 12)).
    __device__ __forceinline__ uint64_t peek8(uint32_t pos) const {
        uint32_t w = pos >> 2;
        uint32_t a = word_at(w, 0), b = word_at(w, 1), c = word_at(w, 2);
        uint32_t sh = 8 * (pos & 3);
        uint64_t lo = ((uint64_t)b << 32) | a;
        uint64_t r = sh ? (lo >> sh) | ((uint64_t)c << (64 - sh)) : lo;
        return uni64(r);
    }
};
using InRing = InRingT<kFetchBytes>;

// An input ring without a landing buffer or fetch-ahead: each fetch of F
// bytes (F = 512, or a multiple of 1 KiB) lands straight in the ring half
// whose bytes are no longer needed, and the wave waits for it.  For decoders
// that spend tens of microseconds on a kilobyte of input (Deflate, LZ4) the
// wait costs a few percent, and the LDS it saves (a landing buffer and, at
// F = 512, half the ring) is what limits how many of their waves a CU holds.
// Same interface and guarantee as InRingT: after ensure(end), bytes
// [end - F, end) are readable; bytes past the chunk read as zero.
template <uint32_t F>
struct DirectRing {
    static_assert(F == 512 || F % 1024 == 0, "fetch size");
    static constexpr uint32_t kFetch = F, kBytes = 2 * F, kWords = kBytes / 4;
    static constexpr uint32_t kLdsWords = kWords + 4, kLand = 0;
    static constexpr uint32_t kLanes = F < 1024 ? F / 16 : kWave;  // lanes per fetch instruction
    static constexpr uint32_t kIssues = (F + 1023) / 1024;

    const uint8_t *gbase;  // 16-byte aligned
    uint32_t skip;         // chunk start relative to gbase (0..15)
    uint32_t gend;         // one past the chunk's last byte, relative to gbase
    uint32_t loaded;       // bytes [loaded - F, loaded) are in the ring (and
                           // [loaded - 2F, loaded - F) after two fetches in a row)
    uint32_t *ring;        // this wave's ring (kLdsWords words)

    __device__ __forceinline__ void init(const uint8_t *chunk, uint32_t len, uint32_t *ring_lds, uint32_t *) {
        skip = (uint32_t)(reinterpret_cast<uintptr_t>(chunk) & 15);
        gbase = chunk - skip;
        gend = skip + len;
        loaded = 0;
        ring = ring_lds;
    }

    // Fetch [loaded, loaded + F) into the half that held [loaded - 2F,
    // loaded - F): every caller needs only bytes at or past loaded + 1 - F
    // from here on.  The half's earlier LDS reads have returned (their values
    // were consumed), so the fetch cannot overtake them.
    __device__ __forceinline__ void commit() {
        const uint32_t half = (loaded / F) & 1;
        uint32_t *dst = ring + half * (F / 4);
#pragma unroll
        for (uint32_t k = 0; k < kIssues; k++) {
            const uint32_t at = loaded + 1024 * k + 16 * lane();
            if (lane() < kLanes && at < gend)
                __builtin_amdgcn_global_load_lds(gbase + at, (lds_void *)(dst + 256 * k), 16, 0, 0);
        }
        wait_vm();
        if (loaded + F > gend) {  // zero the bytes past the end of the chunk
#pragma unroll
            for (uint32_t k = 0; k < kIssues; k++) {
                const uint32_t at = loaded + 1024 * k + 16 * lane();
                if (lane() < kLanes && at + 16 > gend) {
                    const uint32_t valid = at < gend ? gend - at : 0;
                    uint4 v = valid ? reinterpret_cast<const uint4 *>(dst)[64 * k + lane()] : make_uint4(0, 0, 0, 0);
                    uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        int keep = (int)valid - 4 * j;
                        uint32_t m = keep >= 4 ? 0xffffffffu : keep <= 0 ? 0u : ((1u << (8 * keep)) - 1);
                        w[j] &= m;
                    }
                    reinterpret_cast<uint4 *>(dst)[64 * k + lane()] = make_uint4(w[0], w[1], w[2], w[3]);
                }
            }
        }
        if (half == 0 && lane() == 0)  // mirror of the first 16 bytes past the ring's end
            reinterpret_cast<uint4 *>(ring)[kBytes / 16] = reinterpret_cast<const uint4 *>(ring)[0];
        loaded += F;
    }

    __device__ __forceinline__ void ensure(uint32_t end) {
        while (loaded < end) commit();
    }

    __device__ __forceinline__ void restart(uint32_t pos) { loaded = pos & ~(F - 1); }

    __device__ __forceinline__ uint32_t word(uint32_t w) const { return ring[w & (kWords - 1)]; }
    __device__ __forceinline__ uint32_t word_next(uint32_t w) const {
        return ring[(w & (kWords - 1)) + 1];
    }
    __device__ __forceinline__ uint32_t word_at(uint32_t w, uint32_t k) const {
        return ring[(w & (kWords - 1)) + k];
    }
};

// Sixteen bytes at position pos as little-endian (lo, hi) pairs, per lane
// (needs the five words from pos >> 2 readable).
template <class Ring>
__device__ __forceinline__ void ring_read16(const Ring &in, uint32_t pos, uint64_t &lo, uint64_t &hi) {
    const uint32_t w = pos >> 2, sh = 8 * (pos & 3);
    const uint32_t a = in.word_at(w, 0), b = in.word_at(w, 1), c = in.word_at(w, 2),
                   d = in.word_at(w, 3), e = in.word_at(w, 4);
    lo = ((uint64_t)__builtin_amdgcn_alignbit(c, b, sh) << 32) | __builtin_amdgcn_alignbit(b, a, sh);
    hi = ((uint64_t)__builtin_amdgcn_alignbit(e, d, sh) << 32) | __builtin_amdgcn_alignbit(d, c, sh);
}

__device__ __forceinline__ uint64_t ring_bits_msb(const InRing &in, uint64_t bit, uint32_t w) {
    uint32_t byte = (uint32_t)(bit >> 3);
    uint32_t wi = byte >> 2;
    uint32_t o = 8 * (byte & 3) + (uint32_t)(bit & 7);  // 0..31
    uint64_t hi = ((uint64_t)bswap32(in.word_at(wi, 0)) << 32) | bswap32(in.word_at(wi, 1));
    uint32_t lo = bswap32(in.word_at(wi, 2));
    uint64_t top = o ? (hi << o) | ((uint64_t)lo >> (32 - o)) : hi;
    return w >= 64 ? top : top >> (64 - w);
}

// Stores a little-endian value of `n` (1..4) bytes at an arbitrary address.
__device__ __forceinline__ void store_bytes(uint8_t *p, uint32_t v, uint32_t n) {
    for (uint32_t k = 0; k < n; k++) p[k] = (uint8_t)(v >> (8 * k));
}

// input_stream of the prefetch-wave ablation (CODAG Section V-F): a second
// wave of the workgroup loads the chunk into an LDS ring of kPrefetchSlots
// kilobytes, as far ahead of the decoding wave as the ring allows, and the
// decoding wave only waits for bytes to arrive.  The two waves meet through
// LDS counters: `filled` (bytes loaded, set by the loader) and `need` (the
// decoder's read frontier).  The decoder's side has the InRing interface.
constexpr uint32_t kPrefetchSlots = 4;
struct PrefetchShared {
    uint32_t ring[kPrefetchSlots * 256 + 4];  // + mirror of the first 16 bytes
    uint32_t filled, need, done;
};

__device__ __forceinline__ uint32_t lds_acquire(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_release(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

struct PrefetchRing {
    static constexpr uint32_t kFetch = 1024, kBytes = kPrefetchSlots * kFetch, kWords = kBytes / 4;
    uint32_t skip, gend, loaded;  // loaded: bytes known to be in the ring
    PrefetchShared *sh;

    __device__ __forceinline__ void init(const uint8_t *chunk, uint32_t len, PrefetchShared *s) {
        skip = (uint32_t)(reinterpret_cast<uintptr_t>(chunk) & 15);
        gend = skip + len;
        loaded = 0;
        sh = s;
    }
    // Bytes [end - 2 KiB, end) readable: publish the frontier, wait for the loader.
    __device__ __forceinline__ void ensure(uint32_t end) {
        if (loaded >= end) return;
        if (lane() == 0) lds_release(&sh->need, end);
        while ((loaded = uni(lds_acquire(&sh->filled))) < end) __builtin_amdgcn_s_sleep(1);
    }
    __device__ __forceinline__ void commit() { ensure(loaded + kFetch); }
    __device__ __forceinline__ void restart(uint32_t) {}  // the loader streams every byte anyway
    __device__ __forceinline__ void finish() {
        if (lane() == 0) lds_release(&sh->done, 1u);
    }
    __device__ __forceinline__ uint32_t word(uint32_t w) const { return sh->ring[w & (kWords - 1)]; }
    __device__ __forceinline__ uint32_t word_next(uint32_t w) const {
        return sh->ring[(w & (kWords - 1)) + 1];
    }
    __device__ __forceinline__ uint32_t word_at(uint32_t w, uint32_t k) const {
        return sh->ring[(w & (kWords - 1)) + k];
    }
    __device__ __forceinline__ uint64_t peek8(uint32_t pos) const {
        uint32_t w = pos >> 2;
        uint32_t a = word_at(w, 0), b = word_at(w, 1), c = word_at(w, 2);
        uint32_t sh8 = 8 * (pos & 3);
        uint64_t lo = ((uint64_t)b << 32) | a;
        uint64_t r = sh8 ? (lo >> sh8) | ((uint64_t)c << (64 - sh8)) : lo;
        return uni64(r);
    }
};

// The loader wave: kilobyte k of the chunk's 16-byte hull goes to slot
// k % kPrefetchSlots once the decoder no longer reads the kilobyte it held
// (its frontier is at least (k - 1) KiB: the decoder reads at most 2 KiB
// behind its frontier).  Bytes past the chunk read as zero, and the loader
// keeps supplying zero kilobytes past the end (decoders read a little
// beyond the last byte) until the decoder says it is done.
__device__ __forceinline__ void prefetch_loader(const uint8_t *chunk, uint32_t len, PrefetchShared *sh) {
    const uint32_t skip = (uint32_t)(reinterpret_cast<uintptr_t>(chunk) & 15);
    const uint8_t *gbase = chunk - skip;
    const uint32_t gend = skip + len, l = lane();
    for (uint32_t k = 0;; k++) {
        if (k >= kPrefetchSlots) {
            while (lds_acquire(&sh->need) < (k - 1) * PrefetchRing::kFetch && !lds_acquire(&sh->done))
                __builtin_amdgcn_s_sleep(1);
        }
        if (lds_acquire(&sh->done)) break;
        const uint32_t at = k * PrefetchRing::kFetch + 16 * l;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (at < gend) v = *reinterpret_cast<const uint4 *>(gbase + at);
        if (at + 16 > gend) {
            const uint32_t valid = at < gend ? gend - at : 0;
            uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int keep = (int)valid - 4 * j;
                w[j] &= keep >= 4 ? 0xffffffffu : keep <= 0 ? 0u : ((1u << (8 * keep)) - 1);
            }
            v = make_uint4(w[0], w[1], w[2], w[3]);
        }
        const uint32_t s = k % kPrefetchSlots;
        reinterpret_cast<uint4 *>(sh->ring)[s * 64 + l] = v;
        if (s == 0 && l == 0) reinterpret_cast<uint4 *>(sh->ring)[kPrefetchSlots * 64] = v;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (l == 0) lds_release(&sh->filled, (k + 1) * PrefetchRing::kFetch);
    }
}

}  // namespace codag
