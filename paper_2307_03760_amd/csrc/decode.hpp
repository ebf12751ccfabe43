// Per-chunk decoding shared by the plain and the batched launches.
#pragma once

#include "../../include/codag.h"
#include "deflate.hpp"
#include "lz4.hpp"
#include "rle.hpp"

namespace codag {

// Per-wave LDS beyond the input ring and its landing buffer.
// For Deflate, TB is the literal/length table bits and H the history
// window bytes.
template <int Codec, int TB, uint32_t H>
struct WaveScratch {
    uint32_t unused;
};
template <int TB, uint32_t H>
struct WaveScratch<CODAG_DEFLATE, TB, H> {
    DeflateLds<TB, H> t;
};
// The LZ4 window is the first member of both, so a Deflate slice (as the
// batched launch allocates) serves LZ4 too.
template <int TB, uint32_t H>
struct WaveScratch<CODAG_LZ4, TB, H> {
    Lz4Lds<H> t;
};

__device__ __forceinline__ uint64_t error_key(uint64_t chunk, int st) {
    return (chunk << 4) | (uint64_t)(uint32_t)(-st);
}

// The input ring each codec decodes from.  Deflate and LZ4 spend tens of
// microseconds per input kilobyte and are held to fewer waves per CU by
// their LDS, so they fetch synchronously into a 1 KiB ring; the RLE decoders
// read input fast and keep the fetch-ahead ring.
template <int Codec>
struct RingOf {
    using T = InRing;
};
template <>
struct RingOf<CODAG_DEFLATE> {
    using T = DirectRing<512>;
};
template <>
struct RingOf<CODAG_LZ4> {
    using T = DirectRing<512>;
};
// LDS words of a codec's ring and landing buffer (at least one word each,
// for the kernels' arrays).
template <int Codec>
constexpr uint32_t ring_lds_words() {
    return RingOf<Codec>::T::kLdsWords;
}
template <int Codec>
constexpr uint32_t land_lds_words() {
    return RingOf<Codec>::T::kLand ? RingOf<Codec>::T::kLand : 1u;
}

// Decodes chunk c with the calling wave; returns its status.  E is the
// element type of the RLE codecs (int64 unless a typed launch says
// otherwise).
template <int Codec, int TB, uint32_t H, class E = I64>
__device__ __forceinline__ int decode_one(const uint8_t *comp, const uint64_t *coff, uint8_t *out,
                                          const uint64_t *ooff, uint32_t c, uint32_t *ring,
                                          uint32_t *land, WaveScratch<Codec, TB, H> *scratch) {
    uint64_t i0 = coff[c], i1 = coff[c + 1], o0 = ooff[c], o1 = ooff[c + 1];
    // Decreasing offsets wrap to huge differences: one test covers both.
    if ((((i1 - i0) | (o1 - o0)) >> 31) != 0) return CODAG_E_INVALID_ARGUMENT;
    uint32_t in_len = (uint32_t)(i1 - i0), out_len = (uint32_t)(o1 - o0);
    uint8_t *dst = out + o0;
    typename RingOf<Codec>::T in;
    int st;
    if constexpr (Codec == CODAG_DEFLATE) {
        if (in_len >= (1u << 28)) return CODAG_E_INVALID_ARGUMENT;  // bit counts fit 31 bits
        in.init(comp + i0, in_len, ring, land);
        st = decode_deflate<TB, H>(in, dst, out_len, &scratch->t);
    } else if constexpr (Codec == CODAG_LZ4) {
        in.init(comp + i0, in_len, ring, land);
        st = decode_lz4<H>(in, dst, out_len, &scratch->t);
    } else if constexpr (Codec == CODAG_BYTE_RLE) {
        in.init(comp + i0, in_len, ring, land);
        st = decode_byte_rle(in, dst, out_len);
    } else {
        constexpr uint32_t B = E::kBytes;
        if ((out_len % B) || (reinterpret_cast<uintptr_t>(dst) % B)) return CODAG_E_INVALID_ARGUMENT;
        in.init(comp + i0, in_len, ring, land);
        typename E::T *dstv = reinterpret_cast<typename E::T *>(dst);
        if constexpr (Codec == CODAG_RLE_V1)
            st = decode_rle_v1<E>(in, dstv, out_len / B);
        else
            st = decode_rle_v2<E>(in, dstv, out_len / B);
    }
    // The landing buffer may still have a fetch in flight: let it land before
    // the wave moves on or exits.
    __builtin_amdgcn_s_waitcnt(0);
    return st;
}

__device__ __forceinline__ void report(uint32_t c, int st, int32_t *status,
                                       unsigned long long *err) {
    if (lane() == 0) {
        if (status) status[c] = st;
        if (st != CODAG_OK) atomicMin(err, (unsigned long long)error_key(c, st));
    }
}

}  // namespace codag
