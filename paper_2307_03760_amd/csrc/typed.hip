// Element types of the integer encodings, ORC byte RLE, and the compressed
// ORC stream (the read path around the decoders, CODAG Section I).
#include <hip/hip_runtime.h>

#include "../../include/codag.h"
#include "decode.hpp"
#include "internal.hpp"

namespace codag {

constexpr int kTypedWpb = 4;

// One chunk per wave, like decode_plain, for byte RLE and for RLE element
// types other than signed 8-byte values.
template <int Codec, class E>
__global__ void __launch_bounds__(kWave * kTypedWpb)
    decode_typed(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
                 uint32_t n, int32_t *status, unsigned long long *err, uint64_t *ticks) {
    __shared__ __align__(16) uint32_t s_ring[kTypedWpb][kRingLdsWords];
    __shared__ __align__(16) uint32_t s_land[kTypedWpb][kLandWords];
    __shared__ __align__(16) WaveScratch<Codec, 9, 0> s_scratch[kTypedWpb];
    const uint32_t wave = uni(threadIdx.x / kWave), c = blockIdx.x * kTypedWpb + wave;
    if (c >= n) return;
    const uint64_t t0 = ticks ? __builtin_amdgcn_s_memtime() : 0;
    const int st = decode_one<Codec, 9, 0, E>(comp, coff, out, ooff, c, s_ring[wave], s_land[wave],
                                             &s_scratch[wave]);
    if (ticks && lane() == 0) ticks[c] = __builtin_amdgcn_s_memtime() - t0;
    report(c, st, status, err);
}

template <int Codec, class E>
int launch_t(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff, uint32_t n,
             int32_t *status, unsigned long long *err, uint64_t *ticks, hipStream_t s) {
    hipLaunchKernelGGL((decode_typed<Codec, E>), dim3((n + kTypedWpb - 1) / kTypedWpb),
                       dim3(kWave * kTypedWpb), 0, s, comp, coff, out, ooff, n, status, err, ticks);
    return hipGetLastError() == hipSuccess ? CODAG_OK : CODAG_E_HIP;
}

template <int Codec, bool SIGNED>
int launch_width(int eb, const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
                 uint32_t n, int32_t *status, unsigned long long *err, uint64_t *ticks, hipStream_t s) {
    switch (eb) {
        case 1: return launch_t<Codec, Elem<1, SIGNED>>(comp, coff, out, ooff, n, status, err, ticks, s);
        case 2: return launch_t<Codec, Elem<2, SIGNED>>(comp, coff, out, ooff, n, status, err, ticks, s);
        case 4: return launch_t<Codec, Elem<4, SIGNED>>(comp, coff, out, ooff, n, status, err, ticks, s);
        default: return launch_t<Codec, Elem<8, SIGNED>>(comp, coff, out, ooff, n, status, err, ticks, s);
    }
}

int launch_typed(int codec, int elem_bytes, bool is_unsigned, const uint8_t *comp, const uint64_t *coff,
                 uint8_t *out, const uint64_t *ooff, uint32_t n, int32_t *status,
                 unsigned long long *err, uint64_t *ticks, hipStream_t s) {
    if (codec == CODAG_BYTE_RLE)
        return launch_t<CODAG_BYTE_RLE, I64>(comp, coff, out, ooff, n, status, err, ticks, s);
    if (codec == CODAG_RLE_V1)
        return is_unsigned
                   ? launch_width<CODAG_RLE_V1, false>(elem_bytes, comp, coff, out, ooff, n, status, err, ticks, s)
                   : launch_width<CODAG_RLE_V1, true>(elem_bytes, comp, coff, out, ooff, n, status, err, ticks, s);
    return is_unsigned
               ? launch_width<CODAG_RLE_V2, false>(elem_bytes, comp, coff, out, ooff, n, status, err, ticks, s)
               : launch_width<CODAG_RLE_V2, true>(elem_bytes, comp, coff, out, ooff, n, status, err, ticks, s);
}

// ---- compressed ORC streams ------------------------------------------------

struct OrcFrame {
    uint64_t src;  // first byte of the chunk's payload in the framed stream
    uint32_t len;  // payload bytes
    uint32_t original;
};

struct OrcMeta {
    uint32_t count;     // chunks found
    uint32_t complete;  // the last chunk found ends the stream (no bytes after it)
    unsigned long long key;  // first failure: chunk << 4 | -status, or all ones
    uint64_t last;           // bytes the last chunk produced
};

// One wave walks the chunk headers (a few per megabyte of stream).
__global__ void __launch_bounds__(kWave)
    orc_frames(const uint8_t *framed, uint64_t len, OrcFrame *frames, uint32_t max_frames, OrcMeta *meta) {
    uint64_t pos = 0;
    uint32_t k = 0;
    unsigned long long key = ~0ull;
    while (pos < len) {
        if (len - pos < 3) {
            key = error_key(k, CODAG_E_TRUNCATED);
            break;
        }
        const uint32_t h = (uint32_t)framed[pos] | (uint32_t)framed[pos + 1] << 8 | (uint32_t)framed[pos + 2] << 16;
        pos += 3;
        const uint32_t n = h >> 1;
        if (len - pos < n) {
            key = error_key(k, CODAG_E_TRUNCATED);
            break;
        }
        if (k >= max_frames) {  // more chunks than the output can hold
            key = error_key(k, CODAG_E_OVERFLOW);
            break;
        }
        if (lane() == 0) {
            frames[k].src = pos;
            frames[k].len = n;
            frames[k].original = h & 1;
        }
        pos += n;
        k++;
    }
    if (lane() == 0) {
        meta->count = k;
        meta->complete = key == ~0ull;
        meta->key = key;
        meta->last = 0;
    }
}

// Chunk f (one wave per chunk, persistent grid) into out + f * block; a
// compressed chunk is a raw Deflate stream (ZLIB) or an LZ4 block (LZ4).
template <int Codec>
__global__ void __launch_bounds__(kWave)
    orc_frame_decode(const uint8_t *framed, uint32_t block, uint8_t *out, uint64_t out_cap,
                     const OrcFrame *frames, OrcMeta *meta) {
    __shared__ __align__(16) uint32_t s_ring[ring_lds_words<Codec>()];
    __shared__ __align__(16) uint32_t s_land[land_lds_words<Codec>()];
    __shared__ __align__(16) WaveScratch<Codec, 9, 4096> s_lds;
    const uint32_t count = uni(meta->count), complete = uni(meta->complete);
    for (uint32_t f = blockIdx.x; f < count; f += gridDim.x) {
        const uint64_t at = (uint64_t)f * block;
        const uint32_t len = uni(frames[f].len), original = uni(frames[f].original);
        const uint64_t src = ((uint64_t)uni((uint32_t)(frames[f].src >> 32)) << 32) | uni((uint32_t)frames[f].src);
        const bool last = f + 1 == count && complete;  // the chunk that ends the stream
        const uint32_t room = at >= out_cap ? 0u : (uint32_t)min((uint64_t)block, out_cap - at);
        int st = CODAG_OK;
        uint32_t made = 0;
        if (original) {
            if (len > room) {
                st = CODAG_E_OVERFLOW;
            } else {
                for (uint32_t i = lane(); i < len; i += kWave) out[at + i] = framed[src + i];
                made = len;
            }
        } else if (len >= (1u << 28)) {
            st = CODAG_E_INVALID_ARGUMENT;
        } else {
            typename RingOf<Codec>::T in;
            in.init(framed + src, len, s_ring, s_land);
            if constexpr (Codec == CODAG_DEFLATE)
                st = decode_deflate<9, 4096>(in, out + at, room, &s_lds.t, &made);
            else
                st = decode_lz4<4096>(in, out + at, room, &s_lds.t, &made);
            __builtin_amdgcn_s_waitcnt(0);
        }
        if (st == CODAG_OK && !last && made != block) st = made < block ? CODAG_E_UNDERFLOW : CODAG_E_OVERFLOW;
        if (lane() == 0) {
            if (st != CODAG_OK) atomicMin(&meta->key, (unsigned long long)error_key(f, st));
            else if (last) meta->last = made;
        }
    }
}

__global__ void orc_finish(uint32_t block, const OrcMeta *meta, uint64_t *out_len, int32_t *status) {
    if (threadIdx.x != 0) return;
    const unsigned long long k = meta->key;
    const int st = k == ~0ull ? CODAG_OK : -(int)(k & 15);
    *status = st;
    *out_len = st != CODAG_OK || meta->count == 0 ? 0 : (uint64_t)(meta->count - 1) * block + meta->last;
}

}  // namespace codag

extern "C" int codag_orc_decompress_stream(int codec, const uint8_t *framed, uint64_t framed_len,
                                           uint32_t block_size, uint8_t *out, uint64_t out_cap,
                                           uint64_t *out_len, int32_t *status, void *stream) {
    using namespace codag;
    if (!out_len || !status || (framed_len && (!framed || !out)) || block_size == 0 ||
        block_size >= (1u << 23) || (codec != CODAG_DEFLATE && codec != CODAG_LZ4))
        return CODAG_E_INVALID_ARGUMENT;
    const uint64_t max_frames64 = out_cap / block_size + 2;
    if (max_frames64 >= (1ull << 31)) return CODAG_E_INVALID_ARGUMENT;
    const uint32_t max_frames = (uint32_t)max_frames64;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *ws = nullptr;
    const size_t bytes = sizeof(OrcMeta) + (size_t)max_frames * sizeof(OrcFrame);
    if (hipMallocAsync(&ws, bytes, s) != hipSuccess) return CODAG_E_HIP;
    OrcMeta *meta = static_cast<OrcMeta *>(ws);
    OrcFrame *frames = reinterpret_cast<OrcFrame *>(static_cast<char *>(ws) + sizeof(OrcMeta));
    hipLaunchKernelGGL(orc_frames, dim3(1), dim3(kWave), 0, s, framed, framed_len, frames, max_frames, meta);
    const uint32_t grid = max_frames < 2048 ? max_frames : 2048;
    if (codec == CODAG_DEFLATE)
        hipLaunchKernelGGL(orc_frame_decode<CODAG_DEFLATE>, dim3(grid), dim3(kWave), 0, s, framed,
                           block_size, out, out_cap, frames, meta);
    else
        hipLaunchKernelGGL(orc_frame_decode<CODAG_LZ4>, dim3(grid), dim3(kWave), 0, s, framed,
                           block_size, out, out_cap, frames, meta);
    hipLaunchKernelGGL(orc_finish, dim3(1), dim3(kWave), 0, s, block_size, meta, out_len, status);
    const hipError_t e = hipGetLastError();
    if (hipFreeAsync(ws, s) != hipSuccess) return CODAG_E_HIP;
    return e == hipSuccess ? CODAG_OK : CODAG_E_HIP;
}

extern "C" int codag_orc_inflate_stream(const uint8_t *framed, uint64_t framed_len, uint32_t block_size,
                                        uint8_t *out, uint64_t out_cap, uint64_t *out_len,
                                        int32_t *status, void *stream) {
    return codag_orc_decompress_stream(CODAG_DEFLATE, framed, framed_len, block_size, out, out_cap,
                                       out_len, status, stream);
}
