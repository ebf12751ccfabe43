// Wave64 primitives for gfx950.
//
// CODAG (Section IV-C, IV-D) makes one warp the decompression unit and has
// every lane run the same serial decode.  On CDNA the natural form of that is
// a 64-lane wavefront whose decode state is wave-uniform: it lives in scalar
// registers (values pulled out of vector registers with readfirstlane), while
// the vector lanes do the lane-parallel parts (cooperative fetch, bit
// unpacking, prefix sums, stores).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace codag {

constexpr int kWave = 64;

__device__ __forceinline__ uint32_t lane() { return __lane_id(); }

// Value of lane 0 (the value is the same on every active lane by construction).
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int32_t uni(int32_t v) { return (int32_t)__builtin_amdgcn_readfirstlane((uint32_t)v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}

__device__ __forceinline__ uint32_t readlane(uint32_t v, uint32_t l) {
    return __builtin_amdgcn_readlane(v, l);
}
__device__ __forceinline__ uint64_t readlane64(uint64_t v, uint32_t l) {
    return ((uint64_t)readlane((uint32_t)(v >> 32), l) << 32) | readlane((uint32_t)v, l);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Value of v in lane `from` (its low 6 bits), for every lane at once.  A
// lane permute reads 0 from a lane that is switched off, so call this with
// every lane on and select afterwards.
__device__ __forceinline__ uint32_t lane_pull(uint32_t v, uint32_t from) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)((from & 63) << 2), (int)v);
}

// One doubling step over a table of links: a lane whose link `at` points at
// a lane (below 64) takes that lane's entry of v; a link at 64 or beyond is
// an end and stays as it is.
__device__ __forceinline__ uint32_t lane_follow(uint32_t v, uint32_t at) {
    const uint32_t r = lane_pull(v, at);
    return at < 64 ? r : at;
}

// Number of set bits of m in lanes below this one.
__device__ __forceinline__ uint32_t count_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// DPP lane moves (GFX9 encodings): row_shr:n and the cross-row broadcasts.
enum : int {
    kDppRowShr1 = 0x111,
    kDppRowShr2 = 0x112,
    kDppRowShr4 = 0x114,
    kDppRowShr8 = 0x118,
    kDppRowBcast15 = 0x142,
    kDppRowBcast31 = 0x143,
    kDppWaveShr1 = 0x138,
};

template <int Ctrl, int RowMask>
__device__ __forceinline__ uint64_t dpp64(uint64_t x) {
    uint32_t lo = __builtin_amdgcn_update_dpp(0u, (uint32_t)x, Ctrl, RowMask, 0xf, true);
    uint32_t hi = __builtin_amdgcn_update_dpp(0u, (uint32_t)(x >> 32), Ctrl, RowMask, 0xf, true);
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive prefix sum over the 64 lanes (modulo 2^64); all lanes active.
__device__ __forceinline__ uint64_t wave_inclusive_sum(uint64_t x) {
    x += dpp64<kDppRowShr1, 0xf>(x);
    x += dpp64<kDppRowShr2, 0xf>(x);
    x += dpp64<kDppRowShr4, 0xf>(x);
    x += dpp64<kDppRowShr8, 0xf>(x);
    x += dpp64<kDppRowBcast15, 0xa>(x);
    x += dpp64<kDppRowBcast31, 0xc>(x);
    return x;
}

template <int Ctrl, int RowMask>
__device__ __forceinline__ uint32_t dpp32(uint32_t x) {
    return __builtin_amdgcn_update_dpp(0u, x, Ctrl, RowMask, 0xf, true);
}

// Inclusive prefix sum over the 64 lanes (modulo 2^32); all lanes active.
__device__ __forceinline__ uint32_t wave_inclusive_sum32(uint32_t x) {
    x += dpp32<kDppRowShr1, 0xf>(x);
    x += dpp32<kDppRowShr2, 0xf>(x);
    x += dpp32<kDppRowShr4, 0xf>(x);
    x += dpp32<kDppRowShr8, 0xf>(x);
    x += dpp32<kDppRowBcast15, 0xa>(x);
    x += dpp32<kDppRowBcast31, 0xc>(x);
    return x;
}

// Inclusive running maximum over the 64 lanes; all lanes active.
__device__ __forceinline__ uint32_t wave_inclusive_max32(uint32_t x) {
    x = max(x, dpp32<kDppRowShr1, 0xf>(x));
    x = max(x, dpp32<kDppRowShr2, 0xf>(x));
    x = max(x, dpp32<kDppRowShr4, 0xf>(x));
    x = max(x, dpp32<kDppRowShr8, 0xf>(x));
    x = max(x, dpp32<kDppRowBcast15, 0xa>(x));
    x = max(x, dpp32<kDppRowBcast31, 0xc>(x));
    return x;
}

// The previous lane's value (0 on lane 0); all lanes active.
__device__ __forceinline__ uint32_t wave_shift_up1(uint32_t x) { return dpp32<kDppWaveShr1, 0xf>(x); }

__device__ __forceinline__ uint32_t bswap32(uint32_t x) { return __builtin_bswap32(x); }

// Zigzag: 0, 1, 2, 3, 4 code 0, -1, 1, -2, 2.
__device__ __forceinline__ uint64_t unzigzag(uint64_t z) { return (z >> 1) ^ (0 - (z & 1)); }

}  // namespace codag
