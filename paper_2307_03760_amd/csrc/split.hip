// Group-parallel RLE v1 for launches with few chunks.
//
// With one wave per chunk, a launch of a few dozen chunks keeps a few dozen
// SIMDs busy and each wave's decode is a long chain of dependent steps.
// Here the chunk is decoded in two passes: an index pass (one wave per
// chunk) walks the group headers -- runs fully, literal lists by counting
// varint terminators without decoding them -- and records where every
// group starts in the input and in the output; then kSplitWaves waves per
// chunk decode the groups in parallel, each from its own input ring.  A
// last pass combines, per chunk, the first error either pass saw (errors are
// keyed by group index, so the earliest group wins, as in a sequential
// decode).
#include <hip/hip_runtime.h>

#include "../../include/codag.h"
#include "decode.hpp"
#include "internal.hpp"

namespace codag {

constexpr uint32_t kSplitGroups = 2048;      // group descriptors kept per chunk
constexpr uint32_t kSplitWaves = 16;         // decoding waves per chunk
constexpr uint32_t kSplitWholeChunk = ~0u;   // count: too many groups, one wave decodes the chunk
constexpr int kSplitWpb = 4;

// Index pass.  desc[c * kSplitGroups + k] = (input position, first value) of
// group k of chunk c; count[c] = number of groups recorded; keys[2c] = the
// first structural error (group << 4 | -status), or all ones.
__global__ void __launch_bounds__(kWave * kSplitWpb)
    rle_v1_index(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
                 uint32_t n, uint2 *desc, uint32_t *count, unsigned long long *keys) {
    __shared__ __align__(16) uint32_t s_ring[kSplitWpb][kRingLdsWords];
    __shared__ __align__(16) uint32_t s_land[kSplitWpb][kLandWords];
    const uint32_t wave = uni(threadIdx.x / kWave), l = lane();
    const uint32_t c = blockIdx.x * kSplitWpb + wave;
    if (c >= n) return;
    keys[2 * c + 1] = ~0ull;  // the decode pass's key, same value from every lane
    const uint64_t i0 = coff[c], i1 = coff[c + 1], o0 = ooff[c], o1 = ooff[c + 1];
    const uint32_t in_len = (uint32_t)(i1 - i0), out_len = (uint32_t)(o1 - o0);
    if ((((i1 - i0) | (o1 - o0)) >> 31) != 0 || (out_len & 7) ||
        (reinterpret_cast<uintptr_t>(out + o0) & 7)) {
        count[c] = 0;
        keys[2 * c] = error_key(0, CODAG_E_INVALID_ARGUMENT);
        return;
    }
    InRing in;
    in.init(comp + i0, in_len, s_ring[wave], s_land[wave]);
    const uint32_t end = in.gend, cap = out_len / 8;
    uint2 *d = desc + (size_t)c * kSplitGroups;
    uint32_t pos = in.skip, nv = 0, k = 0, dpos = 0, dn = 0;
    unsigned long long key = ~0ull;
    bool whole = false, open_end = false;
    while (nv < cap) {
        if (k == kSplitGroups) {
            whole = true;
            break;
        }
        if (pos >= end) {
            key = error_key(k, CODAG_E_TRUNCATED);
            break;
        }
        in.ensure(pos + 24);
        uint64_t lo, hi;
        ring_read16(in, pos, lo, hi);
        lo = uni64(lo);
        const int32_t h = (int8_t)(lo & 0xff);
        const uint32_t gp = pos, gn = nv;
        if (h >= 0) {
            const uint32_t len = (uint32_t)h + 3;
            if (pos + 2 > end) {
                key = error_key(k, CODAG_E_TRUNCATED);
                break;
            }
            hi = uni64(hi);
            uint64_t z;
            const uint32_t nb = varint_bytes((lo >> 16) | (hi << 48), (uint32_t)(hi >> 16), z);
            if (nb == 0 || pos + 2 + nb > end || nv + len > cap) {
                key = error_key(k, nb == 0               ? CODAG_E_CORRUPT
                                   : pos + 2 + nb > end ? CODAG_E_TRUNCATED
                                                        : CODAG_E_OVERFLOW);
                break;
            }
            pos += 2 + nb;
            nv += len;
        } else {
            const uint32_t len = (uint32_t)(-h);
            if (nv + len > cap) {
                key = error_key(k, CODAG_E_OVERFLOW);
                break;
            }
            // A list that does not end inside the chunk is still recorded:
            // its decode reports where it fails.
            const uint32_t q = rle_skip_varints(in, pos + 1, end, len);
            open_end = q == 0;
            pos = q;
            nv += len;
        }
        // Descriptor k goes to lane k % 64; 64 of them are stored at once.
        dpos = l == (k & 63) ? gp : dpos;
        dn = l == (k & 63) ? gn : dn;
        if ((k & 63) == 63) d[(k & ~63u) + l] = make_uint2(dpos, dn);
        k++;
        if (open_end) break;
    }
    if ((k & 63) != 0 && l < (k & 63)) d[(k & ~63u) + l] = make_uint2(dpos, dn);
    if (!whole && !open_end && key == ~0ull && pos != end) key = error_key(k, CODAG_E_CORRUPT);
    count[c] = whole ? kSplitWholeChunk : k;
    keys[2 * c] = whole ? ~0ull : key;
    __builtin_amdgcn_s_waitcnt(0);
}

// Decode pass: wave j of chunk c decodes groups j, j + kSplitWaves, ...
__global__ void __launch_bounds__(kWave * kSplitWpb)
    rle_v1_groups(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
                  uint32_t n, const uint2 *desc, const uint32_t *count, unsigned long long *keys) {
    __shared__ __align__(16) uint32_t s_ring[kSplitWpb][kRingLdsWords];
    __shared__ __align__(16) uint32_t s_land[kSplitWpb][kLandWords];
    __shared__ __align__(16) WaveScratch<CODAG_RLE_V1, 10, 0> s_scratch[kSplitWpb];
    const uint32_t wave = uni(threadIdx.x / kWave);
    const uint32_t gid = blockIdx.x * kSplitWpb + wave;
    const uint32_t c = gid / kSplitWaves, j = gid % kSplitWaves;
    if (c >= n) return;
    const uint32_t cnt = uni(count[c]);
    if (cnt == kSplitWholeChunk) {
        if (j == 0) {
            int st = decode_one<CODAG_RLE_V1, 10, 0>(comp, coff, out, ooff, c, s_ring[wave],
                                                      s_land[wave], &s_scratch[wave]);
            if (st != CODAG_OK) atomicMin(&keys[2 * c + 1], (unsigned long long)error_key(0, st));
        }
        return;
    }
    if (j >= cnt) return;
    const uint64_t i0 = coff[c], i1 = coff[c + 1], o0 = ooff[c], o1 = ooff[c + 1];
    InRing in;
    in.init(comp + i0, (uint32_t)(i1 - i0), s_ring[wave], s_land[wave]);
    const uint32_t end = in.gend, cap = (uint32_t)(o1 - o0) / 8;
    uint64_t *dst = reinterpret_cast<uint64_t *>(out + o0);
    const uint2 *d = desc + (size_t)c * kSplitGroups;
    for (uint32_t g = j; g < cnt; g += kSplitWaves) {
        const uint2 dd = d[g];
        uint32_t pos = uni(dd.x), nv = uni(dd.y);
        in.restart(pos);
        int st = rle_v1_group(in, pos, end, dst, nv, cap);
        if (st != CODAG_OK) {
            // Later groups of this wave come later in the stream.
            atomicMin(&keys[2 * c + 1], (unsigned long long)error_key(g, st));
            break;
        }
    }
    __builtin_amdgcn_s_waitcnt(0);
}

// Per chunk, the earlier of the two passes' errors.
__global__ void rle_v1_finish(uint32_t n, const unsigned long long *keys, int32_t *status,
                              unsigned long long *err) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const unsigned long long k = min(keys[2 * c], keys[2 * c + 1]);
    const int st = k == ~0ull ? CODAG_OK : -(int)(k & 15);
    if (status) status[c] = st;
    if (st != CODAG_OK) atomicMin(err, (unsigned long long)error_key(c, st));
}

int launch_rle_v1_split(const uint8_t *comp, const uint64_t *coff, uint8_t *out,
                        const uint64_t *ooff, uint32_t n, int32_t *status, unsigned long long *err,
                        hipStream_t s) {
    // Workspace from the stream-ordered allocator: concurrent launches on
    // other streams get their own.
    const size_t desc_bytes = (size_t)n * kSplitGroups * sizeof(uint2);
    const size_t bytes = desc_bytes + (size_t)n * (sizeof(uint32_t) + 2 * sizeof(unsigned long long)) + 64;
    void *ws = nullptr;
    if (hipMallocAsync(&ws, bytes, s) != hipSuccess) return CODAG_E_HIP;
    uint2 *desc = static_cast<uint2 *>(ws);
    unsigned long long *keys =
        reinterpret_cast<unsigned long long *>(static_cast<char *>(ws) + desc_bytes);
    uint32_t *count = reinterpret_cast<uint32_t *>(keys + 2 * (size_t)n);
    const uint32_t ib = (n + kSplitWpb - 1) / kSplitWpb;
    hipLaunchKernelGGL(rle_v1_index, dim3(ib), dim3(kWave * kSplitWpb), 0, s, comp, coff, out, ooff,
                       n, desc, count, keys);
    const uint32_t gb = (n * kSplitWaves + kSplitWpb - 1) / kSplitWpb;
    hipLaunchKernelGGL(rle_v1_groups, dim3(gb), dim3(kWave * kSplitWpb), 0, s, comp, coff, out,
                       ooff, n, desc, count, keys);
    hipLaunchKernelGGL(rle_v1_finish, dim3((n + 255) / 256), dim3(256), 0, s, n, keys, status, err);
    hipError_t e = hipGetLastError();
    if (hipFreeAsync(ws, s) != hipSuccess || e != hipSuccess) return CODAG_E_HIP;
    return CODAG_OK;
}

}  // namespace codag
