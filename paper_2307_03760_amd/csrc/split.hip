// Group-parallel RLE v1 for launches with few chunks.
//
// With one wave per chunk, a launch of a few dozen chunks keeps a few dozen
// SIMDs busy and each wave's decode is a long chain of dependent steps.
// Here the chunk is decoded in two passes: an index pass (one wave per
// chunk) walks the group headers -- runs fully, literal lists by counting
// varint terminators without decoding them -- and cuts the groups into
// kSplitWaves ranges of about equal output, recording where each range
// starts in the input and in the output; then kSplitWaves waves per chunk
// decode the ranges in parallel, each streaming through its own part of the
// input.  A last pass combines, per chunk, the first error either pass saw
// (errors are keyed by group index, so the earliest group wins, as in a
// sequential decode).
#include <hip/hip_runtime.h>

#include "../../include/codag.h"
#include "decode.hpp"
#include "internal.hpp"

namespace codag {

constexpr uint32_t kSplitWaves = 16;  // decoding waves per chunk
constexpr int kSplitWpb = 4;          // decode pass: waves per block

// With a few dozen waves on the chip each wave waits on every fetch it
// makes, so the passes read their input in larger pieces than the one-wave
// decoder: the index pass 8 KiB at a time (a chunk is a few dozen KiB), the
// decode waves 4 KiB (each decodes a few KiB).
using IndexRing = InRingT<8192>;
using GroupRing = InRingT<4096>;

// The index pass's view of the input: 512 bytes starting at w (8-aligned),
// 8 per lane in registers.  Varint terminators (bytes with bit 7 clear) are
// counted, per lane, as running counts in the bytes of c0 (bytes 0-3) and c1
// (bytes 4-7), and over the wave as excl/incl (before / through this lane).
// Headers are read with lane reads and literal lists are skipped by
// counting terminators, so the serial walk touches LDS once per 512 bytes
// and each group is one chain of lane reads and scalar instructions.
struct IndexWindow {
    uint32_t w, total;              // wave-uniform
    uint32_t w0, w1, c0, c1, excl, incl;  // per lane

    __device__ __forceinline__ void load(IndexRing &in, uint32_t at) {
        w = at & ~7u;
        in.ensure(w + 528);
        const uint32_t wb = (w >> 2) + 2 * lane();
        w0 = in.word(wb);
        w1 = in.word(wb + 1);
        // One per terminator byte; times 0x01010101 gives running counts.
        c0 = ((~w0 & 0x80808080u) >> 7) * 0x01010101u;
        c1 = ((~w1 & 0x80808080u) >> 7) * 0x01010101u + (c0 >> 24) * 0x01010101u;
        incl = wave_inclusive_sum32(c1 >> 24);
        excl = incl - (c1 >> 24);
        total = readlane(incl, kWave - 1);
    }
    // Byte at x (inside the window).
    __device__ __forceinline__ uint32_t byte(uint32_t x) const {
        const uint32_t L = (x - w) >> 3, o = (x - w) & 7;
        const uint32_t v = o < 4 ? readlane(w0, L) : readlane(w1, L);
        return (v >> (8 * (o & 3))) & 0xff;
    }
    // Terminators in [w, x) (x inside the window).
    __device__ __forceinline__ uint32_t before(uint32_t x) const {
        const uint32_t L = (x - w) >> 3, o = (x - w) & 7;
        const uint64_t cc = ((uint64_t)readlane(c1, L) << 32) | readlane(c0, L);
        return readlane(excl, L) + (o ? (uint32_t)(cc >> (8 * o - 8)) & 0xff : 0);
    }
    // Position of terminator number k (1-based, k <= total): in the first
    // lane whose count through it reaches k, the first byte whose running
    // count reaches the rest (a bytewise compare; counts are at most 8, so
    // no borrow crosses a byte).
    __device__ __forceinline__ uint32_t nth(uint32_t k) const {
        const uint32_t L = (uint32_t)__builtin_ctzll(ballot(incl >= k));
        const uint64_t r = k - readlane(excl, L);
        const uint64_t cc = ((uint64_t)readlane(c1, L) << 32) | readlane(c0, L);
        const uint64_t ge = ((cc | 0x8080808080808080ull) - r * 0x0101010101010101ull) & 0x8080808080808080ull;
        return w + 8 * L + ((uint32_t)__builtin_ctzll(ge) >> 3);
    }
};

// Index pass, one wave per chunk.  The groups it walks are cut into
// kSplitWaves ranges of about equal output: range[c * kSplitWaves + j] =
// (first group, end group, input position and first value of the first
// group).  keys[2c] = the first structural error (group << 4 | -status), or
// all ones; groups from that one on are in no range.
__global__ void __launch_bounds__(kWave)
    rle_v1_index(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
                 uint32_t n, uint4 *range, unsigned long long *keys) {
    __shared__ __align__(16) uint32_t s_ring[IndexRing::kLdsWords];
    __shared__ __align__(16) uint32_t s_land[IndexRing::kLand];
    const uint32_t l = lane(), c = blockIdx.x;
    if (c >= n) return;
    keys[2 * c + 1] = ~0ull;  // the decode pass's key, same value from every lane
    const uint64_t i0 = coff[c], i1 = coff[c + 1], o0 = ooff[c], o1 = ooff[c + 1];
    const uint32_t in_len = (uint32_t)(i1 - i0), out_len = (uint32_t)(o1 - o0);
    if ((((i1 - i0) | (o1 - o0)) >> 31) != 0 || (out_len & 7) ||
        (reinterpret_cast<uintptr_t>(out + o0) & 7)) {
        if (l < kSplitWaves) range[(size_t)c * kSplitWaves + l] = make_uint4(0, 0, 0, 0);
        keys[2 * c] = error_key(0, CODAG_E_INVALID_ARGUMENT);
        return;
    }
    IndexRing in;
    in.init(comp + i0, in_len, s_ring, s_land);
    const uint32_t end = in.gend, cap = out_len / 8;
    uint32_t pos = in.skip, nv = 0, k = 0;
    // Lane j < kSplitWaves: the first group of range j and where it starts.
    uint32_t rg = 0, rpos = 0, rnv = 0, j = 0;
    uint32_t next = 0;  // first value at which range j starts
    unsigned long long key = ~0ull;
    bool open_end = false;
    IndexWindow win;
    win.load(in, pos);
    while (nv < cap) {
        if (pos >= end) {
            key = error_key(k, CODAG_E_TRUNCATED);
            break;
        }
        if (pos + 16 > win.w + 512) win.load(in, pos);
        const int32_t h = (int8_t)win.byte(pos);
        const uint32_t gp = pos, gn = nv;
        if (h >= 0) {
            // Run: header, delta byte, base varint ending at terminator e.
            const uint32_t len = (uint32_t)h + 3, x = pos + 2;
            const uint32_t t = win.before(x) + 1;
            const uint32_t e = t <= win.total ? win.nth(t) : ~0u;
            const uint32_t nb = e - x + 1;  // varint bytes (huge: none in the window)
            if (x > end || nb >= 10 || e >= end || nv + len > cap) {
                // The checks in decoding order; a 10-byte varint is valid
                // when its last byte is 0 or 1.
                const int st = x > end                                        ? CODAG_E_TRUNCATED
                               : nb > 10 || (nb == 10 && win.byte(e) > 1) ? CODAG_E_CORRUPT
                               : e >= end                                     ? CODAG_E_TRUNCATED
                               : nv + len > cap                               ? CODAG_E_OVERFLOW
                                                                              : CODAG_OK;
                if (st != CODAG_OK) {
                    key = error_key(k, st);
                    break;
                }
            }
            pos = e + 1;
            nv += len;
        } else {
            const uint32_t len = (uint32_t)(-h);
            if (nv + len > cap) {
                key = error_key(k, CODAG_E_OVERFLOW);
                break;
            }
            // Skip `len` varints: the list ends at terminator number t
            // counted from the window start.  A list that does not end
            // inside the chunk is still recorded: its decode reports where
            // it fails.
            uint32_t t = win.before(pos + 1) + len;
            while (t > win.total && win.w + 512 < end) {
                t -= win.total;
                win.load(in, win.w + 512);
            }
            if (t > win.total) {
                open_end = true;
            } else {
                const uint32_t e = win.nth(t);
                open_end = e >= end;
                pos = e + 1;
            }
            nv += len;
        }
        // Ranges that start at or before this group's first value start here.
        while (j < kSplitWaves && gn >= next) {
            rg = l == j ? k : rg;
            rpos = l == j ? gp : rpos;
            rnv = l == j ? gn : rnv;
            j++;
            next = cap * j / kSplitWaves;  // cap < 2^28
        }
        k++;
        if (open_end) break;
    }
    if (!open_end && key == ~0ull && pos != end) key = error_key(k, CODAG_E_CORRUPT);
    // Ranges not started are empty; each ends where the next one starts.
    rg = l >= j ? k : rg;
    const uint32_t rend = __shfl_down(rg, 1, kWave);
    if (l < kSplitWaves) range[(size_t)c * kSplitWaves + l] = make_uint4(rg, rend, rpos, rnv);
    keys[2 * c] = key;
    __builtin_amdgcn_s_waitcnt(0);
}

// Decode pass: wave j of chunk c decodes range j of its groups, in order,
// streaming through the input from the range's first group.
__global__ void __launch_bounds__(kWave * kSplitWpb)
    rle_v1_groups(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
                  uint32_t n, const uint4 *range, unsigned long long *keys) {
    __shared__ __align__(16) uint32_t s_ring[kSplitWpb][GroupRing::kLdsWords];
    __shared__ __align__(16) uint32_t s_land[kSplitWpb][GroupRing::kLand];
    const uint32_t wave = uni(threadIdx.x / kWave);
    const uint32_t gid = blockIdx.x * kSplitWpb + wave;
    const uint32_t c = gid / kSplitWaves, j = gid % kSplitWaves;
    if (c >= n) return;
    const uint4 r = range[(size_t)c * kSplitWaves + j];
    const uint32_t g0 = uni(r.x), g1 = uni(r.y);
    if (g0 >= g1) return;
    const uint64_t i0 = coff[c], i1 = coff[c + 1], o0 = ooff[c], o1 = ooff[c + 1];
    uint32_t pos = uni(r.z), nv = uni(r.w);
    GroupRing in;
    in.init_at(comp + i0, (uint32_t)(i1 - i0), s_ring[wave], s_land[wave], pos);
    const uint32_t end = in.gend, cap = (uint32_t)(o1 - o0) / 8;
    uint64_t *dst = reinterpret_cast<uint64_t *>(out + o0);
    for (uint32_t g = g0; g < g1; g++) {
        int st = rle_v1_group(in, pos, end, dst, nv, cap);
        if (st != CODAG_OK) {
            // Later groups of this range come later in the stream.
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

size_t rle_v1_split_workspace(uint32_t n) {
    return (size_t)n * kSplitWorkspacePerChunk;
}

int launch_rle_v1_split(const uint8_t *comp, const uint64_t *coff, uint8_t *out,
                        const uint64_t *ooff, uint32_t n, int32_t *status, unsigned long long *err,
                        hipStream_t s, void *workspace) {
    static_assert(kSplitWorkspacePerChunk == kSplitWaves * sizeof(uint4) + 2 * sizeof(unsigned long long),
                  "workspace layout");
    // Without a caller's workspace it comes from the stream-ordered
    // allocator, so concurrent launches on other streams get their own.
    const size_t range_bytes = (size_t)n * kSplitWaves * sizeof(uint4);
    void *ws = workspace;
    if (!ws && hipMallocAsync(&ws, rle_v1_split_workspace(n), s) != hipSuccess) return CODAG_E_HIP;
    uint4 *range = static_cast<uint4 *>(ws);
    unsigned long long *keys =
        reinterpret_cast<unsigned long long *>(static_cast<char *>(ws) + range_bytes);
    hipLaunchKernelGGL(rle_v1_index, dim3(n), dim3(kWave), 0, s, comp, coff, out, ooff, n, range,
                       keys);
    const uint32_t gb = (n * kSplitWaves + kSplitWpb - 1) / kSplitWpb;
    hipLaunchKernelGGL(rle_v1_groups, dim3(gb), dim3(kWave * kSplitWpb), 0, s, comp, coff, out,
                       ooff, n, range, keys);
    hipLaunchKernelGGL(rle_v1_finish, dim3((n + 255) / 256), dim3(256), 0, s, n, keys, status, err);
    hipError_t e = hipGetLastError();
    if (!workspace && hipFreeAsync(ws, s) != hipSuccess) return CODAG_E_HIP;
    return e == hipSuccess ? CODAG_OK : CODAG_E_HIP;
}

}  // namespace codag
