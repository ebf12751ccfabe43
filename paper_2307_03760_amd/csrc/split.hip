// Group-parallel RLE v1 and v2 for launches with few chunks.
//
// With one wave per chunk, a launch of a few dozen (RLE v1) or a thousand
// (RLE v2) chunks keeps at most one wave on each SIMD, and each wave's
// decode is a long chain of dependent steps.  Here a chunk is decoded in
// two passes: an index pass finds where the groups (runs) start -- without
// decoding their values -- and cuts them into ranges of about equal output,
// recording where each range starts in the input and in the output; then
// one wave per range decodes the ranges in parallel, each streaming through
// its own part of the input.  A last pass combines, per chunk, the first
// error either pass saw (errors are keyed by stream position, so the
// earliest group wins, as in a sequential decode).
#include <hip/hip_runtime.h>

#include "../../include/codag.h"
#include "decode.hpp"
#include "internal.hpp"

namespace codag {

constexpr uint32_t kSplitWaves = 32;  // decoding waves per chunk
constexpr int kSplitWpb = 4;          // decode pass: waves per block

// With a few dozen waves on the chip each wave waits on every fetch it
// makes, so the decode waves read their input 4 KiB at a time (each decodes
// a few KiB), more than the one-wave decoder's 1 KiB.
using GroupRing = InRingT<4096>;

// Index pass, one workgroup per chunk: one walker wave and kIdxHelpers
// helper waves.  The chunk is taken in windows of kIdxStep byte positions
// on a fixed grid.  For every position p of a window the helpers work out,
// in parallel, the group that would start at p -- its length in bytes and
// in values, and what its header and run base say about errors (runs), or
// where its last varint ends (literal lists) -- from a count of varint
// terminator bytes (bit 7 clear) over the window and a lookahead long
// enough for any valid group.  The walker follows the real groups through
// those entries, one LDS read per group, and cuts them into kSplitWaves
// ranges of about equal output.  The helpers prepare window t + 1 while the
// walker walks window t (the two sides meet through LDS counters, not
// workgroup barriers, so neither waits for the other's whole step), and
// each window's bytes arrive by direct-to-LDS loads issued one window
// ahead.
constexpr uint32_t kIdxHelpers = 15;
constexpr uint32_t kIdxThreads = kWave * (kIdxHelpers + 1);
constexpr uint32_t kIdxStep = 4096;                    // positions per window
constexpr uint32_t kIdxAhead = 1536;                   // a valid group spans at most 1 + 10 * 128 bytes
constexpr uint32_t kIdxRegion = kIdxStep + kIdxAhead;  // bytes read per window
constexpr uint32_t kIdxWords = kIdxRegion / 4;
constexpr uint32_t kIdxPieces = kIdxRegion / 16;       // 16-byte loads per window
static_assert(kIdxRegion % 16 == 0 && kIdxStep >= kIdxAhead, "window shape");

// Entry of a position: byte length (13 bits), value count (8 bits) and a
// code: 0 = valid so far, 1 = truncated, 2 = corrupt (both for the header
// and base of a run), 3 = a list whose end is not in the chunk.
enum : uint32_t { kEntOk = 0, kEntTruncated = 1, kEntCorrupt = 2, kEntOpen = 3 };
__device__ __forceinline__ uint32_t make_ent(uint32_t off, uint32_t len, uint32_t code) {
    return off | (len << 13) | (code << 21);
}

// One bit per terminator byte (bit 7 clear) of a little-endian word.
__device__ __forceinline__ uint32_t term_bits(uint32_t w) {
    const uint32_t t = (~w & 0x80808080u) >> 7;  // bits 0, 8, 16, 24
    return (t | (t >> 7) | (t >> 14) | (t >> 21)) & 15;
}

// Counters the walker and the helpers meet at (LDS, monotone).
__device__ __forceinline__ uint32_t lds_load_acquire(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_store_release(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void wait_at_least(const uint32_t *p, uint32_t v) {
    while (lds_load_acquire(p) < v) __builtin_amdgcn_s_sleep(1);
}
// A barrier of the helper waves alone: the counter only grows, each
// crossing adds one per helper wave.
__device__ __forceinline__ void helper_barrier(uint32_t *ctr, uint32_t &gen) {
    gen++;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane() == 0) __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    wait_at_least(ctr, gen * kIdxHelpers);
}

// Index pass.  The groups are cut into kSplitWaves ranges of about equal
// output: range[c * kSplitWaves + j] = (first group, end group, input
// position and first value of the first group).  keys[2c] = the first
// structural error (group << 4 | -status), or all ones; groups from that
// one on are in no range.
__global__ void __launch_bounds__(kIdxThreads)
    rle_v1_index(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
                 uint32_t n, uint4 *range, unsigned long long *keys) {
    __shared__ __align__(16) uint32_t s_buf[2][kIdxWords];
    __shared__ __align__(16) uint32_t s_before[kIdxWords];  // terminators before each word
    __shared__ uint16_t s_tpos[kIdxRegion];                 // region position of each terminator
    __shared__ __align__(16) uint32_t s_ent[2][kIdxStep];
    __shared__ uint32_t s_wsum[kIdxHelpers];
    __shared__ uint32_t s_sync[4];  // helper barrier, windows ready, windows walked, walk done
    __shared__ uint32_t s_stop;     // the walk-done flag as the helpers see it this window
    const uint32_t tid = threadIdx.x, wave = uni(tid / kWave), l = lane();
    const uint32_t c = blockIdx.x;
    if (c >= n) return;
    if (tid == 0) keys[2 * c + 1] = ~0ull;  // the decode pass's key
    const uint64_t i0 = coff[c], i1 = coff[c + 1], o0 = ooff[c], o1 = ooff[c + 1];
    const uint32_t in_len = (uint32_t)(i1 - i0), out_len = (uint32_t)(o1 - o0);
    if ((((i1 - i0) | (o1 - o0)) >> 31) != 0 || (out_len & 7) ||
        (reinterpret_cast<uintptr_t>(out + o0) & 7)) {
        if (tid < kSplitWaves) range[(size_t)c * kSplitWaves + tid] = make_uint4(0, 0, 0, 0);
        if (tid == 0) keys[2 * c] = error_key(0, CODAG_E_INVALID_ARGUMENT);
        return;
    }
    const uint8_t *chunk = comp + i0;
    const uint32_t skip = (uint32_t)(reinterpret_cast<uintptr_t>(chunk) & 15);
    const uint8_t *gbase = chunk - skip;  // positions are relative to the 16-byte hull
    const uint32_t end = skip + in_len, cap = out_len / 8;
    if (tid < 4) s_sync[tid] = 0;
    if (tid == 0) s_stop = 0;
    __syncthreads();

    if (wave != 0) {
        // ---- helpers: prepare each window's entries, one window ahead of
        // the walker.
        const uint32_t h = wave - 1, ht = tid - kWave;  // helper index, helper thread index
        uint32_t gen = 0;
        // Region of window t into buffer t & 1: 1 KiB blocks of 16-byte
        // loads, one per helper wave instruction.
        auto issue = [&](uint32_t t) {
            const uint32_t W = t * kIdxStep;
            for (uint32_t b = h; b * kWave < kIdxPieces; b += kIdxHelpers) {
                const uint32_t q = b * kWave + l, at = W + 16 * q;
                if (q < kIdxPieces && at < end)
                    __builtin_amdgcn_global_load_lds(gbase + at, (lds_void *)(&s_buf[t & 1][b * 256]), 16, 0, 0);
            }
        };
        issue(0);
        wait_vm();
        helper_barrier(&s_sync[0], gen);  // window 0's region has landed
        for (uint32_t t = 0; t * kIdxStep < end; t++) {
            const uint32_t W = t * kIdxStep;
            uint32_t *buf = s_buf[t & 1];
            // s_stop was sampled before the barrier that ended the previous
            // window, so every helper takes the same decision here.
            if (s_stop) break;
            // The other buffer held window t - 1, whose entries are done.
            if (W + kIdxStep < end) issue(t + 1);
            // Bytes past the end of the chunk read as zero (terminators).
            if (W + kIdxRegion > end) {
                for (uint32_t q = ht; q < kIdxPieces; q += kWave * kIdxHelpers) {
                    const uint32_t at = W + 16 * q;
                    if (at + 16 > end) {
                        uint4 v = reinterpret_cast<uint4 *>(buf)[q];
                        const uint32_t valid = at < end ? end - at : 0;
                        uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                        for (int i = 0; i < 4; i++) {
                            const int keep = (int)valid - 4 * i;
                            w[i] &= keep >= 4 ? 0xffffffffu : keep <= 0 ? 0u : ((1u << (8 * keep)) - 1);
                        }
                        reinterpret_cast<uint4 *>(buf)[q] = make_uint4(w[0], w[1], w[2], w[3]);
                    }
                }
                helper_barrier(&s_sync[0], gen);
            }
            // Terminator counts: helper thread ht takes region bytes
            // [16 ht, 16 ht + 16).
            uint32_t tb[4] = {0, 0, 0, 0};
            if (ht < kIdxPieces) {
                const uint4 v = reinterpret_cast<const uint4 *>(buf)[ht];
                tb[0] = term_bits(v.x);
                tb[1] = term_bits(v.y);
                tb[2] = term_bits(v.z);
                tb[3] = term_bits(v.w);
            }
            const uint32_t c0 = __builtin_popcount(tb[0]), c1 = __builtin_popcount(tb[1]);
            const uint32_t c2 = __builtin_popcount(tb[2]), c3 = __builtin_popcount(tb[3]);
            const uint32_t cnt = c0 + c1 + c2 + c3;
            const uint32_t incl = wave_inclusive_sum32(cnt);
            if (l == kWave - 1) s_wsum[h] = incl;
            helper_barrier(&s_sync[0], gen);
            uint32_t base = 0, total = 0;
#pragma unroll
            for (uint32_t w = 0; w < kIdxHelpers; w++) {
                const uint32_t sw = s_wsum[w];
                base += w < h ? sw : 0;
                total += sw;
            }
            if (ht < kIdxPieces) {
                const uint32_t ex = base + incl - cnt;
                reinterpret_cast<uint4 *>(s_before)[ht] =
                    make_uint4(ex, ex + c0, ex + c0 + c1, ex + c0 + c1 + c2);
                uint32_t r = ex;
#pragma unroll
                for (uint32_t i = 0; i < 4; i++) {
                    uint32_t m = tb[i];
                    while (m) {
                        const uint32_t bb = (uint32_t)__builtin_ctz(m);
                        m &= m - 1;
                        s_tpos[r++] = (uint16_t)(16 * ht + 4 * i + bb);
                    }
                }
            }
            // Entries go to buffer t & 1, which held window t - 2: wait
            // until the walker is done with it.
            if (t >= 2) {
                while (lds_load_acquire(&s_sync[2]) < t - 1 && !lds_load_acquire(&s_sync[3]))
                    __builtin_amdgcn_s_sleep(1);
            }
            helper_barrier(&s_sync[0], gen);
            // Entries, four positions (one word) per thread.  A run is a
            // header, a delta byte and a base varint from r = p + 2 to its
            // terminator e; a literal list of 256 - h varints from r = p + 1
            // ends at its last terminator.  Both take one count of the
            // terminators before r, so every position is one path.
            uint32_t *ent = s_ent[t & 1];
            for (uint32_t q = ht; q < kIdxStep / 4; q += kWave * kIdxHelpers) {
                const uint32_t w0 = buf[q], w1 = buf[q + 1];
                const uint32_t sb0 = s_before[q], sb1 = s_before[q + 1];
                const uint32_t tb0 = term_bits(w0), tb1 = term_bits(w1);
                uint32_t e4[4];
#pragma unroll
                for (uint32_t i = 0; i < 4; i++) {
                    const uint32_t p = 4 * q + i;
                    const uint32_t hb = (w0 >> (8 * i)) & 0xff;
                    const bool run = hb < 128;
                    const uint32_t rr = i + 1 + (run ? 1u : 0u);  // r - 4q, 1..5
                    const uint32_t r = 4 * q + rr, rb = rr & 3;
                    const uint32_t tcnt = rr < 4 ? sb0 + __builtin_popcount(tb0 & ((1u << rb) - 1))
                                                 : sb1 + __builtin_popcount(tb1 & ((1u << rb) - 1));
                    const uint32_t cntl = 256 - hb;
                    const uint32_t ti = tcnt + (run ? 0u : cntl - 1);
                    // Every lane looks up (index clamped into the table) and
                    // builds both kinds of entry; selects pick one, so there
                    // are no lane-masked branches.
                    const uint32_t tp = s_tpos[min(ti, kIdxRegion - 1)];
                    const uint32_t e = ti < total ? tp : kIdxRegion;
                    const uint32_t nb = e - r + 1;
                    uint32_t eb = 0;  // a 10-byte varint's last byte (rare: read only when some lane needs it)
                    if (ballot(run && nb == 10)) eb = (buf[min(e >> 2, kIdxWords - 1)] >> (8 * (e & 3))) & 0xff;
                    const uint32_t rcode = W + r > end                        ? kEntTruncated
                                           : nb > 10 || (nb == 10 && eb > 1) ? kEntCorrupt
                                           : W + e >= end                    ? kEntTruncated
                                                                              : kEntOk;
                    const uint32_t ent_run = make_ent(rcode == kEntOk ? e + 1 - p : 0, hb + 3, rcode);
                    const bool open = e >= kIdxRegion || W + e >= end;
                    const uint32_t ent_lit = make_ent(open ? 0 : e + 1 - p, cntl, open ? kEntOpen : kEntOk);
                    e4[i] = run ? ent_run : ent_lit;
                }
                reinterpret_cast<uint4 *>(ent)[q] = make_uint4(e4[0], e4[1], e4[2], e4[3]);
            }
            // One barrier ends the window: its entries are complete, the next
            // window's region (issued above) has landed, and every helper
            // sees the same walk-done sample.
            wait_vm();
            if (h == 0 && l == 0) s_stop = lds_load_acquire(&s_sync[3]);
            helper_barrier(&s_sync[0], gen);
            if (h == 0 && l == 0) lds_store_release(&s_sync[1], t + 1);  // window t ready
        }
        wait_vm();  // a load issued one window ahead may still be landing
        return;
    }

    // ---- walker (wave 0): wave-uniform state; per lane j < kSplitWaves the
    // first group of range j and where it starts.
    __builtin_amdgcn_s_setprio(3);
    uint32_t pos = skip, nv = 0, k = 0, j = 0, next = 0;
    uint32_t rg = 0, rpos = 0, rnv = 0;
    unsigned long long key = ~0ull;
    bool open_end = false;
    for (uint32_t t = 0;; t++) {
        const uint32_t W = t * kIdxStep;
        bool done = false;
        // Leave windows behind without waiting for them (a group jump
        // never passes a whole window, but an empty chunk starts past 0).
        if (nv < cap && pos < end && pos < W + kIdxStep) wait_at_least(&s_sync[1], t + 1);
        const uint32_t *ent = s_ent[t & 1];
        const uint32_t lim = min(end, W + kIdxStep);
        while (true) {
            // Fast path, scalar state only: groups that are valid, fit the
            // output and start no range (the checks below, all passing).
            const uint32_t fastlim = uni(j < kSplitWaves ? min(next, cap) : cap);
            while (pos < lim && nv < fastlim) {
                const uint32_t e = uni(ent[pos - W]);
                const uint32_t len = (e >> 13) & 0xff;
                if ((e >> 21) != kEntOk || nv + len > cap) break;
                nv += len;
                k++;
                pos += e & 0x1fff;
            }
            if (nv >= cap) {
                done = true;
                break;
            }
            if (pos >= end) {
                key = error_key(k, CODAG_E_TRUNCATED);
                done = true;
                break;
            }
            if (pos >= W + kIdxStep) break;  // on in the next window
            const uint32_t e = uni(ent[pos - W]);
            const uint32_t code = e >> 21, len = (e >> 13) & 0xff, off = e & 0x1fff;
            if (code == kEntTruncated || code == kEntCorrupt) {
                key = error_key(k, code == kEntTruncated ? CODAG_E_TRUNCATED : CODAG_E_CORRUPT);
                done = true;
                break;
            }
            if (nv + len > cap) {
                key = error_key(k, CODAG_E_OVERFLOW);
                done = true;
                break;
            }
            const uint32_t gp = pos, gn = nv;
            nv += len;
            // Ranges that start at or before this group's first value start here.
            while (j < kSplitWaves && gn >= next) {
                rg = l == j ? k : rg;
                rpos = l == j ? gp : rpos;
                rnv = l == j ? gn : rnv;
                j++;
                next = uni((uint32_t)((uint64_t)cap * j / kSplitWaves));
            }
            k++;
            if (code == kEntOpen) {
                // A list that does not end inside the chunk is still
                // recorded: its decode reports where it fails.
                open_end = true;
                done = true;
                break;
            }
            pos += off;
        }
        if (done) {
            if (l == 0) lds_store_release(&s_sync[3], 1u);
            break;
        }
        if (l == 0) lds_store_release(&s_sync[2], t + 1);  // window t walked
    }
    if (!open_end && key == ~0ull && pos != end) key = error_key(k, CODAG_E_CORRUPT);
    // Ranges not started are empty; each ends where the next one starts.
    rg = l >= j ? k : rg;
    const uint32_t rend = __shfl_down(rg, 1, kWave);
    if (l < kSplitWaves) range[(size_t)c * kSplitWaves + l] = make_uint4(rg, rend, rpos, rnv);
    if (l == 0) keys[2 * c] = key;
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

// Per chunk, the earlier of the two passes' errors (both passes key errors
// the same way: RLE v1 by group index, RLE v2 by the failing run's first
// value).
__global__ void split_finish(uint32_t n, const unsigned long long *keys, int32_t *status,
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
    hipLaunchKernelGGL(rle_v1_index, dim3(n), dim3(kIdxThreads), 0, s, comp, coff, out, ooff, n,
                       range, keys);
    const uint32_t gb = (n * kSplitWaves + kSplitWpb - 1) / kSplitWpb;
    hipLaunchKernelGGL(rle_v1_groups, dim3(gb), dim3(kWave * kSplitWpb), 0, s, comp, coff, out,
                       ooff, n, range, keys);
    hipLaunchKernelGGL(split_finish, dim3((n + 255) / 256), dim3(256), 0, s, n, keys, status, err);
    hipError_t e = hipGetLastError();
    if (!workspace && hipFreeAsync(ws, s) != hipSuccess) return CODAG_E_HIP;
    return e == hipSuccess ? CODAG_OK : CODAG_E_HIP;
}

// ---- RLE v2 ------------------------------------------------------------
//
// The same two passes for RLE v2.  A run's header gives its byte length
// (DELTA after two varints), so the index pass parses headers only: long
// runs are stepped over, and SHORT_REPEAT stretches are walked 64 bytes at
// a time with every lane parsing the header at its own byte (the decoder's
// chain walk without the values and stores).  It cuts the runs into
// kV2Ranges ranges of about equal output at run boundaries; each range is
// then decoded by one wave of the plain decoder, started at the range's
// first run and stopped at its last value.  Errors are keyed by the first
// value of the failing run (every run has at least one value, so that order
// is the stream order): the index pass reports structural errors (and
// leftover input, keyed at the end), the decoding waves the rest.

constexpr uint32_t kV2Ranges = 8;  // decoding waves per chunk
constexpr int kV2IndexWpb = 4;     // index pass: waves per block
constexpr int kV2DecodeWpb = 4;    // decode pass: waves per block
using V2IndexRing = InRingT<4096>;

// Where each range starts (byte position, first value) and the value at
// which the index pass stopped (the chunk's value count, or the first value
// of the run where it found an error).
struct V2Split {
    uint2 start[kV2Ranges];
    uint32_t stop, pad[3];
};
static_assert(sizeof(V2Split) + 2 * sizeof(unsigned long long) == kSplitV2WorkspacePerChunk,
              "workspace layout");

__device__ __forceinline__ uint32_t v2_threshold(uint32_t cap, uint32_t j) {
    return (uint32_t)((uint64_t)cap * j / kV2Ranges);
}

// Ranges whose first value is at most nv start at the run at (pos, nv).
__device__ __forceinline__ void v2_cut(uint32_t &j, uint32_t cap, uint32_t pos, uint32_t nv,
                                       V2Split *sp) {
    while (j < kV2Ranges && nv >= v2_threshold(cap, j)) {
        if (lane() == 0) sp->start[j] = make_uint2(pos, nv);
        j++;
    }
}

// A stretch of SHORT_REPEAT runs from pos, as the decoder walks it: lane l
// parses the header at pos + l, the chain of runs is followed from lane 0
// with one lane read per run, and a wave prefix sum gives each run's first
// value (for the cuts).  Stops like the decoder: at the first header that is
// not a SHORT_REPEAT, at the end of input, or with the output full.  On an
// error, errnv is the first value of the failing run.
template <class Ring>
__device__ __forceinline__ int v2_index_short_repeats(Ring &in, uint32_t &pos, uint32_t end,
                                                      uint32_t &nv, uint32_t cap, uint32_t &j,
                                                      V2Split *sp, uint32_t &errnv) {
    const uint32_t l = lane();
    for (;;) {
        in.ensure(pos + 72);
        const uint32_t at_b = pos + l;
        const uint32_t h = (in.word(at_b >> 2) >> (8 * (at_b & 3))) & 0xff;
        const uint32_t w = ((h >> 3) & 7) + 1, cs = (h & 7) + 3;
        const uint32_t nxt = (h >> 6) == 0 && at_b + 1 + w <= end ? l + 1 + w : 128 + l;
        // Fast path: a window that holds no range start and stays inside the
        // output needs only the chain's end and its value count.  Each lane
        // gathers, by link doubling, where its chain is after 8 runs (or
        // where it ended) and how many values those runs hold, so the walk
        // reads two lanes per 8 runs.
        {
            const uint32_t c1 = nxt < 128 ? cs : 0u;
            const uint32_t n2 = lane_follow(nxt, nxt), g1 = lane_pull(c1, nxt);
            const uint32_t c2 = c1 + (nxt < 64 ? g1 : 0u);
            const uint32_t n4 = lane_follow(n2, n2), g2 = lane_pull(c2, n2);
            const uint32_t c4 = c2 + (n2 < 64 ? g2 : 0u);
            const uint32_t n8 = lane_follow(n4, n4), g4 = lane_pull(c4, n4);
            const uint32_t c8 = c4 + (n4 < 64 ? g4 : 0u);
            uint32_t t = 0, acc = nv;
            for (uint32_t step = 0; step < 64; step++) {  // links only lead forward
                acc += readlane(c8, t);
                t = readlane(n8, t);
                if (t >= kWave) break;
            }
            if (acc <= cap && (j >= kV2Ranges || v2_threshold(cap, j) >= acc)) {
                nv = acc;
                if (t >= 128) {
                    t -= 128;
                    int st = CODAG_OK;
                    if (pos + t < end && nv < cap) {
                        const uint32_t hs = readlane(h, t);
                        if ((hs >> 6) == 0) {
                            st = nv + (hs & 7) + 3 > cap ? CODAG_E_OVERFLOW : CODAG_E_TRUNCATED;
                            errnv = nv;
                        }
                    }
                    pos += t;
                    return st;
                }
                pos += t;
                if (nv >= cap || pos >= end) return CODAG_OK;
                continue;
            }
        }
        // The window fills the output or holds a range start: every run's
        // first value, by a prefix sum over the lanes where runs start.
        uint32_t s = 0;
        uint64_t starts = 0;
        do {
            starts |= 1ull << s;
            s = readlane(nxt, s);
        } while (s < kWave);
        if (s >= 128) {
            s -= 128;
            starts &= ~(1ull << s);
        }
        const bool mine = (starts >> l) & 1;
        const uint32_t c = mine ? cs : 0;
        const uint32_t at = nv + wave_inclusive_sum32(c) - c;
        const uint32_t n1 = uni(readlane(at + c, kWave - 1));
        uint32_t ff = kWave, fo = kWave;
        if (n1 > cap) {
            const uint64_t full = ballot(mine && at >= cap), over = ballot(mine && at < cap && at + c > cap);
            ff = full ? (uint32_t)__builtin_ctzll(full) : kWave;
            fo = over ? (uint32_t)__builtin_ctzll(over) : kWave;
        }
        const uint32_t lim = min(ff, fo);
        while (j < kV2Ranges && v2_threshold(cap, j) < n1) {
            const uint64_t m = ballot(mine && l < lim && at >= v2_threshold(cap, j));
            if (!m) break;
            const uint32_t L = (uint32_t)__builtin_ctzll(m);
            const uint32_t a = uni(readlane(at, L));
            if (l == 0) sp->start[j] = make_uint2(pos + L, a);
            j++;
        }
        if (fo < ff) {
            errnv = uni(readlane(at, fo));
            return CODAG_E_OVERFLOW;
        }
        if (ff < kWave) {
            nv = cap;
            pos += ff;
            return CODAG_OK;
        }
        nv = n1;
        if (s < kWave) {
            int st = CODAG_OK;
            if (pos + s < end && nv < cap) {
                const uint32_t hs = readlane(h, s);
                if ((hs >> 6) == 0) {
                    st = nv + (hs & 7) + 3 > cap ? CODAG_E_OVERFLOW : CODAG_E_TRUNCATED;
                    errnv = nv;
                }
            }
            pos += s;
            return st;
        }
        pos += s;
        if (nv >= cap || pos >= end) return CODAG_OK;
    }
}

// Bit width of a 5-bit width code, and the width PATCHED_BASE patches are
// stored at (0 when none fits), as scalar selects.
__device__ __forceinline__ uint32_t v2_width(uint32_t code) {
    const uint32_t high = (uint32_t)(0x40383028201E1C1Aull >> (8 * ((code - 24) & 7))) & 0xff;
    return code < 24 ? code + 1 : high;  // 26, 28, 30, 32, 40, 48, 56, 64
}
__device__ __forceinline__ uint32_t v2_fit_width(uint32_t n) {
    const uint32_t w = n <= 32 ? (n + 1) & ~1u : (n + 7) & ~7u;
    return n <= 24 ? n : n <= 64 ? w : 0u;
}

// Bytes and value count of the DIRECT, PATCHED_BASE or DELTA run whose
// header starts x (bytes 0-7 of the run; y and z bytes 8-23), without
// branches; ok false where the run needs the step-by-step checks (a
// PATCHED_BASE patch width that fits nothing, a DELTA varint longer than 8
// bytes).
__device__ __forceinline__ uint32_t v2_long_run(uint64_t x, uint64_t y, uint64_t z, uint32_t &len, bool &ok) {
    const uint32_t b0 = (uint32_t)x & 0xff, b1 = (uint32_t)(x >> 8) & 0xff;
    const uint32_t b2 = (uint32_t)(x >> 16) & 0xff, b3 = (uint32_t)(x >> 24) & 0xff;
    const uint32_t type = b0 >> 6, code = (b0 >> 1) & 31, w = v2_width(code);
    len = (((b0 & 1) << 8) | b1) + 1;
    const uint32_t data = (len * w + 7) >> 3;
    // PATCHED_BASE: 4 header bytes, the base, the data, the patches.
    const uint32_t ew = v2_fit_width(((b3 >> 5) + 1) + v2_width(b2 & 31));
    const uint32_t adv_p = 4 + ((b2 >> 5) + 1) + data + (((b3 & 31) * ew + 7) >> 3);
    // DELTA: two varints from byte 2, then len - 2 deltas of width w (none
    // for width code 0).
    const uint64_t u1 = (x >> 16) | (y << 48);
    const uint64_t t1 = ~u1 & 0x8080808080808080ull;
    const uint32_t s2 = 2 + (uint32_t)(__builtin_ctzll(t1 | (1ull << 63)) >> 3) + 1;  // 3..10
    const uint32_t sh = 8 * (s2 & 7);
    const uint64_t lo = s2 < 8 ? x : y, hi = s2 < 8 ? y : z;
    const uint64_t u2 = sh ? (lo >> sh) | (hi << (64 - sh)) : lo;
    const uint64_t t2 = ~u2 & 0x8080808080808080ull;
    const uint32_t s3 = s2 + (uint32_t)(__builtin_ctzll(t2 | (1ull << 63)) >> 3) + 1;
    const uint32_t nd = len >= 2 ? len - 2 : 0u;
    const uint32_t adv_t = s3 + ((nd * (code ? w : 0u) + 7) >> 3);
    ok = type == 1 || (type == 2 && ew != 0) || (type == 3 && t1 != 0 && t2 != 0);
    return type == 1 ? 2 + data : type == 2 ? adv_p : adv_t;
}

// Index pass, one wave per chunk: the checks of the decoder's header parse,
// in its order.
__global__ void __launch_bounds__(kWave * kV2IndexWpb)
    rle_v2_index(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
                 uint32_t n, V2Split *split, unsigned long long *keys) {
    __shared__ __align__(16) uint32_t s_ring[kV2IndexWpb][V2IndexRing::kLdsWords];
    __shared__ __align__(16) uint32_t s_land[kV2IndexWpb][V2IndexRing::kLand];
    const uint32_t wave = uni(threadIdx.x / kWave);
    const uint32_t c = blockIdx.x * kV2IndexWpb + wave;
    if (c >= n) return;
    V2Split *sp = &split[c];
    if (lane() == 0) keys[2 * c + 1] = ~0ull;  // the decode pass's key
    const uint64_t i0 = coff[c], i1 = coff[c + 1], o0 = ooff[c], o1 = ooff[c + 1];
    const uint32_t in_len = (uint32_t)(i1 - i0), out_len = (uint32_t)(o1 - o0);
    if ((((i1 - i0) | (o1 - o0)) >> 31) != 0 || (out_len & 7) ||
        (reinterpret_cast<uintptr_t>(out + o0) & 7)) {
        if (lane() < kV2Ranges) sp->start[lane()] = make_uint2(0, 0);
        if (lane() == 0) {
            sp->stop = 0;
            keys[2 * c] = error_key(0, CODAG_E_INVALID_ARGUMENT);
        }
        return;
    }
    V2IndexRing in;
    in.init(comp + i0, in_len, s_ring[wave], s_land[wave]);
    const uint32_t end = in.gend, cap = out_len / 8;
    uint32_t pos = in.skip, nv = 0, j = 0, errnv = 0;
    int st = CODAG_OK;
    while (nv < cap) {
        if (pos >= end) {
            st = CODAG_E_TRUNCATED;
            errnv = nv;
            break;
        }
        in.ensure(pos + 24);
        // The 24 bytes from pos: lane k aligns their word k, and six lane
        // reads bring them out (one LDS round trip).
        const uint32_t wa = pos >> 2;
        const uint32_t al = __builtin_amdgcn_alignbit(in.word(wa + lane() + 1), in.word(wa + lane()), 8 * (pos & 3));
        const uint64_t x = ((uint64_t)readlane(al, 1) << 32) | readlane(al, 0);
        const uint32_t b0 = (uint32_t)(x & 0xff), type = b0 >> 6;
        if (type == 0) {
            st = v2_index_short_repeats(in, pos, end, nv, cap, j, sp, errnv);
            if (st) break;
            continue;
        }
        {
            // A run that passes every check and starts no range moves on
            // here; anything else takes the checks below.
            const uint64_t y = ((uint64_t)readlane(al, 3) << 32) | readlane(al, 2);
            const uint64_t z = ((uint64_t)readlane(al, 5) << 32) | readlane(al, 4);
            uint32_t len;
            bool ok;
            const uint32_t adv = v2_long_run(x, y, z, len, ok);
            const bool cut = j < kV2Ranges && nv >= v2_threshold(cap, j);
            if (ok && !cut && len <= cap - nv && adv <= end - pos) {
                pos += adv;
                nv += len;
                continue;
            }
        }
        v2_cut(j, cap, pos, nv, sp);
        errnv = nv;
        if (pos + 2 > end) {
            st = CODAG_E_TRUNCATED;
            break;
        }
        const uint32_t b1 = (uint32_t)((x >> 8) & 0xff);
        const uint32_t len = (((b0 & 1) << 8) | b1) + 1;
        if (type == 1) {
            const uint32_t w = orc_width((b0 >> 1) & 31);
            if (nv + len > cap) { st = CODAG_E_OVERFLOW; break; }
            const uint32_t nbytes = (len * w + 7) >> 3;
            if (pos + 2 + nbytes > end) { st = CODAG_E_TRUNCATED; break; }
            pos += 2 + nbytes;
        } else if (type == 2) {
            if (pos + 4 > end) { st = CODAG_E_TRUNCATED; break; }
            const uint32_t b2 = (uint32_t)((x >> 16) & 0xff), b3 = (uint32_t)((x >> 24) & 0xff);
            const uint32_t w = orc_width((b0 >> 1) & 31);
            const uint32_t bw = (b2 >> 5) + 1, pw = orc_width(b2 & 31);
            const uint32_t pgw = (b3 >> 5) + 1, pll = b3 & 31;
            const uint32_t ew = orc_fit_width(pgw + pw);
            if (ew == 0) { st = CODAG_E_CORRUPT; break; }
            if (nv + len > cap) { st = CODAG_E_OVERFLOW; break; }
            const uint32_t bsec = pos + 4;
            if (bsec + bw > end) { st = CODAG_E_TRUNCATED; break; }
            const uint32_t dsec = bsec + bw, dbytes = (len * w + 7) >> 3;
            if (dsec + dbytes > end) { st = CODAG_E_TRUNCATED; break; }
            const uint32_t psec = dsec + dbytes, pbytes = (pll * ew + 7) >> 3;
            if (psec + pbytes > end) { st = CODAG_E_TRUNCATED; break; }
            pos = psec + pbytes;
        } else {
            const uint32_t code = (b0 >> 1) & 31;
            const uint32_t w = code ? orc_width(code) : 0;
            uint32_t p = pos + 2;
            uint64_t z;
            st = read_varint(in, p, end, z);
            if (st) break;
            st = read_varint(in, p, end, z);
            if (st) break;
            if (nv + len > cap) { st = CODAG_E_OVERFLOW; break; }
            if (w) {
                const uint32_t nd = len >= 2 ? len - 2 : 0, nbytes = (nd * w + 7) >> 3;
                if (p + nbytes > end) { st = CODAG_E_TRUNCATED; break; }
                p += nbytes;
            }
            pos = p;
        }
        nv += len;
    }
    if (st == CODAG_OK && pos != end) {
        st = CODAG_E_CORRUPT;  // input left over once the output is full
        errnv = nv;
    }
    const uint32_t stop = st == CODAG_OK ? nv : errnv;
    // Ranges not started are empty.
    for (uint32_t k = j; k < kV2Ranges; k++)
        if (lane() == 0) sp->start[k] = make_uint2(pos, stop);
    if (lane() == 0) {
        sp->stop = stop;
        keys[2 * c] = st == CODAG_OK ? ~0ull : error_key(errnv, st);
    }
    __builtin_amdgcn_s_waitcnt(0);
}

// Decode pass: wave j of chunk c decodes range j with the plain decoder,
// from its first run to the next range's first value.
__global__ void __launch_bounds__(kWave * kV2DecodeWpb)
    rle_v2_ranges(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
                  uint32_t n, const V2Split *split, unsigned long long *keys) {
    __shared__ __align__(16) uint32_t s_ring[kV2DecodeWpb][kRingLdsWords];
    __shared__ __align__(16) uint32_t s_land[kV2DecodeWpb][kLandWords];
    const uint32_t wave = uni(threadIdx.x / kWave);
    const uint32_t gid = blockIdx.x * kV2DecodeWpb + wave;
    const uint32_t c = gid / kV2Ranges, j = gid % kV2Ranges;
    if (c >= n) return;
    const V2Split *sp = &split[c];
    const uint2 r = sp->start[j];
    const uint32_t e = uni(j + 1 < kV2Ranges ? sp->start[j + 1].y : sp->stop);
    uint32_t pos = uni(r.x), nv = uni(r.y);
    if (nv >= e) return;
    const uint64_t i0 = coff[c], i1 = coff[c + 1], o0 = ooff[c];
    InRing in;
    in.init_at(comp + i0, (uint32_t)(i1 - i0), s_ring[wave], s_land[wave], pos);
    uint64_t *dst = reinterpret_cast<uint64_t *>(out + o0);
    const int st = decode_rle_v2_runs(in, pos, in.gend, dst, nv, e);
    if (st != CODAG_OK && lane() == 0) atomicMin(&keys[2 * c + 1], (unsigned long long)error_key(nv, st));
    __builtin_amdgcn_s_waitcnt(0);
}

size_t rle_v2_split_workspace(uint32_t n) {
    return (size_t)n * kSplitV2WorkspacePerChunk;
}

int launch_rle_v2_split(const uint8_t *comp, const uint64_t *coff, uint8_t *out,
                        const uint64_t *ooff, uint32_t n, int32_t *status, unsigned long long *err,
                        hipStream_t s, void *workspace) {
    void *ws = workspace;
    if (!ws && hipMallocAsync(&ws, rle_v2_split_workspace(n), s) != hipSuccess) return CODAG_E_HIP;
    V2Split *split = static_cast<V2Split *>(ws);
    unsigned long long *keys =
        reinterpret_cast<unsigned long long *>(static_cast<char *>(ws) + (size_t)n * sizeof(V2Split));
    hipLaunchKernelGGL(rle_v2_index, dim3((n + kV2IndexWpb - 1) / kV2IndexWpb),
                       dim3(kWave * kV2IndexWpb), 0, s, comp, coff, out, ooff, n, split, keys);
    const uint32_t gb = (uint32_t)(((uint64_t)n * kV2Ranges + kV2DecodeWpb - 1) / kV2DecodeWpb);
    hipLaunchKernelGGL(rle_v2_ranges, dim3(gb), dim3(kWave * kV2DecodeWpb), 0, s, comp, coff, out,
                       ooff, n, split, keys);
    hipLaunchKernelGGL(split_finish, dim3((n + 255) / 256), dim3(256), 0, s, n, keys, status, err);
    hipError_t e = hipGetLastError();
    if (!workspace && hipFreeAsync(ws, s) != hipSuccess) return CODAG_E_HIP;
    return e == hipSuccess ? CODAG_OK : CODAG_E_HIP;
}

}  // namespace codag
