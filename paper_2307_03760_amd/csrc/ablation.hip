// The paper's decoding-unit ablations, on the same chunks and with the same
// statuses as the main decoders:
//
//   * Leader lane (CODAG Section V-E, single-thread decoding): one lane
//     parses every header, varint and Huffman token and hands each result to
//     the wave through LDS; the other lanes only write output.  (The main
//     decoders have every lane take part in decoding: ballot-split varints,
//     a candidate token per lane.)
//   * Prefetch wave (Section V-F): a second wave per chunk loads the input
//     into an LDS ring ahead of the decoding wave, which runs the main
//     decoder unchanged and only waits for bytes.
//   * Block leader (Section II-C, the design CODAG argues against): a
//     256-thread workgroup per chunk whose thread 0 parses every group while
//     the other threads wait at a barrier, then all of them write it.
//     RLE v1 only.
#include <hip/hip_runtime.h>

#include "../../include/codag.h"
#include "decode.hpp"
#include "internal.hpp"

namespace codag {

// ---- RLE v1 by a leader thread --------------------------------------------

constexpr uint32_t kLeadWindow = 2048;  // staged input bytes
constexpr uint32_t kLeadGroupMax = 1300;  // a group's bytes: at most 1 + 10 * 128

struct LeadLds {
    uint32_t buf[kLeadWindow / 4];
    uint64_t vals[128];
    uint64_t base, delta;
    uint32_t req;                      // window requested by the leader (~0: none)
    uint32_t st, kind, len, n0, done;  // the leader's result for the group
};

template <int UNIT>
__device__ __forceinline__ void unit_barrier() {
    if constexpr (UNIT == kWave) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// One varint at p read by the leader from the staged window (bytes past the
// end of the chunk are zero): the sequential decoder's rules.
__device__ __forceinline__ int lead_varint(const LeadLds *L, uint32_t wb, uint32_t p, uint32_t end,
                                           uint64_t &z, uint32_t &nb) {
    z = 0;
    uint32_t b = 0, i = 0;
    for (; i < 10; i++) {
        const uint32_t r = p + i - wb;
        b = (L->buf[r >> 2] >> (8 * (r & 3))) & 0xff;
        z |= (uint64_t)(b & 0x7f) << (7 * i);
        if (b < 128) break;
    }
    if (i == 10) return CODAG_E_CORRUPT;  // no terminator in ten bytes
    nb = i + 1;
    if (nb == 10 && b > 1) return CODAG_E_CORRUPT;  // bits above bit 63
    if (p + nb > end) return CODAG_E_TRUNCATED;
    return CODAG_OK;
}

// RLE v1 decoded by thread 0 of a unit of UNIT threads (a wave, or a
// 256-thread workgroup): per group, the unit stages input if the leader
// asks, the leader parses the group into LDS, and after a barrier the unit
// writes it.
template <int UNIT>
__device__ int rle_v1_leader(const uint8_t *chunk, uint32_t in_len, uint64_t *out, uint32_t cap,
                             LeadLds *L) {
    const uint32_t t = UNIT == kWave ? lane() : threadIdx.x;
    const uint32_t skip = (uint32_t)(reinterpret_cast<uintptr_t>(chunk) & 15);
    const uint8_t *gbase = chunk - skip;
    const uint32_t end = skip + in_len;
    uint32_t pos = skip, n = 0, wb = 0;  // the leader's state (thread 0)
    bool staged = false;
    for (;;) {
        if (t == 0) {
            uint32_t req = ~0u;
            if (!staged || pos + kLeadGroupMax > wb + kLeadWindow) {
                req = pos & ~15u;
                wb = req;
                staged = true;
            }
            L->req = req;
        }
        unit_barrier<UNIT>();
        const uint32_t req = L->req;
        if (req != ~0u) {
            for (uint32_t q = t; q < kLeadWindow / 16; q += UNIT) {
                const uint32_t at = req + 16 * q;
                uint4 v = make_uint4(0, 0, 0, 0);
                if (at < end) v = *reinterpret_cast<const uint4 *>(gbase + at);
                if (at + 16 > end) {
                    const uint32_t valid = at < end ? end - at : 0;
                    uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const int keep = (int)valid - 4 * j;
                        w[j] &= keep >= 4 ? 0xffffffffu : keep <= 0 ? 0u : ((1u << (8 * keep)) - 1);
                    }
                    v = make_uint4(w[0], w[1], w[2], w[3]);
                }
                reinterpret_cast<uint4 *>(L->buf)[q] = v;
            }
            unit_barrier<UNIT>();
        }
        if (t == 0) {
            // The group at pos: header, validity, capacity, payload.
            int st = CODAG_OK;
            uint32_t kind = 0, len = 0;
            const uint32_t n0 = n;
            if (n >= cap) {
                // Nothing to decode (an empty output range): only leftover
                // input can be wrong, checked below.
            } else if (pos >= end) {
                st = CODAG_E_TRUNCATED;
            } else {
                const uint32_t r = pos - wb;
                const int32_t h = (int8_t)((L->buf[r >> 2] >> (8 * (r & 3))) & 0xff);
                if (h >= 0) {
                    len = (uint32_t)h + 3;
                    if (pos + 2 > end) {
                        st = CODAG_E_TRUNCATED;
                    } else {
                        const uint32_t r1 = r + 1;
                        const int32_t delta = (int8_t)((L->buf[r1 >> 2] >> (8 * (r1 & 3))) & 0xff);
                        uint64_t z;
                        uint32_t nb = 0;
                        st = lead_varint(L, wb, pos + 2, end, z, nb);
                        if (st == CODAG_OK) {
                            pos += 2 + nb;
                            if (n + len > cap) {
                                st = CODAG_E_OVERFLOW;
                            } else {
                                L->base = unzigzag(z);
                                L->delta = (uint64_t)(int64_t)delta;
                                kind = 1;
                                n += len;
                            }
                        }
                    }
                } else {
                    len = (uint32_t)(-h);
                    pos += 1;
                    if (n + len > cap) {
                        st = CODAG_E_OVERFLOW;
                    } else {
                        for (uint32_t i = 0; i < len; i++) {
                            uint64_t z;
                            uint32_t nb = 0;
                            st = lead_varint(L, wb, pos, end, z, nb);
                            if (st != CODAG_OK) break;
                            L->vals[i] = unzigzag(z);
                            pos += nb;
                        }
                        if (st == CODAG_OK) {
                            kind = 2;
                            n += len;
                        }
                    }
                }
            }
            uint32_t done = st != CODAG_OK || n >= cap;
            if (st == CODAG_OK && n >= cap && pos != end) st = CODAG_E_CORRUPT;  // input left over
            L->st = (uint32_t)st;
            L->kind = kind;
            L->len = len;
            L->n0 = n0;
            L->done = done;
        }
        unit_barrier<UNIT>();
        const uint32_t kind = L->kind, len = L->len, n0 = L->n0;
        if (kind == 1) {
            const uint64_t base = L->base, delta = L->delta;
            for (uint32_t i = t; i < len; i += UNIT) out[n0 + i] = base + (uint64_t)i * delta;
        } else if (kind == 2) {
            for (uint32_t i = t; i < len; i += UNIT) out[n0 + i] = L->vals[i];
        }
        const uint32_t done = L->done, st = L->st;
        unit_barrier<UNIT>();  // the next group's staging and results overwrite LDS
        if (done) return (int)st;
    }
}

__device__ __forceinline__ bool rle_args_ok(const uint64_t *coff, const uint64_t *ooff, uint8_t *out,
                                            uint32_t c, uint32_t &in_len, uint32_t &out_len) {
    const uint64_t i0 = coff[c], i1 = coff[c + 1], o0 = ooff[c], o1 = ooff[c + 1];
    if ((((i1 - i0) | (o1 - o0)) >> 31) != 0) return false;
    in_len = (uint32_t)(i1 - i0);
    out_len = (uint32_t)(o1 - o0);
    return !((out_len & 7) || (reinterpret_cast<uintptr_t>(out + o0) & 7));
}

// Leader lane: WPB independent waves per workgroup, one chunk each.
template <int WPB>
__global__ void __launch_bounds__(kWave * WPB)
    rle_v1_leader_lane(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
                       uint32_t n, int32_t *status, unsigned long long *err) {
    __shared__ LeadLds s_lead[WPB];
    const uint32_t wave = uni(threadIdx.x / kWave), c = blockIdx.x * WPB + wave;
    if (c >= n) return;
    uint32_t in_len, out_len;
    int st = CODAG_E_INVALID_ARGUMENT;
    if (rle_args_ok(coff, ooff, out, c, in_len, out_len))
        st = rle_v1_leader<kWave>(comp + coff[c], in_len, reinterpret_cast<uint64_t *>(out + ooff[c]),
                                  out_len / 8, &s_lead[wave]);
    report(c, st, status, err);
}

// Block leader: one 256-thread workgroup per chunk.
constexpr int kBlockLeaderThreads = 256;
__global__ void __launch_bounds__(kBlockLeaderThreads)
    rle_v1_block_leader(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
                        uint32_t n, int32_t *status, unsigned long long *err) {
    __shared__ LeadLds s_lead;
    const uint32_t c = blockIdx.x;
    if (c >= n) return;
    uint32_t in_len, out_len;
    int st = CODAG_E_INVALID_ARGUMENT;
    if (rle_args_ok(coff, ooff, out, c, in_len, out_len))
        st = rle_v1_leader<kBlockLeaderThreads>(comp + coff[c], in_len,
                                                reinterpret_cast<uint64_t *>(out + ooff[c]), out_len / 8,
                                                &s_lead);
    if (threadIdx.x < kWave) report(c, st, status, err);
}

// ---- Deflate by a leader lane ----------------------------------------------

template <int TB, uint32_t H>
__global__ void __launch_bounds__(kWave)
    deflate_leader_lane(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
                        uint32_t n, int32_t *status, unsigned long long *err) {
    __shared__ __align__(16) uint32_t s_ring[kRingLdsWords];
    __shared__ __align__(16) uint32_t s_land[kLandWords];
    __shared__ __align__(16) DeflateLds<TB, H> s_lds;
    const uint32_t c = blockIdx.x;
    if (c >= n) return;
    const uint64_t i0 = coff[c], i1 = coff[c + 1], o0 = ooff[c], o1 = ooff[c + 1];
    int st = CODAG_E_INVALID_ARGUMENT;
    if (((((i1 - i0) | (o1 - o0)) >> 31) == 0) && (i1 - i0) < (1u << 28)) {
        InRing in;
        in.init(comp + i0, (uint32_t)(i1 - i0), s_ring, s_land);
        st = decode_deflate<TB, H, kLeaderLane>(in, out + o0, (uint32_t)(o1 - o0), &s_lds);
        __builtin_amdgcn_s_waitcnt(0);
    }
    report(c, st, status, err);
}

// ---- the main decoders behind a prefetch wave ------------------------------

template <int Codec, int TB, uint32_t H>
__global__ void __launch_bounds__(2 * kWave)
    decode_prefetch(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
                    uint32_t n, int32_t *status, unsigned long long *err) {
    __shared__ __align__(16) PrefetchShared s_pf;
    __shared__ __align__(16) WaveScratch<Codec, TB, H> s_scratch;
    const uint32_t wave = uni(threadIdx.x / kWave), c = blockIdx.x;
    if (c >= n) return;
    const uint64_t i0 = coff[c], i1 = coff[c + 1], o0 = ooff[c], o1 = ooff[c + 1];
    bool ok = ((((i1 - i0) | (o1 - o0)) >> 31) == 0);
    if (Codec == CODAG_DEFLATE) ok = ok && (i1 - i0) < (1u << 28);
    else ok = ok && !(((o1 - o0) & 7) || (reinterpret_cast<uintptr_t>(out + o0) & 7));
    if (threadIdx.x == 0) {
        s_pf.filled = 0;
        s_pf.need = 0;
        s_pf.done = ok ? 0u : 1u;
    }
    __syncthreads();
    if (wave == 1) {
        if (ok) prefetch_loader(comp + i0, (uint32_t)(i1 - i0), &s_pf);
        return;
    }
    int st = CODAG_E_INVALID_ARGUMENT;
    if (ok) {
        PrefetchRing in;
        in.init(comp + i0, (uint32_t)(i1 - i0), &s_pf);
        if constexpr (Codec == CODAG_DEFLATE)
            st = decode_deflate<TB, H>(in, out + o0, (uint32_t)(o1 - o0), &s_scratch.t);
        else
            st = decode_rle_v1(in, reinterpret_cast<uint64_t *>(out + o0), (uint32_t)(o1 - o0) / 8);
        in.finish();
        __builtin_amdgcn_s_waitcnt(0);
    }
    report(c, st, status, err);
}

int launch_variant(int variant, int codec, const uint8_t *comp, const uint64_t *coff, uint8_t *out,
                   const uint64_t *ooff, uint32_t n, int32_t *status, unsigned long long *err,
                   hipStream_t s) {
    if (codec == CODAG_RLE_V1) {
        if (variant == CODAG_VARIANT_LEADER_LANE)
            hipLaunchKernelGGL(rle_v1_leader_lane<4>, dim3((n + 3) / 4), dim3(4 * kWave), 0, s, comp, coff,
                               out, ooff, n, status, err);
        else if (variant == CODAG_VARIANT_PREFETCH_WAVE)
            hipLaunchKernelGGL((decode_prefetch<CODAG_RLE_V1, 10, 0>), dim3(n), dim3(2 * kWave), 0, s, comp,
                               coff, out, ooff, n, status, err);
        else if (variant == CODAG_VARIANT_BLOCK_LEADER)
            hipLaunchKernelGGL(rle_v1_block_leader, dim3(n), dim3(kBlockLeaderThreads), 0, s, comp, coff,
                               out, ooff, n, status, err);
        else
            return CODAG_E_INVALID_ARGUMENT;
    } else if (codec == CODAG_DEFLATE) {
        if (variant == CODAG_VARIANT_LEADER_LANE)
            hipLaunchKernelGGL((deflate_leader_lane<9, 4096>), dim3(n), dim3(kWave), 0, s, comp, coff, out,
                               ooff, n, status, err);
        else if (variant == CODAG_VARIANT_PREFETCH_WAVE)
            hipLaunchKernelGGL((decode_prefetch<CODAG_DEFLATE, 9, 4096>), dim3(n), dim3(2 * kWave), 0, s,
                               comp, coff, out, ooff, n, status, err);
        else
            return CODAG_E_INVALID_ARGUMENT;
    } else {
        return CODAG_E_INVALID_ARGUMENT;
    }
    return hipGetLastError() == hipSuccess ? CODAG_OK : CODAG_E_HIP;
}

}  // namespace codag
