// Kernels and the C ABI of the chunk-parallel decompressor.
//
// One 64-lane wavefront decodes one chunk (CODAG Section IV-C: the warp is
// the decompression unit); a workgroup holds `waves_per_block` independent
// waves that never synchronize with each other, so workgroups are only a
// dispatch and LDS-allocation unit.  Chunk i of the plain launch is handled
// by wave (blockIdx.x * waves_per_block + wave) and the hardware dispatcher
// balances uneven chunks by handing out workgroups as slots free up.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/codag.h"
#include "decode.hpp"
#include "internal.hpp"

namespace codag {

// Plain launch: one chunk per wave, WPB waves per workgroup, every chunk of
// one codec.  Each wave's LDS is a slice of three distinct arrays so the
// compiler can tell ring reads from landing-buffer fetches.
template <int Codec, int TB, uint32_t H, int WPB>
__global__ void __launch_bounds__(kWave * WPB)
    decode_plain(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
                 uint32_t n, int32_t *status, unsigned long long *err, uint64_t *ticks) {
    __shared__ __align__(16) uint32_t s_ring[WPB][ring_lds_words<Codec>()];
    __shared__ __align__(16) uint32_t s_land[WPB][land_lds_words<Codec>()];
    __shared__ __align__(16) WaveScratch<Codec, TB, H> s_scratch[WPB];
    uint32_t wave = uni(threadIdx.x / kWave);
    uint32_t c = blockIdx.x * WPB + wave;
    if (c >= n) return;
    uint64_t t0 = ticks ? __builtin_amdgcn_s_memtime() : 0;
    int st = decode_one<Codec, TB, H>(comp, coff, out, ooff, c, s_ring[wave], s_land[wave],
                                      &s_scratch[wave]);
    if (ticks && lane() == 0) ticks[c] = __builtin_amdgcn_s_memtime() - t0;
    report(c, st, status, err);
}

}  // namespace codag

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

namespace codag {

// The per-device first-error word, (chunk << 4) | -status of the smallest
// failing chunk, all ones when there is none; and the slot codag_get_error's
// exchange writes the taken value to.  Device globals, so the library
// allocates nothing for them; each device holds its own copy.
__device__ unsigned long long g_error_word[2] = {~0ull, ~0ull};

// Scratch memory of codag_decompress_noalloc: the workspace of the
// group-parallel RLE paths at their default chunk limits (RLE v1: 256
// chunks; RLE v2: 2048 chunks, the larger), held by every device the library
// runs on until the process ends.  Host code never uses this name as an
// address: device_state looks up each device's copy once.
constexpr size_t kNoAllocScratchBytes =
    kSplitMaxChunks * kSplitWorkspacePerChunk > kSplitV2MaxChunks * kSplitV2WorkspacePerChunk
        ? kSplitMaxChunks * kSplitWorkspacePerChunk
        : kSplitV2MaxChunks * kSplitV2WorkspacePerChunk;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
static_assert(kNoAllocScratchBytes == CODAG_NOALLOC_SCRATCH_BYTES, "header limit");

// Takes the error word and leaves "no error" in one atomic step, so a
// failure recorded by a kernel on another stream is either taken here or
// stays for the next call.
__global__ void take_error(unsigned long long *word) {
    if (threadIdx.x == 0) word[1] = atomicExch(&word[0], ~0ull);
}

std::mutex g_mu;
DeviceState g_dev[kMaxDevices];

int device_state(DeviceState **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CODAG_E_HIP;
    std::lock_guard<std::mutex> lock(g_mu);
    DeviceState &s = g_dev[dev];
    if (!s.err) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_error_word)) != hipSuccess || !p) return CODAG_E_HIP;
        void *q = nullptr;
        if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return CODAG_E_HIP;
        s.scratch = q;
        s.err = static_cast<unsigned long long *>(p);
    }
    *out = &s;
    return CODAG_OK;
}

}  // namespace codag

namespace {

using namespace codag;

template <int Codec, int TB, uint32_t H, int WPB>
int launch_wpb(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
               uint64_t n, int32_t *status, unsigned long long *err, uint64_t *ticks,
               hipStream_t stream) {
    uint64_t grid = (n + WPB - 1) / WPB;
    hipLaunchKernelGGL((decode_plain<Codec, TB, H, WPB>), dim3((uint32_t)grid), dim3(kWave * WPB),
                       0, stream, comp, coff, out, ooff, (uint32_t)n, status, err, ticks);
    return hipGetLastError() == hipSuccess ? CODAG_OK : CODAG_E_HIP;
}

template <int Codec, int TB, uint32_t H>
int launch_plain(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
                 uint64_t n, int wpb, int32_t *status, unsigned long long *err, uint64_t *ticks,
                 hipStream_t stream) {
    switch (wpb) {
        case 1: return launch_wpb<Codec, TB, H, 1>(comp, coff, out, ooff, n, status, err, ticks, stream);
        case 2: return launch_wpb<Codec, TB, H, 2>(comp, coff, out, ooff, n, status, err, ticks, stream);
        default: return launch_wpb<Codec, TB, H, 4>(comp, coff, out, ooff, n, status, err, ticks, stream);
    }
}

// LZ4 keeps the Deflate window sizes (its offsets reach 64 KiB; farther
// matches read the written output from HBM).
int launch_lz4(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
               uint64_t n, int wpb, int hist_kib, int32_t *status, unsigned long long *err,
               uint64_t *ticks, hipStream_t stream) {
    switch (hist_kib) {
        case 2: return launch_plain<CODAG_LZ4, 9, 2048>(comp, coff, out, ooff, n, wpb, status, err, ticks, stream);
        case 4: return launch_plain<CODAG_LZ4, 9, 4096>(comp, coff, out, ooff, n, wpb, status, err, ticks, stream);
        case 8: return launch_plain<CODAG_LZ4, 9, 8192>(comp, coff, out, ooff, n, wpb, status, err, ticks, stream);
        case 16: return launch_plain<CODAG_LZ4, 9, 16384>(comp, coff, out, ooff, n, wpb, status, err, ticks, stream);
        default: return launch_wpb<CODAG_LZ4, 9, 32768, 1>(comp, coff, out, ooff, n, status, err, ticks, stream);
    }
}

template <int TB>
int launch_deflate(const uint8_t *comp, const uint64_t *coff, uint8_t *out, const uint64_t *ooff,
                   uint64_t n, int wpb, int hist_kib, int32_t *status, unsigned long long *err,
                   uint64_t *ticks, hipStream_t stream) {
    if (hist_kib == 16)
        return launch_plain<CODAG_DEFLATE, TB, 16384>(comp, coff, out, ooff, n, wpb, status, err,
                                                      ticks, stream);
    if (hist_kib == 2)
        return launch_plain<CODAG_DEFLATE, TB, 2048>(comp, coff, out, ooff, n, wpb, status, err,
                                                     ticks, stream);
    if (hist_kib == 4)
        return launch_plain<CODAG_DEFLATE, TB, 4096>(comp, coff, out, ooff, n, wpb, status, err,
                                                     ticks, stream);
    if (hist_kib == 32)
        return launch_wpb<CODAG_DEFLATE, TB, 32768, 1>(comp, coff, out, ooff, n, status, err,
                                                       ticks, stream);
    return launch_plain<CODAG_DEFLATE, TB, 8192>(comp, coff, out, ooff, n, wpb, status, err, ticks,
                                                 stream);
}

}  // namespace

namespace {

// codag_decompress_ex, and with noalloc its variant that takes every
// workspace from the device's static scratch array.
int decompress(int codec, const uint8_t *comp_buf, const uint64_t *chunk_offsets, uint8_t *out_buf,
               const uint64_t *out_offsets, uint64_t n_chunks, void *stream, int32_t *chunk_status,
               const codag_opts *opts, bool noalloc) {
    if (codec < CODAG_RLE_V1 || codec > CODAG_LZ4) return CODAG_E_INVALID_ARGUMENT;
    const bool lz77 = codec == CODAG_DEFLATE || codec == CODAG_LZ4;
    const int eb = opts && opts->elem_bytes ? opts->elem_bytes : 8;
    const int uns = opts ? opts->unsigned_values : 0;
    if ((eb != 1 && eb != 2 && eb != 4 && eb != 8) || (uns != 0 && uns != 1)) return CODAG_E_INVALID_ARGUMENT;
    // Byte RLE, and RLE element types other than signed 8-byte values, take
    // the one-wave-per-chunk typed decoder.
    const bool typed = codec == CODAG_BYTE_RLE || (!lz77 && (eb != 8 || uns));
    if (typed && opts && (opts->variant || opts->group_parallel == 2)) return CODAG_E_INVALID_ARGUMENT;
    if (n_chunks == 0) return CODAG_OK;
    if (!comp_buf || !chunk_offsets || !out_buf || !out_offsets) return CODAG_E_INVALID_ARGUMENT;
    if (n_chunks >= (1ull << 32) - 64) return CODAG_E_INVALID_ARGUMENT;
    // Defaults: RLE waves share a workgroup; Deflate and LZ4 waves go one
    // per workgroup with a small window (and table), for the most resident
    // waves.
    int wpb = opts && opts->waves_per_block ? opts->waves_per_block : lz77 ? 1 : 4;
    int tb = opts && opts->lit_table_bits ? opts->lit_table_bits : 9;
    // LZ4 batches fit a 2 KiB window, and the smaller window keeps more
    // waves resident; Deflate's token batches want 4 KiB.
    int hist = opts && opts->history_kib ? opts->history_kib : codec == CODAG_LZ4 ? 2 : 4;
    if (opts && (opts->group_parallel < 0 || opts->group_parallel > 2)) return CODAG_E_INVALID_ARGUMENT;
    if (opts && opts->group_parallel == 2 && opts->chunk_ticks) return CODAG_E_INVALID_ARGUMENT;
    if ((wpb != 1 && wpb != 2 && wpb != 4) || (tb != 9 && tb != 10) ||
        (hist != 2 && hist != 4 && hist != 8 && hist != 16 && hist != 32))
        return CODAG_E_INVALID_ARGUMENT;
    uint64_t *ticks = opts ? opts->chunk_ticks : nullptr;
    const int variant = opts ? opts->variant : 0;
    if (variant < 0 || variant > CODAG_VARIANT_BLOCK_LEADER || (variant && ticks))
        return CODAG_E_INVALID_ARGUMENT;
    DeviceState *ds = nullptr;
    int st = device_state(&ds);
    if (st) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (variant)
        return launch_variant(variant, codec, comp_buf, chunk_offsets, out_buf, out_offsets,
                              (uint32_t)n_chunks, chunk_status, ds->err, s);
    if (typed)
        return launch_typed(codec, eb, uns != 0, comp_buf, chunk_offsets, out_buf, out_offsets,
                            (uint32_t)n_chunks, chunk_status, ds->err, ticks, s);
    switch (codec) {
        case CODAG_RLE_V1: {
            const int gp = opts ? opts->group_parallel : 0;
            if (gp == 2 || (gp == 0 && !ticks && n_chunks <= kSplitMaxChunks)) {
                if (noalloc && rle_v1_split_workspace((uint32_t)n_chunks) > kNoAllocScratchBytes)
                    return CODAG_E_INVALID_ARGUMENT;
                return launch_rle_v1_split(comp_buf, chunk_offsets, out_buf, out_offsets,
                                           (uint32_t)n_chunks, chunk_status, ds->err, s,
                                           noalloc ? ds->scratch : nullptr);
            }
        }
            return launch_plain<CODAG_RLE_V1, 10, 0>(comp_buf, chunk_offsets, out_buf, out_offsets,
                                                     n_chunks, wpb, chunk_status, ds->err, ticks, s);
        case CODAG_RLE_V2: {
            const int gp = opts ? opts->group_parallel : 0;
            if (gp == 2 || (gp == 0 && !ticks && n_chunks <= kSplitV2MaxChunks)) {
                if (noalloc && rle_v2_split_workspace((uint32_t)n_chunks) > kNoAllocScratchBytes)
                    return CODAG_E_INVALID_ARGUMENT;
                return launch_rle_v2_split(comp_buf, chunk_offsets, out_buf, out_offsets,
                                           (uint32_t)n_chunks, chunk_status, ds->err, s,
                                           noalloc ? ds->scratch : nullptr);
            }
        }
            return launch_plain<CODAG_RLE_V2, 10, 0>(comp_buf, chunk_offsets, out_buf, out_offsets,
                                                     n_chunks, wpb, chunk_status, ds->err, ticks, s);
        case CODAG_LZ4:
            return launch_lz4(comp_buf, chunk_offsets, out_buf, out_offsets, n_chunks, wpb, hist,
                              chunk_status, ds->err, ticks, s);
        default:
            if (tb == 9)
                return launch_deflate<9>(comp_buf, chunk_offsets, out_buf, out_offsets, n_chunks,
                                         wpb, hist, chunk_status, ds->err, ticks, s);
            return launch_deflate<10>(comp_buf, chunk_offsets, out_buf, out_offsets, n_chunks, wpb,
                                      hist, chunk_status, ds->err, ticks, s);
    }
}

}  // namespace

extern "C" {

int codag_decompress_ex(int codec, const uint8_t *comp_buf, const uint64_t *chunk_offsets,
                        uint8_t *out_buf, const uint64_t *out_offsets, uint64_t n_chunks,
                        void *stream, int32_t *chunk_status, const codag_opts *opts) {
    return decompress(codec, comp_buf, chunk_offsets, out_buf, out_offsets, n_chunks, stream,
                      chunk_status, opts, false);
}

int codag_decompress_noalloc(int codec, const uint8_t *comp_buf, const uint64_t *chunk_offsets,
                             uint8_t *out_buf, const uint64_t *out_offsets, uint64_t n_chunks,
                             void *stream, int32_t *chunk_status, const codag_opts *opts) {
    return decompress(codec, comp_buf, chunk_offsets, out_buf, out_offsets, n_chunks, stream,
                      chunk_status, opts, true);
}

int codag_decompress(int codec, const uint8_t *comp_buf, const uint64_t *chunk_offsets,
                     uint8_t *out_buf, const uint64_t *out_offsets, uint64_t n_chunks,
                     void *stream) {
    return codag_decompress_ex(codec, comp_buf, chunk_offsets, out_buf, out_offsets, n_chunks,
                               stream, nullptr, nullptr);
}

int codag_get_error(void *stream, uint64_t *first_bad_chunk) {
    if (first_bad_chunk) *first_bad_chunk = UINT64_MAX;
    DeviceState *ds = nullptr;
    int st = device_state(&ds);
    if (st) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned long long key = ~0ull;
    {
        // One taker at a time per process: the result slot is shared.
        static std::mutex take_mu;
        std::lock_guard<std::mutex> lock(take_mu);
        hipLaunchKernelGGL(take_error, dim3(1), dim3(64), 0, s, ds->err);
        if (hipGetLastError() != hipSuccess) return CODAG_E_HIP;
        if (hipMemcpyAsync(&key, ds->err + 1, sizeof(key), hipMemcpyDeviceToHost, s) != hipSuccess)
            return CODAG_E_HIP;
        if (hipStreamSynchronize(s) != hipSuccess) return CODAG_E_HIP;
    }
    if (key == ~0ull) return CODAG_OK;
    if (first_bad_chunk) *first_bad_chunk = key >> 4;
    return -(int)(key & 15);
}

const char *codag_status_string(int status) {
    switch (status) {
        case CODAG_OK: return "ok";
        case CODAG_E_INVALID_ARGUMENT: return "invalid argument";
        case CODAG_E_HIP: return "HIP runtime error";
        case CODAG_E_CORRUPT: return "corrupt stream";
        case CODAG_E_TRUNCATED: return "truncated stream";
        case CODAG_E_OVERFLOW: return "output range too small";
        case CODAG_E_UNDERFLOW: return "output range too large";
        default: return "unknown status";
    }
}

void codag_shutdown(void) {
    // Nothing is allocated per device; forget the looked-up addresses.
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto &s : g_dev) s = DeviceState{};
}

}  // extern "C"
