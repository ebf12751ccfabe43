/*
 * codag.h -- chunk-parallel decompression on AMD Instinct MI355X (gfx950).
 *
 * The operation (CODAG, Section II-B and Section IV-A): the input is a set of
 * independently compressed chunks described by offset metadata; every chunk
 * is decoded by one decompression unit (here one 64-lane wavefront) whose
 * lanes all take part in decoding, reading and writing.  Codecs (Section
 * V-A): ORC integer RLE v1 and RLE v2 (signed int64 columns) and raw Deflate
 * (RFC 1951), one independent stream per chunk.
 *
 * All entry points are plain C.  Buffers are caller-owned device memory;
 * the library never frees them and keeps no pointer to them once the
 * enqueued work has completed.  "stream" is a hipStream_t (NULL = the null
 * stream).  Calls enqueue work and return without synchronizing, except
 * codag_get_error, which synchronizes the given stream.
 */
#ifndef CODAG_H
#define CODAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Codecs. */
enum {
    CODAG_RLE_V1 = 1,  /* ORC integer RLE v1, signed int64 (zigzag varints) */
    CODAG_RLE_V2 = 2,  /* ORC integer RLE v2, signed int64 */
    CODAG_DEFLATE = 3  /* raw RFC 1951 stream per chunk */
};

/* Status codes: return values and per-chunk statuses. */
enum {
    CODAG_OK = 0,
    CODAG_E_INVALID_ARGUMENT = -1, /* bad codec/pointer/size; per chunk: bad output range */
    CODAG_E_HIP = -2,              /* a HIP runtime call or kernel launch failed */
    CODAG_E_CORRUPT = -3,          /* the chunk's stream violates its format */
    CODAG_E_TRUNCATED = -4,        /* the chunk's stream ends before its output is complete */
    CODAG_E_OVERFLOW = -5,         /* the stream decodes to more bytes than the output range */
    CODAG_E_UNDERFLOW = -6         /* Deflate: the final block ends before the output range is full */
};

/*
 * Tuning knobs; a zeroed struct (or NULL) selects the defaults.
 *   waves_per_block   wavefronts per workgroup: 1, 2 or 4 (default 4); waves
 *                     never synchronize with each other, so this only
 *                     shapes occupancy and dispatch.
 *   lit_table_bits    Deflate literal/length lookup-table bits, 9 or 10
 *                     (default 10); longer codes take a slower path.
 *   history_kib       Deflate history window kept in LDS per wave: 8, 16 or
 *                     32 KiB (default 8).  Back-references reaching further
 *                     read the already written output from HBM.  With 32 the
 *                     workgroup holds one wave.
 *   chunk_ticks       optional device array (n_chunks uint64): receives each
 *                     chunk's decode time in shader clock cycles.
 */
typedef struct codag_opts {
    int waves_per_block;
    int lit_table_bits;
    uint64_t *chunk_ticks;
    int history_kib;
    int reserved[7];
} codag_opts;

/*
 * Decompress n_chunks chunks of one codec.
 *
 *   comp_buf       device, the compressed bytes.
 *   chunk_offsets  device, n_chunks + 1 non-decreasing uint64: chunk i is
 *                  comp_buf[chunk_offsets[i] .. chunk_offsets[i+1]).  Input
 *                  ranges may overlap.  Loads stay inside the 16-byte-aligned
 *                  hull of each chunk's range.  A chunk's compressed length
 *                  is below 2^31 bytes (Deflate: below 2^28), otherwise the
 *                  chunk fails with CODAG_E_INVALID_ARGUMENT.
 *   out_buf        device, the decompressed bytes.
 *   out_offsets    device, n_chunks + 1 non-decreasing uint64: chunk i
 *                  decodes into out_buf[out_offsets[i] .. out_offsets[i+1]),
 *                  which it must fill exactly (below 2^31 bytes).  Output
 *                  ranges must not
 *                  overlap.  For the RLE codecs each range is a whole number
 *                  of little-endian int64 values and starts 8-byte aligned
 *                  (otherwise the chunk fails with CODAG_E_INVALID_ARGUMENT
 *                  and nothing is written for it).
 *   n_chunks       number of chunks, below 2^32 - 64 (0 is a no-op).
 *   stream         hipStream_t the work is enqueued on.
 *
 * Returns CODAG_OK once the work is enqueued, CODAG_E_INVALID_ARGUMENT for an
 * unknown codec or a NULL pointer with n_chunks > 0, or CODAG_E_HIP if the
 * launch fails.  Per-chunk failures are reported asynchronously: they are
 * latched into a per-device error word read by codag_get_error.  Whatever
 * the input bytes, no chunk writes outside its output range and every chunk
 * finishes in bounded time; a failed chunk's output bytes are unspecified.
 */
int codag_decompress(int codec, const uint8_t *comp_buf, const uint64_t *chunk_offsets,
                     uint8_t *out_buf, const uint64_t *out_offsets, uint64_t n_chunks,
                     void *stream);

/*
 * As codag_decompress, plus:
 *   chunk_status   device, n_chunks int32 (may be NULL): receives each
 *                  chunk's status (CODAG_OK or a CODAG_E_* code).
 *   opts           tuning knobs (may be NULL).
 */
int codag_decompress_ex(int codec, const uint8_t *comp_buf, const uint64_t *chunk_offsets,
                        uint8_t *out_buf, const uint64_t *out_offsets, uint64_t n_chunks,
                        void *stream, int32_t *chunk_status, const codag_opts *opts);

/*
 * Synchronize `stream`, then return the status of the lowest-indexed chunk
 * that failed in any call on the current device since the previous
 * codag_get_error (CODAG_OK if none), storing that chunk's index in
 * *first_bad_chunk (may be NULL; UINT64_MAX if none).  Clears the error word.
 * Returns CODAG_E_HIP if synchronization or the read fails.
 */
int codag_get_error(void *stream, uint64_t *first_bad_chunk);

/* A static, human-readable name for a status code. */
const char *codag_status_string(int status);

/* Release the library's per-device resources (error words).  Any later call
 * re-creates them. */
void codag_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* CODAG_H */
