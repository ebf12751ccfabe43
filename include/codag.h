/*
 * codag.h -- chunk-parallel decompression on AMD Instinct MI355X (gfx950).
 *
 * The operation (CODAG, Section II-B and Section IV-A): the input is a set of
 * independently compressed chunks described by offset metadata; every chunk
 * is decoded by one decompression unit (here one 64-lane wavefront) whose
 * lanes all take part in decoding, reading and writing.  Codecs (Section
 * V-A): ORC integer RLE v1 and RLE v2 (signed int64 columns) and raw Deflate
 * (RFC 1951), one independent stream per chunk; beside them ORC byte RLE and
 * LZ4 blocks, written against the same input and output primitives
 * (Section III's extensibility: a codec is a device function over them).
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
    CODAG_RLE_V1 = 1,   /* ORC integer RLE v1, signed int64 (zigzag varints) unless codag_opts
                           names another element type */
    CODAG_RLE_V2 = 2,   /* ORC integer RLE v2, likewise */
    CODAG_DEFLATE = 3,  /* raw RFC 1951 stream per chunk */
    CODAG_BYTE_RLE = 4, /* ORC byte RLE (byte columns, PRESENT bitmaps): a header 0..127 is a
                           run of header + 3 copies of the next byte, -1..-128 is followed by
                           -header literal bytes; output is bytes */
    CODAG_LZ4 = 5       /* one LZ4 block per chunk (the byte-aligned LZ77 codec ORC and Parquet
                           call LZ4): sequences of a token byte, literals, a 2-byte offset of
                           1..65535 and the match length; no dictionary, so an offset past the
                           bytes already produced is CORRUPT; output is bytes */
};

/* Status codes: return values and per-chunk statuses. */
enum {
    CODAG_OK = 0,
    CODAG_E_INVALID_ARGUMENT = -1, /* bad codec/pointer/size; per chunk: bad output range */
    CODAG_E_HIP = -2,              /* a HIP runtime call or kernel launch failed */
    CODAG_E_CORRUPT = -3,          /* the chunk's stream violates its format */
    CODAG_E_TRUNCATED = -4,        /* the chunk's stream ends before its output is complete */
    CODAG_E_OVERFLOW = -5,         /* the stream decodes to more bytes than the output range */
    CODAG_E_UNDERFLOW = -6         /* Deflate, LZ4: the stream ends before the output range is full */
};

/*
 * Tuning knobs; a zeroed struct (or NULL) selects the defaults.
 *   waves_per_block   wavefronts per workgroup: 1, 2 or 4 (default 1 for
 *                     Deflate and LZ4, 4 for RLE); waves never synchronize with each
 *                     other, so this only shapes occupancy and dispatch.
 *   lit_table_bits    Deflate literal/length lookup-table bits, 9 or 10
 *                     (default 9); longer codes take a slower path.
 *   history_kib       Deflate and LZ4 output window kept in LDS per wave: 2,
 *                     4, 8, 16 or 32 KiB (default 4 for Deflate, 2 for
 *                     LZ4).  Back-references reaching
 *                     further read the already written output from HBM.
 *                     With 32 the workgroup holds one wave.
 *   chunk_ticks       optional device array (n_chunks uint64): receives each
 *                     chunk's decode time in shader clock cycles.
 *   group_parallel    RLE codecs: 0 = automatic (RLE v1 launches of at
 *                     most 256 chunks and RLE v2 launches of at most 2048
 *                     chunks, without chunk_ticks, are decoded
 *                     group-parallel), 1 = one wave per chunk,
 *                     2 = group-parallel (not with chunk_ticks).
 *                     Group-parallel: an index pass finds where the groups
 *                     (RLE v1 runs and literal lists; RLE v2 runs) start,
 *                     without decoding values, and cuts them into ranges of
 *                     about equal output -- 32 per RLE v1 chunk, 8 per RLE
 *                     v2 chunk -- then one wave per range decodes it.  The
 *                     path takes its workspace (528 bytes per RLE v1 chunk,
 *                     96 per RLE v2 chunk) from the stream-ordered allocator
 *                     (hipMallocAsync) on `stream`.  Ignored for Deflate
 *                     and LZ4.
 *   variant           0 = the decoders above.  The others are the decoding-
 *                     unit designs CODAG measures its own against, for
 *                     comparison on the same chunks (same output and
 *                     statuses; no chunk_ticks; waves_per_block,
 *                     group_parallel, lit_table_bits and history_kib are
 *                     ignored -- Deflate uses 9 table bits and a 4 KiB
 *                     window):
 *                       CODAG_VARIANT_LEADER_LANE (Section V-E, single-
 *                       thread decoding): one lane of each chunk's wave
 *                       parses every header, varint and Huffman token and
 *                       hands each result to the wave through LDS; the
 *                       other lanes only write.  RLE v1 and Deflate.
 *                       CODAG_VARIANT_PREFETCH_WAVE (Section V-F): a second
 *                       wave per chunk loads the input into an LDS ring
 *                       ahead of the decoding wave, which runs the main
 *                       one-wave decoder.  RLE v1 and Deflate.
 *                       CODAG_VARIANT_BLOCK_LEADER (Section II-C): a
 *                       256-thread workgroup per chunk; thread 0 parses each
 *                       group while the others wait at a barrier, then all
 *                       write it.  RLE v1 only.
 *                     Other codecs, or a variant a codec lacks, return
 *                     CODAG_E_INVALID_ARGUMENT.
 *   elem_bytes        RLE codecs: bytes per output value, 1, 2, 4 or 8 (0 =
 *                     8).  Each value is stored as the low bytes of its
 *                     64-bit decoded value, little-endian (how an ORC
 *                     short/int column holds it); output ranges must be a
 *                     multiple of elem_bytes and aligned to it.
 *   unsigned_values   RLE codecs: 1 = the stream is unsigned (no zigzag;
 *                     ORC writes string lengths and other unsigned streams
 *                     so; the RLE v2 DELTA delta base stays signed).
 *                     Element types other than signed 8-byte values use the
 *                     one-wave-per-chunk decoder (group_parallel 2 and the
 *                     variants return CODAG_E_INVALID_ARGUMENT).
 */
enum {
    CODAG_VARIANT_DEFAULT = 0,
    CODAG_VARIANT_LEADER_LANE = 1,
    CODAG_VARIANT_PREFETCH_WAVE = 2,
    CODAG_VARIANT_BLOCK_LEADER = 3
};
typedef struct codag_opts {
    int waves_per_block;
    int lit_table_bits;
    uint64_t *chunk_ticks;
    int history_kib;
    int group_parallel;
    int variant;
    int elem_bytes;
    int unsigned_values;
    int reserved[3];
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
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * decode as codag_decompress_ex (same arguments, results and errors), but
 * the call allocates nothing.  The launches that need a workspace, the
 * group-parallel RLE paths (by default RLE v1 launches of at most 256
 * chunks and RLE v2 launches of at most 2048 chunks, without chunk_ticks;
 * any count with group_parallel = 2), take it from a static per-device
 * array of CODAG_NOALLOC_SCRATCH_BYTES bytes that the library holds on every
 * device it runs on until the process ends; a launch needing more than that
 * (group_parallel = 2 with more than 372 RLE v1 or 2048 RLE v2 chunks)
 * returns CODAG_E_INVALID_ARGUMENT.  Every call on one device shares that
 * array: calls that overlap in time on one device (on different streams or
 * threads) race and must not be made.
 */
#define CODAG_NOALLOC_SCRATCH_BYTES (2048u * 96u)
int codag_decompress_noalloc(int codec, const uint8_t *comp_buf, const uint64_t *chunk_offsets,
                             uint8_t *out_buf, const uint64_t *out_offsets, uint64_t n_chunks,
                             void *stream, int32_t *chunk_status, const struct codag_opts *opts);

/*
 * The read path around the decoders (CODAG Section I places decoding inside
 * ORC/Parquet reads): one compressed ORC stream, ZLIB codec, decompressed
 * into out[0 .. out_cap) on the device.  The stream is a sequence of
 * compression chunks, each a 3-byte little-endian header (length << 1 |
 * original) and `length` bytes -- the bytes themselves if `original`, else
 * a raw Deflate stream (codag_orc_decompress_stream: or an LZ4 block).  Every chunk but the last holds exactly block_size
 * uncompressed bytes (as Apache ORC's writers produce them; a shorter one
 * is CODAG_E_UNDERFLOW, a longer one CODAG_E_OVERFLOW), the last at most
 * block_size; a header or chunk cut off by the end of the stream is
 * CODAG_E_TRUNCATED; output past out_cap is CODAG_E_OVERFLOW.  The chunks
 * are located by one wave and decoded in parallel, one wave per chunk, each
 * straight into its place in out.
 *   framed       device, framed_len bytes (the stream as stored in the file).
 *   out_len      device uint64: bytes produced (valid when *status is OK).
 *   status       device int32: CODAG_OK or the status of the first chunk
 *                that failed, in stream order.
 * block_size must be 1..2^23 - 1 (the file's compressionBlockSize).  Takes a
 * workspace of 16 bytes per possible chunk (out_cap / block_size + 2) from
 * the stream-ordered allocator.  Enqueued on `stream`; returns
 * CODAG_E_INVALID_ARGUMENT for bad arguments, CODAG_E_HIP on a launch
 * failure.  The decompressed stream is then decoded with codag_decompress
 * (for example as RLE v2, or byte RLE for a PRESENT stream).
 */
int codag_orc_inflate_stream(const uint8_t *framed, uint64_t framed_len, uint32_t block_size,
                             uint8_t *out, uint64_t out_cap, uint64_t *out_len, int32_t *status,
                             void *stream);

/* As codag_orc_inflate_stream for a stream of either ORC codec the library
 * decodes: codec CODAG_DEFLATE (ORC's ZLIB) or CODAG_LZ4 (ORC's LZ4, one
 * LZ4 block per compression chunk); other codecs return
 * CODAG_E_INVALID_ARGUMENT. */
int codag_orc_decompress_stream(int codec, const uint8_t *framed, uint64_t framed_len,
                                uint32_t block_size, uint8_t *out, uint64_t out_cap,
                                uint64_t *out_len, int32_t *status, void *stream);

/*
 * Return the status of the lowest-indexed chunk that failed in any call on
 * the current device since the previous codag_get_error (CODAG_OK if none),
 * storing that chunk's index in *first_bad_chunk (may be NULL; UINT64_MAX if
 * none), and clear the error word.  The read-and-clear is one atomic
 * exchange enqueued on `stream` after its pending work; the call then
 * synchronizes `stream`.  A failure recorded concurrently by work on another
 * stream is either returned here or kept for the next call, never lost.
 * Returns CODAG_E_HIP if the launch, the copy or the synchronization fails.
 */
int codag_get_error(void *stream, uint64_t *first_bad_chunk);

/* A static, human-readable name for a status code. */
const char *codag_status_string(int status);

/* Forget the library's per-device state (the looked-up addresses of its
 * static error word and scratch array; it allocates no device memory of its
 * own outside plans).  Any later call looks them up again. */
void codag_shutdown(void);


/* ------------------------------------------------------------------------
 * Batched launch: many chunks of mixed codecs in one persistent kernel.
 *
 * A persistent grid (resident waves on every CU) takes chunk indices from a
 * device-side work queue; each wave decodes its chunk with the chunk's codec
 * and takes the next.  The queue order decides how uneven chunks balance
 * across the CUs.  Output bytes are identical whatever the order.
 * ------------------------------------------------------------------------ */

/* Queue orders. */
enum {
    CODAG_ORDER_INDEX = 0,   /* chunk index order (plain atomic queue) */
    CODAG_ORDER_GIVEN = 1,   /* the caller's permutation (`order` argument) */
    CODAG_ORDER_LEARNED = 2, /* longest predicted decode time first, predicted by
                                the plan's cost model (see codag_sched_*); a
                                plan whose model was never trained or set runs
                                in index order */
    CODAG_ORDER_CODEC = 3    /* chunks grouped by codec (every RLE v1 chunk, then
                                every RLE v2 chunk, ...; any order within a
                                codec), sorted on the device at each launch */
};

/*
 * Launch configuration of a plan; zero fields select defaults.
 *   waves_per_cu      resident waves per CU in the persistent grid (default:
 *                     as many as the per-wave LDS allows, at most 16).
 *   waves_per_block   1, 2 or 4 (default 2).
 *   lit_table_bits    Deflate literal/length table bits, 9 or 10 (default 9).
 *   history_kib       Deflate and LZ4 LDS output window, 4, 8 or 16 KiB
 *                     (default 4).
 *   order             CODAG_ORDER_* (default CODAG_ORDER_INDEX).
 *   use_graph         nonzero: capture the launch sequence (queue reset,
 *                     scheduling steps, decode) in a hipGraph once per set of
 *                     arguments and replay it.
 *   chunks_per_claim  queue positions a wave takes with one atomic add, 1..64
 *                     (default 1): packs small chunks onto one claim at the
 *                     cost of coarser balancing.
 */
typedef struct codag_batch_opts {
    int waves_per_cu;
    int waves_per_block;
    int lit_table_bits;
    int history_kib;
    int order;
    int use_graph;
    int chunks_per_claim;
    int reserved[9];
} codag_batch_opts;

typedef struct codag_plan codag_plan;

/* Create a plan on the current device (its device buffers are allocated
 * here and grown on demand by later calls).  opts may be NULL. */
int codag_plan_create(codag_plan **plan, const codag_batch_opts *opts);
/* Synchronize the plan's work and release it. */
void codag_plan_destroy(codag_plan *plan);
/* Read or replace the plan's launch configuration (replacing drops any
 * captured graph). */
int codag_plan_get_opts(const codag_plan *plan, codag_batch_opts *opts);
int codag_plan_set_opts(codag_plan *plan, const codag_batch_opts *opts);

/*
 * Decompress n_chunks chunks whose codecs are codecs[i] (device, uint8,
 * CODAG_RLE_V1/V2/DEFLATE/LZ4; anything else fails that chunk with
 * CODAG_E_INVALID_ARGUMENT).  Buffers, offsets and output rules are those of
 * codag_decompress.
 *   chunk_status  device, n_chunks int32, may be NULL.
 *   order         device, n_chunks uint32 permutation of 0..n_chunks-1, used
 *                 with CODAG_ORDER_GIVEN (ignored otherwise).  An entry
 *                 >= n_chunks is skipped and recorded as an
 *                 CODAG_E_INVALID_ARGUMENT error (codag_get_error) naming
 *                 its queue position; with repeated entries some chunks are
 *                 decoded twice and others not at all.
 *   chunk_ticks   device, n_chunks uint64, may be NULL: each chunk's decode
 *                 time in shader clock cycles.
 * Enqueued on `stream`; returns CODAG_E_INVALID_ARGUMENT for bad arguments,
 * CODAG_E_HIP if a launch or graph operation fails.  Calls that share a plan
 * must not overlap in time (they share its queue).
 */
int codag_decompress_batch(codag_plan *plan, const uint8_t *codecs, const uint8_t *comp_buf,
                           const uint64_t *chunk_offsets, uint8_t *out_buf,
                           const uint64_t *out_offsets, uint64_t n_chunks,
                           int32_t *chunk_status, const uint32_t *order,
                           uint64_t *chunk_ticks, void *stream);

/*
 * Time candidate launch configurations on these buffers (each `reps` times,
 * on `stream`, which is synchronized) and keep the fastest in the plan:
 * a coordinate search over history_kib, lit_table_bits, waves_per_block,
 * chunks_per_claim, index against codec-grouped order (when the plan's
 * order is CODAG_ORDER_INDEX) and waves_per_cu.  *best_ms (may be NULL)
 * receives its time per launch.  The buffers are decoded many times; the
 * output is the same each time.
 *
 * Results are cached for the process, keyed by the device's architecture
 * name, its CU count and the chunk array's shape (each codec's share of the
 * chunks in eighths, log2 of the mean output bytes per chunk and of the
 * chunk count, the plan's order).  A call whose key is cached applies the
 * cached configuration without timing anything and returns its time.
 */
int codag_autotune(codag_plan *plan, const uint8_t *codecs, const uint8_t *comp_buf,
                   const uint64_t *chunk_offsets, uint8_t *out_buf, const uint64_t *out_offsets,
                   uint64_t n_chunks, const uint32_t *order, int reps, double *best_ms,
                   void *stream);

/* The autotune cache as text (host memory), one line per entry:
 * "key|history_kib|lit_table_bits|waves_per_block|chunks_per_claim|
 * waves_per_cu|order|ms".  *len (may be NULL) receives the bytes needed,
 * terminating NUL included; returns CODAG_E_INVALID_ARGUMENT when buf is
 * NULL or shorter. */
int codag_autotune_cache_save(char *buf, size_t cap, size_t *len);
/* Merge entries in that format into the cache (an entry with a key already
 * cached replaces it).  A malformed line, or a configuration the batched
 * launch rejects, returns CODAG_E_INVALID_ARGUMENT and merges nothing. */
int codag_autotune_cache_load(const char *text);
/* Forget every cached entry. */
void codag_autotune_cache_clear(void);

/* ------------------------------------------------------------------------
 * Learned scheduling: a per-plan cost model.
 *
 * The model predicts log2 of a chunk's decode time (shader clock cycles, as
 * codag_decompress_batch reports them) from 16 features that a header-only
 * pre-pass reads from each chunk:
 *   0 log2(1 + compressed bytes)   1 log2(1 + output bytes)   2 = 1 - 0
 *   3..5  codec one-hot (RLE v1, RLE v2, Deflate)
 *   6..8  BTYPE one-hot of the first Deflate block (stored, fixed, dynamic)
 *   9 HLIT/286  10 HDIST/30  11 HCLEN/19 of a dynamic first block
 *   12..15 shares of that block's literal/length code lengths in
 *          1-6, 7-8, 9-10 and 11-15 bits
 * (Deflate header fields as in RFC 1951 section 3.2.7; zero where absent.)
 *
 * Network: x' = (x - mu) * s per feature; h1 = relu(W1 x' + b1),
 * h2 = relu(W2 h1 + b2), y = w3 . h2 + b3 (16-64-64-1, FP32); prediction =
 * y * sy + my.  Parameters are packed as W1[64][16], b1[64], W2[64][64],
 * b2[64], w3[64], b3 (CODAG_SCHED_PARAMS floats, row-major, W[out][in]);
 * normalization as mu[16], s[16], my, sy (CODAG_SCHED_NORM floats).
 * Loss: mean over samples of (y - (t - my) / sy)^2 for targets t.
 * All feat/target/pred buffers are device memory; features are n x 16
 * row-major floats.  Calls are enqueued on `stream` and synchronize it where
 * they return host values.  Like codag_decompress_batch, calls that share a
 * plan must not overlap in time.
 * ------------------------------------------------------------------------ */

#define CODAG_SCHED_FEATURES 16
#define CODAG_SCHED_PARAMS 5313
#define CODAG_SCHED_NORM 34

/* Features of n chunks (arguments as codag_decompress_batch) into feat. */
int codag_sched_features(codag_plan *plan, const uint8_t *codecs, const uint8_t *comp_buf,
                         const uint64_t *chunk_offsets, const uint64_t *out_offsets,
                         uint64_t n_chunks, float *feat, void *stream);

/* Replace the model: params (CODAG_SCHED_PARAMS floats) and norm
 * (CODAG_SCHED_NORM floats) are host arrays.  Marks the model trained. */
int codag_sched_set_params(codag_plan *plan, const float *params, const float *norm);
/* Copy the model out (either pointer may be NULL).  Returns
 * CODAG_E_INVALID_ARGUMENT if the plan has no model yet. */
int codag_sched_get_params(const codag_plan *plan, float *params, float *norm);

/*
 * Serialize the model into host memory, CODAG_SCHED_BLOB_BYTES bytes: the
 * 8 bytes "CODAGMLP", uint32 format version 1, uint32 feature, parameter and
 * normalization counts (16, 5313, 34), the parameters and the normalization
 * as little-endian floats (the codag_sched_set_params layout), then a
 * uint64 FNV-1a hash of all bytes before it.  *len (may be NULL) receives
 * CODAG_SCHED_BLOB_BYTES.  Returns CODAG_E_INVALID_ARGUMENT if buf is NULL
 * or shorter, or the plan has no model.
 */
#define CODAG_SCHED_BLOB_BYTES (8 + 16 + 4 * (5313 + 34) + 8)
int codag_sched_save(const codag_plan *plan, void *buf, size_t cap, size_t *len);
/* Replace the model from such bytes (as codag_sched_set_params).  A wrong
 * length, magic, version, count or hash, or a non-finite value, returns
 * CODAG_E_INVALID_ARGUMENT and leaves the model as it was. */
int codag_sched_load(codag_plan *plan, const void *buf, size_t len);

/*
 * Fit the model to n samples: when seed is nonzero, first re-initialize the
 * weights (uniform in +-sqrt(6/fan_in), biases zero, from the given seed) and
 * the normalization (feature and target means and standard deviations of
 * these samples; a constant feature gets scale 0).  Then take `steps`
 * full-batch Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr,
 * moments reset at the start of the call).  losses (host, may be NULL)
 * receives the loss before each step.  Deterministic for given inputs.
 * n must be at least 2 and below 2^24.
 */
int codag_sched_train(codag_plan *plan, const float *feat, const float *target, uint64_t n,
                      int steps, float lr, uint64_t seed, float *losses, void *stream);

/* Loss and its gradient with respect to the packed parameters (host grad of
 * CODAG_SCHED_PARAMS floats, may be NULL; host loss, may be NULL) at the
 * current model, for n samples. */
int codag_sched_grad(codag_plan *plan, const float *feat, const float *target, uint64_t n,
                     float *grad, float *loss, void *stream);

/* Predicted log2 decode cycles of n feature rows into pred (device). */
int codag_sched_predict(codag_plan *plan, const float *feat, uint64_t n, float *pred,
                        void *stream);

/* The queue order CODAG_ORDER_LEARNED uses for these chunks, into order
 * (device, n_chunks uint32): features, prediction, and a descending counting
 * sort of the prediction over 4096 buckets spanning my +- 4 sy (ties in any
 * order). */
int codag_sched_order(codag_plan *plan, const uint8_t *codecs, const uint8_t *comp_buf,
                      const uint64_t *chunk_offsets, const uint64_t *out_offsets,
                      uint64_t n_chunks, uint32_t *order, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CODAG_H */
