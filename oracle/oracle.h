/*
 * Oracle decoders: TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU decoder per codec.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it;
 * the GPU library never links or calls it, and it includes no header and
 * shares no helper, table or constant with the GPU library.
 *
 * What is decoded (CODAG, Section V-A): ORC integer RLE v1 and RLE v2, and
 * Deflate, each chunk compressed independently (Section II-B).  The paper
 * names the formats but does not define their bits; the bit layouts
 * followed here are the Apache ORC integer run-length encodings and
 * RFC 1951.  RLE columns are signed 64-bit little-endian integers unless
 * the _ex entry points say otherwise; ORC's byte RLE and its compressed
 * stream framing (the read path around the decoders) are here too.
 */
#ifndef CODAG_ORACLE_H
#define CODAG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Codec identifiers (same numbering as the public library). */
#define ORACLE_RLE_V1 1
#define ORACLE_RLE_V2 2
#define ORACLE_DEFLATE 3
#define ORACLE_BYTE_RLE 4
#define ORACLE_LZ4 5

/* Per-chunk status values (same numbering as the public library). */
#define ORACLE_OK 0
#define ORACLE_E_INVALID_ARGUMENT (-1)
#define ORACLE_E_CORRUPT (-3)
#define ORACLE_E_TRUNCATED (-4)
#define ORACLE_E_OVERFLOW (-5)
#define ORACLE_E_UNDERFLOW (-6)

/*
 * Decode one chunk: in[0..in_len) -> out[0..out_cap).  Returns a status.
 * *produced receives the number of output bytes written before the
 * decoder stopped (equal to out_cap on success).
 */
int oracle_decode_chunk(int codec, const uint8_t *in, uint64_t in_len,
                        uint8_t *out, uint64_t out_cap, uint64_t *produced);

/*
 * Chunk-array form on host memory, mirroring the library's entry point:
 * chunk i is comp[chunk_offsets[i] .. chunk_offsets[i+1]) and decodes into
 * out[out_offsets[i] .. out_offsets[i+1]).  status[i] receives chunk i's
 * status (status may be NULL).  Returns 0, or -1 if an argument is invalid.
 */
int oracle_decompress(int codec, const uint8_t *comp,
                      const uint64_t *chunk_offsets, uint8_t *out,
                      const uint64_t *out_offsets, uint64_t n_chunks,
                      int32_t *status);

/*
 * As above, with the element type of the RLE codecs -- elem_bytes 1, 2, 4
 * or 8 (the low bytes of each decoded value, little-endian) and is_unsigned
 * (values read without zigzag, as ORC writes unsigned streams; the DELTA
 * delta base stays signed) -- and, with capacity_mode, Deflate output
 * ranges as upper bounds (status OK when the final block ends inside the
 * range).  produced[i] (may be NULL) receives chunk i's output bytes.
 * Codec ORACLE_BYTE_RLE decodes ORC byte RLE and ORACLE_LZ4 the LZ4 block
 * format (elem_bytes and is_unsigned ignored; LZ4 honours capacity_mode).
 */
int oracle_decode_chunk_ex(int codec, int elem_bytes, int is_unsigned, int capacity_mode,
                           const uint8_t *in, uint64_t in_len, uint8_t *out, uint64_t out_cap,
                           uint64_t *produced);
int oracle_decompress_ex(int codec, int elem_bytes, int is_unsigned, int capacity_mode,
                         const uint8_t *comp, const uint64_t *chunk_offsets, uint8_t *out,
                         const uint64_t *out_offsets, uint64_t n_chunks, int32_t *status,
                         uint64_t *produced);

/*
 * One compressed ORC stream (ZLIB codec) into out[0..out_cap): its
 * compression chunks -- 3-byte header (length << 1 | original), then the
 * original bytes or a raw Deflate stream -- in order.  *out_len receives the
 * bytes produced.  Returns a status (see oracle.c for the readings).
 */
int oracle_orc_inflate_stream(const uint8_t *in, uint64_t in_len, uint64_t block_size,
                              uint8_t *out, uint64_t out_cap, uint64_t *out_len);
/* The same for a stream whose compressed chunks are ORACLE_DEFLATE (ORC's
 * ZLIB codec) or ORACLE_LZ4 (ORC's LZ4 codec: one LZ4 block per chunk). */
int oracle_orc_decompress_stream(int codec, const uint8_t *in, uint64_t in_len, uint64_t block_size,
                                 uint8_t *out, uint64_t out_cap, uint64_t *out_len);

#ifdef __cplusplus
}
#endif

#endif
