/*
 * hiputf.h - validating UTF-8 <-> UTF-16LE transcoding on AMD Instinct MI355X
 * (gfx950). C ABI: plain pointers and sizes, no C++ or framework types.
 *
 * The operations are those of Lemire & Mula, "Transcoding Billions of Unicode
 * Characters per Second with SIMD Instructions":
 *   - UTF-8 validity: the six rules of section 3 (lead byte length classes,
 *     continuation bytes, no overlong forms, nothing above U+10FFFF, no
 *     U+D800..DFFF);
 *   - UTF-16 validity and surrogate pairs: section 3;
 *   - UTF-8 -> UTF-16 transcoding: section 4 (Algorithms "core component" and
 *     "non-validating transcoder", validated as described there);
 *   - UTF-16 -> UTF-8 transcoding: section 5 (Algorithm "UTF-16 to UTF-8");
 *   - the output placement across independently decoded pieces follows the
 *     interleaved decoding with precomputed offsets named as future work in
 *     section 7.
 * The paper reports validity as a yes/no answer; this interface adds the first
 * error's kind and byte position and the output length (see hu_result).
 *
 * Memory: every data pointer (src, dst, results, workspaces, document tables)
 * is a DEVICE pointer on the current HIP device. `stream` is a hipStream_t
 * passed as void* (NULL = the default stream). UTF-16LE buffers must be 2-byte
 * aligned; UTF-8 buffers may have any alignment. The caller owns all buffers.
 *
 * Errors: no function throws, aborts or prints. Invalid arguments come back as
 * HU_ERR_INVALID_ARGUMENT, HIP runtime failures as HU_ERR_DEVICE.
 */
#ifndef HIPUTF_H
#define HIPUTF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Result of a call (16 bytes, plain data).
 *   error == HU_OK:
 *     convert_* and *_length_*: count = output code units (UTF-16 words or
 *                               UTF-8 bytes);
 *     validate_*:               count = input code units (bytes or words).
 *   error in HU_ERR_BAD_LEAD .. HU_ERR_UNPAIRED_SURROGATE:
 *     count = BYTE offset of the first ill-formed sequence, i.e. the end of the
 *     longest valid prefix (for UTF-16 input: 2 x word index).
 *   error == HU_ERR_OUTPUT_TOO_SMALL: the input is valid and count = the output
 *     code units required. Validation errors take precedence over it.
 *   other errors: count = 0. */
typedef struct {
    int32_t error;
    int32_t reserved;
    uint64_t count;
} hu_result;

/* Error kinds. For UTF-8 the kind names the first of the six rules of
 * section 3 that the sequence at the error position breaks, the rules being
 * tested in reading order: a continuation byte where a character must start
 * (STRAY_CONTINUATION), a byte F8..FF (BAD_LEAD), a lead byte without all its
 * continuation bytes, also at end of input (TRUNCATED), a value that fits a
 * shorter sequence (OVERLONG), a value above U+10FFFF (TOO_LARGE), a value in
 * U+D800..DFFF (SURROGATE). */
enum {
    HU_OK = 0,
    HU_ERR_BAD_LEAD = 1,
    HU_ERR_TRUNCATED = 2,
    HU_ERR_STRAY_CONTINUATION = 3,
    HU_ERR_OVERLONG = 4,
    HU_ERR_TOO_LARGE = 5,
    HU_ERR_SURROGATE = 6,
    HU_ERR_UNPAIRED_SURROGATE = 7, /* UTF-16: high not followed by low, or low not after high */
    HU_ERR_OUTPUT_TOO_SMALL = 16,
    HU_ERR_INVALID_ARGUMENT = 17,
    HU_ERR_DEVICE = 18
};

/* ------------------------------------------------------------------------
 * Synchronous calls. Each enqueues its kernels on `stream`, waits for that
 * stream, and returns the result. Scratch memory (a few bytes per 4 KiB of
 * input) comes from a per-device, per-stream cache owned by the library
 * (freed by hu_shutdown). n = 0 returns {HU_OK, 0}; pointers may then be NULL.
 * A NULL src (or dst with a non-zero capacity) with n > 0 is
 * HU_ERR_INVALID_ARGUMENT. On success exactly `count` units are written to
 * dst and dst[count, cap) is untouched; on any error the contents of
 * dst[0, cap) are unspecified. Nothing is ever written outside [dst, dst+cap).
 * Calls on one stream are serialised by the stream; calls on different
 * streams may run concurrently.
 * ---------------------------------------------------------------------- */

/* UTF-8 well-formedness (section 3, six rules). */
hu_result validate_utf8(const uint8_t *src, size_t n_bytes, void *stream);

/* Number of UTF-16 words the UTF-8 input converts to (validates first). */
hu_result utf16_length_from_utf8(const uint8_t *src, size_t n_bytes, void *stream);

/* Validating UTF-8 -> UTF-16LE (section 4). dst holds dst_cap_words words;
 * n_bytes words always suffice. */
hu_result convert_utf8_to_utf16le(const uint8_t *src, size_t n_bytes,
                                  uint16_t *dst, size_t dst_cap_words, void *stream);

/* UTF-16LE well-formedness (section 3, surrogate pairing). src: n_words words. */
hu_result validate_utf16le(const uint16_t *src, size_t n_words, void *stream);

/* Number of UTF-8 bytes the UTF-16LE input converts to (validates first). */
hu_result utf8_length_from_utf16le(const uint16_t *src, size_t n_words, void *stream);

/* Validating UTF-16LE -> UTF-8 (section 5). dst holds dst_cap_bytes bytes;
 * 3 x n_words bytes always suffice. */
hu_result convert_utf16le_to_utf8(const uint16_t *src, size_t n_words,
                                  uint8_t *dst, size_t dst_cap_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Asynchronous calls (allocate nothing, never synchronise, safe to record
 * into a HIP graph). Same operations as above; the result is written to the
 * device record *d_result when the enqueued kernels complete.
 *   ws / ws_bytes: caller-owned device workspace of at least
 *   hu_workspace_bytes(op, n) bytes, zero-filled before its first use
 *   (hipMemset or hu_workspace_init). Every completed call leaves it ready for
 *   the next call. Calls that share a workspace must be ordered (same stream
 *   or events); concurrent calls need separate workspaces.
 * Return value: HU_OK once enqueued, HU_ERR_INVALID_ARGUMENT (nothing
 * enqueued) or HU_ERR_DEVICE.
 * ---------------------------------------------------------------------- */

enum {
    HU_OP_VALIDATE_UTF8 = 0,
    HU_OP_UTF16_LENGTH_FROM_UTF8 = 1,
    HU_OP_CONVERT_UTF8_TO_UTF16LE = 2,
    HU_OP_VALIDATE_UTF16LE = 3,
    HU_OP_UTF8_LENGTH_FROM_UTF16LE = 4,
    HU_OP_CONVERT_UTF16LE_TO_UTF8 = 5
};

/* Workspace bytes for one call of `op` on n input code units. */
size_t hu_workspace_bytes(int op, size_t n_units);

/* Zero-fills a workspace with a kernel on `stream` (capturable). */
int hu_workspace_init(void *ws, size_t ws_bytes, void *stream);

int validate_utf8_async(const uint8_t *src, size_t n_bytes, hu_result *d_result,
                        void *ws, size_t ws_bytes, void *stream);
int utf16_length_from_utf8_async(const uint8_t *src, size_t n_bytes, hu_result *d_result,
                                 void *ws, size_t ws_bytes, void *stream);
int convert_utf8_to_utf16le_async(const uint8_t *src, size_t n_bytes, uint16_t *dst,
                                  size_t dst_cap_words, hu_result *d_result,
                                  void *ws, size_t ws_bytes, void *stream);
int validate_utf16le_async(const uint16_t *src, size_t n_words, hu_result *d_result,
                           void *ws, size_t ws_bytes, void *stream);
int utf8_length_from_utf16le_async(const uint16_t *src, size_t n_words, hu_result *d_result,
                                   void *ws, size_t ws_bytes, void *stream);
int convert_utf16le_to_utf8_async(const uint16_t *src, size_t n_words, uint8_t *dst,
                                  size_t dst_cap_bytes, hu_result *d_result,
                                  void *ws, size_t ws_bytes, void *stream);

/* Library-wide: a human-readable name for an error code (static string). */
const char *hu_error_name(int error);

/* Frees the library's cached workspaces and pinned result slots on every
 * device. Calls may follow; caches are rebuilt on demand. */
void hu_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* HIPUTF_H */
