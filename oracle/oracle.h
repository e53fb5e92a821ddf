/*
 * oracle.h - scalar CPU reference for validating UTF-8 <-> UTF-16LE transcoding.
 *
 * TEST INFRASTRUCTURE. This header and oracle.c exist to check the GPU library;
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load them. The library never includes, links or calls anything here, and this
 * code includes nothing from the library.
 *
 * Source of truth: Lemire & Mula, "Transcoding Billions of Unicode Characters per
 * Second with SIMD Instructions", section 3 (the UTF-8 and UTF-16 formats, the six
 * UTF-8 validation rules, surrogate pairs, Table "utfsummary"), together with
 * RFC 3629 (UTF-8) and RFC 2781 (UTF-16).
 *
 * All pointers are host pointers. UTF-16LE data is passed as raw bytes
 * (2 bytes per code unit, least significant byte first) so that the byte order
 * is explicit in this code and independent of the host.
 */
#ifndef TRANSCODE_ORACLE_H
#define TRANSCODE_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Result of every entry point.
 *   error == ORACLE_OK:  count = output code units (convert / length functions),
 *                        or input code units (validate functions).
 *   error in 1..7:       count = byte offset of the first ill-formed sequence,
 *                        i.e. of the end of the longest valid prefix. For UTF-16
 *                        input that is 2 x (word index).
 *   ORACLE_ERR_OUTPUT_TOO_SMALL: count = output code units required.           */
typedef struct {
    int32_t error;
    int32_t reserved;
    uint64_t count;
} oracle_result;

/* Error kinds. A UTF-8 error kind names the first of the six rules of section 3
 * that the sequence at the error position breaks, tested in reading order. */
enum {
    ORACLE_OK = 0,
    ORACLE_ERR_BAD_LEAD = 1,            /* rule 1: byte F8..FF                       */
    ORACLE_ERR_TRUNCATED = 2,           /* rule 2: lead without all its continuations */
    ORACLE_ERR_STRAY_CONTINUATION = 3,  /* rule 3: continuation byte with no lead     */
    ORACLE_ERR_OVERLONG = 4,            /* rule 4: value fits a shorter sequence      */
    ORACLE_ERR_TOO_LARGE = 5,           /* rule 5: value above U+10FFFF               */
    ORACLE_ERR_SURROGATE = 6,           /* rule 6: value in U+D800..DFFF              */
    ORACLE_ERR_UNPAIRED_SURROGATE = 7,  /* UTF-16: high not followed by low, or lone low */
    ORACLE_ERR_OUTPUT_TOO_SMALL = 16
};

oracle_result oracle_validate_utf8(const uint8_t *src, size_t n_bytes);
oracle_result oracle_utf16_length_from_utf8(const uint8_t *src, size_t n_bytes);
/* dst receives 2*dst_cap_words bytes at most; the valid prefix is converted
 * even when an error follows (tests do not rely on that). */
oracle_result oracle_convert_utf8_to_utf16le(const uint8_t *src, size_t n_bytes,
                                             uint8_t *dst, size_t dst_cap_words);

/* src holds 2*n_words bytes. */
oracle_result oracle_validate_utf16le(const uint8_t *src, size_t n_words);
oracle_result oracle_utf8_length_from_utf16le(const uint8_t *src, size_t n_words);
oracle_result oracle_convert_utf16le_to_utf8(const uint8_t *src, size_t n_words,
                                             uint8_t *dst, size_t dst_cap_bytes);

/* Many independent inputs in one call (test and baseline convenience only):
 * document d is src[offsets[d] .. offsets[d+1]) in the function's input units
 * (bytes for UTF-8, words for UTF-16LE, offsets counted in those units).
 * op: 0 = validate, 1 = length. out[d] receives the per-document result. */
void oracle_many_utf8(int op, const uint8_t *src, const uint64_t *offsets,
                      size_t n_docs, oracle_result *out);
void oracle_many_utf16le(int op, const uint8_t *src, const uint64_t *offsets,
                         size_t n_docs, oracle_result *out);
/* The same over inputs anywhere in host memory: input i starts at address
 * src[i] and holds n_units[i] code units; utf16 selects the encoding. */
void oracle_many_at(int op, int utf16, const uint64_t *src, const uint64_t *n_units,
                    size_t n, oracle_result *out);
/* Conversion of many inputs: input i (address src[i], n_units[i] code units,
 * UTF-16LE -> UTF-8 if utf16 else UTF-8 -> UTF-16LE) is converted into the
 * buffer at address dst[i] of dst_cap[i] output code units. */
void oracle_many_convert_at(int utf16, const uint64_t *src, const uint64_t *n_units,
                            const uint64_t *dst, const uint64_t *dst_cap, size_t n,
                            oracle_result *out);

#ifdef __cplusplus
}
#endif

#endif
