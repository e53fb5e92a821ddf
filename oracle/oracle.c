/*
 * oracle.c - scalar CPU reference for validating UTF-8 <-> UTF-16LE transcoding.
 *
 * TEST INFRASTRUCTURE: see oracle.h. Plain branching code, one character at a
 * time, the scalar branching approach that section 4 of the paper opens with:
 * look at the lead byte, branch on the number of continuation bytes.
 * No tables, no intrinsics, no blocking.
 *
 * Citations:
 *  - UTF-8 layout: section 3 - the lead byte's top bits give the sequence length
 *    (0 -> 1 byte, 110 -> 2, 1110 -> 3, 11110 -> 4), continuation bytes start
 *    with 10, payloads of 7/11/16/21 bits are stored most significant first
 *    (worked example: U+93E1 is E9 8F A1).
 *  - UTF-8 validity: the six rules listed in section 3 (exhaustive).
 *  - UTF-16: section 3 - BMP values outside D800..DFFF are one code unit; others
 *    are a surrogate pair, high word D800..DBFF then low word DC00..DFFF, whose
 *    10-bit payloads (high first) plus 0x10000 give the value. Little-endian
 *    byte order per code unit.
 *  - UTF-16 validity: section 3 - a high surrogate must be followed by a low
 *    one and a low one preceded by a high one.
 *  - UTF-8 encoding from UTF-16: section 5 - split the value into 3/4/5 payload
 *    bits for the lead byte and 6 for each continuation byte, and add the
 *    prefixes 11110 / 1110 / 110 / 10.
 */
#include "oracle.h"

/* ---- UTF-16LE code units as explicit byte pairs (low byte first) ---- */

static uint32_t word_at(const uint8_t *s, size_t i)
{
    return (uint32_t)s[2 * i] | ((uint32_t)s[2 * i + 1] << 8);
}

static void put_word(uint8_t *d, size_t i, uint32_t w)
{
    d[2 * i] = (uint8_t)(w & 0xFF);
    d[2 * i + 1] = (uint8_t)(w >> 8);
}

/* ---- UTF-8 decoding of one character ----
 * Reads the character that starts at s[p] (p < n). On success returns
 * ORACLE_OK with the scalar value in *cp and its length in *len. Otherwise
 * returns the kind of the first rule (section 3, in reading order) that the
 * sequence starting at p breaks. */
static int decode_utf8_at(const uint8_t *s, size_t n, size_t p,
                          uint32_t *cp, size_t *len)
{
    uint32_t b = s[p];
    size_t L, k;
    uint32_t v;

    if (b < 0x80) {                 /* most significant bit 0: ASCII, one byte */
        *cp = b;
        *len = 1;
        return ORACLE_OK;
    }
    if (b < 0xC0)                   /* 10xxxxxx where a character must start */
        return ORACLE_ERR_STRAY_CONTINUATION;          /* rule 3 */
    if (b >= 0xF8)                  /* five most significant bits all ones */
        return ORACLE_ERR_BAD_LEAD;                    /* rule 1 */

    if (b < 0xE0) {                 /* 110xxxxx: two bytes, 5 payload bits here */
        L = 2;
        v = b & 0x1F;
    } else if (b < 0xF0) {          /* 1110xxxx: three bytes, 4 payload bits */
        L = 3;
        v = b & 0x0F;
    } else {                        /* 11110xxx: four bytes, 3 payload bits */
        L = 4;
        v = b & 0x07;
    }

    if (p + L > n)
        return ORACLE_ERR_TRUNCATED;                   /* rule 2 */
    for (k = 1; k < L; k++) {
        uint32_t c = s[p + k];
        if ((c & 0xC0) != 0x80)
            return ORACLE_ERR_TRUNCATED;               /* rule 2 */
        v = (v << 6) | (c & 0x3F);  /* big-endian: later bytes are lower bits */
    }

    if ((L == 2 && v <= 0x7F) || (L == 3 && v <= 0x7FF) || (L == 4 && v <= 0xFFFF))
        return ORACLE_ERR_OVERLONG;                    /* rule 4 */
    if (v >= 0x110000)
        return ORACLE_ERR_TOO_LARGE;                   /* rule 5 */
    if (v >= 0xD800 && v <= 0xDFFF)
        return ORACLE_ERR_SURROGATE;                   /* rule 6 */

    *cp = v;
    *len = L;
    return ORACLE_OK;
}

/* ---- UTF-16 decoding of one character ----
 * Reads the character starting at word i (i < n). On success returns
 * ORACLE_OK with the value in *cp and its length in words in *len. */
static int decode_utf16_at(const uint8_t *s, size_t n, size_t i,
                           uint32_t *cp, size_t *len)
{
    uint32_t w = word_at(s, i);

    if (w < 0xD800 || w > 0xDFFF) {        /* stored as is */
        *cp = w;
        *len = 1;
        return ORACLE_OK;
    }
    if (w <= 0xDBFF && i + 1 < n) {        /* high surrogate: needs a low one next */
        uint32_t w2 = word_at(s, i + 1);
        if (w2 >= 0xDC00 && w2 <= 0xDFFF) {
            /* low word gives the 10 least significant bits, high word the next
             * 10, then 0x10000 is added */
            *cp = 0x10000 + (((w & 0x3FF) << 10) | (w2 & 0x3FF));
            *len = 2;
            return ORACLE_OK;
        }
    }
    return ORACLE_ERR_UNPAIRED_SURROGATE;
}

/* Number of UTF-16 code units for a scalar value (Table utfsummary: 2 bytes for
 * the basic multilingual plane, 4 bytes for U+10000..10FFFF). */
static size_t utf16_units(uint32_t cp)
{
    return cp < 0x10000 ? 1 : 2;
}

/* Number of UTF-8 bytes for a scalar value (Table utfsummary). */
static size_t utf8_units(uint32_t cp)
{
    if (cp < 0x80)
        return 1;
    if (cp < 0x800)
        return 2;
    if (cp < 0x10000)
        return 3;
    return 4;
}

static oracle_result make_result(int error, uint64_t count)
{
    oracle_result r;
    r.error = error;
    r.reserved = 0;
    r.count = count;
    return r;
}

/* ---- UTF-8 input ---- */

oracle_result oracle_validate_utf8(const uint8_t *src, size_t n)
{
    size_t p = 0;
    while (p < n) {
        uint32_t cp;
        size_t len;
        int e = decode_utf8_at(src, n, p, &cp, &len);
        if (e != ORACLE_OK)
            return make_result(e, p);
        p += len;
    }
    return make_result(ORACLE_OK, n);
}

oracle_result oracle_utf16_length_from_utf8(const uint8_t *src, size_t n)
{
    size_t p = 0;
    uint64_t words = 0;
    while (p < n) {
        uint32_t cp;
        size_t len;
        int e = decode_utf8_at(src, n, p, &cp, &len);
        if (e != ORACLE_OK)
            return make_result(e, p);
        words += utf16_units(cp);
        p += len;
    }
    return make_result(ORACLE_OK, words);
}

oracle_result oracle_convert_utf8_to_utf16le(const uint8_t *src, size_t n,
                                             uint8_t *dst, size_t cap)
{
    size_t p = 0;
    uint64_t q = 0;
    while (p < n) {
        uint32_t cp;
        size_t len;
        int e = decode_utf8_at(src, n, p, &cp, &len);
        if (e != ORACLE_OK)
            return make_result(e, p);
        if (cp < 0x10000) {
            if (q < cap)
                put_word(dst, q, cp);
            q += 1;
        } else {
            uint32_t v = cp - 0x10000;            /* 20 bits */
            uint32_t hi = 0xD800 | (v >> 10);     /* top 10 bits in the first word */
            uint32_t lo = 0xDC00 | (v & 0x3FF);   /* low 10 bits in the second word */
            if (q < cap)
                put_word(dst, q, hi);
            if (q + 1 < cap)
                put_word(dst, q + 1, lo);
            q += 2;
        }
        p += len;
    }
    if (q > cap)
        return make_result(ORACLE_ERR_OUTPUT_TOO_SMALL, q);
    return make_result(ORACLE_OK, q);
}

/* ---- UTF-16LE input ---- */

oracle_result oracle_validate_utf16le(const uint8_t *src, size_t n)
{
    size_t i = 0;
    while (i < n) {
        uint32_t cp;
        size_t len;
        int e = decode_utf16_at(src, n, i, &cp, &len);
        if (e != ORACLE_OK)
            return make_result(e, 2 * (uint64_t)i);
        i += len;
    }
    return make_result(ORACLE_OK, n);
}

oracle_result oracle_utf8_length_from_utf16le(const uint8_t *src, size_t n)
{
    size_t i = 0;
    uint64_t bytes = 0;
    while (i < n) {
        uint32_t cp;
        size_t len;
        int e = decode_utf16_at(src, n, i, &cp, &len);
        if (e != ORACLE_OK)
            return make_result(e, 2 * (uint64_t)i);
        bytes += utf8_units(cp);
        i += len;
    }
    return make_result(ORACLE_OK, bytes);
}

oracle_result oracle_convert_utf16le_to_utf8(const uint8_t *src, size_t n,
                                             uint8_t *dst, size_t cap)
{
    size_t i = 0;
    uint64_t q = 0;
    while (i < n) {
        uint32_t cp;
        size_t len, k, m;
        uint8_t out[4];
        int e = decode_utf16_at(src, n, i, &cp, &len);
        if (e != ORACLE_OK)
            return make_result(e, 2 * (uint64_t)i);
        m = utf8_units(cp);
        if (m == 1) {
            out[0] = (uint8_t)cp;
        } else if (m == 2) {                 /* 110 + 5 bits, 10 + 6 bits */
            out[0] = (uint8_t)(0xC0 | (cp >> 6));
            out[1] = (uint8_t)(0x80 | (cp & 0x3F));
        } else if (m == 3) {                 /* 1110 + 4 bits, then two 10 + 6 */
            out[0] = (uint8_t)(0xE0 | (cp >> 12));
            out[1] = (uint8_t)(0x80 | ((cp >> 6) & 0x3F));
            out[2] = (uint8_t)(0x80 | (cp & 0x3F));
        } else {                             /* 11110 + 3 bits, then three 10 + 6 */
            out[0] = (uint8_t)(0xF0 | (cp >> 18));
            out[1] = (uint8_t)(0x80 | ((cp >> 12) & 0x3F));
            out[2] = (uint8_t)(0x80 | ((cp >> 6) & 0x3F));
            out[3] = (uint8_t)(0x80 | (cp & 0x3F));
        }
        for (k = 0; k < m; k++) {
            if (q + k < cap)
                dst[q + k] = out[k];
        }
        q += m;
        i += len;
    }
    if (q > cap)
        return make_result(ORACLE_ERR_OUTPUT_TOO_SMALL, q);
    return make_result(ORACLE_OK, q);
}

/* ---- many documents per call ---- */

void oracle_many_utf8(int op, const uint8_t *src, const uint64_t *offsets,
                      size_t n_docs, oracle_result *out)
{
    size_t d;
    for (d = 0; d < n_docs; d++) {
        const uint8_t *s = src + offsets[d];
        size_t n = (size_t)(offsets[d + 1] - offsets[d]);
        out[d] = op == 0 ? oracle_validate_utf8(s, n) : oracle_utf16_length_from_utf8(s, n);
    }
}

void oracle_many_utf16le(int op, const uint8_t *src, const uint64_t *offsets,
                         size_t n_docs, oracle_result *out)
{
    size_t d;
    for (d = 0; d < n_docs; d++) {
        const uint8_t *s = src + 2 * offsets[d];
        size_t n = (size_t)(offsets[d + 1] - offsets[d]);
        out[d] = op == 0 ? oracle_validate_utf16le(s, n) : oracle_utf8_length_from_utf16le(s, n);
    }
}

void oracle_many_at(int op, int utf16, const uint64_t *src, const uint64_t *n_units,
                    size_t n, oracle_result *out)
{
    size_t i;
    for (i = 0; i < n; i++) {
        const uint8_t *s = (const uint8_t *)(uintptr_t)src[i];
        size_t m = (size_t)n_units[i];
        if (utf16)
            out[i] = op == 0 ? oracle_validate_utf16le(s, m) : oracle_utf8_length_from_utf16le(s, m);
        else
            out[i] = op == 0 ? oracle_validate_utf8(s, m) : oracle_utf16_length_from_utf8(s, m);
    }
}

void oracle_many_convert_at(int utf16, const uint64_t *src, const uint64_t *n_units,
                            const uint64_t *dst, const uint64_t *dst_cap, size_t n,
                            oracle_result *out)
{
    size_t i;
    for (i = 0; i < n; i++) {
        const uint8_t *s = (const uint8_t *)(uintptr_t)src[i];
        uint8_t *d = (uint8_t *)(uintptr_t)dst[i];
        if (utf16)
            out[i] = oracle_convert_utf16le_to_utf8(s, (size_t)n_units[i], d, (size_t)dst_cap[i]);
        else
            out[i] = oracle_convert_utf8_to_utf16le(s, (size_t)n_units[i], d, (size_t)dst_cap[i]);
    }
}
