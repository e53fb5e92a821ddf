// u16_dir.hpp - UTF-16LE input side of the tile engine: validation, counting
// and encoding of one 16-byte chunk (8 words) per thread (gfx950).
//
// Method (Lemire & Mula, section 5, Algorithm "UTF-16 to UTF-8"): words below
// U+0080 give one byte, below U+0800 two, other words outside D800..DFFF three,
// a surrogate pair four; the value's bits are split into 3/4/5 lead-byte
// payload bits and 6-bit continuation payloads with the prefixes 11110 / 1110
// / 110 / 10. Validation (section 3): a word in D800..DBFF must be followed by
// one in DC00..DFFF and a word in DC00..DFFF must follow one in D800..DBFF.
// The paper sends blocks with surrogates to a scalar path (vectorising them is
// its stated future work, section 7); here each lane composes its pairs in
// registers: the high word emits all four bytes and the low word none. The
// first flagged word is exactly the first error.
#pragma once

#include "device_common.hpp"

namespace hu {

__device__ __forceinline__ bool is_high(unsigned int w) { return (w & 0xFC00u) == 0xD800u; }
__device__ __forceinline__ bool is_low(unsigned int w) { return (w & 0xFC00u) == 0xDC00u; }

// UTF-8 length of the character that starts at word w: 0 for the low half of
// a pair (its high half emits the four bytes).
__device__ __forceinline__ unsigned int utf8_bytes_of(unsigned int w)
{
    return w < 0x80u ? 1u : w < 0x800u ? 2u : is_high(w) ? 4u : is_low(w) ? 0u : 3u;
}

struct U16Dir {
    using Out = unsigned char;
    static constexpr int kInUnit = 2;
    static constexpr int kOutUnit = 1;
    static constexpr bool kNeedsTable = false;
    static constexpr int kOpValidate = HU_OP_VALIDATE_UTF16LE;
    static constexpr int kOpLength = HU_OP_UTF8_LENGTH_FROM_UTF16LE;
    static constexpr int kOpConvert = HU_OP_CONVERT_UTF16LE_TO_UTF8;
    // staging bound per 4 KiB sub-tile (2048 words): valid input gives at most
    // three bytes per word plus one (a high surrogate in the last word)
    static constexpr unsigned int kStageUnits = 3 * (kSub / 2) + 48;
    // the same bound for one 1 KiB piece (a wave's share of a small document)
    static constexpr unsigned int kPieceStageUnits = 3 * (64 * kChunk / 2) + 48;

    // word i (-2..9) of x[0..5]
    __device__ __forceinline__ static unsigned int word(const unsigned int x[6], int i)
    {
        const int h = i + 2;
        return (x[h >> 1] >> (16 * (h & 1))) & 0xFFFFu;
    }

    // UTF-8 bytes of the chunk's words, without any validation (a high
    // surrogate four, a low one none): analyze's count, whose flag is not
    // looked at (its surrogate-free waves take the cheap path; the others
    // count word by word as below).
    __device__ __forceinline__ static unsigned int count_only(const unsigned int x[6])
    {
        int f;
        unsigned int cls;
        return analyze<true>(x, nullptr, &f, &cls);
    }

    // x[0..5] as for UTF-8 input (8 words per chunk, words outside the input
    // read as zero). Positions in the flag are in words relative to the chunk
    // start. Called by whole waves (the surrogate test below is a wave vote).
    template <bool COUNT>
    __device__ __forceinline__ static unsigned int analyze(const unsigned int x[6], const unsigned char * /*table*/,
                                                           int *flag, unsigned int *cls)
    {
        *cls = kClassUnknown;   // emit finds its own path
        // Waves without any word in D800..DFFF have nothing to flag; each
        // word then takes 1 + (w >= 0x80) + (w >= 0x800) UTF-8 bytes. The two
        // words of a dword are tested together as 16-bit halves: the top bit
        // of a half of ((x & m) + m) | x, with m = 0x7F80 (0x7800), is set
        // exactly when its word is >= 0x80 (0x800), and no sum carries into
        // the next half.
        const u16x2 one = {1, 1}, sur = {0x1B, 0x1B};   // w >> 11 of D800..DFFF
        u16x2 plain = {1, 1};
#pragma unroll
        for (int k = 1; k <= 4; ++k) {
            const u16x2 w = __builtin_bit_cast(u16x2, x[k]);
            plain = __builtin_elementwise_min(plain, __builtin_elementwise_min((w >> 11) ^ sur, one));
        }
        if (!__any(__builtin_bit_cast(unsigned int, plain) != 0x00010001u)) {
            *flag = kNoFlag;
            unsigned int count = 8;
            if (COUNT) {
#pragma unroll
                for (int k = 1; k <= 4; ++k) {
                    const unsigned int g80 = ((x[k] & 0x7F807F80u) + 0x7F807F80u) | x[k];
                    const unsigned int g800 = ((x[k] & 0x78007800u) + 0x78007800u) | x[k];
                    count += __popc(g80 & 0x80008000u) + __popc(g800 & 0x80008000u);
                }
            }
            return COUNT ? count : 0u;
        }
        unsigned int count = 0;
        int f = kNoFlag;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const unsigned int w = word(x, j), pw = word(x, j - 1), nw = word(x, j + 1);
            const bool bad = (is_high(w) && !is_low(nw)) || (is_low(w) && !is_high(pw));
            if (bad && f == kNoFlag)
                f = j;
            if (COUNT)
                count += utf8_bytes_of(w);
        }
        *flag = f;
        return count;
    }

    // A high surrogate in the last word is flagged by analyze itself (its
    // successor reads as zero): nothing to add at the end of the input.
    __device__ __forceinline__ static long long end_truncation(const uint8_t * /*base*/, unsigned long long /*off_b*/,
                                                               unsigned long long /*end_b*/)
    {
        return -1;
    }

    // Only called for tiles without any flagged word: the output of a sub-tile
    // then fits the staging buffer. Called by whole waves.
    __device__ __forceinline__ static void emit(const unsigned int x[6], Out *out, unsigned int o, unsigned int /*cls*/)
    {
        // words of three UTF-8 bytes or surrogates anywhere in the wave?
        const unsigned int all = x[1] | x[2] | x[3] | x[4];
        if (!__any((all & 0xF800F800u) != 0)) {
            emit_direct2(x, out, o);
            return;
        }
        bool sur = false;
#pragma unroll
        for (int k = 1; k <= 4; ++k) {
            // a 16-bit half equal to 0xD800 after masking: a surrogate
            const unsigned int v = (x[k] & 0xF800F800u) ^ 0xD800D800u;
            sur |= ((v - 0x00010001u) & ~v & 0x80008000u) != 0;
        }
        if (!__any(sur)) {
            emit_direct<3>(x, out, o);
            return;
        }
        // Surrogates in the wave: one word at a time (text dense in pairs has
        // a high word and an empty low word per character, where a branch-free
        // form would store four bytes for every word).
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const unsigned int w = word(x, j), nw = word(x, j + 1);
            const unsigned int m = utf8_bytes_of(w);
            unsigned int b0, b1 = 0, b2 = 0, b3 = 0;
            if (m == 4) {
                const unsigned int cp = 0x10000u + (((w & 0x3FFu) << 10) | (nw & 0x3FFu));
                b0 = 0xF0u | (cp >> 18);
                b1 = 0x80u | ((cp >> 12) & 0x3Fu);
                b2 = 0x80u | ((cp >> 6) & 0x3Fu);
                b3 = 0x80u | (cp & 0x3Fu);
            } else if (m == 3) {
                b0 = 0xE0u | (w >> 12);
                b1 = 0x80u | ((w >> 6) & 0x3Fu);
                b2 = 0x80u | (w & 0x3Fu);
            } else if (m == 2) {
                b0 = 0xC0u | (w >> 6);
                b1 = 0x80u | (w & 0x3Fu);
            } else {
                b0 = w;
            }
            if (m != 0) {
                out[o] = (Out)b0;
                if (m > 1) out[o + 1] = (Out)b1;
                if (m > 2) out[o + 2] = (Out)b2;
                if (m > 3) out[o + 3] = (Out)b3;
            }
            o += m;
        }
    }

    // Encoding of waves whose words are all below U+0800 (one or two bytes,
    // the first two cases of section 5), two words per register: as 16-bit
    // halves, the lead byte is w (w < 0x80) or 0xC0 | w >> 6, the second byte
    // 0x80 | (w & 0x3F). Each word stores both bytes at its output offset,
    // words in ascending order; the second byte of a one-byte word lands
    // where the next word starts and is overwritten by it. The last word of
    // the chunk stores its second byte only if it has one (the next thread's
    // output starts right after it).
    __device__ __forceinline__ static void emit_direct2(const unsigned int x[6], Out *out, unsigned int o)
    {
#pragma unroll
        for (int k = 1; k <= 4; ++k) {
            const unsigned int v = x[k];
            const u16x2 w = __builtin_bit_cast(u16x2, v);
            // 0xFFFF in the halves whose word is below 0x80 (all are below 0x800)
            const unsigned int small = __builtin_bit_cast(unsigned int, __builtin_bit_cast(i16x2, w - (u16x2)(0x80)) >> 15);
            const unsigned int lead = __builtin_bit_cast(unsigned int, w >> 6) | 0x00C000C0u;
            // bitop3 truth tables: 0xE4 (a & c) | (b & ~c), 0xEA (a & b) | c
            const unsigned int b0 = __builtin_amdgcn_bitop3_b32(v, lead, small, 0xE4);
            const unsigned int b1 = __builtin_amdgcn_bitop3_b32(v, 0x003F003Fu, 0x00800080u, 0xEA);
            // bytes per word in each half: 2 - 1 for the small ones
            const unsigned int n = __builtin_bit_cast(unsigned int, __builtin_bit_cast(u16x2, small) + (u16x2)(2));
            out[o] = (Out)b0;
            out[o + 1] = (Out)b1;
            o += n & 0xFFFFu;
            out[o] = (Out)(b0 >> 16);
            if (k < 4 || (n >> 16) == 2u)
                out[o + 1] = (Out)(b1 >> 16);
            o += n >> 16;
        }
    }

    // Encoding without a branch per word, for waves whose words need at most
    // MAXB bytes: 2 is the paper's section 5 cases of one and two output
    // bytes, 3 adds three-byte words (no surrogates). Bytes of a word w:
    // b0 = w (w < 0x80), 0xC0 | w >> 6 (w < 0x800) or 0xE0 | w >> 12; the
    // following bytes 0x80 | six bits each, most significant first. MAXB
    // bytes are stored for every word, words in ascending order, at the
    // word's output offset: bytes past a word's length land where the next
    // words start, and those overwrite them. Nothing may spill past the
    // chunk's output (the next thread's): the last MAXB - 1 words store a
    // byte only where the chunk's remaining words still reach (words before
    // them are followed by at least MAXB - 1 words of at least one byte).
    // emit uses MAXB = 3; for waves below U+0800 emit_direct2 is the same
    // encoding two words at a time.
    template <int MAXB>
    __device__ __forceinline__ static void emit_direct(const unsigned int x[6], Out *out, unsigned int o)
    {
        static_assert(MAXB == 2 || MAXB == 3, "no surrogates");
        constexpr int kSafe = 9 - MAXB;
        unsigned int len[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const unsigned int w = word(x, j);
            len[j] = 1u + (w >= 0x80u ? 1u : 0u) + (MAXB == 3 && w >= 0x800u ? 1u : 0u);
        }
        // reach[j]: output bytes of words j..7 (only j >= kSafe matter)
        unsigned int reach[8];
        reach[7] = len[7];
#pragma unroll
        for (int j = 6; j >= 0; --j)
            reach[j] = reach[j + 1] + len[j];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const unsigned int w = word(x, j);
            const unsigned int n = len[j];
            const bool three = n == 3u;
            unsigned int b[3];
            b[0] = three ? (0xE0u | (w >> 12)) : n == 2u ? (0xC0u | (w >> 6)) : w;
            b[1] = 0x80u | ((three ? (w >> 6) : w) & 0x3Fu);
            b[2] = 0x80u | (w & 0x3Fu);
#pragma unroll
            for (int i = 0; i < MAXB; ++i) {
                if (j < kSafe || (unsigned int)i < reach[j])
                    out[o + i] = (Out)b[i];
            }
            o += n;
        }
    }
};

}  // namespace hu
