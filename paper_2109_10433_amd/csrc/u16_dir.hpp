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
// its stated future work, section 7); here a pair's four bytes are split two
// and two between its words: the high word gives the lead byte and the first
// continuation byte (bits 20..12 of the code point, which come from the high
// word alone), the low word the last two (bits 11..0: two bits of the high
// word, ten of its own). Every word then stands for one to three bytes and
// waves with surrogates encode without a branch per word. The first flagged
// word is exactly the first error.
#pragma once

#include "device_common.hpp"

namespace hu {

__device__ __forceinline__ bool is_high(unsigned int w) { return (w & 0xFC00u) == 0xD800u; }
__device__ __forceinline__ bool is_low(unsigned int w) { return (w & 0xFC00u) == 0xDC00u; }

struct U16Dir {
    using Out = unsigned char;
    static constexpr int kInUnit = 2;
    static constexpr int kOutUnit = 1;
    static constexpr bool kNeedsTable = false;
    static constexpr int kOpValidate = HU_OP_VALIDATE_UTF16LE;
    static constexpr int kOpLength = HU_OP_UTF8_LENGTH_FROM_UTF16LE;
    static constexpr int kOpConvert = HU_OP_CONVERT_UTF16LE_TO_UTF8;
    // staging bound per 4 KiB sub-tile (2048 words): at most three bytes per
    // word, whatever the input
    static constexpr unsigned int kStageUnits = 3 * (kSub / 2) + 48;
    // the same bound for one 1 KiB piece (a wave's share of a small document)
    static constexpr unsigned int kPieceStageUnits = 3 * (64 * kChunk / 2) + 48;

    // word i (-2..9) of x[0..5]
    __device__ __forceinline__ static unsigned int word(const unsigned int x[6], int i)
    {
        const int h = i + 2;
        return (x[h >> 1] >> (16 * (h & 1))) & 0xFFFFu;
    }

    // UTF-8 bytes of the chunk's words, without any validation (two for
    // each surrogate): analyze's count, whose flag is not looked at.
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
        // Waves without any word in D800..DFFF have nothing to flag:
        // min((w >> 11) ^ 0x1B, 1) is 0 for a surrogate and 1 otherwise.
        const u16x2 one = {1, 1}, sur = {0x1B, 0x1B};   // w >> 11 of D800..DFFF
        u16x2 plain = {1, 1};
#pragma unroll
        for (int k = 1; k <= 4; ++k) {
            const u16x2 w = __builtin_bit_cast(u16x2, x[k]);
            plain = __builtin_elementwise_min(plain, __builtin_elementwise_min((w >> 11) ^ sur, one));
        }
        if (!__any(__builtin_bit_cast(unsigned int, plain) != 0x00010001u)) {
            *flag = kNoFlag;
            return COUNT ? 8u + extra_bytes(x) : 0u;
        }
        // Pairing, two words per dword operation: c = (w >> 10) ^ 0x36 is 0
        // for a high surrogate and 1 for a low one (6 bits per 16-bit half);
        // bit 6 of c + 0x3F is set when the word is not high, of
        // (c ^ 1) + 0x3F when it is not low. Word j + 1 must be low exactly
        // when word j is high, for the pairs (-1, 0) .. (7, 8); waves where
        // every lane passes have no flagged word (a mismatch may also be word
        // -1's or word 8's alone, which the search below then clears).
        unsigned int mism = 0, nh_prev = 0;
#pragma unroll
        for (int k = 0; k <= 5; ++k) {
            const unsigned int c = ((x[k] >> 10) & 0x003F003Fu) ^ 0x00360036u;
            const unsigned int nh = (c + 0x003F003Fu) & 0x00400040u;
            const unsigned int nl = ((c ^ 0x00010001u) + 0x003F003Fu) & 0x00400040u;
            // halves: words 2k - 3 and 2k - 2 (not high) against words 2k - 2
            // and 2k - 1 (not low)
            if (k >= 1)
                mism |= (__builtin_amdgcn_alignbit(nh, nh_prev, 16) ^ nl) & (k == 5 ? 0x40u : 0x00400040u);
            nh_prev = nh;
        }
        int f = kNoFlag;
        if (__any(mism != 0)) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const unsigned int w = word(x, j), pw = word(x, j - 1), nw = word(x, j + 1);
                const bool bad = (is_high(w) && !is_low(nw)) || (is_low(w) && !is_high(pw));
                if (bad && f == kNoFlag)
                    f = j;
            }
        }
        *flag = f;
        if (!COUNT)
            return 0u;
        // a surrogate takes two bytes: one less than the other words >= 0x800
        u16x2 kept = {0, 0};   // words outside D800..DFFF
#pragma unroll
        for (int k = 1; k <= 4; ++k)
            kept += __builtin_elementwise_min((__builtin_bit_cast(u16x2, x[k]) >> 11) ^ sur, one);
        return extra_bytes(x) + kept.x + kept.y;
    }

    // UTF-8 bytes beyond the first of the chunk's words, each word counted as
    // (w >= 0x80) + (w >= 0x800). The two words of a dword are tested together
    // as 16-bit halves: the top bit of a half of ((x & m) + m) | x, with
    // m = 0x7F80 (0x7800), is set exactly when its word is >= 0x80 (0x800),
    // and no sum carries into the next half.
    __device__ __forceinline__ static unsigned int extra_bytes(const unsigned int x[6])
    {
        unsigned int count = 0;
#pragma unroll
        for (int k = 1; k <= 4; ++k) {
            const unsigned int g80 = ((x[k] & 0x7F807F80u) + 0x7F807F80u) | x[k];
            const unsigned int g800 = ((x[k] & 0x78007800u) + 0x78007800u) | x[k];
            count += __popc(g80 & 0x80008000u) + __popc(g800 & 0x80008000u);
        }
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
        if (!__any(sur))
            emit_direct<3>(x, out, o);
        else
            emit_direct<3, true>(x, out, o);
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
    // bytes, 3 adds three-byte words. A word w of n bytes is shifted left by
    // 6(3 - n) bits into v; its lead byte is P ^ (v >> 12), with P = 0x00,
    // 0xC0, 0xE0 for n = 1, 2, 3 (no payload bit meets a prefix bit, so the
    // exclusive or is an or), its next bytes 0x80 | (v >> 6 & 0x3F) and
    // 0x80 | (v & 0x3F). MAXB bytes are stored for every word, words in
    // ascending order, at the word's output offset: bytes past a word's length
    // land where the next words start, and those overwrite them. Nothing may
    // spill past the chunk's output (the next thread's): the last MAXB - 1
    // words store a byte only where the chunk's remaining words still reach
    // (words before them are followed by at least MAXB - 1 words of at least
    // one byte). emit uses MAXB = 3; for waves below U+0800 emit_direct2 is
    // the same encoding two words at a time.
    // With SUR, surrogates are two-byte words (P = 0xC0) with a value of
    // their own in place of w. A high word h stands for bits 20..12 of the
    // code point, u >> 2 with u = (h & 0x3FF) + 0x40; with 0xC00 added, its
    // lead byte is 0xC0 ^ (0x30 | u >> 8) = 0xF0 | u >> 8. A low word l after h
    // stands for bits 11..0, (h & 3) << 10 | (l & 0x3FF); with 0x1000 added,
    // its first byte is 0xC0 ^ 0x40 ^ (bits 11..6) = 0x80 | bits 11..6.
    template <int MAXB, bool SUR = false>
    __device__ __forceinline__ static void emit_direct(const unsigned int x[6], Out *out, unsigned int o)
    {
        static_assert(MAXB == 2 || MAXB == 3, "at most three bytes per word");
        static_assert(!SUR || MAXB == 3, "surrogates only beside three-byte words");
        constexpr int kSafe = 9 - MAXB;
        unsigned int len[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const unsigned int w = word(x, j);
            const bool s = SUR && (w & 0xF800u) == 0xD800u;
            len[j] = 1u + (w >= 0x80u ? 1u : 0u) + (MAXB == 3 && w >= 0x800u && !s ? 1u : 0u);
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
            const unsigned int n1 = len[j] - 1u;   // 0, 1, 2
            unsigned int v = w;
            if (SUR) {
                // both values computed, then selected: the compiler keeps
                // selects of plain values as selects, not branches
                const unsigned int t = w & 0x3FFu;
                const unsigned int vh = (t >> 2) + 0xC10u, vl = (((word(x, j - 1) & 3u) | 4u) << 10) | t;
                const unsigned int vs = (w & 0x400u) == 0 ? vh : vl;
                v = (w & 0xF800u) == 0xD800u ? vs : w;
            }
            v <<= 12u - 6u * n1;
            unsigned int b[3];
            b[0] = __builtin_amdgcn_ubfe(0x00E0C000u, 8u * n1, 8u) ^ (v >> 12);
            b[1] = 0x80u | ((v >> 6) & 0x3Fu);
            b[2] = 0x80u | (v & 0x3Fu);
#pragma unroll
            for (int i = 0; i < MAXB; ++i) {
                if (j < kSafe || (unsigned int)i < reach[j])
                    out[o + i] = (Out)b[i];
            }
            o += len[j];
        }
    }
};

}  // namespace hu
