// u8_dir.hpp - UTF-8 input side of the tile engine: validation, counting and
// decoding of one 16-byte chunk per thread (gfx950).
//
// Method (Lemire & Mula): section 4 transcodes UTF-8 to UTF-16 by finding
// character starts as the bytes that are not continuation bytes (Algorithm
// "non-validating transcoder"), with an ASCII fast path, and validates with
// the Keiser-Lemire nibble tables (the rules are the six of section 3).
//
// Validation of every byte: the class bits of (previous byte high nibble,
// previous byte low nibble, current byte high nibble) from three 16-entry
// nibble tables, AND-ed; the tables are staged in LDS as their 4096-entry
// product so that one LDS lookup per byte replaces three lookups and two ANDs.
// Two continuation bytes in a row are legal exactly where the byte two back is
// E0..FF or the byte three back is F0..FF. A lead byte among the last three
// input bytes that needs more bytes than remain is a truncation.
// The first flagged byte f satisfies P <= f <= P + 3, P = end of the longest
// valid prefix (flags look only backwards, and every ill-formed sequence is
// flagged at its first byte, its second byte or at the first byte within
// three that should have continued it); finish.hpp decodes from just before f
// to recover P and the rule it breaks.
#pragma once

#include "device_common.hpp"

namespace hu {

// ------------------------------------------------------------ nibble tables
// Classes of adjacent byte pairs (p, c) that break a rule of section 3. Each
// class is a product of three nibble sets: p >> 4, p & 15 and c >> 4.
struct PairClass {
    unsigned short bit;
    unsigned short prev_hi, prev_lo, cur_hi;   // sets of nibble values (bit v = value v)
};

constexpr unsigned short kAnyNibble = 0xFFFF;
constexpr unsigned short kContNibbles = 0x0F00;      // 8..B: continuation byte
constexpr unsigned short kAsciiNibbles = 0x00FF;     // 0..7
constexpr unsigned short kLeadNibbles = 0xF000;      // C..F
constexpr unsigned short kTwoConts = 1u << 8;

constexpr PairClass kPairClasses[] = {
    {1u << 0, kAsciiNibbles, kAnyNibble, kContNibbles},           // ASCII then continuation (rule 3)
    {1u << 1, kLeadNibbles, kAnyNibble, (unsigned short)~kContNibbles},  // lead then non-continuation (rule 2)
    {1u << 2, 1u << 0xC, 0x0003, kContNibbles},                   // C0, C1: overlong 2-byte (rule 4)
    {1u << 3, 1u << 0xE, 1u << 0x0, 0x0300},                      // E0 80..9F: overlong 3-byte (rule 4)
    {1u << 4, 1u << 0xE, 1u << 0xD, 0x0C00},                      // ED A0..BF: surrogate (rule 6)
    {1u << 5, 1u << 0xF, 1u << 0x0, 0x0100},                      // F0 80..8F: overlong 4-byte (rule 4)
    {1u << 6, 1u << 0xF, 1u << 0x4, 0x0E00},                      // F4 90..BF: above U+10FFFF (rule 5)
    {1u << 7, 1u << 0xF, 0xFFE0, kContNibbles},                   // F5..FF then continuation (rules 1, 5)
    {kTwoConts, kContNibbles, kAnyNibble, kContNibbles},          // two continuations: legal only as 3rd/4th byte
};

struct NibbleTables {
    unsigned short prev_hi[16], prev_lo[16], cur_hi[16];
};

constexpr NibbleTables make_nibble_tables()
{
    NibbleTables t{};
    for (int v = 0; v < 16; ++v) {
        unsigned short a = 0, b = 0, c = 0;
        for (const PairClass &pc : kPairClasses) {
            if (pc.prev_hi & (1u << v)) a |= pc.bit;
            if (pc.prev_lo & (1u << v)) b |= pc.bit;
            if (pc.cur_hi & (1u << v)) c |= pc.bit;
        }
        t.prev_hi[v] = a;
        t.prev_lo[v] = b;
        t.cur_hi[v] = c;
    }
    return t;
}

// Product table, entry (p << 4) | (c >> 4): bit 7 = the pair breaks a rule,
// bit 6 = both bytes are continuation bytes (bit positions chosen so that four
// entries packed into a dword line up with the per-byte SWAR masks). Built at
// compile time from the three nibble tables; each workgroup copies it into LDS.
struct PairTable {
    alignas(16) unsigned char e[4096];
};

constexpr PairTable make_pair_table()
{
    const NibbleTables t = make_nibble_tables();
    PairTable p{};
    for (unsigned int idx = 0; idx < 4096; ++idx) {
        const unsigned int cls = t.prev_hi[idx >> 8] & t.prev_lo[(idx >> 4) & 15] & t.cur_hi[idx & 15];
        p.e[idx] = (unsigned char)(((cls & ~kTwoConts) ? 0x80u : 0u) | ((cls & kTwoConts) ? 0x40u : 0u));
    }
    return p;
}

__device__ const PairTable g_pair_table = make_pair_table();

// ------------------------------------------------------------ SWAR helpers
// bit 7 of each byte of the result is set iff that byte of x is >= 0xE0 / 0xF0
__device__ __forceinline__ unsigned int ge_e0(unsigned int x) { return x & (x << 1) & (x << 2) & 0x80808080u; }
__device__ __forceinline__ unsigned int ge_f0(unsigned int x) { return ge_e0(x) & (x << 3); }
// bit 7 of each byte set iff bits 1..4 of that byte are not all zero (for a
// lead C0..DF: false exactly for C0 and C1, the overlong two-byte leads)
__device__ __forceinline__ unsigned int payload_nonzero(unsigned int x)
{
    return ((x & 0x1E1E1E1Eu) + 0x7F7F7F7Fu) & 0x80808080u;
}
// bit 7 of each byte set iff that byte is not a continuation byte (10xxxxxx)
__device__ __forceinline__ unsigned int not_cont(unsigned int x)
{
    unsigned int y = (x & 0xC0C0C0C0u) ^ 0x80808080u;
    return (y | (y << 1)) & 0x80808080u;
}

struct U8Dir {
    using Out = unsigned short;                       // output code unit
    static constexpr int kInUnit = 1;                 // bytes per input unit
    static constexpr int kOutUnit = 2;                // bytes per output unit
    static constexpr bool kNeedsTable = true;
    static constexpr int kOpValidate = HU_OP_VALIDATE_UTF8;
    static constexpr int kOpLength = HU_OP_UTF16_LENGTH_FROM_UTF8;
    static constexpr int kOpConvert = HU_OP_CONVERT_UTF8_TO_UTF16LE;
    // staging bound per 4 KiB sub-tile: valid input gives at most one word per
    // byte plus one (a four-byte lead in the last byte)
    static constexpr unsigned int kStageUnits = kSub + 40;
    // the same bound for one 1 KiB piece (a wave's share of a small document)
    static constexpr unsigned int kPieceStageUnits = 64 * kChunk + 40;

    // UTF-16 words of the characters that start in the chunk, without any
    // validation (words per lead as in the paper's non-validating transcoder:
    // one, two for a lead F0..FF).
    __device__ __forceinline__ static unsigned int count_only(const unsigned int x[6])
    {
        unsigned int n = 0;
#pragma unroll
        for (int k = 1; k <= 4; ++k)
            n += __popc(not_cont(x[k])) + __popc(ge_e0(x[k]) & (x[k] << 3));
        return n;
    }

    // x[0]: the 4 bytes before the chunk, x[1..4]: the chunk, x[5]: the 4
    // bytes after (bytes outside the input read as zero). Returns the number
    // of UTF-16 words of the characters that start in the chunk (if COUNT) and
    // sets *flag to the first flagged position relative to the chunk start
    // (kNoFlag if none). Truncation at the input's end is end_truncation's.
    // *cls receives the wave's class for emit: 0 no byte >= E0 in x[0..4], 1
    // no byte >= F0, 4 bytes >= F0 but no lead of two or three bytes (C0..EF)
    // in x[1..4], 2 otherwise. Called by whole waves (the tests below are wave
    // votes).
    template <bool COUNT>
    __device__ __forceinline__ static unsigned int analyze(const unsigned int x[6], const unsigned char *table,
                                                           int *flag, unsigned int *cls)
    {
        // Waves with no byte >= E0 hold one- and two-byte characters only
        // (or errors). There the rules of section 3 reduce to: a byte is a
        // continuation exactly when the byte before it is a lead, and the byte
        // before it is not C0 or C1. That check needs no table; a wave that
        // fails it goes through the general check below, which places the
        // flag. Every test looks at the byte and the one before it, as the
        // general check does, so a chunk passes exactly when that check
        // would flag nothing in it that comes first (a pair split across two
        // chunks is judged by the second, in either check).
        // per dword: bytes >= E0 (bit 7 of each byte)
        unsigned int G[5];
#pragma unroll
        for (int k = 0; k < 5; ++k)
            G[k] = ge_e0(x[k]);
        if (!__any(G[0] | G[1] | G[2] | G[3] | G[4])) {
            unsigned int bad = 0, n_cont = 0;   // continuation bytes: 16 - n_cont characters start here
            unsigned int lead_prev = x[0] & (x[0] << 1) & 0x80808080u;
            unsigned int c01_prev = lead_prev & ~payload_nonzero(x[0]);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const unsigned int cur = x[k + 1];
                const unsigned int hib = cur & 0x80808080u;
                const unsigned int lead = hib & (cur << 1);   // C0..DF
                const unsigned int cont = hib ^ lead;         // 80..BF
                const unsigned int c01 = lead & ~payload_nonzero(cur);   // C0, C1
                bad |= (cont ^ __builtin_amdgcn_alignbyte(lead, lead_prev, 3)) |
                       __builtin_amdgcn_alignbyte(c01, c01_prev, 3);
                if (COUNT)
                    n_cont += __popc(cont);
                lead_prev = lead;
                c01_prev = c01;
            }
            if (!__any(bad)) {
                *flag = kNoFlag;
                *cls = 0;
                return COUNT ? 16u - n_cont : 0u;
            }
        }
        // per dword: bytes >= F0
        unsigned int F[5];
#pragma unroll
        for (int k = 0; k < 5; ++k)
            F[k] = G[k] & (x[k] << 3);
        unsigned int k_cls = 1;
        if (__any(F[0] | F[1] | F[2] | F[3] | F[4])) {
            // leads C0..EF in the chunk? (bit 7 of x & x << 1: byte >= C0)
            unsigned int mid = 0;
#pragma unroll
            for (int k = 1; k <= 4; ++k)
                mid |= x[k] & (x[k] << 1) & ~F[k];
            k_cls = __any((mid & 0x80808080u) != 0) ? 2u : 4u;
        }
        *cls = k_cls;
        unsigned int count = 0;
        if (COUNT) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                count += __popc(not_cont(x[k + 1])) + __popc(F[k + 1]);
        }
        // 8 * (first flagged position) + 7, or all ones when nothing is flagged
        unsigned int f8 = ~0u;
        const bool ascii = ((x[1] | x[2] | x[3] | x[4]) & 0x80808080u) == 0;
        if (!ascii || (x[0] & 0x80000000u) != 0) {
            // An all-ASCII chunk can only be flagged if the byte just before
            // it belongs to an unfinished character.
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const unsigned int cur = x[k + 1], prev = x[k];
                const unsigned int p1 = __builtin_amdgcn_alignbyte(cur, prev, 3);   // byte before each byte
                // table index of byte m: (p1_m << 4) | (cur_m >> 4), from the
                // 16-bit pair (p1_m << 8) | cur_m
                const unsigned int y01 = __builtin_amdgcn_perm(p1, cur, 0x05010400u);   // [c0 p0 c1 p1]
                const unsigned int y23 = __builtin_amdgcn_perm(p1, cur, 0x07030602u);   // [c2 p2 c3 p3]
                const unsigned int i0 = (y01 & 0xFFFFu) >> 4, i1 = y01 >> 20;
                const unsigned int i2 = (y23 & 0xFFFFu) >> 4, i3 = y23 >> 20;
                // entries of bytes 0, 2 and 1, 3 loaded into 16-bit halves
                const u16x2 e02 = {table[i0], table[i2]}, e13 = {table[i1], table[i3]};
                const unsigned int e = __builtin_bit_cast(unsigned int, e02) | (__builtin_bit_cast(unsigned int, e13) << 8);
                // a continuation byte is required exactly where the byte two
                // back is E0..FF or the byte three back is F0..FF
                const unsigned int must = __builtin_amdgcn_alignbyte(G[k + 1], G[k], 2) |
                                          __builtin_amdgcn_alignbyte(F[k + 1], F[k], 1);
                const unsigned int flags = (e | ((e << 1) ^ must)) & 0x80808080u;
                // lowest set bit: 8b + 7 for byte b, all ones if none; OR-ing
                // 32k keeps all ones and otherwise adds 32k
                const unsigned int low = lowest_bit_or_ones(flags) | (32u * k);
                f8 = f8 < low ? f8 : low;
            }
        }
        static_assert(kNoFlag == (int)(~0u >> 3), "no flag: all ones, shifted");
        *flag = (int)(f8 >> 3);
        return count;
    }

    // A lead among the last three bytes of the input that needs more bytes
    // than remain (rule 2 at the input's end): its position relative to the
    // input start, else -1. The input is [base + off_b, base + end_b); one
    // thread reads its last bytes from memory.
    __device__ __forceinline__ static long long end_truncation(const uint8_t *base, unsigned long long off_b,
                                                               unsigned long long end_b)
    {
        for (unsigned int back = 3; back >= 1; --back) {
            if (end_b < off_b + back)
                continue;   // before the input
            const unsigned int b = base[end_b - back];
            const unsigned int need = b >= 0xF0u ? 4u : b >= 0xE0u ? 3u : b >= 0xC0u ? 2u : 1u;
            if (need > back)
                return (long long)(end_b - back - off_b);
        }
        return -1;
    }

    // Writes the words of the characters that start in the chunk to out[o..].
    // Only called for tiles without any flagged byte, so the chunk is valid
    // UTF-8 (its last character may end in the next chunk) and the output of a
    // sub-tile fits the staging buffer. cls: the wave's class from analyze, or
    // kClassUnknown (then found here, without class 4). Called by whole waves.
    __device__ __forceinline__ static void emit(const unsigned int x[6], Out *out, unsigned int o, unsigned int cls)
    {
        unsigned int lead[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            lead[k] = not_cont(x[k + 1]);
        if (cls == kClassUnknown) {
            bool wide = false, pairs = false;   // bytes >= E0, bytes >= F0
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const unsigned int g = ge_e0(x[k + 1]);
                wide |= g != 0;
                pairs |= (g & (x[k + 1] << 3)) != 0;
            }
            cls = !__any(wide) ? 0u : !__any(pairs) ? 1u : 2u;
        }
        if (cls == 0) {
            emit_direct<2>(x, lead, out, o);
            return;
        }
        if (cls == 1) {
            emit_direct<3>(x, lead, out, o);
            return;
        }
        if (cls == 4) {
            emit_direct4<false>(x, lead, out, o);
            return;
        }
        emit_direct4<true>(x, lead, out, o);
    }

    // Decoding without a branch per character, for waves whose characters
    // have at most MAXB bytes: 2 is the first case of the paper's Algorithm
    // "core component", 3 its second (one 16-bit word per character). The
    // word at byte position p, as if p held a lead b followed by n1, n2 (bit
    // layouts of section 3): b < 0x80: b;  C0..DF: ((b & 0x1F) << 6) |
    // (n1 & 0x3F);  E0..EF: ((b & 0x0F) << 12) | ((n1 & 0x3F) << 6) |
    // (n2 & 0x3F). With n1, n2 continuation bytes (10xxxxxx) the first is
    // two = (b << 6) ^ n1 ^ 0x3080, and for E0..EF that is 0x800 | the
    // payload so far, so the second is (two << 6) ^ n2 ^ 0x80 modulo 2^16;
    // neither needs masking. Words are formed two positions per
    // register (16-bit halves, packed 16-bit shifts for the second) for
    // all 16 positions, junk at continuation bytes. Every position then stores
    // its word without a branch, positions in descending order, at the slot of
    // the last lead at or before it: a continuation byte's junk lands in the
    // slot of its lead (or of the character before), which that character,
    // stored later, overwrites. The first bytes of the chunk (up to three,
    // whatever MAXB) can precede its first lead (the rest of a character begun
    // in the previous chunk); they store only when a lead is at or before them.
    template <int MAXB>
    __device__ __forceinline__ static void emit_direct(const unsigned int x[6], const unsigned int lead[4], Out *out,
                                                       unsigned int o)
    {
        static_assert(MAXB == 2 || MAXB == 3, "one word per character");
        // first slot of each dword's characters
        unsigned int first[4];
        first[0] = o;
#pragma unroll
        for (int k = 1; k < 4; ++k)
            first[k] = first[k - 1] + __popc(lead[k - 1]);
        char *base = reinterpret_cast<char *>(out);
#pragma unroll
        for (int k = 3; k >= 0; --k) {
            const unsigned int lo = x[k + 1], hi = x[k + 2];   // this dword and the next
            // bytes (p, p + 1) of hi:lo into the low bytes of the two halves
            const unsigned int a2[2] = {__builtin_amdgcn_perm(hi, lo, 0x0C010C00u),
                                        __builtin_amdgcn_perm(hi, lo, 0x0C030C02u)};
            const unsigned int b2[2] = {__builtin_amdgcn_perm(hi, lo, 0x0C020C01u),
                                        __builtin_amdgcn_perm(hi, lo, 0x0C040C03u)};
            // 0xFFFF in the halves whose byte is >= 0x80: permute selectors 8..11
            // copy the top bit of bytes 1, 3, 5, 7 of (lo : lo << 8)
            const unsigned int lo8 = lo << 8;
            const unsigned int m[2] = {__builtin_amdgcn_perm(lo, lo8, 0x0A0A0808u),
                                       __builtin_amdgcn_perm(lo, lo8, 0x0B0B0909u)};
            unsigned int W[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                // bitop3 truth tables: 0x96 a ^ b ^ c, 0xE4 (a & c) | (b & ~c)
                const unsigned int two = __builtin_amdgcn_bitop3_b32(a2[h] << 6, b2[h], 0x30803080u, 0x96);
                unsigned int w = __builtin_amdgcn_bitop3_b32(two, a2[h], m[h], 0xE4);
                if (MAXB >= 3) {
                    const unsigned int c2 = h == 0 ? a2[1] : __builtin_amdgcn_perm(hi, lo, 0x0C050C04u);
                    const u16x2 av = __builtin_bit_cast(u16x2, a2[h]);
                    // for a three-byte lead, two = 0x800 | (b & 0x0F) << 6 | (n1 & 0x3F),
                    // so (two << 6) ^ n2 ^ 0x80 is its word modulo 2^16
                    const u16x2 t6 = __builtin_bit_cast(u16x2, two) << 6;
                    const unsigned int three = __builtin_amdgcn_bitop3_b32(__builtin_bit_cast(unsigned int, t6), c2,
                                                                           0x00800080u, 0x96);
                    // 0xFFFF in the halves whose byte is below 0xE0
                    const unsigned int below =
                        __builtin_bit_cast(unsigned int, __builtin_bit_cast(i16x2, av - (u16x2)(0xE0)) >> 15);
                    w = __builtin_amdgcn_bitop3_b32(w, three, below, 0xE4);
                }
                W[h] = w;
            }
            // byte b of incl2: twice the leads among bytes 0..b of this dword
            const unsigned int incl2 = byte_prefix_sum(lead[k] >> 6);
            const unsigned int a0 = 2u * first[k] - 2u;   // address of slot (first - 1)
#pragma unroll
            for (int b = 3; b >= 0; --b) {
                const unsigned int ib = (incl2 >> (8 * b)) & 0xFFu;
                unsigned short *p = reinterpret_cast<unsigned short *>(base + a0 + ib);
                const unsigned short v = (unsigned short)((b & 1) ? (W[b >> 1] >> 16) : W[b >> 1]);
                // chunk start: positions before the first lead store nothing
                // (up to three: the chunk before may end with any lead, even
                // in a wave that took another path)
                const bool guard = k == 0 && b < 3;
                if (!guard || ib != 0)
                    *p = v;
            }
        }
    }

    // Decoding without a branch per character where the wave holds
    // four-byte characters (which the paper's vectorised path leaves to its
    // third case or to scalar code). Leads of one to three bytes give one
    // word as in emit_direct. A four-byte lead b n1 n2 n3, of value
    // c = ((b & 7) << 18) | ((n1 & 0x3F) << 12) | ((n2 & 0x3F) << 6) |
    // (n3 & 0x3F), gives the surrogate pair 0xD800 + ((c - 0x10000) >> 10),
    // 0xDC00 + (c & 0x3FF) (section 3). For valid bytes the three-byte
    // formula of emit_direct gives c >> 6 here, so these are (three >> 4) +
    // 0xD7C0 and ((n2 << 6) & 0x3C0) + n3 + 0xDB80, modulo 2^16. Slots count
    // two words per four-byte lead: every position stores its (last) word at
    // the slot of the last word of the character at or before it, in
    // descending order as in emit_direct. Before that it
    // stores its first word one slot lower if it is a four-byte lead, else at
    // that same slot, where its own second store overwrites it: no store
    // needs a mask but the guard at the chunk start. SHORT = false: the wave
    // has no leads of two or three bytes, so a position's word is its byte
    // itself unless it is a four-byte lead.
    template <bool SHORT>
    __device__ __forceinline__ static void emit_direct4(const unsigned int x[6], const unsigned int lead[4], Out *out,
                                                        unsigned int o)
    {
        unsigned int f0[4];   // bytes >= F0
#pragma unroll
        for (int k = 0; k < 4; ++k)
            f0[k] = ge_e0(x[k + 1]) & (x[k + 1] << 3);
        unsigned int first[4];
        first[0] = o;
#pragma unroll
        for (int k = 1; k < 4; ++k)
            first[k] = first[k - 1] + __popc(lead[k - 1]) + __popc(f0[k - 1]);
        char *base = reinterpret_cast<char *>(out);
#pragma unroll
        for (int k = 3; k >= 0; --k) {
            const unsigned int lo = x[k + 1], hi = x[k + 2];
            // bytes (p, p + 1), (p + 1, p + 2), ... of hi:lo into the halves
            const unsigned int a2[2] = {__builtin_amdgcn_perm(hi, lo, 0x0C010C00u),
                                        __builtin_amdgcn_perm(hi, lo, 0x0C030C02u)};
            const unsigned int b2[2] = {__builtin_amdgcn_perm(hi, lo, 0x0C020C01u),
                                        __builtin_amdgcn_perm(hi, lo, 0x0C040C03u)};
            const unsigned int c2[2] = {a2[1], __builtin_amdgcn_perm(hi, lo, 0x0C050C04u)};
            const unsigned int d2[2] = {b2[1], __builtin_amdgcn_perm(hi, lo, 0x0C060C05u)};
            unsigned int W[2], H[2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const u16x2 av = __builtin_bit_cast(u16x2, a2[h]);
                const unsigned int two = __builtin_amdgcn_bitop3_b32(a2[h] << 6, b2[h], 0x30803080u, 0x96);
                const u16x2 t6 = __builtin_bit_cast(u16x2, two) << 6;
                const unsigned int three =
                    __builtin_amdgcn_bitop3_b32(__builtin_bit_cast(unsigned int, t6), c2[h], 0x00800080u, 0x96);
                unsigned int w = a2[h];
                if constexpr (SHORT) {
                    const unsigned int lo8 = lo << 8;
                    const unsigned int m = h == 0 ? __builtin_amdgcn_perm(lo, lo8, 0x0A0A0808u)
                                                  : __builtin_amdgcn_perm(lo, lo8, 0x0B0B0909u);
                    w = __builtin_amdgcn_bitop3_b32(two, a2[h], m, 0xE4);
                    const unsigned int below_e0 =
                        __builtin_bit_cast(unsigned int, __builtin_bit_cast(i16x2, av - (u16x2)(0xE0)) >> 15);
                    w = __builtin_amdgcn_bitop3_b32(w, three, below_e0, 0xE4);
                }
                // for a four-byte lead, three is c >> 6 (15 bits), so the first
                // word is 0xD800 + (c >> 10) - 0x40 = (three >> 4) + 0xD7C0
                const u16x2 hs = (__builtin_bit_cast(u16x2, three) >> 4) + (u16x2)(0xD7C0);
                const unsigned int ls = ((c2[h] << 6) & 0x03C003C0u) + d2[h] + 0xDB80DB80u;
                const unsigned int below_f0 =
                    __builtin_bit_cast(unsigned int, __builtin_bit_cast(i16x2, av - (u16x2)(0xF0)) >> 15);
                W[h] = __builtin_amdgcn_bitop3_b32(w, ls, below_f0, 0xE4);
                H[h] = __builtin_bit_cast(unsigned int, hs);
            }
            // byte b of incl2: twice the words of the characters starting at
            // bytes 0..b; of incl2h: the same less 2 at four-byte leads (no
            // byte borrows: such a byte counts at least 4)
            const unsigned int incl2 = byte_prefix_sum((lead[k] >> 6) + (f0[k] >> 6));
            const unsigned int incl2h = incl2 - (f0[k] >> 6);
            const unsigned int a0 = 2u * first[k] - 2u;   // address of slot (first - 1)
#pragma unroll
            for (int b = 3; b >= 0; --b) {
                const unsigned int ib = (incl2 >> (8 * b)) & 0xFFu;
                const unsigned int ibh = (incl2h >> (8 * b)) & 0xFFu;
                const unsigned short v = (unsigned short)((b & 1) ? (W[b >> 1] >> 16) : W[b >> 1]);
                const unsigned short vh = (unsigned short)((b & 1) ? (H[b >> 1] >> 16) : H[b >> 1]);
                const bool guard = k == 0 && b < 3;
                if (!guard || ib != 0) {
                    *reinterpret_cast<unsigned short *>(base + a0 + ibh) = vh;
                    *reinterpret_cast<unsigned short *>(base + a0 + ib) = v;
                }
            }
        }
    }
};

}  // namespace hu
