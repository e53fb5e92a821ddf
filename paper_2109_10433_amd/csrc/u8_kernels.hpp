// u8_kernels.hpp - validating UTF-8 -> UTF-16LE on gfx950.
//
// Method (Lemire & Mula): section 4 transcodes UTF-8 to UTF-16 block by block,
// finding character starts as the bytes that are not continuation bytes
// (Algorithm "non-validating transcoder"), with an ASCII fast path, and
// validates each block with the Keiser-Lemire nibble tables (section 4, last
// paragraphs; the rules themselves are the six of section 3). The output of
// each block goes where the block's characters start in UTF-16; here every
// 4 KiB tile finds that place with a decoupled look-back (device_common.hpp).
//
// Per tile (256 threads, 16 bytes each):
//   1. coalesced 16-byte loads into LDS, plus the 16-byte granules before and
//      after the tile (3-byte look-behind for validation, 3-byte look-ahead
//      for decoding: a tile owns the characters whose lead byte it holds);
//   2. validation: for every byte, the class bits of (previous byte high
//      nibble, previous byte low nibble, current byte high nibble) from the
//      three nibble tables, AND-ed, staged in LDS as their 4096-entry product;
//      plus the "third / fourth byte must be a continuation" check from the
//      bytes two and three back, and the truncation check at end of input.
//      The first flagged byte f of the input satisfies P <= f <= P + 3 where P
//      is the end of the longest valid prefix; the finalize kernel decodes
//      from just before f to find P and the rule it breaks;
//   3. count UTF-16 words: one per lead byte, two for F0..F7 leads;
//   4. workgroup scan of the counts, publish the tile aggregate;
//   5. decode every lead into one word or a surrogate pair (section 3) and
//      stage the words in LDS at their scanned offsets;
//   6. look-back for the tile's output offset, then coalesced stores.
#pragma once

#include "finish.hpp"

namespace hu {

enum Mode { kValidate = 0, kLength = 1, kConvert = 2 };

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

__constant__ NibbleTables c_nibble = make_nibble_tables();

// Product table entry for index (p << 4) | (c >> 4):
// bit 0 = the pair breaks a rule, bit 1 = both bytes are continuation bytes.
__device__ __forceinline__ unsigned char pair_entry(unsigned int idx)
{
    unsigned int cls = c_nibble.prev_hi[idx >> 8] & c_nibble.prev_lo[(idx >> 4) & 15] & c_nibble.cur_hi[idx & 15];
    return (unsigned char)(((cls & ~kTwoConts) ? 1u : 0u) | ((cls & kTwoConts) ? 2u : 0u));
}

// ------------------------------------------------------------ SWAR helpers
// bit 7 of each byte of the result is set iff that byte of x is >= 0xE0 / 0xF0
__device__ __forceinline__ unsigned int ge_e0(unsigned int x) { return x & (x << 1) & (x << 2) & 0x80808080u; }
__device__ __forceinline__ unsigned int ge_f0(unsigned int x) { return ge_e0(x) & (x << 3); }
// bit 7 of each byte set iff that byte is not a continuation byte (10xxxxxx)
__device__ __forceinline__ unsigned int not_cont(unsigned int x)
{
    unsigned int y = (x & 0xC0C0C0C0u) ^ 0x80808080u;
    return (y | (y << 1)) & 0x80808080u;
}

__device__ __forceinline__ unsigned int inrange_mask(int k, unsigned int lo, unsigned int hi)
{
    unsigned int m = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        unsigned int pos = 4 * k + b;
        m |= (pos >= lo && pos < hi) ? (0xFFu << (8 * b)) : 0u;
    }
    return m;
}

// Decode the character whose lead byte is the low byte of w (little-endian
// window of the next four bytes) into one UTF-16 word or a surrogate pair.
// Bit layouts: section 3 (7/11/16/21 payload bits, most significant first;
// values above U+FFFF become D800 | high ten bits, DC00 | low ten bits of
// value - 0x10000). Returns the word count; garbage in -> garbage out.
__device__ __forceinline__ int decode_utf8_char(unsigned int w, unsigned int *u0, unsigned int *u1)
{
    unsigned int b0 = w & 0xFFu;
    unsigned int b1 = (w >> 8) & 0x3Fu, b2 = (w >> 16) & 0x3Fu, b3 = (w >> 24) & 0x3Fu;
    unsigned int cp2 = ((b0 & 0x1Fu) << 6) | b1;
    unsigned int cp3 = ((b0 & 0x0Fu) << 12) | (b1 << 6) | b2;
    unsigned int cp4 = ((b0 & 0x07u) << 18) | (b1 << 12) | (b2 << 6) | b3;
    unsigned int cp = b0 < 0x80u ? b0 : (b0 < 0xE0u ? cp2 : cp3);
    unsigned int v = cp4 - 0x10000u;
    bool pair = b0 >= 0xF0u;
    *u0 = pair ? (0xD800u | ((v >> 10) & 0x3FFu)) : cp;
    *u1 = 0xDC00u | (v & 0x3FFu);
    return pair ? 2 : 1;
}

// ------------------------------------------------------------ one tile
struct U8Doc {
    const uint8_t *base;          // 16-byte aligned base
    unsigned long long off;       // first byte of the document relative to base
    unsigned long long n;         // bytes
    uint16_t *dst;                // output words
    unsigned long long cap;       // output capacity in words
};

constexpr unsigned int kOutWords = kTile + 8;

struct U8Shared {
    unsigned int in[(kTile + 32) / 4];
    // Valid input gives at most one word per tile byte plus one (a four-byte
    // lead in the last byte). Invalid input can count more; writes past the
    // array are dropped (its output is unspecified anyway).
    unsigned short out[kOutWords];
    unsigned char table[4096];
    unsigned int tmp[kWaves];
    unsigned long long tmp64[kWaves];
    unsigned long long prefix;
    unsigned long long tile;
    int flag;
};

template <int MODE>
__device__ void u8_tile(U8Shared &s, const U8Doc &d, long long tile, unsigned long long *status,
                        long long chain_first, unsigned int epoch, WsHeader *hdr,
                        unsigned long long *err_key, unsigned long long *total)
{
    const int tid = threadIdx.x;
    const unsigned long long end = d.off + d.n;
    const unsigned long long tv = (unsigned long long)tile * kTile;
    const unsigned long long cv = tv + (unsigned long long)tid * kChunk;

    // 1. loads: own chunk, plus the neighbouring granules of the tile
    uint4 q = load_granule(d.base, cv, d.off, end);
    s.in[4 + 4 * tid + 0] = q.x;
    s.in[4 + 4 * tid + 1] = q.y;
    s.in[4 + 4 * tid + 2] = q.z;
    s.in[4 + 4 * tid + 3] = q.w;
    if (tid == 0) {
        uint4 p = tv >= 16 ? load_granule(d.base, tv - 16, d.off, end) : make_uint4(0, 0, 0, 0);
        s.in[0] = p.x; s.in[1] = p.y; s.in[2] = p.z; s.in[3] = p.w;
    } else if (tid == kBlock - 1) {
        uint4 p = load_granule(d.base, tv + kTile, d.off, end);
        s.in[4 + kTile / 4 + 0] = p.x; s.in[4 + kTile / 4 + 1] = p.y;
        s.in[4 + kTile / 4 + 2] = p.z; s.in[4 + kTile / 4 + 3] = p.w;
    }
    __syncthreads();

    unsigned int x[6];
    x[0] = s.in[4 + 4 * tid - 1];
    x[1] = q.x; x[2] = q.y; x[3] = q.z; x[4] = q.w;
    x[5] = s.in[4 + 4 * tid + 4];

    // in-range positions [lo, hi) of this chunk
    unsigned int lo = cv < d.off ? (unsigned int)min(d.off - cv, 16ull) : 0u;
    unsigned int hi = cv + 16 <= end ? 16u : (cv >= end ? 0u : (unsigned int)(end - cv));
    if (hi < lo) hi = lo;

    // 2. validation flags and 3. counts
    const unsigned char *in_bytes = reinterpret_cast<const unsigned char *>(s.in);
    long long flag_rel = 0x7FFFFFFFFFFFFFFFll;   // first flagged position, relative to cv
    unsigned int count = 0;
    unsigned int leads[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        unsigned int rm = inrange_mask(k, lo, hi);
        leads[k] = not_cont(x[k + 1]) & rm;
        if (MODE != kValidate)
            count += __popc(leads[k]) + __popc(ge_f0(x[k + 1]) & rm);
    }
    const bool ascii = ((x[1] | x[2] | x[3] | x[4]) & 0x80808080u) == 0;
    if (!ascii || (x[0] & 0x80000000u) != 0) {
        // An all-ASCII chunk can only be flagged if the byte just before it is
        // part of an unfinished character; otherwise the full check runs.
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            unsigned int cur = x[k + 1], prev = x[k];
            unsigned int p1 = __builtin_amdgcn_alignbyte(cur, prev, 3);   // byte before each byte
            unsigned int p2 = __builtin_amdgcn_alignbyte(cur, prev, 2);   // two before
            unsigned int p3 = __builtin_amdgcn_alignbyte(cur, prev, 1);   // three before
            unsigned int err = 0, two = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                unsigned int idx = (((p1 >> (8 * m)) & 0xFFu) << 4) | ((cur >> (8 * m + 4)) & 0xFu);
                unsigned int e = s.table[idx];
                err |= (e & 1u) << (8 * m + 7);
                two |= (e & 2u) << (8 * m + 6);
            }
            // a continuation byte is required exactly where the byte two back
            // is E0..FF or the byte three back is F0..FF
            unsigned int must = ge_e0(p2) | ge_f0(p3);
            unsigned int flags = (err | (two ^ must)) & inrange_mask(k, lo, 32u);
            if (flags && flag_rel == 0x7FFFFFFFFFFFFFFFll)
                flag_rel = 4 * k + (__builtin_ctz(flags) >> 3);
        }
    }
    // truncation at the end of the input: a lead byte among the last three
    // bytes that needs more bytes than remain
    if (cv < end && cv + 16 >= end) {
        const int e = (int)(end - cv);   // 1..16
#pragma unroll
        for (int back = 3; back >= 1; --back) {
            const int j = e - back;       // >= -2
            if ((long long)cv + j >= (long long)d.off) {
                unsigned int b = in_bytes[16 + kChunk * tid + j];
                unsigned int need = b >= 0xF0u ? 4u : b >= 0xE0u ? 3u : b >= 0xC0u ? 2u : 1u;
                if (need > (unsigned int)back) {
                    if (j < flag_rel)
                        flag_rel = j;
                    break;
                }
            }
        }
    }

    // errors: smallest flagged input position of the tile
    unsigned long long my_flag = ~0ull;
    if (flag_rel != 0x7FFFFFFFFFFFFFFFll)
        my_flag = (unsigned long long)((long long)cv + flag_rel - (long long)d.off);
    unsigned long long tile_flag = block_min_u64(my_flag, s.tmp64);
    if (tid == 0 && tile_flag != ~0ull)
        atomicMax(err_key, ~tile_flag);

    if (MODE == kValidate)
        return;

    // 4. scan
    unsigned int agg;
    unsigned int my_off = block_exclusive_sum(count, s.tmp, &agg);
    if (MODE == kLength) {
        if (tid == 0)
            atomicAdd(total, (unsigned long long)agg);
        return;
    }
    if (tid == 0) {
        atomicAdd(total, (unsigned long long)agg);
        publish(&status[tile], pack_status(epoch, tile == chain_first ? kFlagInclusive : kFlagAggregate, agg));
    }

    // 5. decode into LDS at the scanned offsets
    unsigned int o = my_off;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        unsigned int l = leads[k];
        while (l) {
            unsigned int m = __builtin_ctz(l) >> 3;
            l &= l - 1;
            unsigned int w = __builtin_amdgcn_alignbyte(x[k + 2], x[k + 1], m);
            unsigned int u0, u1;
            int nw = decode_utf8_char(w, &u0, &u1);
            if (o + 1 < kOutWords) {
                s.out[o] = (unsigned short)u0;
                if (nw == 2)
                    s.out[o + 1] = (unsigned short)u1;
            }
            o += nw;
        }
    }

    // 6. output offset of the tile
    if (tid < 64) {
        unsigned long long excl = 0;
        if (tile != chain_first)
            excl = lookback(status, chain_first, tile, epoch, &hdr->hang);
        if (tid == 0) {
            if (tile != chain_first)
                publish(&status[tile], pack_status(epoch, kFlagInclusive, excl + agg));
            s.prefix = excl;
        }
    }
    __syncthreads();
    const unsigned long long pref = s.prefix;
    const unsigned int staged = agg < kOutWords ? agg : kOutWords;
    for (unsigned int i = tid; i < staged; i += kBlock) {
        unsigned long long g = pref + i;
        if (g < d.cap)
            d.dst[g] = s.out[i];
    }
}

// ------------------------------------------------------------ kernels
__device__ __forceinline__ void build_pair_table(unsigned char *table)
{
    for (int i = threadIdx.x; i < 4096; i += kBlock)
        table[i] = pair_entry((unsigned int)i);
}

// One document; persistent workgroups take tiles from the workspace counter;
// the last workgroup to finish writes the call's result.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_u8_single(U8Doc d, unsigned long long n_tiles, WsHeader *hdr,
                                                      unsigned long long *status, unsigned long long status_cap,
                                                      hu_result *out)
{
    __shared__ U8Shared s;
    build_pair_table(s.table);
    const unsigned int epoch = __hip_atomic_load(&hdr->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (threadIdx.x == 0)
            s.tile = atomicAdd(&hdr->tile_counter, 1ull);
        __syncthreads();
        const unsigned long long tile = s.tile;
        if (tile >= n_tiles)
            break;
        u8_tile<MODE>(s, d, (long long)tile, status, 0, epoch, hdr, &hdr->err_key, &hdr->total);
        __syncthreads();
    }
    const CallInfo c{d.base + d.off, d.n, d.cap,
                     MODE == kValidate ? HU_OP_VALIDATE_UTF8
                                       : (MODE == kLength ? HU_OP_UTF16_LENGTH_FROM_UTF8 : HU_OP_CONVERT_UTF8_TO_UTF16LE)};
    finish_launch(c, hdr, status, status_cap, out, &s.flag);
}

}  // namespace hu
