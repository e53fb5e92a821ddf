// u16_kernels.hpp - validating UTF-16LE -> UTF-8 on gfx950.
//
// Method (Lemire & Mula, section 5, Algorithm "UTF-16 to UTF-8"): words below
// U+0080 give one byte, below U+0800 two, other words outside D800..DFFF three,
// a surrogate pair four; the bits are split into 3/4/5 lead-byte payload bits
// and 6-bit continuation payloads with the prefixes 11110 / 1110 / 110 / 10.
// Validation (section 3): a word in D800..DBFF must be followed by one in
// DC00..DFFF and a word in DC00..DFFF must follow one in D800..DBFF. The paper
// leaves pairs to a scalar path (and names vectorising them as future work in
// section 7); here every lane handles its pairs in registers: the high word
// emits all four bytes and the low word none.
//
// Per tile (256 threads, 8 words each): coalesced loads into LDS with a
// one-granule halo on each side; per word byte counts and the unpaired-
// surrogate flag (the first flagged word is exactly the first error); scan;
// encode into LDS; look-back; coalesced stores.
#pragma once

#include "u8_kernels.hpp"

namespace hu {

constexpr int kTileWords = kTile / 2;

struct U16Doc {
    const uint8_t *base;          // 16-byte aligned base
    unsigned long long off;       // first word of the document relative to base, in words
    unsigned long long n;         // words
    uint8_t *dst;                 // output bytes
    unsigned long long cap;       // output capacity in bytes
};

constexpr unsigned int kOutBytes = 3 * kTileWords + 8;

struct U16Shared {
    unsigned int in[(kTile + 32) / 4];
    // Valid input gives at most three bytes per word plus one (a high
    // surrogate in the last word, its low half in the next tile); invalid
    // input can count more and the excess is dropped.
    unsigned char out[kOutBytes];
    unsigned int tmp[kWaves];
    unsigned long long tmp64[kWaves];
    unsigned long long prefix;
    unsigned long long tile;
    int flag;
};

__device__ __forceinline__ bool is_high(unsigned int w) { return (w & 0xFC00u) == 0xD800u; }
__device__ __forceinline__ bool is_low(unsigned int w) { return (w & 0xFC00u) == 0xDC00u; }

// UTF-8 length of the character that starts at word w (followed by nw):
// 0 for the low half of a pair (its high half emits the four bytes).
__device__ __forceinline__ unsigned int utf8_bytes_of(unsigned int w)
{
    return w < 0x80u ? 1u : w < 0x800u ? 2u : is_high(w) ? 4u : is_low(w) ? 0u : 3u;
}

template <int MODE>
__device__ void u16_tile(U16Shared &s, const U16Doc &d, long long tile, unsigned long long *status,
                         long long chain_first, unsigned int epoch, WsHeader *hdr,
                         unsigned long long *err_key, unsigned long long *total)
{
    const int tid = threadIdx.x;
    // byte-granular virtual positions relative to base
    const unsigned long long off_b = 2 * d.off, end_b = 2 * (d.off + d.n);
    const unsigned long long tv = (unsigned long long)tile * kTile;
    const unsigned long long cv = tv + (unsigned long long)tid * kChunk;

    uint4 q = load_granule(d.base, cv, off_b, end_b);
    s.in[4 + 4 * tid + 0] = q.x;
    s.in[4 + 4 * tid + 1] = q.y;
    s.in[4 + 4 * tid + 2] = q.z;
    s.in[4 + 4 * tid + 3] = q.w;
    if (tid == 0) {
        uint4 p = tv >= 16 ? load_granule(d.base, tv - 16, off_b, end_b) : make_uint4(0, 0, 0, 0);
        s.in[0] = p.x; s.in[1] = p.y; s.in[2] = p.z; s.in[3] = p.w;
    } else if (tid == kBlock - 1) {
        uint4 p = load_granule(d.base, tv + kTile, off_b, end_b);
        s.in[4 + kTile / 4 + 0] = p.x; s.in[4 + kTile / 4 + 1] = p.y;
        s.in[4 + kTile / 4 + 2] = p.z; s.in[4 + kTile / 4 + 3] = p.w;
    }
    __syncthreads();

    // words -1 .. 8 of this chunk (word -1 from the previous chunk, 8 from the next)
    unsigned int x[6];
    x[0] = s.in[4 + 4 * tid - 1];
    x[1] = q.x; x[2] = q.y; x[3] = q.z; x[4] = q.w;
    x[5] = s.in[4 + 4 * tid + 4];
    unsigned int wv[10];
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        int j = i + 1;   // index into the 12 half-words of x
        wv[i] = (x[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
    }
    // in-range words [lo, hi) of this chunk
    const unsigned long long cw = cv / 2, offw = d.off, endw = d.off + d.n;
    unsigned int lo = cw < offw ? (unsigned int)min(offw - cw, 8ull) : 0u;
    unsigned int hi = cw + 8 <= endw ? 8u : (cw >= endw ? 0u : (unsigned int)(endw - cw));
    if (hi < lo) hi = lo;

    unsigned int count = 0;
    int first_flag = -1;
    unsigned int nbytes[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        unsigned int w = wv[j + 1], pw = wv[j], nw = wv[j + 2];
        bool in = (unsigned int)j >= lo && (unsigned int)j < hi;
        bool bad = (is_high(w) && !is_low(nw)) || (is_low(w) && !is_high(pw));
        if (in && bad && first_flag < 0)
            first_flag = j;
        nbytes[j] = in ? utf8_bytes_of(w) : 0u;
        count += nbytes[j];
    }
    unsigned long long my_flag = first_flag < 0 ? ~0ull : 2 * (cw + (unsigned int)first_flag - offw);
    unsigned long long tile_flag = block_min_u64(my_flag, s.tmp64);
    if (tid == 0 && tile_flag != ~0ull)
        atomicMax(err_key, ~tile_flag);
    if (MODE == kValidate)
        return;

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

    // encode into LDS at the scanned offsets
    unsigned int o = my_off;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        unsigned int w = wv[j + 1], nw = wv[j + 2], m = nbytes[j];
        unsigned int b[4];
        if (m == 4) {
            unsigned int cp = 0x10000u + (((w & 0x3FFu) << 10) | (nw & 0x3FFu));
            b[0] = 0xF0u | (cp >> 18);
            b[1] = 0x80u | ((cp >> 12) & 0x3Fu);
            b[2] = 0x80u | ((cp >> 6) & 0x3Fu);
            b[3] = 0x80u | (cp & 0x3Fu);
        } else if (m == 3) {
            b[0] = 0xE0u | (w >> 12);
            b[1] = 0x80u | ((w >> 6) & 0x3Fu);
            b[2] = 0x80u | (w & 0x3Fu);
        } else if (m == 2) {
            b[0] = 0xC0u | (w >> 6);
            b[1] = 0x80u | (w & 0x3Fu);
        } else {
            b[0] = w;
        }
        if (o + 3 < kOutBytes) {
#pragma unroll
            for (unsigned int k = 0; k < 4; ++k)
                if (k < m)
                    s.out[o + k] = (unsigned char)b[k];
        }
        o += m;
    }

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
    const unsigned int staged = agg < kOutBytes ? agg : kOutBytes;
    for (unsigned int i = tid; i < staged; i += kBlock) {
        unsigned long long g = pref + i;
        if (g < d.cap)
            d.dst[g] = s.out[i];
    }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_u16_single(U16Doc d, unsigned long long n_tiles, WsHeader *hdr,
                                                       unsigned long long *status, unsigned long long status_cap,
                                                       hu_result *out)
{
    __shared__ U16Shared s;
    const unsigned int epoch = __hip_atomic_load(&hdr->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (threadIdx.x == 0)
            s.tile = atomicAdd(&hdr->tile_counter, 1ull);
        __syncthreads();
        const unsigned long long tile = s.tile;
        if (tile >= n_tiles)
            break;
        u16_tile<MODE>(s, d, (long long)tile, status, 0, epoch, hdr, &hdr->err_key, &hdr->total);
        __syncthreads();
    }
    const CallInfo c{d.base + 2 * d.off, d.n, d.cap,
                     MODE == kValidate ? HU_OP_VALIDATE_UTF16LE
                                       : (MODE == kLength ? HU_OP_UTF8_LENGTH_FROM_UTF16LE : HU_OP_CONVERT_UTF16LE_TO_UTF8)};
    finish_launch(c, hdr, status, status_cap, out, &s.flag);
}

}  // namespace hu
