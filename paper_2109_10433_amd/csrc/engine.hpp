// engine.hpp - tile engine shared by both transcoding directions (gfx950).
//
// An input is cut into tiles of U sub-tiles of 4 KiB. A workgroup of 256
// threads loads a whole tile with U coalesced 16-byte loads per thread, and
// every thread also needs the 4 bytes before and after its 16-byte chunk. The
// direction policy (u8_dir.hpp / u16_dir.hpp) validates and counts each chunk.
//
//  - validate / length: no tile needs another's output offset, so every
//    wave works alone on wave-tiles of a few 1 KiB pieces, grid-stride, with
//    the next wave-tile's loads in flight while it analyses the current one;
//    the wave-tile stays in registers (neighbouring dwords by DPP rotations);
//    counts and the first flagged position are reduced per workgroup and
//    added once at exit.
//  - convert: one workgroup per tile, and the tile stays in registers from
//    the load to the output: the neighbouring dwords come from the adjacent
//    lanes (DPP) and, across wave and sub-tile boundaries, through a few LDS
//    words, so LDS holds only the output staging and the pair table and more
//    workgroups fit a CU. One scan gives every chunk its offset inside the
//    tile, a decoupled look-back gives the tile's offset in the output
//    (device_common.hpp), then per sub-tile the chunks decode into LDS at
//    their offsets, shifted so that LDS and global addresses agree modulo 16,
//    and the sub-tile's output leaves in 16-byte stores.
#pragma once

#include "finish.hpp"
#include "u16_dir.hpp"
#include "u8_dir.hpp"

namespace hu {

struct Doc {
    const uint8_t *base;          // 16-byte aligned address at or below the input
    unsigned long long off_b;     // first input byte, relative to base
    unsigned long long end_b;     // one past the last input byte, relative to base
    unsigned long long n;         // input code units
    void *dst;                    // output
    unsigned long long cap;       // output capacity in code units
};

template <class Dir>
struct ScanShared {
    alignas(16) unsigned char table[Dir::kNeedsTable ? 4096 : 16];
    unsigned long long red[kWaves];
    int flag;
};

// Output staging starts this many units into its buffer (see emit_tile); 16
// units keep LDS and global addresses congruent modulo 16 bytes.
constexpr unsigned int kStageFront = 16;

// The dwords at the wave and sub-tile boundaries of a register-resident tile.
template <int U>
struct TileEdges {
    unsigned int first[U][kWaves];   // first dword of each wave's part of sub-tile u
    unsigned int last[U][kWaves];    // last dword of it
    unsigned int pre, post;          // the dword just before the tile, just after it
};

template <class Dir, int U>
struct ConvertShared {
    alignas(16) typename Dir::Out out[kStageFront + Dir::kStageUnits];
    alignas(16) unsigned char table[Dir::kNeedsTable ? 4096 : 16];
    TileEdges<U> edges;
    unsigned int scan[U][kWaves];
    unsigned long long red[kWaves];
    unsigned long long prefix;
};

// Global (L2-resident) copy of the pair table -> LDS: one 16-byte load per thread.
__device__ __forceinline__ void build_pair_table(unsigned char *table)
{
    static_assert(4096 == 16 * kBlock, "one granule per thread");
    const uint4 v = reinterpret_cast<const uint4 *>(g_pair_table.e)[threadIdx.x];
    reinterpret_cast<uint4 *>(table)[threadIdx.x] = v;
}

// Issue all loads of tile `tile`: U chunks per thread, plus (thread 0) the
// granules just before and just after the tile. Unmasked: settle_tile zeroes
// what lies outside the document.
// INSIDE_FAST: tiles wholly inside the input load without guards (fewer
// registers; the batch kernel takes it) rather than through the guarded path
// whatever the tile (the single-buffer convert kernels measured 2-3 % faster
// that way).
template <int U, bool INSIDE_FAST = false>
__device__ __forceinline__ void load_tile(const Doc &d, unsigned long long tile, uint4 q[U], uint4 &pre, uint4 &post)
{
    const unsigned long long tv = tile * (unsigned long long)(U * kSub);
    if (INSIDE_FAST && tv >= d.off_b && tv + (unsigned long long)U * kSub <= d.end_b) {
        const uint4 *g = reinterpret_cast<const uint4 *>(d.base + tv) + threadIdx.x;
#pragma unroll
        for (int u = 0; u < U; ++u)
            q[u] = g[u * kBlock];
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u)
            q[u] = load_granule_raw(d.base, tv + (unsigned long long)u * kSub + threadIdx.x * kChunk, d.off_b,
                                    d.end_b);
    }
    if (threadIdx.x == 0) {
        pre = load_granule_raw(d.base, tv >= 16 ? tv - 16 : 0, d.off_b, d.end_b);
        post = load_granule_raw(d.base, tv + (unsigned long long)U * kSub, d.off_b, d.end_b);
    }
}

// A tile held in registers: this thread's chunk of every sub-tile. The
// dwords just before and after a chunk come from the adjacent lanes (DPP)
// each time the chunk is read, and at the ends of a wave from the boundary
// dwords in LDS (settle_tile), so they hold no registers between uses.
template <int U>
struct TileRegs {
    uint4 q[U];
    const TileEdges<U> *e;

    // FRESH: hide the chunk's identity from the compiler, so that values it
    // derived from the chunk in an earlier phase are recomputed instead of
    // being kept in registers across the phases in between.
    template <bool FRESH = false>
    __device__ __forceinline__ void chunk(int u, unsigned int x[6]) const
    {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        const unsigned int *lo = wave > 0 ? &e->last[u][wave - 1] : (u > 0 ? &e->last[u - 1][kWaves - 1] : &e->pre);
        const unsigned int *hi = wave < kWaves - 1 ? &e->first[u][wave + 1] : (u + 1 < U ? &e->first[u + 1][0] : &e->post);
        x[1] = q[u].x; x[2] = q[u].y; x[3] = q[u].z; x[4] = q[u].w;
        if (FRESH) {
#pragma unroll
            for (int k = 1; k <= 4; ++k)
                x[k] = opaque(x[k]);
        }
        const unsigned int p = from_lower_lane(x[4]), n = from_upper_lane(x[1]);
        const unsigned int pe = *lo, ne = *hi;   // same address in every lane: broadcast reads
        x[0] = lane == 0 ? pe : p;
        x[5] = lane == 63 ? ne : n;
    }
};

// After load_tile: zero the bytes outside the document (tiles at its edges
// only) and post the boundary dwords to LDS. A barrier must follow before
// the first TileRegs::chunk. SWAP: big-endian UTF-16 input, brought to
// little endian here.
template <int U, bool SWAP = false>
__device__ __forceinline__ void settle_tile(TileEdges<U> &e, const Doc &d, unsigned long long tile, TileRegs<U> &t,
                                            uint4 pre, uint4 post)
{
    const unsigned long long tv = tile * (unsigned long long)(U * kSub);
    if (tv < d.off_b || tv + (unsigned long long)U * kSub > d.end_b) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            t.q[u] = mask_granule(t.q[u], tv + (unsigned long long)u * kSub + threadIdx.x * kChunk, d.off_b, d.end_b);
    }
    if constexpr (SWAP) {
#pragma unroll
        for (int u = 0; u < U; ++u)
            t.q[u] = swap16(t.q[u]);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (lane == 0)
            e.first[u][wave] = t.q[u].x;
        if (lane == 63)
            e.last[u][wave] = t.q[u].w;
    }
    if (threadIdx.x == 0) {
        const unsigned int pw = tv >= 16 ? mask_granule(pre, tv - 16, d.off_b, d.end_b).w : 0u;
        const unsigned int px = mask_granule(post, tv + (unsigned long long)U * kSub, d.off_b, d.end_b).x;
        e.pre = SWAP ? swap16(pw) : pw;
        e.post = SWAP ? swap16(px) : px;
    }
}

// Input units of the chunk at byte position cv that lie in the input.
template <class Dir>
__device__ __forceinline__ void chunk_range(const Doc &d, unsigned long long cv, unsigned int &lo, unsigned int &hi)
{
    constexpr unsigned int per = kChunk / Dir::kInUnit;
    const unsigned long long c = cv / Dir::kInUnit, o = d.off_b / Dir::kInUnit, e = d.end_b / Dir::kInUnit;
    lo = c < o ? (unsigned int)min(o - c, (unsigned long long)per) : 0u;
    hi = c + per <= e ? per : (c >= e ? 0u : (unsigned int)(e - c));
    if (hi < lo)
        hi = lo;
}

// A tile whose chunks all lie inside the input with the input end beyond them
// needs no count correction and no end-of-input check.
template <int U>
__device__ __forceinline__ bool tile_is_interior(const Doc &d, unsigned long long tile)
{
    const unsigned long long tv = tile * (unsigned long long)(U * kSub);
    return tv >= d.off_b && tv + (unsigned long long)U * kSub < d.end_b;
}

// Truncation at the input's end: thread 0 of the tile that holds the last
// input unit lowers flag_min to the lead of a last character cut short (the
// direction reads the last bytes from memory).
template <class Dir, int U>
__device__ __forceinline__ void end_check(const Doc &d, unsigned long long tile, unsigned long long &flag_min)
{
    const unsigned long long tv = tile * (unsigned long long)(U * kSub);
    if (threadIdx.x == 0 && d.end_b > tv && d.end_b <= tv + (unsigned long long)U * kSub) {
        const long long j = Dir::end_truncation(d.base, d.off_b, d.end_b);
        if (j >= 0 && (unsigned long long)j < flag_min)
            flag_min = (unsigned long long)j;
    }
}

// Validation and counting of a staged tile. Returns the per-chunk counts in
// c[] and lowers flag_min to the first flagged input byte position; cls gets
// each sub-tile's wave class for emit (three bits per sub-tile, in a scalar
// register).
// SKIP_PAST: sub-tiles wholly past the input's end are not analysed (batch
// items, where every document's last tile may be short; the single-buffer
// kernels, whose only such tile is the input's last, measured 2-7 % slower
// with the test in their loops).
template <class Dir, int U, bool COUNT, bool SKIP_PAST = false>
__device__ __forceinline__ void analyze_chunks(const TileRegs<U> &t, const unsigned char *table, const Doc &d,
                                               unsigned long long tile, unsigned int c[U],
                                               unsigned long long &flag_min, unsigned int &cls)
{
    static_assert(3 * U <= 32, "three class bits per sub-tile");
    cls = 0;
    // first flag as a 32-bit position inside the tile (no 64-bit chunk
    // positions kept live across the sub-tiles)
    unsigned int rel_min = ~0u;
    const unsigned long long tv = tile * (unsigned long long)(U * kSub);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (SKIP_PAST && tv + (unsigned long long)u * kSub >= d.end_b) {
            // a sub-tile wholly past the input's end: nothing to validate;
            // counted as its zeros, which the edge correction takes off again
            c[u] = kChunk / Dir::kInUnit;
            continue;
        }
        unsigned int x[6];
        t.chunk(u, x);
        int f;
        unsigned int k;
        c[u] = Dir::template analyze<COUNT>(x, table, &f, &k);
        cls |= __builtin_amdgcn_readfirstlane(k) << (3 * u);
        if (f != kNoFlag) {
            const unsigned int rel = (unsigned int)(u * kSub) + threadIdx.x * kChunk + (unsigned int)f * Dir::kInUnit;
            rel_min = rel < rel_min ? rel : rel_min;
        }
        // keep sub-tiles from being interleaved by the scheduler (register pressure)
        __builtin_amdgcn_sched_barrier(0);
    }
    if (rel_min != ~0u) {
        // zeros before the input are never flagged: the position is >= off_b
        const unsigned long long pos = tile * (unsigned long long)(U * kSub) + rel_min - d.off_b;
        flag_min = pos < flag_min ? pos : flag_min;
    }
}

template <class Dir, int U, bool COUNT, bool SKIP_PAST = false>
__device__ __forceinline__ void analyze_tile(const TileRegs<U> &t, const unsigned char *table, const Doc &d,
                                             unsigned long long tile, unsigned int c[U], unsigned long long &flag_min,
                                             unsigned int &cls)
{
    analyze_chunks<Dir, U, COUNT, SKIP_PAST>(t, table, d, tile, c, flag_min, cls);
    if (!tile_is_interior<U>(d, tile)) {
        // Tiles at the input's edges hold zeros outside the input: each zero
        // counts as one unit (an ASCII byte or word), and the only flags they
        // raise are those of a last character cut short by the end, at a
        // position past it; that truncation is reported at the last unit
        // (the first-error decode in finish.hpp starts up to three bytes
        // before the flag and finds it).
        const unsigned long long tv = tile * (unsigned long long)(U * kSub);
        if (COUNT) {
            // chunk positions recomputed here rather than kept live since the loads
            const unsigned int tid = opaque(threadIdx.x);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const unsigned long long cv = tv + (unsigned long long)u * kSub + (unsigned long long)tid * kChunk;
                unsigned int lo, hi;
                chunk_range<Dir>(d, cv, lo, hi);
                c[u] -= (unsigned int)(kChunk / Dir::kInUnit) - (hi - lo);
            }
        }
        end_check<Dir, U>(d, tile, flag_min);
        const unsigned long long n_b = d.end_b - d.off_b;
        if (flag_min != ~0ull && flag_min >= n_b)
            flag_min = n_b - Dir::kInUnit;
    }
}

// Counts only, for input known to be valid: no validation, no flag. Edge
// tiles corrected as in analyze_tile.
template <class Dir, int U, bool SKIP_PAST = false>
__device__ __forceinline__ void count_tile(const TileRegs<U> &t, const Doc &d, unsigned long long tile,
                                           unsigned int c[U])
{
    const unsigned long long tv0 = tile * (unsigned long long)(U * kSub);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (SKIP_PAST && tv0 + (unsigned long long)u * kSub >= d.end_b) {
            c[u] = kChunk / Dir::kInUnit;   // past the input's end, as in analyze_chunks
            continue;
        }
        unsigned int x[6];
        t.chunk(u, x);
        c[u] = Dir::count_only(x);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (!tile_is_interior<U>(d, tile)) {
        const unsigned long long tv = tile * (unsigned long long)(U * kSub);
        const unsigned int tid = opaque(threadIdx.x);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const unsigned long long cv = tv + (unsigned long long)u * kSub + (unsigned long long)tid * kChunk;
            unsigned int lo, hi;
            chunk_range<Dir>(d, cv, lo, hi);
            c[u] -= (unsigned int)(kChunk / Dir::kInUnit) - (hi - lo);
        }
    }
}

// Exclusive offsets of every thread's count for each of U sub-tiles, and the
// sub-tile totals, with one barrier. Counts are at most 32 per thread, so two
// sub-tiles share one 32-bit scan (a wave's total stays below 2^16). With
// FLAG, the same barrier also yields the workgroup's smallest flag.
template <int U, bool FLAG = false>
__device__ __forceinline__ void block_scan_multi(const unsigned int c[U], unsigned int excl[U], unsigned int tot[U],
                                                 unsigned int (*s_scan)[kWaves], unsigned long long flag = ~0ull,
                                                 unsigned long long *s_red = nullptr,
                                                 unsigned long long *flag_min = nullptr)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    if constexpr (FLAG) {
        const unsigned long long m = wave_min_u64(flag);
        if (lane == 0)
            s_red[wave] = m;
    }
#pragma unroll
    for (int i = 0; i < U; i += 2) {
        if (i + 1 < U) {
            const unsigned int v = c[i] | (c[i + 1] << 16);
            const unsigned int inc = wave_inclusive_sum(v);
            if (lane == 63) {
                s_scan[i][wave] = inc & 0xFFFFu;
                s_scan[i + 1][wave] = inc >> 16;
            }
            const unsigned int e = inc - v;
            excl[i] = e & 0xFFFFu;
            excl[i + 1] = e >> 16;
        } else {                       // odd U: the last sub-tile alone
            const unsigned int inc = wave_inclusive_sum(c[i]);
            if (lane == 63)
                s_scan[i][wave] = inc;
            excl[i] = inc - c[i];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < U; ++u) {
        unsigned int before = 0, all = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const unsigned int x = s_scan[u][w];
            before += (w < wave) ? x : 0u;
            all += x;
        }
        excl[u] += before;
        // done here, not sunk past the look-back with the loaded totals kept live
        asm volatile("" : "+v"(excl[u]) :: "memory");
        tot[u] = __builtin_amdgcn_readfirstlane(all);   // uniform: keep it in a scalar register
    }
    if constexpr (FLAG) {
        unsigned long long m = s_red[0];
#pragma unroll
        for (int w = 1; w < kWaves; ++w)
            m = s_red[w] < m ? s_red[w] : m;
        *flag_min = m;
    }
}

// Copy staged output units out[0, shift + w) (valid from index `shift`) to
// global units [gbase + shift, gbase + shift + w), where unit gbase sits at a
// 16-byte aligned address; nothing at or past `cap` is written. SWAP: 16-bit
// units leave big endian.
// NT threads take part (t: this thread's index among them); STAGE: the
// staging buffer's capacity in units.
template <class Dir, bool SWAP = false, unsigned int NT = kBlock, unsigned int STAGE = Dir::kStageUnits>
__device__ __forceinline__ void copy_out(const typename Dir::Out *out, unsigned int shift, unsigned int w,
                                         typename Dir::Out *dst, long long gbase, unsigned long long cap,
                                         unsigned int t = threadIdx.x)
{
    using Out = typename Dir::Out;
    constexpr unsigned int G = 16 / sizeof(Out);
    unsigned int span = shift + w;
    if (span > STAGE)
        span = STAGE;   // only on invalid input
    const unsigned int groups = (span + G - 1) / G;
    // The usual case: all of [gbase + shift, gbase + span) inside [0, cap).
    // Whole groups are then copied with no tests, and threads 0..2G-1 store
    // the units of the partial groups at either end one by one.
    const bool fits = gbase + (long long)shift >= 0 && (unsigned long long)(gbase + (long long)span) <= cap;
    if (fits) {
        const unsigned int gb = (shift + G - 1) / G, ge = span / G;   // whole groups: [gb, ge)
        for (unsigned int g = gb + t; g < ge; g += NT) {
            const unsigned int i0 = g * G;
            const uint4 v = *reinterpret_cast<const uint4 *>(out + i0);
            *reinterpret_cast<uint4 *>(dst + (gbase + (long long)i0)) = SWAP ? swap16(v) : v;
        }
        const unsigned int head_end = gb * G < span ? gb * G : span;
        const unsigned int tail_begin = ge > gb ? ge * G : head_end;
        static_assert(2 * G <= NT, "threads for both partial groups");
        const unsigned int i = t < G ? shift + t : tail_begin + (t - G);
        if (t < 2 * G && (t < G ? i < head_end : i < span)) {
            const Out v = out[i];
            dst[gbase + (long long)i] = SWAP ? (Out)((v >> 8) | (v << 8)) : v;
        }
        return;
    }
    for (unsigned int g = t; g < groups; g += NT) {
        const unsigned int i0 = g * G;
        const long long j0 = gbase + (long long)i0;
        if (i0 >= shift && i0 + G <= span && j0 >= 0 && (unsigned long long)j0 + G <= cap) {
            const uint4 v = *reinterpret_cast<const uint4 *>(out + i0);
            *reinterpret_cast<uint4 *>(dst + j0) = SWAP ? swap16(v) : v;
        } else {
#pragma unroll
            for (unsigned int k = 0; k < G; ++k) {
                const unsigned int i = i0 + k;
                const long long j = j0 + (long long)k;
                if (i >= shift && i < span && j >= 0 && (unsigned long long)j < cap)
                    dst[j] = SWAP ? (Out)((out[i] >> 8) | (out[i] << 8)) : out[i];
            }
        }
    }
}

// Per-workgroup results at exit: the sum of counts (if any) and the first
// flag, one atomic each, then the end-of-launch protocol.
__device__ __forceinline__ void workgroup_exit(unsigned long long my_total, unsigned long long my_flag,
                                               unsigned long long *red, const CallInfo &c, WsHeader *hdr,
                                               unsigned long long *status, unsigned long long status_cap,
                                               hu_result *out, int *s_flag, bool add_total)
{
    const unsigned long long f = block_min_u64(my_flag, red);
    const unsigned long long t = add_total ? block_sum_u64(my_total, red) : 0ull;
    if (threadIdx.x == 0) {
        // both atomics have returned before finish_launch counts the
        // workgroup done (relaxed, no cache-wide fence: see finish_launch)
        if (f != ~0ull)
            report_flag(&hdr->err_key, f);
        if (add_total && t != 0) {
            const unsigned long long old = atomicAdd(&hdr->total, t);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            if (old == 0x5A5A5A5A5A5A5A5Aull)   // consumes the returned value (forces the wait)
                __builtin_amdgcn_s_sleep(1);
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
        }
    }
    finish_launch(c, hdr, status, status_cap, out, s_flag, &red[0]);
}

// ------------------------------------------------------------ validate / length
// A wave-tile is P pieces of 1 KiB, a piece one 16-byte load per lane; wave w
// of a grid of W waves takes wave-tiles w, w + W, w + 2W, ..., issues all
// loads of the next one before it analyses the current one, each piece as
// soon as its load is in. A lane's
// neighbouring dwords come from the adjacent lanes by DPP rotations:
// lane 0's dword before from lane 63 of the piece before (of the same
// register), lane 63's dword after from lane 0 of the piece after, and at the
// wave-tile's two ends from one load of the same address in every lane.
constexpr int kPiece = 64 * kChunk;

template <int P>
struct WaveTile {
    uint4 q[P];
    unsigned int pre, post;   // the dword just before the wave-tile, just after it
};

// The dword at byte position v (4-byte aligned, relative to the document's
// 16-byte aligned base); a dword with no byte of the document is not read,
// its load goes to the document's first dword instead (as load_granule_raw).
__device__ __forceinline__ unsigned int load_dword_raw(const uint8_t *base, unsigned long long v, unsigned long long off,
                                                       unsigned long long end)
{
    const bool any = v < end && v + 4 > off;
    const unsigned long long a = any ? v : (off & ~3ull);
    // a vector load although the address is uniform: a scalar load would share
    // its wait counter with the LDS reads of the analysis, out of order, so
    // every table lookup would wait for it
    return *reinterpret_cast<const unsigned int *>(base + a + opaque(0u));
}

// Zero the bytes of dword w (at position v) that are outside [off, end).
__device__ __forceinline__ unsigned int mask_dword(unsigned int w, unsigned long long v, unsigned long long off,
                                                   unsigned long long end)
{
    const long long lo_s = (long long)off - (long long)v, hi_s = (long long)end - (long long)v;
    const int lo = lo_s < 0 ? 0 : (lo_s > 4 ? 4 : (int)lo_s);
    const int hi = hi_s < 0 ? 0 : (hi_s > 4 ? 4 : (int)hi_s);
    const unsigned long long m = ((1ull << (8 * hi)) - 1) & ~((1ull << (8 * lo)) - 1);
    return w & (unsigned int)m;
}

// Lane l receives lane l - 1's value, lane 0 lane 63's (DPP wave_ror:1).
__device__ __forceinline__ unsigned int rotate_from_lower_lane(unsigned int v)
{
    return (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, 0x13C, 0xF, 0xF, false);
}

// Lane l receives lane l + 1's value, lane 63 lane 0's (DPP wave_rol:1).
__device__ __forceinline__ unsigned int rotate_from_upper_lane(unsigned int v)
{
    return (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, 0x134, 0xF, 0xF, false);
}

// All loads of wave-tile wt, unmasked (scan_wave_tile zeroes what lies
// outside the document).
template <int P>
__device__ __forceinline__ void load_wave_tile(const Doc &d, unsigned long long wt, WaveTile<P> &t)
{
    const unsigned int lane = threadIdx.x & 63;
    const unsigned long long tv = wt * (unsigned long long)(P * kPiece);
    if (tv >= d.off_b && tv + (unsigned long long)P * kPiece <= d.end_b) {
        // every granule of the wave-tile holds bytes of the document: no guards
        const uint4 *g = reinterpret_cast<const uint4 *>(d.base + tv) + lane;
#pragma unroll
        for (int u = 0; u < P; ++u)
            t.q[u] = g[u * 64];
    } else {
#pragma unroll
        for (int u = 0; u < P; ++u)
            t.q[u] = load_granule_raw(d.base, tv + (unsigned long long)u * kPiece + lane * kChunk, d.off_b, d.end_b);
    }
    t.pre = load_dword_raw(d.base, tv >= 4 ? tv - 4 : 0, d.off_b, d.end_b);
    t.post = load_dword_raw(d.base, tv + (unsigned long long)P * kPiece, d.off_b, d.end_b);
}

// Validation (and counting) of one wave-tile; all lanes of the wave call.
// Tiles at the document's edges zero what lies outside it and correct their
// counts as analyze_tile does; the wave-tile that holds the last input unit
// checks for a last character cut short.
template <class Dir, int P, bool COUNT, bool SWAP>
__device__ __forceinline__ void scan_wave_tile(WaveTile<P> &t, const unsigned char *table, const Doc &d,
                                               unsigned long long wt, unsigned long long &total,
                                               unsigned long long &flag_min)
{
    const unsigned int lane = threadIdx.x & 63;
    const unsigned long long tv = wt * (unsigned long long)(P * kPiece);
    const bool interior = tv >= d.off_b && tv + (unsigned long long)P * kPiece < d.end_b;
    // the dwords beyond the wave-tile are masked whatever the tile (the first
    // wave-tile of a document that starts 16-byte aligned is interior, and has
    // nothing before it)
    const unsigned int pre = tv >= 4 ? mask_dword(t.pre, tv - 4, d.off_b, d.end_b) : 0u;
    const unsigned int post = mask_dword(t.post, tv + (unsigned long long)P * kPiece, d.off_b, d.end_b);
    if (!interior) {
#pragma unroll
        for (int u = 0; u < P; ++u)
            t.q[u] = mask_granule(t.q[u], tv + (unsigned long long)u * kPiece + lane * kChunk, d.off_b, d.end_b);
    }
    if constexpr (SWAP) {
#pragma unroll
        for (int u = 0; u < P; ++u)
            t.q[u] = swap16(t.q[u]);
    }
    unsigned int sum = 0;
    unsigned int rel_min = ~0u;           // first flag, as a byte offset in the wave-tile
    unsigned int before = SWAP ? swap16(pre) : pre;   // lane 0: the dword before the piece
#pragma unroll
    for (int u = 0; u < P; ++u) {
        unsigned int x[6];
        x[1] = t.q[u].x; x[2] = t.q[u].y; x[3] = t.q[u].z; x[4] = t.q[u].w;
        const unsigned int r = rotate_from_lower_lane(x[4]);
        x[0] = lane == 0 ? before : r;
        before = r;                       // at lane 0: lane 63's last dword, the next piece's dword before
        const unsigned int after = u + 1 < P ? rotate_from_upper_lane(t.q[u + 1 < P ? u + 1 : u].x)
                                             : (SWAP ? swap16(post) : post);
        const unsigned int l = rotate_from_upper_lane(x[1]);
        x[5] = lane == 63 ? after : l;
        int f;
        unsigned int cls;
        const unsigned int c = Dir::template analyze<COUNT>(x, table, &f, &cls);
        if (f != kNoFlag) {
            const unsigned int rel = (unsigned int)(u * kPiece) + lane * kChunk + (unsigned int)f * Dir::kInUnit;
            rel_min = rel < rel_min ? rel : rel_min;
        }
        sum += c;
        // keep pieces from being interleaved by the scheduler (register pressure)
        __builtin_amdgcn_sched_barrier(0);
    }
    if (COUNT) {
        total += sum;
        if (!interior && lane == 0) {
            // each zero outside the input counted as one unit (a byte or word
            // below 0x80): the wave-tile's units outside it, taken off once
            const unsigned long long te = tv + (unsigned long long)P * kPiece;
            const unsigned long long lo = tv > d.off_b ? tv : d.off_b, hi = te < d.end_b ? te : d.end_b;
            const unsigned long long inside = hi > lo ? (hi - lo) / Dir::kInUnit : 0ull;
            total -= (unsigned long long)(P * kPiece / Dir::kInUnit) - inside;
        }
    }
    if (rel_min != ~0u) {
        // zeros before the input are never flagged: the position is >= off_b
        const unsigned long long pos = tv + rel_min - d.off_b;
        flag_min = pos < flag_min ? pos : flag_min;
    }
    if (!interior) {
        if (lane == 0 && d.end_b > tv && d.end_b <= tv + (unsigned long long)P * kPiece) {
            const long long j = Dir::end_truncation(d.base, d.off_b, d.end_b);
            if (j >= 0 && (unsigned long long)j < flag_min)
                flag_min = (unsigned long long)j;
        }
        const unsigned long long n_b = d.end_b - d.off_b;
        if (flag_min != ~0ull && flag_min >= n_b)
            flag_min = n_b - Dir::kInUnit;
    }
}

// n_tiles: wave-tiles of P pieces covering the document.
template <class Dir, int MODE, int P, bool SWAP = false>
__global__ __launch_bounds__(kBlock) void k_scan(Doc d, unsigned long long n_tiles, WsHeader *hdr,
                                                 unsigned long long *status, unsigned long long status_cap,
                                                 hu_result *out)
{
    __shared__ ScanShared<Dir> s;
    if (Dir::kNeedsTable)
        build_pair_table(s.table);
    __syncthreads();
    unsigned long long my_total = 0, my_flag = ~0ull;
    const unsigned long long stride = (unsigned long long)gridDim.x * kWaves;
    // the wave's index, known to the compiler as uniform: the wave-tile
    // index and everything derived from it stay in scalar registers
    const unsigned int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    unsigned long long wt = (unsigned long long)blockIdx.x * kWaves + wave;
    // the loads of the next wave-tile are issued before this one is
    // analysed (the last round reloads its own wave-tile, never used)
    if (wt < n_tiles) {
        WaveTile<P> t;
        load_wave_tile<P>(d, wt, t);
        for (;;) {
            const unsigned long long wn = wt + stride;
            WaveTile<P> nx;
            load_wave_tile<P>(d, wn < n_tiles ? wn : wt, nx);
            scan_wave_tile<Dir, P, MODE == kLength, SWAP>(t, s.table, d, wt, my_total, my_flag);
            if (wn >= n_tiles)
                break;
            t = nx;
            wt = wn;
        }
    }
    const CallInfo c{d.base + d.off_b, d.n, d.cap, MODE == kLength ? Dir::kOpLength : Dir::kOpValidate};
    workgroup_exit(my_total, my_flag, s.red, c, hdr, status, status_cap, out, &s.flag, MODE == kLength);
}

// Output phase of a convert tile: per sub-tile, chunks decode into LDS at
// their offsets (shifted so that LDS and global addresses agree modulo 16),
// then the sub-tile's output leaves in aligned 16-byte stores. `stage` points
// kStageFront units into the staging buffer. Units outside the input are
// zeros and decode like any other (one output unit each): those after the
// input's end land past the sub-tile's output, which is never copied out;
// those before its start (only in the first chunk of the first tile, fewer
// than 16 bytes of alignment) land just before the chunk's output, in the
// staging buffer's front margin.
template <class Dir, int U, bool SWAP = false, bool SKIP_PAST = false>
__device__ __forceinline__ void emit_tile(const TileRegs<U> &t, typename Dir::Out *stage, const Doc &d,
                                          unsigned long long tile, const unsigned int excl[U], const unsigned int tot[U],
                                          unsigned long long pos, typename Dir::Out *dst, unsigned int cls)
{
    using Out = typename Dir::Out;
    // output units between dst and the 16-byte aligned address below it
    const unsigned int dst_mis = (unsigned int)(((uintptr_t)d.dst & 15u) / sizeof(Out));
    constexpr unsigned int G = 16 / sizeof(Out);
    const unsigned int skip = (tile == 0 && threadIdx.x == 0) ? (unsigned int)(d.off_b / Dir::kInUnit) : 0u;
    const unsigned long long tv = tile * (unsigned long long)(U * kSub);
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (SKIP_PAST && tv + (unsigned long long)u * kSub >= d.end_b)
            break;   // this and the later sub-tiles lie past the input's end: no output
        const unsigned int shift = (unsigned int)((dst_mis + pos) % G);
        unsigned int x[6];
        t.template chunk<true>(u, x);
        Dir::emit(x, stage, shift + excl[u] - (u == 0 ? skip : 0u), (cls >> (3 * u)) & 7u);
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();
        copy_out<Dir, SWAP>(stage, shift, tot[u], dst, (long long)pos - (long long)shift, d.cap);
        __syncthreads();
        pos += tot[u];
    }
}

// ------------------------------------------------------------ chained tiles
// Where a tile sits in a look-back chain: one chain per document.
struct Chain {
    unsigned long long *status;      // status words: item i at status[i * stride]
    unsigned long long first;        // item index of the document's first tile
    unsigned long long item;         // item index of this tile
    unsigned int epoch;
    unsigned long long *err_key;     // the document's error key
    unsigned int *hang;
    unsigned int stride;
};

// One tile of a document in a look-back chain: load, validate, count, scan,
// publish, look back; thread 0 of the document's last tile then calls
// fin(total output units); in convert mode the tile's output is written.
// The pair table must already be in `table` (LDS). All threads must call.
// SWAP_IN: big-endian UTF-16 input; SWAP_OUT: big-endian UTF-16 output.
// ITEM: a batch work item (interior tiles load without guards); SKIP_PAST:
// sub-tiles wholly past the document's end are skipped (batches of UTF-8
// documents: 5 % faster on the 100k documents; the UTF-16 documents, long
// ones, measured 3 % slower with it).
template <class Dir, int U, int MODE, bool SWAP_IN = false, bool SWAP_OUT = false, bool ITEM = false,
          bool SKIP_PAST = false, class Shared, class Finisher>
__device__ __forceinline__ void chained_tile(Shared &s, const unsigned char *table, const Doc &d,
                                             unsigned long long tile, unsigned long long n_tiles, const Chain &cx,
                                             Finisher fin)
{
    using Out = typename Dir::Out;
    const int tid = threadIdx.x;
    TileRegs<U> t;
    t.e = &s.edges;
    uint4 pre = make_uint4(0, 0, 0, 0), post = make_uint4(0, 0, 0, 0);
    load_tile<U, ITEM>(d, tile, t.q, pre, post);
    settle_tile<U, SWAP_IN>(s.edges, d, tile, t, pre, post);
    __syncthreads();

    unsigned long long my_flag = ~0ull;
    unsigned int c[U];
    unsigned int cls = ~0u;   // wave class per sub-tile; all 7 (unknown) without analysis
    if (MODE == kTrusted)
        count_tile<Dir, U, SKIP_PAST>(t, d, tile, c);
    else
        analyze_tile<Dir, U, MODE != kValidate, SKIP_PAST>(t, table, d, tile, c, my_flag, cls);
    unsigned long long tile_flag = ~0ull;
    unsigned int excl[U], tot[U];
    block_scan_multi<U, MODE != kTrusted>(c, excl, tot, s.scan, my_flag, s.red, &tile_flag);
    unsigned int agg = 0;
#pragma unroll
    for (int u = 0; u < U; ++u)
        agg += tot[u];
    const bool first = cx.item == cx.first;
    if (tid == 0) {
        if (tile_flag != ~0ull)
            report_flag(cx.err_key, tile_flag);
        publish(&cx.status[cx.item * cx.stride], pack_status(cx.epoch, first ? kFlagInclusive : kFlagAggregate, agg));
    }
    if (tid < 64) {
        unsigned long long excl_tile = 0;
        if (!first)
            excl_tile = lookback(cx.status, cx.stride, (long long)cx.first, (long long)cx.item, cx.epoch, cx.hang);
        if (tid == 0) {
            if (!first)
                publish(&cx.status[cx.item * cx.stride], pack_status(cx.epoch, kFlagInclusive, excl_tile + agg));
            s.prefix = excl_tile;
        }
    }
    __syncthreads();
    const unsigned long long pos = s.prefix;   // output units before this tile
    if (tile == n_tiles - 1 && tid == 0)
        fin(pos + agg);
    // A tile with a flagged position makes the call fail, and the output of a
    // failed call is unspecified: only flag-free (valid) tiles are decoded.
    // Unvalidated input (kTrusted) is decoded as it is, as long as every
    // sub-tile's count leaves room in the staging buffer for the alignment
    // shift and the zeros past the input's end (always so for valid input;
    // invalid input can count more, and then its tile is not decoded).
    bool decode = MODE == kConvert && tile_flag == ~0ull;
    if (MODE == kTrusted) {
        decode = true;
#pragma unroll
        for (int u = 0; u < U; ++u)
            decode = decode && tot[u] + 2 * kChunk <= Dir::kStageUnits;
    }
    if (decode) {
        Out *dst = reinterpret_cast<Out *>(d.dst);
        emit_tile<Dir, U, SWAP_OUT, SKIP_PAST>(t, s.out + kStageFront, d, tile, excl, tot, pos, dst, cls);
    }
}

// ------------------------------------------------------------ convert
// One workgroup per tile, tile = blockIdx.x. A tile only waits (in the
// look-back) for tiles with smaller ids; workgroups are dispatched in id order
// on each XCD, so the lowest unfinished tile always has a running workgroup and
// all its predecessors done. No tile counter, no per-workgroup atomics: the
// output total is the last tile's inclusive prefix, and the workgroup of the
// last tile writes the call's result once its look-back is complete (every
// tile publishes its status only after its error report has landed, so by
// then all reports are in).
//
// When the last tile's look-back ends, tiles between its nearest inclusive
// predecessor and itself may still be in theirs. They hold this call's epoch
// in a register and read status words tagged with it, so advancing the epoch
// under them is harmless. Clearing the status words is not: the call that
// wraps the epoch to 0 (it starts at the largest epoch, which every tile
// reads before it publishes anything, hence before the last tile can finish)
// lets each other tile count itself done once its inclusive prefix is out, and
// the last tile finishes the call and clears the words only when all have.
// Everything else pays nothing for it.
template <class Dir, int U, int MODE, bool SWAP_IN, bool SWAP_OUT>
__device__ __forceinline__ void convert_body(Doc d, unsigned long long n_tiles, WsHeader *hdr,
                                             unsigned long long *status, unsigned long long status_cap, hu_result *out)
{
    __shared__ ConvertShared<Dir, U> s;
    const unsigned long long tile = blockIdx.x;
    const CallInfo call{d.base + d.off_b, d.n, d.cap, Dir::kOpConvert};
    if (n_tiles == 0) {
        if (threadIdx.x == 0)
            finish_call(call, hdr, 0ull, out, &s.red[0]);
        __syncthreads();
        wrap_clear(status, status_cap, &s.red[0]);
        return;
    }
    if (Dir::kNeedsTable)
        build_pair_table(s.table);
    const unsigned int epoch = __hip_atomic_load(&hdr->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool wraps = epoch == kEpochMask;
    const Chain cx{status, 0ull, tile, epoch, &hdr->err_key, &hdr->hang, kStatusStride};
    unsigned long long *s_wrap = &s.red[0];
    unsigned long long wrap_total = 0;   // thread 0 of the last tile, in the wrapping call
    chained_tile<Dir, U, MODE, SWAP_IN, SWAP_OUT>(s, s.table, d, tile, n_tiles, cx, [&](unsigned long long total) {
        if (wraps)
            wrap_total = total;
        else
            finish_call(call, hdr, total, out, s_wrap);
    });
    if (!wraps)
        return;
    if (tile != n_tiles - 1) {
        // release: this tile's status words and error report precede the count
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&hdr->done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        return;
    }
    // every other tile is resident or finished (each published before the
    // last tile's look-back could end), so this bounded wait only covers the
    // rest of their look-backs
    if (threadIdx.x == 0) {
        unsigned int spins = 0;
        while (__hip_atomic_load(&hdr->done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) <
               (unsigned int)(n_tiles - 1)) {
            if (++spins > kSpinLimit) {
                // the result reports a device error
                __hip_atomic_fetch_or(&hdr->hang, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(4);
        }
        finish_call(call, hdr, wrap_total, out, s_wrap);
    }
    wrap_clear(status, status_cap, s_wrap);
}

// MODE: kConvert, or kTrusted for input known to be valid. BE: the UTF-16
// side is big endian.
template <int U, int MODE, bool BE = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_convert_u8(
    Doc d, unsigned long long n_tiles, WsHeader *hdr, unsigned long long *status, unsigned long long status_cap,
    hu_result *out)
{
    convert_body<U8Dir, U, MODE, false, BE>(d, n_tiles, hdr, status, status_cap, out);
}

template <int U, int MODE, bool BE = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_convert_u16(Doc d, unsigned long long n_tiles, WsHeader *hdr,
                                                        unsigned long long *status, unsigned long long status_cap,
                                                        hu_result *out)
{
    convert_body<U16Dir, U, MODE, BE, false>(d, n_tiles, hdr, status, status_cap, out);
}

}  // namespace hu
