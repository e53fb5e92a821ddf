// device_common.hpp - pieces shared by the UTF-8 and UTF-16 kernels (gfx950).
//
// Tiling: an input is cut into fixed-size tiles that are processed
// independently; each tile counts the output code units it will produce and
// learns where its output starts through a single-pass decoupled look-back over
// the preceding tiles' published counts. This realises the "interleaved
// decoding ... by pre-computing the character offsets" that section 7 of
// Lemire & Mula leaves as future work, with every tile as one piece.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hu {

constexpr int kBlock = 256;       // threads per workgroup: four wave64
constexpr int kWaves = kBlock / 64;
constexpr int kChunk = 16;        // bytes each thread loads per tile (one dwordx4)
constexpr int kTile = kBlock * kChunk;   // tile bytes

// ---------------------------------------------------------------- workspace
// A workspace is a WsHeader followed by one 64-bit status word per tile.
// All-zero is the initial state; the last workgroup of every call restores it
// (apart from the epoch, which advances) so that the next call needs no clearing.
struct alignas(64) WsHeader {
    unsigned long long tile_counter;   // next tile id handed out to workgroups
    unsigned long long err_key;        // ~(first flagged position); 0 = no flag
    unsigned long long total;          // sum of the tiles' output counts
    unsigned int epoch;                // tag of this call's status words
    unsigned int hang;                 // set if a bounded wait gave up
    unsigned int done;                 // workgroups of this launch that have finished
    unsigned int pad0;
    unsigned long long pad[3];
};
static_assert(sizeof(WsHeader) == 64, "header size");
constexpr size_t kHeaderBytes = 256;   // header slot (status array stays 256-byte aligned)

// Status word: [63:42] epoch tag, [41:40] flag, [39:0] value.
constexpr int kFlagShift = 40;
constexpr int kEpochShift = 42;
constexpr unsigned long long kValueMask = (1ull << kFlagShift) - 1;
constexpr unsigned int kEpochMask = (1u << 22) - 1;
constexpr unsigned int kFlagAggregate = 1;   // value = this tile's count
constexpr unsigned int kFlagInclusive = 2;   // value = count of this tile and all before it

__device__ __forceinline__ unsigned long long pack_status(unsigned int epoch, unsigned int flag,
                                                          unsigned long long v)
{
    return ((unsigned long long)epoch << kEpochShift) | ((unsigned long long)flag << kFlagShift) | v;
}

__device__ __forceinline__ void publish(unsigned long long *slot, unsigned long long word)
{
    __hip_atomic_store(slot, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long peek(const unsigned long long *slot)
{
    return __hip_atomic_load(const_cast<unsigned long long *>(slot), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

// Upper bound on polling rounds of one look-back step before it gives up and
// raises WsHeader::hang (a broken predecessor then surfaces as a device error
// instead of a hung GPU). Far above any legitimate wait.
constexpr unsigned int kSpinLimit = 1u << 22;

// Decoupled look-back, executed by one whole wave64 (all 64 lanes active).
// Returns the sum of the values of tiles [first, tile) of the chain, where
// `first` is the chain's first tile (its predecessors belong to nobody).
// Lane i inspects tile (t - 1 - i) of the current window of 64 predecessors.
__device__ unsigned long long lookback(unsigned long long *status, long long first, long long tile,
                                       unsigned int epoch, unsigned int *hang_flag)
{
    const int lane = threadIdx.x & 63;
    unsigned long long sum = 0;
    long long hi = tile - 1;             // newest predecessor not yet accounted
    unsigned int spins = 0;
    while (hi >= first) {
        long long t = hi - lane;
        unsigned long long word = 0;
        unsigned int flag = kFlagInclusive;  // lanes past the chain's start act as a stop of value 0
        if (t >= first) {
            word = peek(&status[t]);
            flag = ((word >> kEpochShift) == epoch) ? (unsigned int)((word >> kFlagShift) & 3u) : 0u;
        }
        unsigned long long pending = __ballot(flag == 0);
        unsigned long long stops = __ballot(flag == kFlagInclusive);
        // lowest lane index = newest tile; everything up to the first stop is needed
        int first_stop = stops ? __ffsll((long long)stops) - 1 : 64;
        unsigned long long needed = first_stop >= 63 ? ~0ull : ((2ull << first_stop) - 1);
        if (pending & needed) {
            if (++spins > kSpinLimit) {
                if (lane == 0)
                    atomicOr(hang_flag, 1u);
                return 0;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        unsigned long long v = (lane <= first_stop && t >= first) ? (word & kValueMask) : 0;
        // wave reduction of the values up to and including the first stop
        for (int off = 32; off > 0; off >>= 1)
            v += __shfl_xor(v, off, 64);
        sum += v;
        if (first_stop < 64)
            break;
        hi -= 64;
        spins = 0;
    }
    return sum;
}

// ---------------------------------------------------------------- scans
__device__ __forceinline__ unsigned int wave_inclusive_sum(unsigned int v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        unsigned int u = __shfl_up(v, d, 64);
        if (lane >= d)
            v += u;
    }
    return v;
}

// Exclusive prefix of `v` over the workgroup and the workgroup total.
// Uses s_tmp[kWaves]; contains barriers (all threads must call it).
__device__ __forceinline__ unsigned int block_exclusive_sum(unsigned int v, unsigned int *s_tmp,
                                                            unsigned int *total)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    unsigned int inc = wave_inclusive_sum(v);
    if (lane == 63)
        s_tmp[wave] = inc;
    __syncthreads();
    unsigned int before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        unsigned int x = s_tmp[w];
        before += (w < wave) ? x : 0u;
        all += x;
    }
    *total = all;
    __syncthreads();
    return before + inc - v;
}

__device__ __forceinline__ unsigned long long block_min_u64(unsigned long long v, unsigned long long *s_tmp)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long u = __shfl_xor(v, off, 64);
        v = u < v ? u : v;
    }
    if (lane == 0)
        s_tmp[wave] = v;
    __syncthreads();
    unsigned long long m = s_tmp[0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w)
        m = s_tmp[w] < m ? s_tmp[w] : m;
    __syncthreads();
    return m;
}

// ---------------------------------------------------------------- loads
// 16-byte aligned load of the granule at virtual byte position `v` of a
// document whose bytes are [off, off + n) relative to the 16-byte aligned base.
// Bytes outside [off, off + n) read as zero. A granule that holds at least one
// byte of the document lies inside the pages that hold it, so the aligned
// access never touches an unmapped page.
__device__ __forceinline__ uint4 load_granule(const uint8_t *base, unsigned long long v,
                                              unsigned long long off, unsigned long long end)
{
    uint4 q = make_uint4(0, 0, 0, 0);
    if (v < end && v + 16 > off) {
        q = *reinterpret_cast<const uint4 *>(base + v);
        if (v < off || v + 16 > end) {
            unsigned int lo = v < off ? (unsigned int)(off - v) : 0u;
            unsigned int hi = v + 16 > end ? (unsigned int)(end - v) : 16u;
            unsigned int w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                unsigned int keep = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    unsigned int pos = 4 * k + b;
                    keep |= (pos >= lo && pos < hi) ? (0xFFu << (8 * b)) : 0u;
                }
                w[k] &= keep;
            }
            q = make_uint4(w[0], w[1], w[2], w[3]);
        }
    }
    return q;
}

}  // namespace hu
