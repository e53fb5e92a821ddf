// device_common.hpp - pieces shared by the UTF-8 and UTF-16 kernels (gfx950).
//
// Tiling: an input is cut into fixed-size tiles that are processed
// independently; each tile counts the output code units it will produce and
// learns where its output starts through a single-pass decoupled look-back over
// the preceding tiles' published counts. This is the interleaved decoding
// from precomputed character offsets that section 7 of Lemire & Mula leaves
// as future work, with every tile as one piece.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hiputf.h"

namespace hu {

constexpr int kBlock = 256;       // threads per workgroup: four wave64
constexpr int kWaves = kBlock / 64;
constexpr int kChunk = 16;        // bytes per thread per sub-tile (one dwordx4)
constexpr int kSub = kBlock * kChunk;    // sub-tile bytes (one coalesced load per thread)
constexpr int kNoFlag = 0x1FFFFFFF;   // no flagged position (all ones >> 3)
constexpr unsigned int kClassUnknown = 7;   // wave class not known: emit finds its own path

// kTrusted: convert input known to be valid (no validation; see the header)
enum Mode { kValidate = 0, kLength = 1, kConvert = 2, kTrusted = 3 };

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
// Each round reads the 32 newest predecessors not yet accounted for, one per
// lane (lane l: tile hi - l), in one memory round trip. Status reads bypass
// the per-XCD caches, and every spinning round re-reads its window: measured
// on the large-buffer convert, rounds of 32 reads beat 64, 128 and 256 (less
// traffic on the hot status lines) and 8 (more rounds to reach an inclusive
// prefix).
constexpr int kLookLanes = 32;

// Status words of the single-buffer calls sit 128 bytes apart (each on its own
// cache line): tiles publishing from different XCDs then never write the same
// line, and the look-back's reads of one round go to distinct lines.
constexpr unsigned int kStatusStride = 16;

// Inlined into every caller: as a call, the UTF-16 conversion kernel kept
// 32 bytes per lane of its tile state in scratch memory around it.
__device__ __forceinline__ unsigned long long lookback(unsigned long long *status, unsigned int stride, long long first,
                                       long long tile, unsigned int epoch, unsigned int *hang_flag)
{
    const int lane = threadIdx.x & 63;
    unsigned long long sum = 0;
    long long hi = tile - 1;             // newest predecessor not yet accounted
    unsigned int spins = 0;
    while (hi >= first) {
        const long long t = hi - lane;
        unsigned int flag = kFlagAggregate;   // lanes past the window: neutral
        unsigned long long val = 0;
        if (lane < kLookLanes) {
            flag = kFlagInclusive;            // before the chain's start: a stop of value 0
            if (t >= first) {
                const unsigned long long w = peek(&status[(unsigned long long)t * stride]);
                flag = ((w >> kEpochShift) == epoch) ? (unsigned int)((w >> kFlagShift) & 3u) : 0u;
                val = w & kValueMask;
            }
        }
        const unsigned long long stops = __ballot(flag == kFlagInclusive);
        const int first_lane = stops ? __ffsll((long long)stops) - 1 : 64;
        if (__ballot(lane <= first_lane && flag == 0)) {
            if (++spins > kSpinLimit) {
                if (lane == 0) {
                    // completes before the caller publishes anything
                    const unsigned int old = atomicOr(hang_flag, 1u);
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                    if (old == 0x5A5A5A5Au)
                        __builtin_amdgcn_s_sleep(1);
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);
                }
                return 0;
            }
            // another wait already gave up: the call ends in a device error,
            // so stop waiting too instead of spinning to the limit
            if ((spins & 4095u) == 0 &&
                __hip_atomic_load(hang_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
                return 0;
            if (spins > 8)
                __builtin_amdgcn_s_sleep(4);
            continue;
        }
        unsigned long long v = lane <= first_lane ? val : 0ull;
        for (int off = 16; off > 0; off >>= 1)      // lanes 32..63 hold 0
            v += __shfl_xor(v, off, 64);
        sum += v;                                   // lane 0 holds the window's sum
        if (first_lane < 64)
            break;
        hi -= kLookLanes;
        spins = 0;
    }
    return sum;
}

// The same value, but opaque to the compiler: expressions of it are computed
// anew instead of being reused from earlier (and kept in registers till then).
__device__ __forceinline__ unsigned int opaque(unsigned int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// The same for a value common to the wave, held in a scalar register.
__device__ __forceinline__ unsigned int opaque_uniform(unsigned int v)
{
    asm volatile("" : "+s"(v));
    return v;
}

// Both bytes of every 16-bit word swapped (UTF-16 big endian <-> little endian).
__device__ __forceinline__ unsigned int swap16(unsigned int v)
{
    return __builtin_amdgcn_perm(v, v, 0x02030001u);
}
__device__ __forceinline__ uint4 swap16(uint4 v)
{
    return make_uint4(swap16(v.x), swap16(v.y), swap16(v.z), swap16(v.w));
}

// Two 16-bit lanes of a register, for packed 16-bit integer arithmetic.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));

// Byte b of the result: the number of set bytes among bytes 0..b of q, whose
// bytes are each 0 or a small count (no byte of the result may exceed 255).
// Two shift-adds; written out so that they do not become a (slower) full
// 32-bit multiply by 0x01010101.
__device__ __forceinline__ unsigned int byte_prefix_sum(unsigned int q)
{
    unsigned int s, r;
    asm("v_lshl_add_u32 %0, %1, 8, %1" : "=v"(s) : "v"(q));
    asm("v_lshl_add_u32 %0, %1, 16, %1" : "=v"(r) : "v"(s));
    return r;
}

// Index of the lowest set bit of v, all ones when v is 0 (the instruction's
// own result for 0, which the compiler would otherwise test for separately).
__device__ __forceinline__ unsigned int lowest_bit_or_ones(unsigned int v)
{
    unsigned int r;
    asm("v_ffbl_b32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

// ---------------------------------------------------------------- lanes
// Lane l receives lane l - 1's value (DPP wave shift; lane 0 receives 0).
__device__ __forceinline__ unsigned int from_lower_lane(unsigned int v)
{
    return (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xF, 0xF, true);
}

// Lane l receives lane l + 1's value (lane 63 receives 0).
__device__ __forceinline__ unsigned int from_upper_lane(unsigned int v)
{
    return (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xF, 0xF, true);
}

// ---------------------------------------------------------------- scans
// Inclusive prefix sum over the wave's 64 lanes with DPP moves: shifts by 1,
// 2, 4 and 8 lanes inside each row of 16 (lanes shifted in from outside the
// row read 0), then the last lane of row 0 and of row 2 added to rows 1 and 3
// (row_bcast:15), and lane 31 added to rows 2 and 3 (row_bcast:31). Rows the
// row mask leaves out keep the 0 they start from.
__device__ __forceinline__ unsigned int wave_inclusive_sum(unsigned int v)
{
    v += (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);   // row_shr:1
    v += (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);   // row_shr:2
    v += (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);   // row_shr:4
    v += (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);   // row_shr:8
    v += (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    v += (unsigned int)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return v;
}

// Minimum over the wave. Flags are rare: a wave whose lanes all hold ~0 (no
// flag) settles it with one vote.
__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v)
{
    if (__any(v != ~0ull)) {
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long u = __shfl_xor(v, off, 64);
            v = u < v ? u : v;
        }
    }
    return v;
}

__device__ __forceinline__ unsigned long long block_min_u64(unsigned long long v, unsigned long long *s_tmp)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    v = wave_min_u64(v);
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

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v, unsigned long long *s_tmp)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    if (lane == 0)
        s_tmp[wave] = v;
    __syncthreads();
    unsigned long long m = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w)
        m += s_tmp[w];
    __syncthreads();
    return m;
}

// ---------------------------------------------------------------- loads
// Inputs are read in 16-byte aligned granules relative to a 16-byte aligned
// base; a document's bytes are [off, end) relative to that base. A granule
// that holds at least one byte of the document lies inside the pages that hold
// it, so the aligned access never touches an unmapped page. Granules with no
// byte of the document are not read: their load is redirected to the
// document's first granule and the result is masked to zero afterwards.
// Loads carry no branch, so a thread can keep many of them in flight; masking
// happens when the data is used.
__device__ __forceinline__ uint4 load_granule_raw(const uint8_t *base, unsigned long long v, unsigned long long off,
                                                  unsigned long long end)
{
    const bool any = v < end && v + 16 > off;
    const unsigned long long a = any ? v : (off & ~15ull);
    return *reinterpret_cast<const uint4 *>(base + a);
}

// Zero the bytes of granule q (at position v) that are outside [off, end).
__device__ __forceinline__ uint4 mask_granule(uint4 q, unsigned long long v, unsigned long long off,
                                              unsigned long long end)
{
    const long long lo_s = (long long)off - (long long)v;
    const long long hi_s = (long long)end - (long long)v;
    const int lo = lo_s < 0 ? 0 : (lo_s > 16 ? 16 : (int)lo_s);
    const int hi = hi_s < 0 ? 0 : (hi_s > 16 ? 16 : (int)hi_s);
    unsigned int w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int lk = lo - 4 * k < 0 ? 0 : (lo - 4 * k > 4 ? 4 : lo - 4 * k);
        const int hk = hi - 4 * k < 0 ? 0 : (hi - 4 * k > 4 ? 4 : hi - 4 * k);
        const unsigned long long m = ((1ull << (8 * hk)) - 1) & ~((1ull << (8 * lk)) - 1);
        w[k] &= (unsigned int)m;
    }
    return make_uint4(w[0], w[1], w[2], w[3]);
}

__device__ __forceinline__ uint4 load_granule(const uint8_t *base, unsigned long long v, unsigned long long off,
                                              unsigned long long end)
{
    return mask_granule(load_granule_raw(base, v, off, end), v, off, end);
}

}  // namespace hu
