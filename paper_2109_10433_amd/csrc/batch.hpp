// batch.hpp - many documents, any of the six operations each, in one call.
//
// Three steps, all on the device (nothing is read back, so a call can be
// recorded into a HIP graph and replayed with new document tables):
//   plan: every document gets its work: none (empty, or invalid arguments:
//         its result is written here), one small-document item (all its
//         bytes fit one wave's tile of four 1 KiB pieces), or tiles (work
//         items of U sub-tiles of 4 KiB). Items are numbered UTF-8 tiles
//         first, then UTF-16 tiles, then small documents, each in document
//         order. The plan also advances the workspace epoch.
//   fill: one record per item: the document, its index, the tile.
//   run:  one fused kernel for both input encodings: one workgroup per tile
//         item, in item order, then one wave per small document. A tile
//         waits (look-back) only for earlier tiles of its own document; a
//         small document is done by its wave alone (validate, count, wave
//         scan, decode, store: no look-back, no barrier). Each document has
//         its own look-back chain and error key; the workgroup that runs a
//         document's last tile writes its result.
#pragma once

#include <type_traits>

#include "engine.hpp"

namespace hu {

struct BatchDoc {                     // mirrors hu_doc
    unsigned long long src_off, n_units, dst_off, dst_cap;
    unsigned int op, reserved;
};
static_assert(sizeof(BatchDoc) == sizeof(hu_doc), "hu_doc layout");

// Workspace of a batch call:
//   [BatchHeader (256 B) | status, item_cap words | first_item | err | items
//    (48 B each) | three words per block of documents (planning)]
// The status array starts at a fixed offset; everything after it moves with
// the call's shape (document count, item capacity). Status words must never
// hold anything but status words or zeros, so memory that earlier calls used
// for the per-document arrays is cleared before it becomes status words.
struct BatchHeader {
    unsigned long long items8;        // UTF-8 tile items of this call
    unsigned long long items16;       // UTF-16 tile items
    unsigned long long smalls;        // small-document items
    unsigned long long dirty_from;    // 1 + first status word that may hold other data (0: none)
    unsigned long long clear_lo;      // status words [clear_lo, clear_hi) to clear in this call
    unsigned long long clear_hi;
    unsigned int epoch;               // tag of this call's status words
    unsigned int hang;                // set if a bounded wait gave up
    unsigned long long overflow;      // 1 if the call's items exceed the item capacity
};
static_assert(sizeof(BatchHeader) <= kHeaderBytes, "batch header size");

// Work item record, written by the fill kernel: the document's table entry
// beside its index and the tile's, so that a run workgroup reads one record
// (scalar loads) instead of an index and then the document table.
struct BatchItem {
    BatchDoc doc;
    unsigned int di;                  // document index
    unsigned int tile;                // tile of the document (0 for a small document)
};
static_assert(sizeof(BatchItem) == 48, "item record");

struct BatchWs {
    BatchHeader *hdr;
    unsigned int *first_item;         // per document
    unsigned long long *err;          // per document error key
    BatchItem *items;                 // per item
    unsigned long long *status;       // per tile item look-back status
    unsigned long long *block;        // per block of documents: UTF-8, UTF-16, small items (then their offsets)
    unsigned long long item_cap;
};

constexpr unsigned int kNoItem = 0xFFFFFFFFu;

// Small documents: all bytes (with the offset in the first 16-byte granule)
// within one wave-tile of kSmallPieces pieces.
constexpr int kSmallPieces = 4;
constexpr unsigned long long kSmallDocBytes = (unsigned long long)kSmallPieces * kPiece;

__device__ __forceinline__ bool op_is_u16(unsigned int op) { return op >= HU_OP_VALIDATE_UTF16LE; }
__device__ __forceinline__ int op_mode(unsigned int op) { return (int)(op % 3u); }   // kValidate/kLength/kConvert

__device__ __forceinline__ Doc make_doc(const BatchDoc &b, const uint8_t *src_base, uint8_t *dst_base)
{
    const uint8_t *src = src_base + b.src_off;
    const unsigned long long bytes = op_is_u16(b.op) ? 2 * b.n_units : b.n_units;
    Doc d;
    d.base = (const uint8_t *)((uintptr_t)src & ~(uintptr_t)15);
    d.off_b = (unsigned long long)((uintptr_t)src & 15u);
    d.end_b = d.off_b + bytes;
    d.n = b.n_units;
    d.dst = dst_base ? (void *)(dst_base + b.dst_off) : nullptr;
    d.cap = b.dst_cap;
    return d;
}

// 0 when the document is fine, else the error its result carries.
__device__ __forceinline__ int doc_check(const BatchDoc &b, const uint8_t *src_base, const uint8_t *dst_base)
{
    if (b.op > HU_OP_CONVERT_UTF16LE_TO_UTF8 || b.n_units > (1ull << 38))
        return HU_ERR_INVALID_ARGUMENT;
    if (b.n_units == 0)
        return 0;
    const uintptr_t src = (uintptr_t)(src_base + b.src_off);
    if (src_base == nullptr || (op_is_u16(b.op) && (src & 1u)))
        return HU_ERR_INVALID_ARGUMENT;
    if (op_mode(b.op) == kConvert && b.dst_cap > 0) {
        if (dst_base == nullptr)
            return HU_ERR_INVALID_ARGUMENT;
        if (b.op == HU_OP_CONVERT_UTF8_TO_UTF16LE && ((uintptr_t)(dst_base + b.dst_off) & 1u))
            return HU_ERR_INVALID_ARGUMENT;
    }
    return 0;
}

// Input bytes of a document counted from its 16-byte aligned base.
__device__ __forceinline__ unsigned long long doc_span(const BatchDoc &b, const uint8_t *src_base)
{
    const unsigned long long off = (unsigned long long)((uintptr_t)(src_base + b.src_off) & 15u);
    return off + (op_is_u16(b.op) ? 2 * b.n_units : b.n_units);
}

__device__ __forceinline__ bool doc_is_small(const BatchDoc &b, const uint8_t *src_base)
{
    return b.n_units > 0 && doc_span(b, src_base) <= kSmallDocBytes;
}

// Tile items of a document (0 for an empty or small one).
__device__ __forceinline__ unsigned long long doc_tiles(const BatchDoc &b, const uint8_t *src_base,
                                                        unsigned long long tile_bytes)
{
    if (b.n_units == 0 || doc_is_small(b, src_base))
        return 0;
    return (doc_span(b, src_base) + tile_bytes - 1) / tile_bytes;
}

constexpr int kPlanBlock = 1024;
constexpr int kCounts = 3;   // UTF-8 tiles, UTF-16 tiles, small documents

// Exclusive prefix over a 1024-thread workgroup of three counters at once;
// t[] receives the workgroup's totals.
__device__ __forceinline__ void plan_scan(const unsigned long long v[kCounts], unsigned long long e[kCounts],
                                          unsigned long long t[kCounts],
                                          unsigned long long (*s_tmp)[kPlanBlock / 64])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long inc[kCounts];
#pragma unroll
    for (int c = 0; c < kCounts; ++c)
        inc[c] = v[c];
    for (int d = 1; d < 64; d <<= 1) {
#pragma unroll
        for (int c = 0; c < kCounts; ++c) {
            const unsigned long long u = __shfl_up(inc[c], d, 64);
            if (lane >= d)
                inc[c] += u;
        }
    }
    if (lane == 63) {
#pragma unroll
        for (int c = 0; c < kCounts; ++c)
            s_tmp[c][wave] = inc[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kCounts; ++c) {
        unsigned long long before = 0, all = 0;
        for (int w = 0; w < kPlanBlock / 64; ++w) {
            const unsigned long long x = s_tmp[c][w];
            before += w < wave ? x : 0ull;
            all += x;
        }
        e[c] = before + inc[c] - v[c];
        t[c] = all;
    }
    __syncthreads();
}

// Planning runs in three steps, so that no single workgroup walks all the
// documents: blocks of kPlanBlock documents (one per thread, coalesced) sum
// their work items; one workgroup turns the block sums into block offsets
// and does the call's bookkeeping; the blocks then give every document its
// first item.

// Work of document d: its three counts (at most one non-zero) and, when it
// fails the argument checks, the error of its result.
__device__ __forceinline__ void doc_work(const BatchDoc &b, const uint8_t *src_base, const uint8_t *dst_base,
                                         unsigned long long tile_bytes, int *err, unsigned long long v[kCounts])
{
    v[0] = v[1] = v[2] = 0;
    *err = doc_check(b, src_base, dst_base);
    if (*err != 0 || b.n_units == 0)
        return;
    if (doc_is_small(b, src_base))
        v[2] = 1;
    else
        v[op_is_u16(b.op) ? 1 : 0] = doc_tiles(b, src_base, tile_bytes);
}

__global__ __launch_bounds__(kPlanBlock) void k_batch_count(const BatchDoc *docs, unsigned int n_docs,
                                                            const uint8_t *src_base, const uint8_t *dst_base, BatchWs w,
                                                            unsigned long long tile_bytes)
{
    __shared__ unsigned long long s_tmp[kCounts][kPlanBlock / 64];
    const unsigned long long d = (unsigned long long)blockIdx.x * kPlanBlock + threadIdx.x;
    unsigned long long v[kCounts] = {0, 0, 0};
    if (d < n_docs) {
        int err;
        doc_work(docs[d], src_base, dst_base, tile_bytes, &err, v);
    }
    unsigned long long e[kCounts], t[kCounts];
    plan_scan(v, e, t, s_tmp);
    if (threadIdx.x < kCounts)
        w.block[kCounts * blockIdx.x + threadIdx.x] = t[threadIdx.x];
}

// The call's totals, the capacity check and the epoch in
// the header; status words cleared when the epoch wraps. All threads of the
// workgroup call it.
__device__ __forceinline__ void plan_bookkeeping(const BatchWs &w, const unsigned long long t[kCounts], int *s_wrap)
{
    const bool overflow = t[0] + t[1] + t[2] > w.item_cap;
    if (threadIdx.x == 0) {
        w.hdr->items8 = overflow ? 0 : t[0];
        w.hdr->items16 = overflow ? 0 : t[1];
        w.hdr->smalls = overflow ? 0 : t[2];
        w.hdr->overflow = overflow ? 1u : 0u;
        w.hdr->hang = 0;
        // status words of earlier calls' per-document arrays: cleared by fill
        const unsigned long long dirty = w.hdr->dirty_from;
        w.hdr->clear_lo = dirty ? dirty - 1 : w.item_cap;
        w.hdr->clear_hi = w.item_cap;
        w.hdr->dirty_from = w.item_cap + 1;
        const unsigned int e = (w.hdr->epoch + 1u) & kEpochMask;
        w.hdr->epoch = e;
        *s_wrap = e == 0;
    }
    __syncthreads();
    if (*s_wrap) {
        for (unsigned long long i = threadIdx.x; i < w.item_cap; i += kPlanBlock)
            w.status[i] = 0;
    }
}

__global__ __launch_bounds__(kPlanBlock) void k_batch_plan(unsigned int n_blocks, BatchWs w)
{
    __shared__ unsigned long long s_tmp[kCounts][kPlanBlock / 64];
    __shared__ int s_wrap;
    unsigned long long run[kCounts] = {0, 0, 0};   // items of the blocks so far
    for (unsigned int g0 = 0; g0 < n_blocks; g0 += kPlanBlock) {
        const unsigned int g = g0 + threadIdx.x;
        unsigned long long v[kCounts], e[kCounts], t[kCounts];
#pragma unroll
        for (int c = 0; c < kCounts; ++c)
            v[c] = g < n_blocks ? w.block[kCounts * g + c] : 0ull;
        plan_scan(v, e, t, s_tmp);
        if (g < n_blocks) {
#pragma unroll
            for (int c = 0; c < kCounts; ++c)
                w.block[kCounts * g + c] = run[c] + e[c];   // block offsets, in place of the sums
        }
#pragma unroll
        for (int c = 0; c < kCounts; ++c)
            run[c] += t[c];
    }
    plan_bookkeeping(w, run, &s_wrap);
}

// Document d's first work item, or its result if it has no work (error,
// empty, or the call's items exceed the workspace's capacity).
__device__ __forceinline__ void assign_doc(const BatchWs &w, hu_result *results, unsigned long long d, int err,
                                           const unsigned long long v[kCounts], bool overflow,
                                           unsigned long long first)
{
    if (err == 0 && overflow)
        err = HU_ERR_INVALID_ARGUMENT;   // work-item capacity of the workspace exceeded
    if (err != 0 || v[0] + v[1] + v[2] == 0) {
        hu_result r;
        r.error = err;
        r.reserved = 0;
        r.count = 0;
        results[d] = r;
        w.first_item[d] = kNoItem;
        return;
    }
    w.first_item[d] = (unsigned int)first;
}

// First item of a document from its category's offset before its block (o8,
// o16, os), its exclusive offset inside the block and the call's totals.
__device__ __forceinline__ unsigned long long first_item_of(const unsigned long long v[kCounts],
                                                            const unsigned long long block_off[kCounts],
                                                            const unsigned long long e[kCounts],
                                                            unsigned long long items8, unsigned long long items16)
{
    if (v[2] != 0)
        return items8 + items16 + block_off[2] + e[2];
    if (v[1] != 0)
        return items8 + block_off[1] + e[1];
    return block_off[0] + e[0];
}

__global__ __launch_bounds__(kPlanBlock) void k_batch_assign(const BatchDoc *docs, unsigned int n_docs,
                                                             const uint8_t *src_base, const uint8_t *dst_base,
                                                             hu_result *results, BatchWs w,
                                                             unsigned long long tile_bytes)
{
    __shared__ unsigned long long s_tmp[kCounts][kPlanBlock / 64];
    const unsigned long long d = (unsigned long long)blockIdx.x * kPlanBlock + threadIdx.x;
    unsigned long long v[kCounts] = {0, 0, 0};
    int err = 0;
    if (d < n_docs)
        doc_work(docs[d], src_base, dst_base, tile_bytes, &err, v);
    unsigned long long e[kCounts], t[kCounts];
    plan_scan(v, e, t, s_tmp);   // every thread takes part
    if (d < n_docs) {
        unsigned long long bo[kCounts];
#pragma unroll
        for (int c = 0; c < kCounts; ++c)
            bo[c] = w.block[kCounts * blockIdx.x + c];
        assign_doc(w, results, d, err, v, w.hdr->overflow != 0, first_item_of(v, bo, e, w.hdr->items8, w.hdr->items16));
    }
}

// Planning of a call of at most kPlanBlock documents, all three steps in one
// workgroup (one launch: small batches, as in serving, wait on it).
__global__ __launch_bounds__(kPlanBlock) void k_batch_plan1(const BatchDoc *docs, unsigned int n_docs,
                                                            const uint8_t *src_base, const uint8_t *dst_base,
                                                            hu_result *results, BatchWs w,
                                                            unsigned long long tile_bytes)
{
    __shared__ unsigned long long s_tmp[kCounts][kPlanBlock / 64];
    __shared__ int s_wrap;
    const unsigned int d = threadIdx.x;
    unsigned long long v[kCounts] = {0, 0, 0};
    int err = 0;
    if (d < n_docs)
        doc_work(docs[d], src_base, dst_base, tile_bytes, &err, v);
    unsigned long long e[kCounts], t[kCounts];
    plan_scan(v, e, t, s_tmp);
    if (d < n_docs) {
        const unsigned long long zero[kCounts] = {0, 0, 0};
        assign_doc(w, results, d, err, v, t[0] + t[1] + t[2] > w.item_cap, first_item_of(v, zero, e, t[0], t[1]));
    }
    plan_bookkeeping(w, t, &s_wrap);
}

// The item records; every error key back to zero; status words the plan
// marked for clearing.
__global__ void k_batch_fill(const BatchDoc *docs, unsigned int n_docs, const uint8_t *src_base, BatchWs w,
                             unsigned long long tile_bytes)
{
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    const unsigned long long me = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (unsigned long long i = w.hdr->clear_lo + me; i < w.hdr->clear_hi; i += stride)
        w.status[i] = 0;
    for (unsigned int d = blockIdx.x * blockDim.x + threadIdx.x; d < n_docs; d += gridDim.x * blockDim.x) {
        w.err[d] = 0;
        const unsigned int first = w.first_item[d];
        if (first == kNoItem)
            continue;
        const BatchDoc b = docs[d];
        const unsigned long long t = doc_tiles(b, src_base, tile_bytes);
        const unsigned long long items = t ? t : 1;   // a small document: one item
        for (unsigned long long k = 0; k < items; ++k)
            w.items[first + k] = BatchItem{b, d, (unsigned int)k};
    }
}

// ------------------------------------------------------------ tile items
// Everything chained_tile needs in LDS but the pair table (kept apart, shared
// by every item and small document a workgroup does).
template <class Dir, int U>
struct BatchTileShared {
    alignas(16) typename Dir::Out out[kStageFront + Dir::kStageUnits];
    TileEdges<U> edges;
    unsigned int scan[U][kWaves];
    unsigned long long red[kWaves];
    unsigned long long prefix;
};

// One tile item (tile `tile` of document di, global item index i).
template <class Dir, int U>
__device__ __forceinline__ void batch_item(BatchTileShared<Dir, U> &s, const unsigned char *table, const BatchDoc &b,
                                           unsigned int di, unsigned long long tile, unsigned long long i,
                                           unsigned int epoch, const uint8_t *src_base, uint8_t *dst_base,
                                           hu_result *results, BatchWs w)
{
    const Doc d = make_doc(b, src_base, dst_base);
    const unsigned long long n_tiles = doc_tiles(b, src_base, (unsigned long long)U * kSub);
    const Chain cx{w.status, i - tile, i, epoch, &w.err[di], &w.hdr->hang, 1u};
    const CallInfo call{d.base + d.off_b, d.n, d.cap, (int)b.op};
    auto fin = [&](unsigned long long total) {
        const unsigned long long key = __hip_atomic_load(&w.err[di], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned int hang = __hip_atomic_load(&w.hdr->hang, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        results[di] = result_from(call, key, hang, total);
        w.err[di] = 0;
    };
    constexpr bool skip = std::is_same<Dir, U8Dir>::value;   // UTF-8 documents only
    switch (op_mode(b.op)) {
    case kValidate: chained_tile<Dir, U, kValidate, false, false, true, skip>(s, table, d, tile, n_tiles, cx, fin); break;
    case kLength: chained_tile<Dir, U, kLength, false, false, true, skip>(s, table, d, tile, n_tiles, cx, fin); break;
    default: chained_tile<Dir, U, kConvert, false, false, true, skip>(s, table, d, tile, n_tiles, cx, fin); break;
    }
}

// ------------------------------------------------------------ small documents
// A wave's staging for one piece's output (either direction).
union SmallStage {
    alignas(16) unsigned short u8[kStageFront + U8Dir::kPieceStageUnits];
    alignas(16) unsigned char u16[kStageFront + U16Dir::kPieceStageUnits];
};

// This lane's chunk of piece u (below P) of a wave-tile, with the dword
// before and after: DPP rotations across the wave, the neighbouring pieces at
// lanes 0 and 63, zeros beyond the wave-tile.
template <int P>
__device__ __forceinline__ void piece_chunk(const WaveTile<P> &t, unsigned int u, unsigned int lane, unsigned int x[6])
{
    uint4 cur = t.q[0];
    unsigned int prev_w = 0u, next_x = P > 1 ? t.q[P > 1 ? 1 : 0].x : 0u;
#pragma unroll
    for (int k = 1; k < P; ++k) {
        if (u == (unsigned int)k) {
            cur = t.q[k];
            prev_w = t.q[k - 1].w;
            next_x = k + 1 < P ? t.q[k + 1 < P ? k + 1 : k].x : 0u;
        }
    }
    x[1] = cur.x; x[2] = cur.y; x[3] = cur.z; x[4] = cur.w;
    const unsigned int r = rotate_from_lower_lane(x[4]);
    const unsigned int before = rotate_from_lower_lane(prev_w);   // lane 0: lane 63's (zero for piece 0)
    x[0] = lane == 0 ? before : r;
    const unsigned int after = rotate_from_upper_lane(next_x);    // lane 63: lane 0's (zero after the last piece)
    const unsigned int l = rotate_from_upper_lane(x[1]);
    x[5] = lane == 63 ? after : l;
}

// One small document, by one whole wave (no barrier; the wave's own LDS
// staging), piece by piece: validate and count the piece, offsets from a wave
// scan, decode into the staging (shifted so that LDS and global addresses
// agree modulo 16) and copy out. The first piece with a flag ends the work:
// every piece before it was valid, so its smallest flag (or a last character
// cut short by the end) is the document's first. A conversion may have
// written the valid pieces before an error is found (the output of a failed
// call is unspecified; nothing goes past the capacity). Lane 0 writes the
// result.
template <class Dir, int MODE>
__device__ __forceinline__ void small_doc(typename Dir::Out *stage, const unsigned char *table, const Doc &d,
                                          const CallInfo &call, hu_result *result)
{
    using Out = typename Dir::Out;
    constexpr int P = kSmallPieces;
    constexpr bool COUNT = MODE != kValidate;
    constexpr unsigned int G = 16 / sizeof(Out);
    const unsigned int lane = threadIdx.x & 63;
    const unsigned int n_pieces = (unsigned int)((d.end_b + kPiece - 1) / kPiece);
    // the document's pieces only (no dwords around the wave-tile: piece_chunk
    // takes zeros there)
    WaveTile<P> t;
#pragma unroll
    for (int u = 0; u < P; ++u) {
        const unsigned long long v = (unsigned long long)u * kPiece + lane * kChunk;
        t.q[u] = (unsigned int)u < n_pieces ? load_granule_raw(d.base, v, d.off_b, d.end_b) : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < P; ++u)
        t.q[u] = mask_granule(t.q[u], (unsigned long long)u * kPiece + lane * kChunk, d.off_b, d.end_b);
    const unsigned long long n_b = d.end_b - d.off_b;
    const unsigned int dst_mis = (unsigned int)(((uintptr_t)d.dst & 15u) / sizeof(Out));
    Out *dst = reinterpret_cast<Out *>(d.dst);
    // whether the output fits the capacity is known only at the end (the
    // count of every piece): pieces are written as they come, each store
    // guarded by the capacity (the output of a call that ends in
    // OUTPUT_TOO_SMALL is unspecified)
    constexpr bool emit_ok = MODE == kConvert;
    unsigned long long total = 0, flag = ~0ull;
#pragma unroll
    for (unsigned int u = 0; u < P; ++u) {
        if (u >= n_pieces)
            break;
        unsigned int x[6];
        piece_chunk<P>(t, u, lane, x);
        int f;
        unsigned int cls;
        unsigned int c = Dir::template analyze<COUNT>(x, table, &f, &cls);
        cls = __builtin_amdgcn_readfirstlane(cls);
        const unsigned long long cv = (unsigned long long)u * kPiece + lane * kChunk;
        if (f != kNoFlag)
            flag = cv + (unsigned long long)f * Dir::kInUnit - d.off_b;   // zeros before the input are never flagged
        if (COUNT) {
            unsigned int lo, hi;
            chunk_range<Dir>(d, cv, lo, hi);
            c -= (unsigned int)(kChunk / Dir::kInUnit) - (hi - lo);
        }
        if (u + 1 == n_pieces && lane == 0) {
            const long long j = Dir::end_truncation(d.base, d.off_b, d.end_b);
            if (j >= 0 && (unsigned long long)j < flag)
                flag = (unsigned long long)j;
        }
        if (flag != ~0ull && flag >= n_b)
            flag = n_b - Dir::kInUnit;   // zeros after a lead at the end: the last unit
        flag = wave_min_u64(flag);
        if (flag != ~0ull)
            break;
        if (COUNT) {
            const unsigned int inc = wave_inclusive_sum(c);
            const unsigned int tot = __builtin_amdgcn_readlane(inc, 63);
            if (emit_ok && tot != 0) {
                // zeros before the document in lane 0's first chunk land in the
                // front margin (offsets counted from the buffer's start)
                const unsigned int skip = (u == 0 && lane == 0) ? (unsigned int)(d.off_b / Dir::kInUnit) : 0u;
                const unsigned int shift = (unsigned int)((dst_mis + total) % G);
                Dir::emit(x, stage, kStageFront + shift + (inc - c) - skip, cls);
                __builtin_amdgcn_wave_barrier();
                copy_out<Dir, false, 64, Dir::kPieceStageUnits>(stage + kStageFront, shift, tot, dst,
                                                                (long long)total - (long long)shift, d.cap, lane);
                __builtin_amdgcn_wave_barrier();
            }
            total += tot;
        }
    }
    if (lane == 0)
        *result = result_from(call, flag != ~0ull ? ~flag : 0ull, 0u, total);
}

// Small document di, its operation's path.
__device__ __forceinline__ void batch_small(SmallStage &stage, const unsigned char *table, const BatchDoc &b,
                                            unsigned int di, const uint8_t *src_base, uint8_t *dst_base,
                                            hu_result *results)
{
    const Doc d = make_doc(b, src_base, dst_base);
    const CallInfo call{d.base + d.off_b, d.n, d.cap, (int)b.op};
    hu_result *r = &results[di];
    switch (b.op) {
    case HU_OP_VALIDATE_UTF8: small_doc<U8Dir, kValidate>(stage.u8, table, d, call, r); break;
    case HU_OP_UTF16_LENGTH_FROM_UTF8: small_doc<U8Dir, kLength>(stage.u8, table, d, call, r); break;
    case HU_OP_CONVERT_UTF8_TO_UTF16LE: small_doc<U8Dir, kConvert>(stage.u8, table, d, call, r); break;
    case HU_OP_VALIDATE_UTF16LE: small_doc<U16Dir, kValidate>(stage.u16, table, d, call, r); break;
    case HU_OP_UTF8_LENGTH_FROM_UTF16LE: small_doc<U16Dir, kLength>(stage.u16, table, d, call, r); break;
    default: small_doc<U16Dir, kConvert>(stage.u16, table, d, call, r); break;
    }
}

// ------------------------------------------------------------ run
template <int U>
struct BatchShared {
    alignas(16) unsigned char table[4096];
    union {
        BatchTileShared<U8Dir, U> u8;
        BatchTileShared<U16Dir, U> u16;
        SmallStage small[kWaves];   // one per wave
    } w;
};

// One fused launch over workgroups numbered base + blockIdx.x: the first nt
// take the tile items in item order, the next ones four small documents each
// (one per wave), and the rest (the host knows only upper bounds on both
// counts) leave at once, before any work. Workgroups are dispatched in id
// order, an item waits only for smaller items of its own document and a
// small document for nothing, so the lowest unfinished item always has a
// running workgroup whose predecessors are done, however few workgroups the
// device holds at a time; the small documents, dispatched after the tiles,
// fill the tail of the tile work. Dynamic LDS (unused) may be requested at
// launch to cap the workgroups resident per CU.
template <int U>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_batch_run(const uint8_t *src_base, uint8_t *dst_base, hu_result *results, BatchWs w, unsigned long long base)
{
    __shared__ BatchShared<U> s;
    const unsigned long long g = base + blockIdx.x;
    const unsigned long long n8 = w.hdr->items8, nt = n8 + w.hdr->items16, smalls = w.hdr->smalls;
    if (g < nt) {
        build_pair_table(s.table);   // the tile path's first barrier comes before its first lookup
        const BatchItem it = w.items[g];
        const unsigned int epoch = w.hdr->epoch;
        if (g < n8)
            batch_item<U8Dir, U>(s.w.u8, s.table, it.doc, it.di, it.tile, g, epoch, src_base, dst_base, results, w);
        else
            batch_item<U16Dir, U>(s.w.u16, s.table, it.doc, it.di, it.tile, g, epoch, src_base, dst_base, results,
                                  w);
        return;
    }
    const unsigned long long j0 = (g - nt) * kWaves;   // this workgroup's first small document
    if (j0 >= smalls)
        return;
    build_pair_table(s.table);
    __syncthreads();
    const unsigned int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned long long j = j0 + wave;
    if (j >= smalls)
        return;
    const BatchItem it = w.items[nt + j];
    batch_small(s.w.small[wave], s.table, it.doc, it.di, src_base, dst_base, results);
}

}  // namespace hu
