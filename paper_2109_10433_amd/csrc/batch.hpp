// batch.hpp - many documents, any of the six operations each, in one call.
//
// Three steps, all on the device (nothing is read back, so a call can be
// recorded into a HIP graph and replayed with new document tables):
//   plan: one workgroup gives every document its tiles (work items): a scan
//         over the documents' tile counts, UTF-8 documents first, then
//         UTF-16 ones; documents with no input or invalid arguments get their
//         result here. It also advances the workspace epoch.
//   fill: item -> (document, tile of the document) map.
//   run:  one fused kernel for both input encodings, one workgroup per work
//         item (workgroup b runs item base + b; the grids cover the host's
//         upper bound on the item count, in as many launches as the grid size
//         limit needs, and surplus workgroups leave at once). An item only
//         waits (look-back) for earlier items of its own document, and
//         workgroups are dispatched in id order, so the lowest unfinished
//         item always has a running workgroup whose predecessors are done,
//         however few workgroups the hardware holds at a time. Each document
//         has its own look-back chain and error key; the workgroup that runs
//         a document's last tile writes its result.
#pragma once

#include "engine.hpp"

namespace hu {

struct BatchDoc {                     // mirrors hu_doc
    unsigned long long src_off, n_units, dst_off, dst_cap;
    unsigned int op, reserved;
};
static_assert(sizeof(BatchDoc) == sizeof(hu_doc), "hu_doc layout");

// Workspace of a batch call:
//   [BatchHeader (256 B) | status, item_cap words | first_item | err | item_map
//    | two words per block of documents (planning)]
// The status array starts at a fixed offset; everything after it moves with
// the call's shape (document count, item capacity). Status words must never
// hold anything but status words or zeros, so memory that earlier calls used
// for the per-document arrays is cleared before it becomes status words.
struct BatchHeader {
    unsigned long long items8;        // UTF-8 work items of this call
    unsigned long long items16;       // UTF-16 work items
    unsigned long long dirty_from;    // 1 + first status word that may hold other data (0: none)
    unsigned long long clear_lo;      // status words [clear_lo, clear_hi) to clear in this call
    unsigned long long clear_hi;
    unsigned int epoch;               // tag of this call's status words
    unsigned int hang;                // set if a bounded wait gave up
    unsigned long long overflow;      // 1 if the call's items exceed the item capacity
    unsigned long long pad;
};
static_assert(sizeof(BatchHeader) <= kHeaderBytes, "batch header size");

struct BatchWs {
    BatchHeader *hdr;
    unsigned int *first_item;         // per document
    unsigned long long *err;          // per document error key
    unsigned long long *item_map;     // per item: document index | tile index << 32
    unsigned long long *status;       // per item look-back status
    unsigned long long *block;        // per block of documents: UTF-8, UTF-16 items (then their offsets)
    unsigned long long item_cap;
};

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

__device__ __forceinline__ unsigned long long doc_tiles(const BatchDoc &b, const uint8_t *src_base,
                                                        unsigned long long tile_bytes)
{
    if (b.n_units == 0)
        return 0;
    const unsigned long long off = (unsigned long long)((uintptr_t)(src_base + b.src_off) & 15u);
    const unsigned long long bytes = op_is_u16(b.op) ? 2 * b.n_units : b.n_units;
    return (off + bytes + tile_bytes - 1) / tile_bytes;
}

constexpr int kPlanBlock = 1024;

// Exclusive prefix over a 1024-thread workgroup of two counters at once.
__device__ __forceinline__ void plan_scan2(unsigned long long a, unsigned long long b, unsigned long long *ea,
                                           unsigned long long *eb, unsigned long long *ta, unsigned long long *tb,
                                           unsigned long long (*s_tmp)[kPlanBlock / 64])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    unsigned long long ia = a, ib = b;
    for (int d = 1; d < 64; d <<= 1) {
        const unsigned long long ua = __shfl_up(ia, d, 64), ub = __shfl_up(ib, d, 64);
        if (lane >= d) {
            ia += ua;
            ib += ub;
        }
    }
    if (lane == 63) {
        s_tmp[0][wave] = ia;
        s_tmp[1][wave] = ib;
    }
    __syncthreads();
    unsigned long long pa = 0, pb = 0, sa = 0, sb = 0;
    for (int w = 0; w < kPlanBlock / 64; ++w) {
        const unsigned long long xa = s_tmp[0][w], xb = s_tmp[1][w];
        if (w < wave) {
            pa += xa;
            pb += xb;
        }
        sa += xa;
        sb += xb;
    }
    *ea = pa + ia - a;
    *eb = pb + ib - b;
    *ta = sa;
    *tb = sb;
    __syncthreads();
}

// Planning runs in three steps, so that no single workgroup walks all the
// documents: blocks of kPlanBlock documents (one per thread, coalesced) sum
// their work items; one workgroup turns the block sums into block offsets
// and does the call's bookkeeping; the blocks then give every document its
// first item. Items are numbered UTF-8 documents first, then UTF-16 ones,
// each in document order.

// Work items of document d (0 if it has none or fails the argument checks,
// whose result goes to *err).
__device__ __forceinline__ unsigned long long doc_items(const BatchDoc &b, const uint8_t *src_base,
                                                        const uint8_t *dst_base, unsigned long long tile_bytes, int *err)
{
    *err = doc_check(b, src_base, dst_base);
    return *err ? 0ull : doc_tiles(b, src_base, tile_bytes);
}

__global__ __launch_bounds__(kPlanBlock) void k_batch_count(const BatchDoc *docs, unsigned int n_docs,
                                                            const uint8_t *src_base, const uint8_t *dst_base, BatchWs w,
                                                            unsigned long long tile_bytes)
{
    __shared__ unsigned long long s_tmp[2][kPlanBlock / 64];
    const unsigned long long d = (unsigned long long)blockIdx.x * kPlanBlock + threadIdx.x;
    unsigned long long c8 = 0, c16 = 0;
    if (d < n_docs) {
        const BatchDoc b = docs[d];
        int err;
        const unsigned long long t = doc_items(b, src_base, dst_base, tile_bytes, &err);
        if (op_is_u16(b.op))
            c16 = t;
        else
            c8 = t;
    }
    unsigned long long e8, e16, t8, t16;
    plan_scan2(c8, c16, &e8, &e16, &t8, &t16, s_tmp);
    if (threadIdx.x == 0) {
        w.block[2 * blockIdx.x] = t8;
        w.block[2 * blockIdx.x + 1] = t16;
    }
}

// The call's totals, the capacity check and the epoch in the header; status
// words cleared when the epoch wraps. All threads of the workgroup call it.
__device__ __forceinline__ void plan_bookkeeping(const BatchWs &w, unsigned long long t8, unsigned long long t16,
                                                 int *s_wrap)
{
    const bool overflow = t8 + t16 > w.item_cap;
    if (threadIdx.x == 0) {
        w.hdr->items8 = overflow ? 0 : t8;
        w.hdr->items16 = overflow ? 0 : t16;
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
    __shared__ unsigned long long s_tmp[2][kPlanBlock / 64];
    __shared__ int s_wrap;
    unsigned long long t8 = 0, t16 = 0;   // items of the blocks so far
    for (unsigned int g0 = 0; g0 < n_blocks; g0 += kPlanBlock) {
        const unsigned int g = g0 + threadIdx.x;
        const unsigned long long a = g < n_blocks ? w.block[2 * g] : 0ull;
        const unsigned long long b = g < n_blocks ? w.block[2 * g + 1] : 0ull;
        unsigned long long ea, eb, ta, tb;
        plan_scan2(a, b, &ea, &eb, &ta, &tb, s_tmp);
        if (g < n_blocks) {
            w.block[2 * g] = t8 + ea;          // block offsets, in place of the sums
            w.block[2 * g + 1] = t16 + eb;
        }
        t8 += ta;
        t16 += tb;
    }
    plan_bookkeeping(w, t8, t16, &s_wrap);
}

// Document d's first work item, or its result if it has no work (error,
// empty, or the call's items exceed the workspace's capacity).
__device__ __forceinline__ void assign_doc(const BatchWs &w, hu_result *results, unsigned long long d, int err,
                                           unsigned long long items, bool overflow, unsigned long long first)
{
    if (err == 0 && overflow)
        err = HU_ERR_INVALID_ARGUMENT;   // work-item capacity of the workspace exceeded
    if (err != 0 || items == 0) {
        hu_result r;
        r.error = err;
        r.reserved = 0;
        r.count = 0;
        results[d] = r;
        w.first_item[d] = 0xFFFFFFFFu;
        return;
    }
    w.first_item[d] = (unsigned int)first;
}

__global__ __launch_bounds__(kPlanBlock) void k_batch_assign(const BatchDoc *docs, unsigned int n_docs,
                                                             const uint8_t *src_base, const uint8_t *dst_base,
                                                             hu_result *results, BatchWs w,
                                                             unsigned long long tile_bytes)
{
    __shared__ unsigned long long s_tmp[2][kPlanBlock / 64];
    const unsigned long long d = (unsigned long long)blockIdx.x * kPlanBlock + threadIdx.x;
    unsigned long long c8 = 0, c16 = 0;
    int err = 0;
    bool u16 = false;
    if (d < n_docs) {
        const BatchDoc b = docs[d];
        u16 = op_is_u16(b.op);
        const unsigned long long t = doc_items(b, src_base, dst_base, tile_bytes, &err);
        if (u16)
            c16 = t;
        else
            c8 = t;
    }
    unsigned long long e8, e16, t8, t16;
    plan_scan2(c8, c16, &e8, &e16, &t8, &t16, s_tmp);   // every thread takes part
    if (d < n_docs)
        assign_doc(w, results, d, err, c8 + c16, w.hdr->overflow != 0,
                   u16 ? w.hdr->items8 + w.block[2 * blockIdx.x + 1] + e16 : w.block[2 * blockIdx.x] + e8);
}

// Planning of a call of at most kPlanBlock documents, all three steps in one
// workgroup (one launch: small batches, as in serving, wait on it).
__global__ __launch_bounds__(kPlanBlock) void k_batch_plan1(const BatchDoc *docs, unsigned int n_docs,
                                                            const uint8_t *src_base, const uint8_t *dst_base,
                                                            hu_result *results, BatchWs w,
                                                            unsigned long long tile_bytes)
{
    __shared__ unsigned long long s_tmp[2][kPlanBlock / 64];
    __shared__ int s_wrap;
    const unsigned int d = threadIdx.x;
    unsigned long long c8 = 0, c16 = 0;
    int err = 0;
    bool u16 = false;
    if (d < n_docs) {
        const BatchDoc b = docs[d];
        u16 = op_is_u16(b.op);
        const unsigned long long t = doc_items(b, src_base, dst_base, tile_bytes, &err);
        if (u16)
            c16 = t;
        else
            c8 = t;
    }
    unsigned long long e8, e16, t8, t16;
    plan_scan2(c8, c16, &e8, &e16, &t8, &t16, s_tmp);
    if (d < n_docs)
        assign_doc(w, results, d, err, c8 + c16, t8 + t16 > w.item_cap, u16 ? t8 + e16 : e8);
    plan_bookkeeping(w, t8, t16, &s_wrap);
}

// item -> (document, tile) map; every error key back to zero; status words
// the plan marked for clearing.
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
        if (first == 0xFFFFFFFFu)
            continue;
        const unsigned long long t = doc_tiles(docs[d], src_base, tile_bytes);
        for (unsigned long long k = 0; k < t; ++k)
            w.item_map[first + k] = (unsigned long long)d | (k << 32);
    }
}

// One work item (tile `tile` of document di, global item index i).
template <class Dir, int U>
__device__ __forceinline__ void batch_item(ConvertShared<Dir, U> &s, const BatchDoc &b, unsigned int di,
                                           unsigned long long tile, unsigned long long i, unsigned int epoch,
                                           const uint8_t *src_base, uint8_t *dst_base, hu_result *results, BatchWs w)
{
    if (Dir::kNeedsTable)
        build_pair_table(s.table);
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
    switch (op_mode(b.op)) {
    case kValidate: chained_tile<Dir, U, kValidate>(s, d, tile, n_tiles, cx, fin); break;
    case kLength: chained_tile<Dir, U, kLength>(s, d, tile, n_tiles, cx, fin); break;
    default: chained_tile<Dir, U, kConvert>(s, d, tile, n_tiles, cx, fin); break;
    }
}

template <int U>
union BatchShared {
    ConvertShared<U8Dir, U> u8;
    ConvertShared<U16Dir, U> u16;
};

// Items [0, n8) are UTF-8 input, [n8, n8 + n16) UTF-16LE. Dynamic LDS (unused)
// may be requested at launch to cap the workgroups resident per CU.
template <int U>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4, 8)))
void k_batch_run(const BatchDoc *docs, const uint8_t *src_base, uint8_t *dst_base, hu_result *results, BatchWs w,
                 unsigned long long item_base)
{
    __shared__ BatchShared<U> s;
    const unsigned long long i = item_base + blockIdx.x;
    const unsigned long long n8 = w.hdr->items8, n16 = w.hdr->items16;
    if (i >= n8 + n16)
        return;
    const unsigned long long m = w.item_map[i];
    const unsigned int di = (unsigned int)m;
    const unsigned long long tile = m >> 32;
    const BatchDoc b = docs[di];
    const unsigned int epoch = w.hdr->epoch;
    if (i < n8)
        batch_item<U8Dir, U>(s.u8, b, di, tile, i, epoch, src_base, dst_base, results, w);
    else
        batch_item<U16Dir, U>(s.u16, b, di, tile, i, epoch, src_base, dst_base, results, w);
}

}  // namespace hu
