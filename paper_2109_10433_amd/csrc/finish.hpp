// finish.hpp - end of a call: the last workgroup of a launch turns the
// workspace's error key and totals into the hu_result and resets the
// workspace for the next call (all in the same kernel launch).
#pragma once

#include "device_common.hpp"
#include "hiputf.h"

namespace hu {

// Kind of the UTF-8 sequence that starts at p (p < n), testing the six rules
// of section 3 in reading order; on success *len is the sequence length.
__device__ inline int utf8_sequence_kind(const uint8_t *s, unsigned long long n, unsigned long long p, int *len)
{
    const unsigned int b = s[p];
    if (b < 0x80u) {
        *len = 1;
        return HU_OK;
    }
    if (b < 0xC0u)
        return HU_ERR_STRAY_CONTINUATION;
    if (b >= 0xF8u)
        return HU_ERR_BAD_LEAD;
    const int L = b >= 0xF0u ? 4 : (b >= 0xE0u ? 3 : 2);
    if (p + (unsigned long long)L > n)
        return HU_ERR_TRUNCATED;
    unsigned int v = b & (L == 2 ? 0x1Fu : (L == 3 ? 0x0Fu : 0x07u));
    for (int i = 1; i < L; ++i) {
        const unsigned int c = s[p + i];
        if ((c & 0xC0u) != 0x80u)
            return HU_ERR_TRUNCATED;
        v = (v << 6) | (c & 0x3Fu);
    }
    const unsigned int smallest = L == 2 ? 0x80u : (L == 3 ? 0x800u : 0x10000u);
    if (v < smallest)
        return HU_ERR_OVERLONG;
    if (v > 0x10FFFFu)
        return HU_ERR_TOO_LARGE;
    if (v >= 0xD800u && v <= 0xDFFFu)
        return HU_ERR_SURROGATE;
    *len = L;
    return HU_OK;
}

// Given the first flagged byte f (P <= f <= P + 3, P = end of the longest
// valid prefix), step back to a character boundary at or before P and decode
// forward to the first ill-formed sequence.
__device__ inline hu_result resolve_utf8(const uint8_t *s, unsigned long long n, unsigned long long f)
{
    hu_result r;
    r.reserved = 0;
    if (f >= n) {                 // flags always lie inside the input
        r.error = HU_ERR_DEVICE;
        r.count = 0;
        return r;
    }
    unsigned long long p = f >= 3 ? f - 3 : 0;
    for (int steps = 0; steps < 4 && p > 0 && (s[p] & 0xC0u) == 0x80u; ++steps)
        --p;
    while (p < n && p <= f) {
        int len = 0;
        const int kind = utf8_sequence_kind(s, n, p, &len);
        if (kind != HU_OK) {
            r.error = kind;
            r.count = p;
            return r;
        }
        p += (unsigned long long)len;
    }
    r.error = HU_ERR_DEVICE;   // flags and decoding disagree: never expected
    r.count = 0;
    return r;
}

struct CallInfo {
    const uint8_t *src;          // first input byte
    unsigned long long n;        // input code units
    unsigned long long cap;      // output capacity in code units
    int op;                      // HU_OP_*
};

// Result of a call (or of one document of a batch) from its error key, the
// hang flag and the output total.
__device__ inline hu_result result_from(const CallInfo &c, unsigned long long key, unsigned int hang,
                                        unsigned long long total)
{
    hu_result r;
    r.reserved = 0;
    if (hang) {
        r.error = HU_ERR_DEVICE;
        r.count = 0;
    } else if (key != 0) {
        const unsigned long long f = ~key;
        if (c.op <= HU_OP_CONVERT_UTF8_TO_UTF16LE) {
            r = resolve_utf8(c.src, c.n, f);
        } else {
            r.error = HU_ERR_UNPAIRED_SURROGATE;   // the first flagged word is the first error
            r.count = f;
        }
    } else if (c.op == HU_OP_VALIDATE_UTF8 || c.op == HU_OP_VALIDATE_UTF16LE) {
        r.error = HU_OK;
        r.count = c.n;
    } else if ((c.op == HU_OP_CONVERT_UTF8_TO_UTF16LE || c.op == HU_OP_CONVERT_UTF16LE_TO_UTF8) &&
               total > c.cap) {
        r.error = HU_ERR_OUTPUT_TOO_SMALL;
        r.count = total;
    } else {
        r.error = HU_OK;
        r.count = total;
    }
    return r;
}

__device__ inline hu_result call_result(const CallInfo &c, WsHeader *hdr, unsigned long long total)
{
    const unsigned long long key = __hip_atomic_load(&hdr->err_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned int hang = __hip_atomic_load(&hdr->hang, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return result_from(c, key, hang, total);
}

// Report a flagged position (smallest wins) and wait until the report has
// landed, so that a status word published afterwards implies it.
__device__ inline void report_flag(unsigned long long *err_key, unsigned long long pos)
{
    const unsigned long long old = atomicMax(err_key, ~pos);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if (old == 0x5A5A5A5A5A5A5A5Aull)   // consumes the returned value (forces the wait)
        __builtin_amdgcn_s_sleep(1);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Thread 0 of the finishing workgroup: write the result, reset the header for
// the next call (the epoch advances). Sets *s_wrap when the epoch wrapped.
__device__ inline void finish_call(const CallInfo &c, WsHeader *hdr, unsigned long long total, hu_result *out,
                                   unsigned long long *s_wrap)
{
    *out = call_result(c, hdr, total);
    hdr->tile_counter = 0;
    hdr->err_key = 0;
    hdr->total = 0;
    hdr->hang = 0;
    hdr->done = 0;
    const unsigned int e = (hdr->epoch + 1u) & kEpochMask;
    hdr->epoch = e;
    *s_wrap = (e == 0) ? 1ull : 0ull;
}

// All threads of the finishing workgroup, after finish_call and a barrier:
// when the epoch wrapped to 0, clear the status words so that none from the
// previous era of tag 0 can look current.
__device__ inline void wrap_clear(unsigned long long *status, unsigned long long status_cap,
                                  const unsigned long long *s_wrap)
{
    __syncthreads();
    if (*s_wrap) {
        for (unsigned long long i = threadIdx.x; i < status_cap; i += blockDim.x)
            status[i] = 0;
    }
}

// Persistent kernels: called by every workgroup after its last tile (all
// threads). The workgroup that arrives last writes the result and resets the
// workspace.
__device__ inline void finish_launch(const CallInfo &c, WsHeader *hdr, unsigned long long *status,
                                     unsigned long long status_cap, hu_result *out, int *s_flag,
                                     unsigned long long *s_wrap)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        // The workgroup's contributions (error key, totals) are device-scope
        // atomics whose results it has already waited for, so they are
        // performed before this count is; the last workgroup reads them with
        // device-scope atomic loads after its own count has returned. Relaxed
        // ordering: a release or acquire at device scope would write back or
        // invalidate the whole L2 of the workgroup's XCD once per workgroup,
        // which stalls every other workgroup's loads there.
        const unsigned int prev = __hip_atomic_fetch_add(&hdr->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *s_flag = (prev == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (*s_flag == 0)
        return;
    if (threadIdx.x == 0) {
        const unsigned long long total = __hip_atomic_load(&hdr->total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        finish_call(c, hdr, total, out, s_wrap);
    }
    wrap_clear(status, status_cap, s_wrap);
}

}  // namespace hu
