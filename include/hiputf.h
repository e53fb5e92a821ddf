/*
 * hiputf.h - validating UTF-8 <-> UTF-16LE transcoding on AMD Instinct MI355X
 * (gfx950). C ABI: plain pointers and sizes, no C++ or framework types.
 *
 * The operations are those of Lemire & Mula, "Transcoding Billions of Unicode
 * Characters per Second with SIMD Instructions":
 *   - UTF-8 validity: the six rules of section 3 (lead byte length classes,
 *     continuation bytes, no overlong forms, nothing above U+10FFFF, no
 *     U+D800..DFFF);
 *   - UTF-16 validity and surrogate pairs: section 3;
 *   - UTF-8 -> UTF-16 transcoding: section 4 (Algorithms "core component" and
 *     "non-validating transcoder", validated as described there);
 *   - UTF-16 -> UTF-8 transcoding: section 5 (Algorithm "UTF-16 to UTF-8");
 *   - the output placement across independently decoded pieces follows the
 *     interleaved decoding with precomputed offsets named as future work in
 *     section 7.
 * The paper reports validity as a yes/no answer; this interface adds the first
 * error's kind and byte position and the output length (see hu_result).
 *
 * Memory: every data pointer (src, dst, results, workspaces, document tables)
 * is a DEVICE pointer on the current HIP device. `stream` is a hipStream_t
 * passed as void* (NULL = the default stream). UTF-16LE buffers must be 2-byte
 * aligned; UTF-8 buffers may have any alignment. The caller owns all buffers.
 *
 * Errors: no function throws, aborts or prints. Invalid arguments come back as
 * HU_ERR_INVALID_ARGUMENT, HIP runtime failures as HU_ERR_DEVICE.
 */
#ifndef HIPUTF_H
#define HIPUTF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Result of a call (16 bytes, plain data).
 *   error == HU_OK:
 *     convert_* and *_length_*: count = output code units (UTF-16 words or
 *                               UTF-8 bytes);
 *     validate_*:               count = input code units (bytes or words).
 *   error in HU_ERR_BAD_LEAD .. HU_ERR_UNPAIRED_SURROGATE:
 *     count = BYTE offset of the first ill-formed sequence, i.e. the end of the
 *     longest valid prefix (for UTF-16 input: 2 x word index).
 *   error == HU_ERR_OUTPUT_TOO_SMALL: the input is valid and count = the output
 *     code units required. Validation errors take precedence over it.
 *   other errors: count = 0. */
typedef struct {
    int32_t error;
    int32_t reserved;
    uint64_t count;
} hu_result;

/* Error kinds. For UTF-8 the kind names the first of the six rules of
 * section 3 that the sequence at the error position breaks, the rules being
 * tested in reading order: a continuation byte where a character must start
 * (STRAY_CONTINUATION), a byte F8..FF (BAD_LEAD), a lead byte without all its
 * continuation bytes, also at end of input (TRUNCATED), a value that fits a
 * shorter sequence (OVERLONG), a value above U+10FFFF (TOO_LARGE), a value in
 * U+D800..DFFF (SURROGATE). */
enum {
    HU_OK = 0,
    HU_ERR_BAD_LEAD = 1,
    HU_ERR_TRUNCATED = 2,
    HU_ERR_STRAY_CONTINUATION = 3,
    HU_ERR_OVERLONG = 4,
    HU_ERR_TOO_LARGE = 5,
    HU_ERR_SURROGATE = 6,
    HU_ERR_UNPAIRED_SURROGATE = 7, /* UTF-16: high not followed by low, or low not after high */
    HU_ERR_OUTPUT_TOO_SMALL = 16,
    HU_ERR_INVALID_ARGUMENT = 17,
    HU_ERR_DEVICE = 18,
    HU_ERR_EXCEEDS_SCRATCH = 19    /* convert_utf8_to_utf16le_noalloc: input above HU_NOALLOC_MAX_BYTES */
};

/* ------------------------------------------------------------------------
 * Synchronous calls. Each enqueues its kernel on `stream`, waits for that
 * stream, and returns the result, which the kernel writes straight into a
 * pinned host record. Scratch memory (a 256-byte header, and for the
 * conversions 128 bytes per tile of 4 to 24 KiB of input, by input size;
 * hu_workspace_bytes gives the exact figure) comes from a per-device,
 * per-stream cache owned by the library
 * (freed by hu_shutdown). n = 0 returns {HU_OK, 0}; pointers may then be NULL.
 * A NULL src (or dst with a non-zero capacity) with n > 0 is
 * HU_ERR_INVALID_ARGUMENT. On success exactly `count` units are written to
 * dst and dst[count, cap) is untouched; on any error the contents of
 * dst[0, cap) are unspecified. Nothing is ever written outside [dst, dst+cap).
 * Calls on one stream are serialised by the stream; calls on different
 * streams may run concurrently.
 * ---------------------------------------------------------------------- */

/* UTF-8 well-formedness (section 3, six rules). */
hu_result validate_utf8(const uint8_t *src, size_t n_bytes, void *stream);

/* Number of UTF-16 words the UTF-8 input converts to (validates first): one
 * word per character of one to three bytes, two for a four-byte character
 * (Table "utfsummary", section 3: code point ranges and their UTF-8 and
 * UTF-16 lengths). On invalid input, the error of validate_utf8. */
hu_result utf16_length_from_utf8(const uint8_t *src, size_t n_bytes, void *stream);

/* Validating UTF-8 -> UTF-16LE (section 4). dst holds dst_cap_words words;
 * n_bytes words always suffice. */
hu_result convert_utf8_to_utf16le(const uint8_t *src, size_t n_bytes,
                                  uint16_t *dst, size_t dst_cap_words, void *stream);

/* UTF-16LE well-formedness (section 3, surrogate pairing). src: n_words words. */
hu_result validate_utf16le(const uint16_t *src, size_t n_words, void *stream);

/* Number of UTF-8 bytes the UTF-16LE input converts to (validates first):
 * one byte for a word below U+0080, two below U+0800, three for any other
 * word outside the surrogates, four for a surrogate pair (Table "utfsummary",
 * section 3). On invalid input, the error of validate_utf16le. */
hu_result utf8_length_from_utf16le(const uint16_t *src, size_t n_words, void *stream);

/* Validating UTF-16LE -> UTF-8 (section 5). dst holds dst_cap_bytes bytes;
 * 3 x n_words bytes always suffice. */
hu_result convert_utf16le_to_utf8(const uint16_t *src, size_t n_words,
                                  uint8_t *dst, size_t dst_cap_bytes, void *stream);

/* Non-validating conversions, for input known to be valid (section 4's
 * non-validating transcoder, and its UTF-16 counterpart of section 5): the
 * same output and count as the validating calls on valid input, without the
 * validation work. On invalid input the result and the contents of
 * dst[0, cap) are unspecified (a tile whose counts do not fit the decoder's
 * staging is left undecoded), but the call completes, never writes outside
 * [dst, dst + cap) and still reports HU_ERR_OUTPUT_TOO_SMALL when its count
 * exceeds cap. Arguments, capacities and argument errors as for
 * convert_utf8_to_utf16le / convert_utf16le_to_utf8; workspace as for the op
 * HU_OP_CONVERT_UTF8_TO_UTF16LE / HU_OP_CONVERT_UTF16LE_TO_UTF8. */
hu_result convert_valid_utf8_to_utf16le(const uint8_t *src, size_t n_bytes,
                                        uint16_t *dst, size_t dst_cap_words, void *stream);
hu_result convert_valid_utf16le_to_utf8(const uint16_t *src, size_t n_words,
                                        uint8_t *dst, size_t dst_cap_bytes, void *stream);

/* UTF-16 big endian (section 3: UTF-16's two byte orders; the experiments
 * section notes that the big-endian format costs a little-endian transcoder
 * only a byte swap per word): the same four operations with every UTF-16 word
 * read from, or written to, memory most significant byte first. Results,
 * error kinds and positions (2 x word index for UTF-16 input) as for the
 * little-endian calls; workspace as for the matching HU_OP_* little-endian
 * op. */
hu_result validate_utf16be(const uint16_t *src, size_t n_words, void *stream);
hu_result utf8_length_from_utf16be(const uint16_t *src, size_t n_words, void *stream);
hu_result convert_utf16be_to_utf8(const uint16_t *src, size_t n_words,
                                  uint8_t *dst, size_t dst_cap_bytes, void *stream);
hu_result convert_utf8_to_utf16be(const uint8_t *src, size_t n_bytes,
                                  uint16_t *dst, size_t dst_cap_words, void *stream);

/* Byte-order mark at the start of a buffer: UTF-16LE FF FE and UTF-16BE
 * FE FF (section 3), UTF-8 EF BB BF (RFC 3629, section 6); checked in the
 * order UTF-8, UTF-16LE, UTF-16BE. `head` is HOST memory holding the
 * first n_bytes (up to 3 are read); returns the encoding and the BOM's
 * length in bytes (HU_BOM_NONE, 0 when there is none or head is NULL). The
 * caller skips the BOM and picks the calls for that encoding. */
enum { HU_BOM_NONE = 0, HU_BOM_UTF8 = 1, HU_BOM_UTF16LE = 2, HU_BOM_UTF16BE = 3 };
typedef struct {
    int32_t encoding;   /* HU_BOM_* */
    int32_t length;     /* bytes */
} hu_bom;
hu_bom hu_detect_bom(const uint8_t *head, size_t n_bytes);

/* ------------------------------------------------------------------------
 * Asynchronous calls (allocate nothing, never synchronise, safe to record
 * into a HIP graph). Same operations as above; the result is written to the
 * device record *d_result when the enqueued kernels complete.
 *   ws / ws_bytes: caller-owned device workspace of at least
 *   hu_workspace_bytes(op, n) bytes, zero-filled before its first use
 *   (hipMemset or hu_workspace_init). Every completed call leaves it ready for
 *   the next call. Calls that share a workspace must be ordered (same stream
 *   or events); concurrent calls need separate workspaces.
 * Return value: HU_OK once enqueued, HU_ERR_INVALID_ARGUMENT (nothing
 * enqueued) or HU_ERR_DEVICE.
 * ---------------------------------------------------------------------- */

enum {
    HU_OP_VALIDATE_UTF8 = 0,
    HU_OP_UTF16_LENGTH_FROM_UTF8 = 1,
    HU_OP_CONVERT_UTF8_TO_UTF16LE = 2,
    HU_OP_VALIDATE_UTF16LE = 3,
    HU_OP_UTF8_LENGTH_FROM_UTF16LE = 4,
    HU_OP_CONVERT_UTF16LE_TO_UTF8 = 5
};

/* Workspace bytes for one call of `op` on n input code units (validation and
 * length need the 256-byte header only; a workspace shared by several
 * operations is sized for the largest). */
size_t hu_workspace_bytes(int op, size_t n_units);

/* Input bytes per tile of the kernel that runs `op` (HU_OP_*) on n_units
 * code units, 0 for an unknown op. A tile is the unit of work that has one
 * status word in the workspace; tile k covers input bytes [k*T, (k+1)*T)
 * counted from the 16-byte aligned address at or below src. Host only: no
 * GPU work, no allocation. */
size_t hu_tile_bytes(int op, size_t n_units);

/* Zero-fills a workspace with a kernel on `stream` (capturable). */
int hu_workspace_init(void *ws, size_t ws_bytes, void *stream);

int validate_utf8_async(const uint8_t *src, size_t n_bytes, hu_result *d_result,
                        void *ws, size_t ws_bytes, void *stream);
int utf16_length_from_utf8_async(const uint8_t *src, size_t n_bytes, hu_result *d_result,
                                 void *ws, size_t ws_bytes, void *stream);
int convert_utf8_to_utf16le_async(const uint8_t *src, size_t n_bytes, uint16_t *dst,
                                  size_t dst_cap_words, hu_result *d_result,
                                  void *ws, size_t ws_bytes, void *stream);
int validate_utf16le_async(const uint16_t *src, size_t n_words, hu_result *d_result,
                           void *ws, size_t ws_bytes, void *stream);
int utf8_length_from_utf16le_async(const uint16_t *src, size_t n_words, hu_result *d_result,
                                   void *ws, size_t ws_bytes, void *stream);
int convert_utf16le_to_utf8_async(const uint16_t *src, size_t n_words, uint8_t *dst,
                                  size_t dst_cap_bytes, hu_result *d_result,
                                  void *ws, size_t ws_bytes, void *stream);
int validate_utf16be_async(const uint16_t *src, size_t n_words, hu_result *d_result,
                           void *ws, size_t ws_bytes, void *stream);
int utf8_length_from_utf16be_async(const uint16_t *src, size_t n_words, hu_result *d_result,
                                   void *ws, size_t ws_bytes, void *stream);
int convert_utf16be_to_utf8_async(const uint16_t *src, size_t n_words, uint8_t *dst,
                                  size_t dst_cap_bytes, hu_result *d_result,
                                  void *ws, size_t ws_bytes, void *stream);
int convert_utf8_to_utf16be_async(const uint8_t *src, size_t n_bytes, uint16_t *dst,
                                  size_t dst_cap_words, hu_result *d_result,
                                  void *ws, size_t ws_bytes, void *stream);
int convert_valid_utf8_to_utf16le_async(const uint8_t *src, size_t n_bytes, uint16_t *dst,
                                        size_t dst_cap_words, hu_result *d_result,
                                        void *ws, size_t ws_bytes, void *stream);
int convert_valid_utf16le_to_utf8_async(const uint16_t *src, size_t n_words, uint8_t *dst,
                                        size_t dst_cap_bytes, hu_result *d_result,
                                        void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory at all (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * validating UTF-8 -> UTF-16LE conversion of convert_utf8_to_utf16le_async
 * with the workspace taken from a static device array of the library
 * (1.5 MiB per device, held until the process ends) instead of a workspace
 * argument. It calls no allocating routine. The array's address is looked up
 * on the first call on each device, and that call also clears it with a
 * kernel on `stream`; every completed call leaves it ready for the next.
 * src, dst, dst_cap_words, d_result (a device record) and the result's
 * meaning are as for convert_utf8_to_utf16le_async; the output is the same.
 * All calls on one device share the one array: calls that may overlap on a
 * device (different streams, or graphs replayed concurrently) race and give
 * wrong results, so they must be ordered on one stream or by events.
 * Returns HU_OK once enqueued, HU_ERR_EXCEEDS_SCRATCH (nothing enqueued) when
 * n_bytes > HU_NOALLOC_MAX_BYTES, HU_ERR_INVALID_ARGUMENT as the async call,
 * or HU_ERR_DEVICE.
 * ---------------------------------------------------------------------- */
#define HU_NOALLOC_MAX_BYTES ((size_t)1 << 28)   /* 256 MiB */
int convert_utf8_to_utf16le_noalloc(const uint8_t *src, size_t n_bytes, uint16_t *dst,
                                    size_t dst_cap_words, hu_result *d_result, void *stream);

/* ------------------------------------------------------------------------
 * Batches: many documents of any lengths, each with its own operation (any of
 * the six, directions may be mixed), in one call of three kernel launches
 * (plan, item map, one fused run kernel with one workgroup per work item;
 * the run kernel takes one more launch per 2^24 - 1 work items) and no host
 * synchronisation; safe to record into a HIP graph and replay (the
 * document table and inputs are read on the device at run time).
 * All pointers except `tuning` are device pointers.
 * ---------------------------------------------------------------------- */

/* One document (40 bytes). Input: src_base + src_off, n_units code units
 * (bytes for UTF-8 operations, 2-byte aligned words for UTF-16 ones). Output
 * (convert operations): dst_base + dst_off, capacity dst_cap output code
 * units. Output regions must not overlap. */
typedef struct {
    uint64_t src_off;
    uint64_t n_units;
    uint64_t dst_off;
    uint64_t dst_cap;
    uint32_t op;          /* HU_OP_* */
    uint32_t reserved;    /* 0 */
} hu_doc;

/* Launch shape of the batch kernels (see hu_tune_batch). */
typedef struct {
    uint32_t sub_tiles;       /* 4 KiB input sub-tiles per tile work item: 1, 2, 4 or 6 (0 = default, 2) */
    uint32_t groups_per_cu;   /* at most this many run-kernel workgroups per compute unit, enforced by
                                 reserving unused LDS (0 = as many as the kernel's resources allow) */
} hu_tuning;

/* Workspace bytes for a batch of n_docs documents whose inputs total at most
 * total_input_bytes bytes (UTF-16 inputs count 2 bytes per word). */
size_t hu_batch_workspace_bytes(uint32_t n_docs, uint64_t total_input_bytes);

/* Runs the batch. results[d] receives document d's result with the same
 * meaning as the single-buffer call of its operation. ws: device workspace of
 * at least hu_batch_workspace_bytes(n_docs, total_input_bytes) bytes,
 * 256-byte aligned, zero-filled before first use; each call leaves it ready
 * for the next. If the documents need more work items than the workspace was
 * sized for, every document reports HU_ERR_INVALID_ARGUMENT. A document with
 * invalid arguments (misaligned UTF-16 input, unknown op, ...) reports
 * HU_ERR_INVALID_ARGUMENT alone. tuning: host pointer or NULL.
 * Returns HU_OK once enqueued, else HU_ERR_INVALID_ARGUMENT or HU_ERR_DEVICE. */
int hu_batch_run(const hu_doc *docs, uint32_t n_docs, uint64_t total_input_bytes, const void *src_base,
                 void *dst_base, hu_result *results, const hu_tuning *tuning, void *ws, size_t ws_bytes,
                 void *stream);

/* Records one hu_batch_run into a HIP graph and instantiates it; *graph_exec
 * receives a hipGraphExec_t. Replays (hu_graph_launch) read the document
 * table, inputs and workspace at the same addresses, so callers may rewrite
 * them in place between replays (same n_docs). */
int hu_batch_graph_create(const hu_doc *docs, uint32_t n_docs, uint64_t total_input_bytes, const void *src_base,
                          void *dst_base, hu_result *results, const hu_tuning *tuning, void *ws, size_t ws_bytes,
                          void **graph_exec);
int hu_graph_launch(void *graph_exec, void *stream);
void hu_graph_destroy(void *graph_exec);

/* Autotuner: times hu_batch_run on the given batch (which it runs several
 * times) for every sub_tiles in {1, 2, 4, 6} and groups_per_cu in {2, 4, 6, 0},
 * writes the fastest to *best and its mean time in microseconds to *best_us.
 * If `key` is non-NULL and the environment variable HIPUTF_TUNE_CACHE names a
 * file, the result is appended to that file as one JSON line
 * {"key": ..., "device": "<arch>/<compute units>", "sub_tiles": ..., "groups_per_cu": ..., "us": ...}. */
int hu_tune_batch(const hu_doc *docs, uint32_t n_docs, uint64_t total_input_bytes, const void *src_base,
                  void *dst_base, hu_result *results, void *ws, size_t ws_bytes, const char *key,
                  hu_tuning *best, double *best_us, void *stream);

/* Reads the last cached tuning stored under `key` for the current device from
 * HIPUTF_TUNE_CACHE. Returns HU_OK and fills *out, or HU_ERR_INVALID_ARGUMENT
 * when there is no such entry. */
int hu_tuning_lookup(const char *key, hu_tuning *out);

/* ------------------------------------------------------------------------
 * Server: transcoding requests from HOST memory, batched on the device as
 * they arrive (continuous batching). A scheduler thread admits requests in
 * arrival order while batch slots, the in-flight request limit and the device
 * pool allow (a request waits at the head of the queue until memory is free;
 * none is overtaken, so none starves), stages each batch in pinned host memory
 * (one host-to-device copy of the document table and inputs), runs it with
 * hu_batch_run, brings outputs and results back in one device-to-host copy and
 * copies each output to the request's dst. Up to `slots` batches are in
 * flight on their own streams, so new arrivals are batched and copied while
 * earlier batches run. Unlike the rest of this interface, request src and dst
 * are HOST pointers; they must stay valid until the request completes.
 * ---------------------------------------------------------------------- */

typedef struct {
    uint64_t pool_bytes;      /* device memory for batch regions (0 = 8 GiB) */
    uint64_t batch_bytes;     /* largest batch region: document table, inputs,
                                 worst-case outputs, results; also the pinned
                                 staging per slot (0 = 256 MiB) */
    uint32_t batch_requests;  /* most requests per batch (0 = 4096) */
    uint32_t max_in_flight;   /* most requests admitted and not completed (0 = 65536) */
    uint32_t slots;           /* batches in flight, one stream each (0 = 3) */
    uint32_t plain;           /* 1: comparison path: one request at a time, each
                                 through the single-buffer async call (one slot,
                                 one request per step) */
    hu_tuning tuning;         /* launch shape of the batch kernels (zeros = defaults) */
} hu_server_config;

/* One request (48 bytes). Output capacity dst_cap is in output code units;
 * dst may be NULL (the result alone is returned). On success exactly
 * result.count units are written to dst; on an error nothing is. */
typedef struct {
    uint64_t tag;             /* returned in the completion */
    uint32_t op;              /* HU_OP_* */
    uint32_t reserved;        /* 0 */
    const void *src;          /* host input: n_units code units */
    uint64_t n_units;
    void *dst;                /* host output or NULL */
    uint64_t dst_cap;
} hu_request;

typedef struct {
    uint64_t tag;
    hu_result result;         /* as from the single-buffer call of the same op;
                                 HU_ERR_INVALID_ARGUMENT for a request that can
                                 never run (unknown op, larger than a batch) */
    int64_t latency_ns;       /* arrival to output in dst, host monotonic clock */
} hu_completion;

typedef struct {
    uint64_t submitted, completed, rejected, batches;
    uint64_t input_bytes, output_bytes;   /* of requests completed without error */
    int64_t p50_ns, p99_ns, max_ns;       /* latency percentiles (nearest rank) */
    int64_t device_ns;                    /* summed device time of the batch steps */
    double mean_batch;                    /* requests per batch */
} hu_server_stats;

/* Creates a server on the current HIP device (cfg may be NULL: defaults).
 * Returns HU_OK and *server, HU_ERR_INVALID_ARGUMENT or HU_ERR_DEVICE (not
 * enough device or pinned memory). */
int hu_server_create(const hu_server_config *cfg, void **server);

/* Queues a request; its arrival time is now. Thread-safe. */
int hu_server_submit(void *server, const hu_request *req);

/* Moves up to `max` completions into out (*n_out of them), waiting up to
 * timeout_ns for the first. Thread-safe. */
int hu_server_poll(void *server, hu_completion *out, uint32_t max, uint32_t *n_out, int64_t timeout_ns);

/* Open-loop replay: submits reqs[i] at arrival_ns[i] nanoseconds after the
 * call starts (non-decreasing), latency counted from that scheduled time, and
 * returns when all n have completed; out[i] receives request i's completion.
 * Completions of a replay are not queued for hu_server_poll. */
int hu_server_replay(void *server, const hu_request *reqs, const int64_t *arrival_ns, uint64_t n,
                     hu_completion *out);

/* Statistics since creation or the last reset. */
int hu_server_stats_get(void *server, hu_server_stats *out);
int hu_server_stats_reset(void *server);

/* Finishes every queued and running request, then frees the server. */
void hu_server_destroy(void *server);

/* Library-wide: a human-readable name for an error code (static string). */
const char *hu_error_name(int error);

/* Frees the library's cached workspaces and pinned result slots on every
 * device. Calls may follow; caches are rebuilt on demand. */
void hu_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* HIPUTF_H */
