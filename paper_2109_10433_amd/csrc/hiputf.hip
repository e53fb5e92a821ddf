// hiputf.hip - C-ABI runtime for validating UTF-8 <-> UTF-16LE transcoding
// (declarations and contracts in include/hiputf.h).
//
// A call = one launch of a tile kernel (engine.hpp) whose last workgroup writes
// the hu_result and resets the workspace for the next call (finish.hpp).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>

#include "batch.hpp"
#include "hiputf.h"
#include "kernel_choice.hpp"

namespace hu {

__global__ void k_fill_zero(unsigned int *p, unsigned long long n_words)
{
    for (unsigned long long i = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; i < n_words;
         i += (unsigned long long)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ------------------------------------------------------------ launch helpers
struct DeviceInfo {
    int cus = 0;
    std::map<const void *, int> blocks_per_cu;
    std::map<std::pair<const void *, unsigned int>, size_t> lds_pads;   // (kernel, groups per CU)
};

size_t lds_pad(const void *fn, unsigned int groups_per_cu);

std::mutex g_info_mu;
std::map<int, DeviceInfo> g_info;

// Resident workgroups of a persistent kernel over the device: per CU, what
// its resources allow, at most cap (0: no cap). *pad: the dynamic LDS per
// workgroup that holds residency to cap (0 without a cap).
int max_resident_blocks(const void *kernel, unsigned int cap = 0, size_t *pad = nullptr)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return 0;
    std::lock_guard<std::mutex> lk(g_info_mu);
    DeviceInfo &di = g_info[dev];
    if (di.cus == 0) {
        if (hipDeviceGetAttribute(&di.cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
    }
    auto it = di.blocks_per_cu.find(kernel);
    if (it == di.blocks_per_cu.end()) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, 0) != hipSuccess || nb < 1)
            nb = 1;
        it = di.blocks_per_cu.emplace(kernel, nb).first;
    }
    if (pad != nullptr) {
        *pad = 0;
        if (cap != 0) {
            auto pt = di.lds_pads.find({kernel, cap});
            if (pt == di.lds_pads.end())
                pt = di.lds_pads.emplace(std::make_pair(kernel, cap), lds_pad(kernel, cap)).first;
            *pad = pt->second;
        }
    }
    return di.cus * (cap != 0 && (int)cap < it->second ? (int)cap : it->second);
}

constexpr unsigned long long kMaxUnits = 1ull << 38;   // status values hold 40 bits

// n_bytes: the input's size, which picks the UTF-8 -> UTF-16LE tile size (0:
// the smallest tile any input of the operation may take).
KernelChoice choose_kernel(int op, unsigned long long n_bytes)
{
#define HU_K(...) reinterpret_cast<const void *>(&__VA_ARGS__)
    if ((op & kOpFlags) != 0) {   // no kernel for the combination: fn stays null
        KernelChoice kc{nullptr, (unsigned long long)kSub, true};
        choose_variant(op, n_bytes, kc);
        return kc;
    }
    switch (op) {
    case HU_OP_VALIDATE_UTF8: return {HU_K(k_scan<U8Dir, kValidate, kPValidate8>), kPValidate8 * kPieceBytes, false};
    case HU_OP_UTF16_LENGTH_FROM_UTF8:
        return {HU_K(k_scan<U8Dir, kLength, kPLength8>), kPLength8 * kPieceBytes, false, kLength8GroupsPerCu};
    case HU_OP_CONVERT_UTF8_TO_UTF16LE: {
        const int u = class_sub_tiles(kConvert8Classes, n_bytes);
        const void *fn = u == 1 ? HU_K(k_convert_u8<1, kConvert>) : u == 2 ? HU_K(k_convert_u8<2, kConvert>)
                       : u == 5 ? HU_K(k_convert_u8<5, kConvert>) : HU_K(k_convert_u8<6, kConvert>);
        return {fn, (unsigned long long)u * kSub, true};
    }
    case HU_OP_VALIDATE_UTF16LE: return {HU_K(k_scan<U16Dir, kValidate, kPValidate16>), kPValidate16 * kPieceBytes, false};
    case HU_OP_UTF8_LENGTH_FROM_UTF16LE:
        return {HU_K(k_scan<U16Dir, kLength, kPLength16>), kPLength16 * kPieceBytes, false, kLength16GroupsPerCu};
    default: {
        const int u = class_sub_tiles(kConvert16Classes, n_bytes);
        const void *fn = u == 1 ? HU_K(k_convert_u16<1, kConvert>) : u == 2 ? HU_K(k_convert_u16<2, kConvert>)
                                                                          : HU_K(k_convert_u16<6, kConvert>);
        return {fn, (unsigned long long)u * kSub, true};
    }
    }
#undef HU_K
}

unsigned long long tiles_for(int op, const void *src, unsigned long long n_units)
{
    const bool u16 = (op & ~kOpFlags) >= HU_OP_VALIDATE_UTF16LE;
    const unsigned long long bytes = u16 ? 2 * n_units : n_units;
    const unsigned long long off = (unsigned long long)((uintptr_t)src & 15u);
    const unsigned long long tb = choose_kernel(op, bytes).tile_bytes;
    return (off + bytes + tb - 1) / tb;
}

// Workspace bytes a call needs: the header, and for the convert kernels one
// status word (on its own 128-byte line) per tile.
unsigned long long workspace_need(int op, const void *src, unsigned long long n_units)
{
    const bool u16 = (op & ~kOpFlags) >= HU_OP_VALIDATE_UTF16LE;
    const unsigned long long bytes = u16 ? 2 * n_units : n_units;
    if (n_units == 0 || !choose_kernel(op, bytes).one_group_per_tile)
        return kHeaderBytes;
    return kHeaderBytes + 8ull * kStatusStride * tiles_for(op, src, n_units);
}

// op: HU_OP_* with the flags above (only on the combinations choose_kernel has)
int enqueue(int op, const void *src, unsigned long long n, void *dst, unsigned long long cap,
            hu_result *d_result, void *ws, size_t ws_bytes, hipStream_t stream)
{
    const int base_op = op & ~kOpFlags;
    const bool u16 = base_op >= HU_OP_VALIDATE_UTF16LE;
    if (base_op < 0 || base_op > HU_OP_CONVERT_UTF16LE_TO_UTF8 || d_result == nullptr || ws == nullptr ||
        ((uintptr_t)ws & 255u) != 0 || n > kMaxUnits)
        return HU_ERR_INVALID_ARGUMENT;
    if (n > 0 && src == nullptr)
        return HU_ERR_INVALID_ARGUMENT;
    if (cap > 0 && dst == nullptr)
        return HU_ERR_INVALID_ARGUMENT;
    if (u16 && ((uintptr_t)src & 1u))
        return HU_ERR_INVALID_ARGUMENT;
    if (base_op == HU_OP_CONVERT_UTF8_TO_UTF16LE && ((uintptr_t)dst & 1u))
        return HU_ERR_INVALID_ARGUMENT;
    const unsigned long long n_bytes = u16 ? 2 * n : n;
    if (choose_kernel(op, n_bytes).fn == nullptr)
        return HU_ERR_INVALID_ARGUMENT;
    const unsigned long long n_tiles = n ? tiles_for(op, src, n) : 0;
    if (ws_bytes < workspace_need(op, src, n))
        return HU_ERR_INVALID_ARGUMENT;

    WsHeader *hdr = reinterpret_cast<WsHeader *>(ws);
    unsigned long long *status = reinterpret_cast<unsigned long long *>((char *)ws + kHeaderBytes);
    unsigned long long status_cap = (ws_bytes - kHeaderBytes) / 8;

    const KernelChoice kc = choose_kernel(op, n_bytes);
    unsigned long long grid_ll = 1;   // at least one workgroup: with no tiles it only writes the result
    size_t pad = 0;                   // dynamic LDS that holds residency to kc.groups_per_cu
    if (kc.one_group_per_tile) {
        if (n_tiles > 0x7FFFFFFFull)
            return HU_ERR_INVALID_ARGUMENT;
        grid_ll = n_tiles ? n_tiles : 1;
    } else {
        const int max_blocks = max_resident_blocks(kc.fn, kc.groups_per_cu, &pad);
        if (max_blocks <= 0)
            return HU_ERR_DEVICE;
        grid_ll = n_tiles == 0 ? 1ull : (n_tiles < (unsigned long long)max_blocks ? n_tiles : max_blocks);
    }
    const unsigned int grid = (unsigned int)grid_ll;
    const uint8_t *base = (const uint8_t *)((uintptr_t)src & ~(uintptr_t)15);
    const unsigned long long off_b = (unsigned long long)((uintptr_t)src & 15u);
    Doc doc{base, off_b, off_b + (u16 ? 2 * n : n), n, dst, cap};
    unsigned long long n_tiles_arg = n_tiles;
    void *args[] = {&doc, &n_tiles_arg, &hdr, &status, &status_cap, &d_result};
    if (hipLaunchKernel(kc.fn, dim3(grid), dim3(kBlock), args, pad, stream) != hipSuccess)
        return HU_ERR_DEVICE;
    return HU_OK;
}

// ------------------------------------------------------------ batches
constexpr unsigned int kBatchDefaultU = 2;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct BatchLayout {
    size_t first, err, map, status, block, total;
    unsigned long long item_cap;
    unsigned int n_blocks;   // blocks of documents for planning
};

BatchLayout batch_layout(uint32_t n_docs, uint64_t total_input_bytes)
{
    BatchLayout l;
    // the smallest tile is one 4 KiB sub-tile; each document adds at most two
    // partial tiles (alignment offset and tail), a small document one item
    l.item_cap = total_input_bytes / kSub + 2ull * n_docs + 1;
    l.status = kHeaderBytes;
    l.first = align256(l.status + 8ull * l.item_cap);
    l.err = align256(l.first + 4ull * n_docs);
    l.map = align256(l.err + 8ull * n_docs);
    l.block = align256(l.map + sizeof(BatchItem) * l.item_cap);
    l.n_blocks = (unsigned int)((n_docs + kPlanBlock - 1ull) / kPlanBlock);
    l.total = align256(l.block + 8ull * kCounts * l.n_blocks);
    return l;
}

// Sub-tiles per tile item that the batch kernel is built for.
bool batch_sub_tiles_ok(unsigned int U) { return U == 1 || U == 2 || U == 4 || U == 6; }

const void *batch_run_kernel(unsigned int U)
{
#define HU_K(...) reinterpret_cast<const void *>(&__VA_ARGS__)
    return U == 1 ? HU_K(k_batch_run<1>) : U == 2 ? HU_K(k_batch_run<2>) : U == 4 ? HU_K(k_batch_run<4>)
                                                                                 : HU_K(k_batch_run<6>);
#undef HU_K
}

// Dynamic LDS that leaves room for at most `groups_per_cu` workgroups of the
// kernel per CU (0: none requested, occupancy set by the kernel's resources).
size_t lds_pad(const void *fn, unsigned int groups_per_cu)
{
    if (groups_per_cu == 0)
        return 0;
    int dev = 0, per_cu = 0, per_block = 0;
    hipFuncAttributes fa;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        hipFuncGetAttributes(&fa, fn) != hipSuccess || per_cu <= 0)
        return 0;
    const size_t fixed = fa.sharedSizeBytes;
    size_t want = (size_t)per_cu / groups_per_cu;
    want = want > 1024 ? want - 1024 : want;          // allocation granularity slack
    if (want > (size_t)per_block)
        want = (size_t)per_block;
    return want > fixed ? want - fixed : 0;
}

int batch_enqueue(const hu_doc *docs, uint32_t n_docs, uint64_t total_input_bytes, const void *src_base,
                  void *dst_base, hu_result *results, const hu_tuning *tuning, void *ws, size_t ws_bytes,
                  hipStream_t stream)
{
    if (n_docs == 0)
        return HU_OK;
    if (docs == nullptr || results == nullptr || ws == nullptr || ((uintptr_t)ws & 255u) != 0)
        return HU_ERR_INVALID_ARGUMENT;
    const BatchLayout l = batch_layout(n_docs, total_input_bytes);
    if (ws_bytes < l.total || l.item_cap >= 0x7FFFFFFFull)
        return HU_ERR_INVALID_ARGUMENT;
    const unsigned int U = (tuning && tuning->sub_tiles) ? tuning->sub_tiles : kBatchDefaultU;
    if (!batch_sub_tiles_ok(U))
        return HU_ERR_INVALID_ARGUMENT;
    char *base = reinterpret_cast<char *>(ws);
    BatchWs w{reinterpret_cast<BatchHeader *>(base), reinterpret_cast<unsigned int *>(base + l.first),
              reinterpret_cast<unsigned long long *>(base + l.err),
              reinterpret_cast<BatchItem *>(base + l.map),
              reinterpret_cast<unsigned long long *>(base + l.status),
              reinterpret_cast<unsigned long long *>(base + l.block), l.item_cap};
    const BatchDoc *bd = reinterpret_cast<const BatchDoc *>(docs);
    const uint8_t *src = reinterpret_cast<const uint8_t *>(src_base);
    uint8_t *dst = reinterpret_cast<uint8_t *>(dst_base);
    const unsigned long long tile_bytes = (unsigned long long)U * kSub;

    if (l.n_blocks == 1) {
        hipLaunchKernelGGL(k_batch_plan1, dim3(1), dim3(kPlanBlock), 0, stream, bd, n_docs, src,
                           (const uint8_t *)dst, results, w, tile_bytes);
    } else {
        hipLaunchKernelGGL(k_batch_count, dim3(l.n_blocks), dim3(kPlanBlock), 0, stream, bd, n_docs, src,
                           (const uint8_t *)dst, w, tile_bytes);
        hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(kPlanBlock), 0, stream, l.n_blocks, w);
        hipLaunchKernelGGL(k_batch_assign, dim3(l.n_blocks), dim3(kPlanBlock), 0, stream, bd, n_docs, src,
                           (const uint8_t *)dst, results, w, tile_bytes);
    }
    // enough workgroups for the documents and for clearing the status array
    unsigned long long fill_grid = (n_docs + 255) / 256;
    if (fill_grid < (l.item_cap + 4095) / 4096)
        fill_grid = (l.item_cap + 4095) / 4096;
    fill_grid = fill_grid < 2048 ? fill_grid : 2048;
    hipLaunchKernelGGL(k_batch_fill, dim3((unsigned int)fill_grid), dim3(256), 0, stream, bd, n_docs, src, w,
                       tile_bytes);
    // Workgroups for upper bounds on the tile items at this tile size and on
    // the small documents (the plan may need fewer: surplus workgroups leave
    // at once). A launch holds at most 2^32 - 1 work-items, so more
    // workgroups take several launches in order.
    const unsigned long long items = total_input_bytes / tile_bytes + 2ull * n_docs + 1;
    const unsigned long long groups = items + ((unsigned long long)n_docs + kWaves - 1) / kWaves;
    constexpr unsigned long long kMaxGrid = 0xFFFFFFFFull / kBlock;
    const void *fn = batch_run_kernel(U);
    const size_t pad = lds_pad(fn, tuning ? tuning->groups_per_cu : 0);
    for (unsigned long long base = 0; base < groups; base += kMaxGrid) {
        const unsigned long long grid = groups - base < kMaxGrid ? groups - base : kMaxGrid;
        void *args[] = {&src, &dst, &results, &w, &base};
        if (hipLaunchKernel(fn, dim3((unsigned int)grid), dim3(kBlock), args, pad, stream) != hipSuccess)
            return HU_ERR_DEVICE;
    }
    return hipGetLastError() == hipSuccess ? HU_OK : HU_ERR_DEVICE;
}

// ------------------------------------------------------------ tuning cache
std::string device_tag()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s/%d", prop.gcnArchName, prop.multiProcessorCount);
    for (char *c = buf; *c; ++c)
        if (*c == '"' || *c == '\\')
            *c = '_';
    return buf;
}

// value of "name": in a JSON line written by tune_store (string or integer)
bool json_field(const std::string &line, const char *name, std::string *out)
{
    const std::string pat = std::string("\"") + name + "\": ";
    size_t p = line.find(pat);
    if (p == std::string::npos)
        return false;
    p += pat.size();
    if (p < line.size() && line[p] == '"') {
        const size_t q = line.find('"', p + 1);
        if (q == std::string::npos)
            return false;
        *out = line.substr(p + 1, q - p - 1);
        return true;
    }
    size_t q = p;
    while (q < line.size() && line[q] != ',' && line[q] != '}')
        ++q;
    *out = line.substr(p, q - p);
    return true;
}

// ------------------------------------------------------------ synchronous path
struct StreamSlot {
    std::mutex mu;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    hu_result *h_result = nullptr;   // pinned host memory the kernel writes the result to
    hu_result *h_result_dev = nullptr;   // its device address
};

std::mutex g_slots_mu;
std::map<std::pair<int, hipStream_t>, StreamSlot *> g_slots;

StreamSlot *slot_for(hipStream_t stream)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_slots_mu);
    StreamSlot *&s = g_slots[std::make_pair(dev, stream)];
    if (s == nullptr)
        s = new StreamSlot();
    return s;
}

hu_result make_result(int error, unsigned long long count)
{
    hu_result r;
    r.error = error;
    r.reserved = 0;
    r.count = count;
    return r;
}

hu_result run_sync(int op, const void *src, unsigned long long n, void *dst, unsigned long long cap,
                   hipStream_t stream)
{
    const int base_op = op & ~kOpFlags;
    const bool u16 = base_op >= HU_OP_VALIDATE_UTF16LE;
    if (n > kMaxUnits || (n > 0 && src == nullptr) || (cap > 0 && dst == nullptr) ||
        (u16 && ((uintptr_t)src & 1u)) || (base_op == HU_OP_CONVERT_UTF8_TO_UTF16LE && ((uintptr_t)dst & 1u)))
        return make_result(HU_ERR_INVALID_ARGUMENT, 0);
    if (n == 0)
        return make_result(HU_OK, 0);
    StreamSlot *slot = slot_for(stream);
    if (slot == nullptr)
        return make_result(HU_ERR_DEVICE, 0);
    std::lock_guard<std::mutex> lk(slot->mu);
    const size_t need = workspace_need(op, src, n);
    if (slot->h_result == nullptr) {
        // the result goes straight to pinned host memory: no device-to-host
        // copy after the kernel
        hu_result *h = nullptr;
        if (hipHostMalloc((void **)&h, sizeof(hu_result), hipHostMallocDefault) != hipSuccess)
            return make_result(HU_ERR_DEVICE, 0);
        if (hipHostGetDevicePointer((void **)&slot->h_result_dev, h, 0) != hipSuccess) {
            (void)hipHostFree(h);
            return make_result(HU_ERR_DEVICE, 0);
        }
        slot->h_result = h;
    }
    if (slot->ws_bytes < need) {
        // the old workspace may still be in use by work queued on this stream
        if (slot->ws != nullptr) {
            if (hipStreamSynchronize(stream) != hipSuccess)
                return make_result(HU_ERR_DEVICE, 0);
            (void)hipFree(slot->ws);
            slot->ws = nullptr;
            slot->ws_bytes = 0;
        }
        size_t bytes = need + need / 4;
        if (hipMalloc(&slot->ws, bytes) != hipSuccess || hipMemset(slot->ws, 0, bytes) != hipSuccess) {
            slot->ws = nullptr;
            return make_result(HU_ERR_DEVICE, 0);
        }
        slot->ws_bytes = bytes;
    }
    const int rc = enqueue(op, src, n, dst, cap, slot->h_result_dev, slot->ws, slot->ws_bytes, stream);
    if (rc != HU_OK)
        return make_result(rc, 0);
    if (hipStreamSynchronize(stream) != hipSuccess)
        return make_result(HU_ERR_DEVICE, 0);
    const volatile hu_result *r = slot->h_result;
    return make_result(r->error, r->count);
}

// ------------------------------------------------------------ static scratch
// Workspace of convert_utf8_to_utf16le_noalloc: a file-scope device array
// (one per device, each at its own address) sized for the largest input it
// takes. In host code `scratch` names a host-side stand-in, never the device
// memory: kernels get the address hipGetSymbolAddress returns for the current
// device, looked up once per device.
constexpr unsigned long long kNoAllocMaxBytes = HU_NOALLOC_MAX_BYTES;
constexpr size_t kScratchBytes = 1536u << 10;
static_assert(kHeaderBytes + 8ull * kStatusStride * class_max_tiles(kConvert8Classes, kNoAllocMaxBytes, kSub) <=
                  kScratchBytes,
              "scratch holds the status words of any input the entry point takes");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];   // device address of `scratch`, per device (null: not set up)

// The current device's scratch address; on the first call on a device, looks
// it up and clears the array with a kernel on `stream`. Null on failure.
void *scratch_for_current_device(hipStream_t stream)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
            return nullptr;
        unsigned int *words = reinterpret_cast<unsigned int *>(p);
        unsigned long long n_words = kScratchBytes / 4;
        void *args[] = {&words, &n_words};
        if (hipLaunchKernel(reinterpret_cast<const void *>(&k_fill_zero), dim3(256), dim3(256), args, 0, stream) !=
            hipSuccess)
            return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace hu

// ------------------------------------------------------------ C ABI
using hu::run_sync;

extern "C" {

hu_result validate_utf8(const uint8_t *src, size_t n_bytes, void *stream)
{
    return run_sync(HU_OP_VALIDATE_UTF8, src, n_bytes, nullptr, 0, (hipStream_t)stream);
}

hu_result utf16_length_from_utf8(const uint8_t *src, size_t n_bytes, void *stream)
{
    return run_sync(HU_OP_UTF16_LENGTH_FROM_UTF8, src, n_bytes, nullptr, 0, (hipStream_t)stream);
}

hu_result convert_utf8_to_utf16le(const uint8_t *src, size_t n_bytes, uint16_t *dst, size_t dst_cap_words,
                                  void *stream)
{
    return run_sync(HU_OP_CONVERT_UTF8_TO_UTF16LE, src, n_bytes, dst, dst_cap_words, (hipStream_t)stream);
}

hu_result validate_utf16le(const uint16_t *src, size_t n_words, void *stream)
{
    return run_sync(HU_OP_VALIDATE_UTF16LE, src, n_words, nullptr, 0, (hipStream_t)stream);
}

hu_result utf8_length_from_utf16le(const uint16_t *src, size_t n_words, void *stream)
{
    return run_sync(HU_OP_UTF8_LENGTH_FROM_UTF16LE, src, n_words, nullptr, 0, (hipStream_t)stream);
}

hu_result convert_utf16le_to_utf8(const uint16_t *src, size_t n_words, uint8_t *dst, size_t dst_cap_bytes,
                                  void *stream)
{
    return run_sync(HU_OP_CONVERT_UTF16LE_TO_UTF8, src, n_words, dst, dst_cap_bytes, (hipStream_t)stream);
}

hu_result convert_valid_utf8_to_utf16le(const uint8_t *src, size_t n_bytes, uint16_t *dst, size_t dst_cap_words,
                                         void *stream)
{
    return run_sync(HU_OP_CONVERT_UTF8_TO_UTF16LE | hu::kTrustedOp, src, n_bytes, dst, dst_cap_words,
                    (hipStream_t)stream);
}

hu_result convert_valid_utf16le_to_utf8(const uint16_t *src, size_t n_words, uint8_t *dst, size_t dst_cap_bytes,
                                         void *stream)
{
    return run_sync(HU_OP_CONVERT_UTF16LE_TO_UTF8 | hu::kTrustedOp, src, n_words, dst, dst_cap_bytes,
                    (hipStream_t)stream);
}

hu_result validate_utf16be(const uint16_t *src, size_t n_words, void *stream)
{
    return run_sync(HU_OP_VALIDATE_UTF16LE | hu::kBigEndianOp, src, n_words, nullptr, 0, (hipStream_t)stream);
}

hu_result utf8_length_from_utf16be(const uint16_t *src, size_t n_words, void *stream)
{
    return run_sync(HU_OP_UTF8_LENGTH_FROM_UTF16LE | hu::kBigEndianOp, src, n_words, nullptr, 0,
                    (hipStream_t)stream);
}

hu_result convert_utf16be_to_utf8(const uint16_t *src, size_t n_words, uint8_t *dst, size_t dst_cap_bytes,
                                  void *stream)
{
    return run_sync(HU_OP_CONVERT_UTF16LE_TO_UTF8 | hu::kBigEndianOp, src, n_words, dst, dst_cap_bytes,
                    (hipStream_t)stream);
}

hu_result convert_utf8_to_utf16be(const uint8_t *src, size_t n_bytes, uint16_t *dst, size_t dst_cap_words,
                                  void *stream)
{
    return run_sync(HU_OP_CONVERT_UTF8_TO_UTF16LE | hu::kBigEndianOp, src, n_bytes, dst, dst_cap_words,
                    (hipStream_t)stream);
}

hu_bom hu_detect_bom(const uint8_t *head, size_t n_bytes)
{
    hu_bom b{HU_BOM_NONE, 0};
    if (head == nullptr)
        return b;
    if (n_bytes >= 3 && head[0] == 0xEF && head[1] == 0xBB && head[2] == 0xBF)
        b = {HU_BOM_UTF8, 3};
    else if (n_bytes >= 2 && head[0] == 0xFF && head[1] == 0xFE)
        b = {HU_BOM_UTF16LE, 2};
    else if (n_bytes >= 2 && head[0] == 0xFE && head[1] == 0xFF)
        b = {HU_BOM_UTF16BE, 2};
    return b;
}

size_t hu_workspace_bytes(int op, size_t n_units)
{
    if (op < 0 || op > HU_OP_CONVERT_UTF16LE_TO_UTF8)
        return 0;
    // worst case over source alignments: 15 bytes of offset
    const unsigned long long bytes = op >= HU_OP_VALIDATE_UTF16LE ? 2ull * n_units : n_units;
    // validate / length keep no status words; a conversion needs one per tile
    // of the most tiles any input of at most n units takes (smaller inputs
    // take smaller tiles)
    if (!hu::choose_kernel(op, 0).one_group_per_tile)
        return hu::kHeaderBytes;
    const unsigned long long tiles = op == HU_OP_CONVERT_UTF8_TO_UTF16LE
                                         ? hu::class_max_tiles(hu::kConvert8Classes, bytes, hu::kSub)
                                         : hu::class_max_tiles(hu::kConvert16Classes, bytes, hu::kSub);
    return hu::kHeaderBytes + 8ull * hu::kStatusStride * tiles;
}

size_t hu_tile_bytes(int op, size_t n_units)
{
    if (op < 0 || op > HU_OP_CONVERT_UTF16LE_TO_UTF8)
        return 0;
    const unsigned long long bytes = op >= HU_OP_VALIDATE_UTF16LE ? 2ull * n_units : n_units;
    return hu::choose_kernel(op, bytes).tile_bytes;
}

int hu_workspace_init(void *ws, size_t ws_bytes, void *stream)
{
    if (ws == nullptr || ((uintptr_t)ws & 255u) != 0 || ws_bytes < hu::kHeaderBytes)
        return HU_ERR_INVALID_ARGUMENT;
    const unsigned long long words = ws_bytes / 4;
    const unsigned int grid = (unsigned int)((words + 255) / 256 < 1024 ? (words + 255) / 256 : 1024);
    hipLaunchKernelGGL(hu::k_fill_zero, dim3(grid), dim3(256), 0, (hipStream_t)stream, (unsigned int *)ws, words);
    return hipGetLastError() == hipSuccess ? HU_OK : HU_ERR_DEVICE;
}

int validate_utf8_async(const uint8_t *src, size_t n_bytes, hu_result *d_result, void *ws, size_t ws_bytes,
                        void *stream)
{
    return hu::enqueue(HU_OP_VALIDATE_UTF8, src, n_bytes, nullptr, 0, d_result, ws, ws_bytes, (hipStream_t)stream);
}

int utf16_length_from_utf8_async(const uint8_t *src, size_t n_bytes, hu_result *d_result, void *ws,
                                 size_t ws_bytes, void *stream)
{
    return hu::enqueue(HU_OP_UTF16_LENGTH_FROM_UTF8, src, n_bytes, nullptr, 0, d_result, ws, ws_bytes,
                       (hipStream_t)stream);
}

int convert_utf8_to_utf16le_async(const uint8_t *src, size_t n_bytes, uint16_t *dst, size_t dst_cap_words,
                                  hu_result *d_result, void *ws, size_t ws_bytes, void *stream)
{
    return hu::enqueue(HU_OP_CONVERT_UTF8_TO_UTF16LE, src, n_bytes, dst, dst_cap_words, d_result, ws, ws_bytes,
                       (hipStream_t)stream);
}

int validate_utf16le_async(const uint16_t *src, size_t n_words, hu_result *d_result, void *ws, size_t ws_bytes,
                           void *stream)
{
    return hu::enqueue(HU_OP_VALIDATE_UTF16LE, src, n_words, nullptr, 0, d_result, ws, ws_bytes,
                       (hipStream_t)stream);
}

int utf8_length_from_utf16le_async(const uint16_t *src, size_t n_words, hu_result *d_result, void *ws,
                                   size_t ws_bytes, void *stream)
{
    return hu::enqueue(HU_OP_UTF8_LENGTH_FROM_UTF16LE, src, n_words, nullptr, 0, d_result, ws, ws_bytes,
                       (hipStream_t)stream);
}

int convert_utf16le_to_utf8_async(const uint16_t *src, size_t n_words, uint8_t *dst, size_t dst_cap_bytes,
                                  hu_result *d_result, void *ws, size_t ws_bytes, void *stream)
{
    return hu::enqueue(HU_OP_CONVERT_UTF16LE_TO_UTF8, src, n_words, dst, dst_cap_bytes, d_result, ws, ws_bytes,
                       (hipStream_t)stream);
}

int convert_valid_utf8_to_utf16le_async(const uint8_t *src, size_t n_bytes, uint16_t *dst, size_t dst_cap_words,
                                        hu_result *d_result, void *ws, size_t ws_bytes, void *stream)
{
    return hu::enqueue(HU_OP_CONVERT_UTF8_TO_UTF16LE | hu::kTrustedOp, src, n_bytes, dst, dst_cap_words, d_result,
                       ws, ws_bytes, (hipStream_t)stream);
}

int convert_valid_utf16le_to_utf8_async(const uint16_t *src, size_t n_words, uint8_t *dst, size_t dst_cap_bytes,
                                        hu_result *d_result, void *ws, size_t ws_bytes, void *stream)
{
    return hu::enqueue(HU_OP_CONVERT_UTF16LE_TO_UTF8 | hu::kTrustedOp, src, n_words, dst, dst_cap_bytes, d_result,
                       ws, ws_bytes, (hipStream_t)stream);
}

int validate_utf16be_async(const uint16_t *src, size_t n_words, hu_result *d_result, void *ws, size_t ws_bytes,
                           void *stream)
{
    return hu::enqueue(HU_OP_VALIDATE_UTF16LE | hu::kBigEndianOp, src, n_words, nullptr, 0, d_result, ws, ws_bytes,
                       (hipStream_t)stream);
}

int utf8_length_from_utf16be_async(const uint16_t *src, size_t n_words, hu_result *d_result, void *ws,
                                   size_t ws_bytes, void *stream)
{
    return hu::enqueue(HU_OP_UTF8_LENGTH_FROM_UTF16LE | hu::kBigEndianOp, src, n_words, nullptr, 0, d_result, ws,
                       ws_bytes, (hipStream_t)stream);
}

int convert_utf16be_to_utf8_async(const uint16_t *src, size_t n_words, uint8_t *dst, size_t dst_cap_bytes,
                                  hu_result *d_result, void *ws, size_t ws_bytes, void *stream)
{
    return hu::enqueue(HU_OP_CONVERT_UTF16LE_TO_UTF8 | hu::kBigEndianOp, src, n_words, dst, dst_cap_bytes, d_result,
                       ws, ws_bytes, (hipStream_t)stream);
}

int convert_utf8_to_utf16be_async(const uint8_t *src, size_t n_bytes, uint16_t *dst, size_t dst_cap_words,
                                  hu_result *d_result, void *ws, size_t ws_bytes, void *stream)
{
    return hu::enqueue(HU_OP_CONVERT_UTF8_TO_UTF16LE | hu::kBigEndianOp, src, n_bytes, dst, dst_cap_words, d_result,
                       ws, ws_bytes, (hipStream_t)stream);
}

int convert_utf8_to_utf16le_noalloc(const uint8_t *src, size_t n_bytes, uint16_t *dst, size_t dst_cap_words,
                                    hu_result *d_result, void *stream)
{
    if (n_bytes > hu::kNoAllocMaxBytes)
        return HU_ERR_EXCEEDS_SCRATCH;
    void *ws = hu::scratch_for_current_device((hipStream_t)stream);
    if (ws == nullptr)
        return HU_ERR_DEVICE;
    return hu::enqueue(HU_OP_CONVERT_UTF8_TO_UTF16LE, src, n_bytes, dst, dst_cap_words, d_result, ws,
                       hu::kScratchBytes, (hipStream_t)stream);
}

size_t hu_batch_workspace_bytes(uint32_t n_docs, uint64_t total_input_bytes)
{
    return hu::batch_layout(n_docs, total_input_bytes).total;
}

int hu_batch_run(const hu_doc *docs, uint32_t n_docs, uint64_t total_input_bytes, const void *src_base,
                 void *dst_base, hu_result *results, const hu_tuning *tuning, void *ws, size_t ws_bytes, void *stream)
{
    return hu::batch_enqueue(docs, n_docs, total_input_bytes, src_base, dst_base, results, tuning, ws, ws_bytes,
                             (hipStream_t)stream);
}

int hu_batch_graph_create(const hu_doc *docs, uint32_t n_docs, uint64_t total_input_bytes, const void *src_base,
                          void *dst_base, hu_result *results, const hu_tuning *tuning, void *ws, size_t ws_bytes,
                          void **graph_exec)
{
    if (graph_exec == nullptr)
        return HU_ERR_INVALID_ARGUMENT;
    *graph_exec = nullptr;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        return HU_ERR_DEVICE;
    int rc = HU_OK;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        rc = HU_ERR_DEVICE;
    } else {
        rc = hu::batch_enqueue(docs, n_docs, total_input_bytes, src_base, dst_base, results, tuning, ws, ws_bytes, s);
        if (hipStreamEndCapture(s, &g) != hipSuccess && rc == HU_OK)
            rc = HU_ERR_DEVICE;
    }
    if (rc == HU_OK && g != nullptr) {
        hipGraphExec_t e = nullptr;
        if (hipGraphInstantiate(&e, g, nullptr, nullptr, 0) != hipSuccess)
            rc = HU_ERR_DEVICE;
        else
            *graph_exec = (void *)e;
    }
    if (g != nullptr)
        (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(s);
    return rc;
}

int hu_graph_launch(void *graph_exec, void *stream)
{
    if (graph_exec == nullptr)
        return HU_ERR_INVALID_ARGUMENT;
    return hipGraphLaunch((hipGraphExec_t)graph_exec, (hipStream_t)stream) == hipSuccess ? HU_OK : HU_ERR_DEVICE;
}

void hu_graph_destroy(void *graph_exec)
{
    if (graph_exec != nullptr)
        (void)hipGraphExecDestroy((hipGraphExec_t)graph_exec);
}

int hu_tune_batch(const hu_doc *docs, uint32_t n_docs, uint64_t total_input_bytes, const void *src_base,
                  void *dst_base, hu_result *results, void *ws, size_t ws_bytes, const char *key, hu_tuning *best,
                  double *best_us, void *stream)
{
    if (best == nullptr || best_us == nullptr)
        return HU_ERR_INVALID_ARGUMENT;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return HU_ERR_DEVICE;
    const unsigned int subs[] = {1, 2, 4, 6};
    const unsigned int gpcs[] = {2, 4, 6, 0};
    const int reps = 3;
    double best_t = 1e300;
    hu_tuning bt{hu::kBatchDefaultU, 0};
    int rc = HU_OK;
    for (unsigned int u : subs) {
        for (unsigned int g : gpcs) {
            const hu_tuning t{u, g};
            rc = hu::batch_enqueue(docs, n_docs, total_input_bytes, src_base, dst_base, results, &t, ws, ws_bytes, st);
            if (rc != HU_OK)
                break;
            (void)hipEventRecord(e0, st);
            for (int r = 0; r < reps && rc == HU_OK; ++r)
                rc = hu::batch_enqueue(docs, n_docs, total_input_bytes, src_base, dst_base, results, &t, ws, ws_bytes,
                                       st);
            (void)hipEventRecord(e1, st);
            float ms = 0.f;
            if (rc != HU_OK || hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                rc = rc != HU_OK ? rc : HU_ERR_DEVICE;
                break;
            }
            const double us = 1000.0 * ms / reps;
            if (us < best_t) {
                best_t = us;
                bt = t;
            }
        }
        if (rc != HU_OK)
            break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != HU_OK)
        return rc;
    *best = bt;
    *best_us = best_t;
    const char *path = std::getenv("HIPUTF_TUNE_CACHE");
    if (key != nullptr && path != nullptr && *path) {
        std::string k(key);
        for (char &c : k)
            if (c == '"' || c == '\\')
                c = '_';
        if (FILE *f = std::fopen(path, "a")) {
            std::fprintf(f, "{\"key\": \"%s\", \"device\": \"%s\", \"sub_tiles\": %u, \"groups_per_cu\": %u, \"us\": %.3f}\n",
                         k.c_str(), hu::device_tag().c_str(), bt.sub_tiles, bt.groups_per_cu, best_t);
            std::fclose(f);
        }
    }
    return HU_OK;
}

int hu_tuning_lookup(const char *key, hu_tuning *out)
{
    const char *path = std::getenv("HIPUTF_TUNE_CACHE");
    if (key == nullptr || out == nullptr || path == nullptr || !*path)
        return HU_ERR_INVALID_ARGUMENT;
    FILE *f = std::fopen(path, "r");
    if (f == nullptr)
        return HU_ERR_INVALID_ARGUMENT;
    const std::string dev = hu::device_tag();
    char buf[1024];
    bool found = false;
    hu_tuning t{0, 0};
    while (std::fgets(buf, sizeof buf, f)) {
        const std::string line(buf);
        std::string k, d, su, gp;
        if (hu::json_field(line, "key", &k) && hu::json_field(line, "device", &d) && k == key && d == dev &&
            hu::json_field(line, "sub_tiles", &su) && hu::json_field(line, "groups_per_cu", &gp)) {
            t.sub_tiles = (uint32_t)std::strtoul(su.c_str(), nullptr, 10);
            t.groups_per_cu = (uint32_t)std::strtoul(gp.c_str(), nullptr, 10);
            found = true;   // the last matching line wins
        }
    }
    std::fclose(f);
    if (!found || !hu::batch_sub_tiles_ok(t.sub_tiles))
        return HU_ERR_INVALID_ARGUMENT;
    *out = t;
    return HU_OK;
}

const char *hu_error_name(int error)
{
    switch (error) {
    case HU_OK: return "OK";
    case HU_ERR_BAD_LEAD: return "BAD_LEAD";
    case HU_ERR_TRUNCATED: return "TRUNCATED";
    case HU_ERR_STRAY_CONTINUATION: return "STRAY_CONTINUATION";
    case HU_ERR_OVERLONG: return "OVERLONG";
    case HU_ERR_TOO_LARGE: return "TOO_LARGE";
    case HU_ERR_SURROGATE: return "SURROGATE";
    case HU_ERR_UNPAIRED_SURROGATE: return "UNPAIRED_SURROGATE";
    case HU_ERR_OUTPUT_TOO_SMALL: return "OUTPUT_TOO_SMALL";
    case HU_ERR_INVALID_ARGUMENT: return "INVALID_ARGUMENT";
    case HU_ERR_DEVICE: return "DEVICE";
    case HU_ERR_EXCEEDS_SCRATCH: return "EXCEEDS_SCRATCH";
    default: return "UNKNOWN";
    }
}

void hu_shutdown(void)
{
    std::lock_guard<std::mutex> lk(hu::g_slots_mu);
    for (auto &kv : hu::g_slots) {
        hu::StreamSlot *s = kv.second;
        std::lock_guard<std::mutex> lk2(s->mu);
        int prev = 0;
        (void)hipGetDevice(&prev);
        if (hipSetDevice(kv.first.first) == hipSuccess) {
            (void)hipDeviceSynchronize();
            if (s->ws) (void)hipFree(s->ws);
            if (s->h_result) (void)hipHostFree(s->h_result);
        }
        (void)hipSetDevice(prev);
        s->ws = nullptr;
        s->h_result = nullptr;
        s->h_result_dev = nullptr;
        s->ws_bytes = 0;
    }
}

}  // extern "C"
