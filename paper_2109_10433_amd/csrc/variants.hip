// variants.hip - kernels of the operation variants: conversions of input
// known to be valid (no validation step), and UTF-16 big endian (every UTF-16
// word byte swapped on load or store). Same engine as the plain operations.
#include <hip/hip_runtime.h>

#include "engine.hpp"
#include "kernel_choice.hpp"

namespace hu {

// Tile sizes by input size as for the plain conversions (kConvert8Classes,
// kConvert16Classes), so that a variant takes the workspace of its plain
// operation.
template <int MODE, bool SWAP>
const void *convert8_kernel(int u)
{
#define HU_K(...) reinterpret_cast<const void *>(&__VA_ARGS__)
    return u == 1 ? HU_K(k_convert_u8<1, MODE, SWAP>) : u == 2 ? HU_K(k_convert_u8<2, MODE, SWAP>)
         : u == 5 ? HU_K(k_convert_u8<5, MODE, SWAP>) : HU_K(k_convert_u8<6, MODE, SWAP>);
#undef HU_K
}

template <int MODE, bool SWAP>
const void *convert16_kernel(int u)
{
#define HU_K(...) reinterpret_cast<const void *>(&__VA_ARGS__)
    return u == 1 ? HU_K(k_convert_u16<1, MODE, SWAP>) : u == 2 ? HU_K(k_convert_u16<2, MODE, SWAP>)
                  : HU_K(k_convert_u16<6, MODE, SWAP>);
#undef HU_K
}

bool choose_variant(int op, unsigned long long n_bytes, KernelChoice &kc)
{
#define HU_K(...) reinterpret_cast<const void *>(&__VA_ARGS__)
    const int u8 = class_sub_tiles(kConvert8Classes, n_bytes), u16 = class_sub_tiles(kConvert16Classes, n_bytes);
    const unsigned long long t8 = (unsigned long long)u8 * kSub, t16 = (unsigned long long)u16 * kSub;
    constexpr unsigned long long tv = kPValidate16 * kPieceBytes;
    constexpr unsigned long long tl = kPLength16 * kPieceBytes;
    switch (op) {
    case HU_OP_CONVERT_UTF8_TO_UTF16LE | kTrustedOp: kc = {convert8_kernel<kTrusted, false>(u8), t8, true}; return true;
    case HU_OP_CONVERT_UTF16LE_TO_UTF8 | kTrustedOp: kc = {convert16_kernel<kTrusted, false>(u16), t16, true}; return true;
    case HU_OP_CONVERT_UTF8_TO_UTF16LE | kBigEndianOp: kc = {convert8_kernel<kConvert, true>(u8), t8, true}; return true;
    case HU_OP_CONVERT_UTF16LE_TO_UTF8 | kBigEndianOp: kc = {convert16_kernel<kConvert, true>(u16), t16, true}; return true;
    case HU_OP_VALIDATE_UTF16LE | kBigEndianOp: kc = {HU_K(k_scan<U16Dir, kValidate, kPValidate16, true>), tv, false}; return true;
    case HU_OP_UTF8_LENGTH_FROM_UTF16LE | kBigEndianOp:
        kc = {HU_K(k_scan<U16Dir, kLength, kPLength16, true>), tl, false, kLength16GroupsPerCu};
        return true;
    default: return false;
    }
#undef HU_K
}

}  // namespace hu
