// variants.hip - kernels of the operation variants: conversions of input
// known to be valid (no validation step), and UTF-16 big endian (every UTF-16
// word byte swapped on load or store). Same engine as the plain operations.
#include <hip/hip_runtime.h>

#include "engine.hpp"
#include "kernel_choice.hpp"

namespace hu {

bool choose_variant(int op, KernelChoice &kc)
{
#define HU_K(...) reinterpret_cast<const void *>(&__VA_ARGS__)
    constexpr unsigned long long t8 = (unsigned long long)kUConvert8 * kSub;
    constexpr unsigned long long t16 = (unsigned long long)kUConvert16 * kSub;
    constexpr unsigned long long tv = kPValidate16 * kPieceBytes;
    constexpr unsigned long long tl = kPLength16 * kPieceBytes;
    switch (op) {
    case HU_OP_CONVERT_UTF8_TO_UTF16LE | kTrustedOp: kc = {HU_K(k_convert_u8<kUConvert8, kTrusted>), t8, true}; return true;
    case HU_OP_CONVERT_UTF16LE_TO_UTF8 | kTrustedOp: kc = {HU_K(k_convert_u16<kUConvert16, kTrusted>), t16, true}; return true;
    case HU_OP_CONVERT_UTF8_TO_UTF16LE | kBigEndianOp: kc = {HU_K(k_convert_u8<kUConvert8, kConvert, true>), t8, true}; return true;
    case HU_OP_CONVERT_UTF16LE_TO_UTF8 | kBigEndianOp: kc = {HU_K(k_convert_u16<kUConvert16, kConvert, true>), t16, true}; return true;
    case HU_OP_VALIDATE_UTF16LE | kBigEndianOp: kc = {HU_K(k_scan<U16Dir, kValidate, kPValidate16, true>), tv, false}; return true;
    case HU_OP_UTF8_LENGTH_FROM_UTF16LE | kBigEndianOp: kc = {HU_K(k_scan<U16Dir, kLength, kPLength16, true>), tl, false}; return true;
    default: return false;
    }
#undef HU_K
}

}  // namespace hu
