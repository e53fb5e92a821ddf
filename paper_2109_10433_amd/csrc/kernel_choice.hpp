// kernel_choice.hpp - which kernel runs an operation, and its tile size.
//
// The plain operations' kernels are instantiated in hiputf.hip; the variants
// (conversions without validation, big-endian UTF-16) in variants.hip, a
// translation unit of their own, so that adding them leaves the code
// generated for the plain kernels unchanged.
#pragma once

namespace hu {

// Convert tiles: sub-tiles of 4 KiB per tile (one per workgroup); bigger
// tiles mean fewer look-backs per byte, more registers fewer waves per SIMD.
// Measured: UTF-8 input is fastest at 6 (68 registers, seven waves per SIMD;
// 5 fits eight waves but leaves one- and two-byte text 5 % slower, 7 and 8
// slow down three- and four-byte text); UTF-16 input at 6 (64 registers; 8
// and 10 are far slower).
constexpr int kUConvert8 = 6;
// UTF-8 -> UTF-16LE inputs below kSmallConvert8Bytes take the 5 sub-tile
// kernel instead: there more, shorter tiles spread a small input over more of
// the chip (1 MiB: 13 instead of 16 us).
constexpr int kUConvert8Small = 5;
constexpr unsigned long long kSmallConvert8Bytes = 64ull << 20;
constexpr int kUConvert16 = 6;
// Validate / length: pieces of 1 KiB (one 16-byte load per lane) per
// wave-tile, the unit a wave works on alone; a wave analyses one wave-tile
// while the loads of its next one are in flight. Measured (P = 1..4 pieces):
// two pieces are fastest for both validations and UTF-8 length, four for
// UTF-16 length (three within 0.1 %).
#ifndef HU_P_VALIDATE8
#define HU_P_VALIDATE8 2
#endif
#ifndef HU_P_LENGTH8
#define HU_P_LENGTH8 2
#endif
#ifndef HU_P_VALIDATE16
#define HU_P_VALIDATE16 2
#endif
#ifndef HU_P_LENGTH16
#define HU_P_LENGTH16 4
#endif
constexpr int kPValidate8 = HU_P_VALIDATE8;
constexpr int kPLength8 = HU_P_LENGTH8;
constexpr int kPValidate16 = HU_P_VALIDATE16;
constexpr int kPLength16 = HU_P_LENGTH16;
constexpr unsigned long long kPieceBytes = 1024;

// Internal op flags on top of HU_OP_*: convert without validating (input
// known to be valid); the UTF-16 side is big endian.
constexpr int kTrustedOp = 0x100;
constexpr int kBigEndianOp = 0x200;
constexpr int kOpFlags = kTrustedOp | kBigEndianOp;

struct KernelChoice {
    const void *fn;
    unsigned long long tile_bytes;
    bool one_group_per_tile;   // convert: one workgroup per tile, a status word per tile;
                               // else: persistent, each wave grid-stride over wave-tiles, no status words
};

// An op with flags (variants.hip): false when the combination has no kernel.
bool choose_variant(int op, KernelChoice &kc);

}  // namespace hu
