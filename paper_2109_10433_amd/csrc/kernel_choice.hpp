// kernel_choice.hpp - which kernel runs an operation, and its tile size.
//
// The plain operations' kernels are instantiated in hiputf.hip; the variants
// (conversions without validation, big-endian UTF-16) in variants.hip, a
// translation unit of their own, so that adding them leaves the code
// generated for the plain kernels unchanged.
#pragma once

namespace hu {

// Sub-tiles of 4 KiB per tile. Convert tiles: bigger tiles mean fewer
// look-backs per byte, more registers fewer waves per SIMD. Measured: UTF-8
// input is fastest at 6 (68 registers, seven waves per SIMD; 5 fits eight
// waves but leaves one- and two-byte text 5 % slower, 7 and 8 slow down
// three- and four-byte text); UTF-16 input at 6 (64 registers; 8 and 10 are
// far slower). Validate / length tiles are staged in LDS; their sizes were
// measured per kernel (4 to 16 sub-tiles; larger tiles keep more bytes in
// flight per workgroup but fewer workgroups fit a CU).
constexpr int kUConvert8 = 6;
// UTF-8 -> UTF-16LE inputs below kSmallConvert8Bytes take the 5 sub-tile
// kernel instead: there more, shorter tiles spread a small input over more of
// the chip (1 MiB: 13 instead of 16 us).
constexpr int kUConvert8Small = 5;
constexpr unsigned long long kSmallConvert8Bytes = 64ull << 20;
constexpr int kUConvert16 = 6;
constexpr int kUValidate8 = 12;
constexpr int kULength8 = 10;
constexpr int kUValidate16 = 16;
constexpr int kULength16 = 10;

// Internal op flags on top of HU_OP_*: convert without validating (input
// known to be valid); the UTF-16 side is big endian.
constexpr int kTrustedOp = 0x100;
constexpr int kBigEndianOp = 0x200;
constexpr int kOpFlags = kTrustedOp | kBigEndianOp;

struct KernelChoice {
    const void *fn;
    unsigned long long tile_bytes;
    bool one_group_per_tile;   // else: persistent, grid-stride over tiles
};

// An op with flags (variants.hip): false when the combination has no kernel.
bool choose_variant(int op, KernelChoice &kc);

}  // namespace hu
