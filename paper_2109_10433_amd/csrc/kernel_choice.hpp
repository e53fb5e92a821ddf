// kernel_choice.hpp - which kernel runs an operation, and its tile size.
//
// The plain operations' kernels are instantiated in hiputf.hip; the variants
// (conversions without validation, big-endian UTF-16) in variants.hip, a
// translation unit of their own, so that adding them leaves the code
// generated for the plain kernels unchanged.
#pragma once

namespace hu {

// Sub-tiles of 4 KiB per tile. Convert tiles: the largest that still fit 64
// registers (eight waves per SIMD); bigger tiles mean fewer look-backs per
// byte. UTF-8 input at 6 would spill; UTF-16 input fits 6 when held to eight
// waves. Validate / length tiles are staged in LDS; their sizes were measured
// per kernel (4 to 16 sub-tiles; larger tiles keep more bytes in flight per
// workgroup but fewer workgroups fit a CU).
constexpr int kUConvert8 = 5;
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
