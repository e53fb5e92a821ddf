// kernel_choice.hpp - which kernel runs an operation, and its tile size.
//
// The plain operations' kernels are instantiated in hiputf.hip; the variants
// (conversions without validation, big-endian UTF-16) in variants.hip, a
// translation unit of their own, so that adding them leaves the code
// generated for the plain kernels unchanged.
#pragma once

namespace hu {

// Convert tiles: sub-tiles of 4 KiB per tile (one per workgroup); bigger
// tiles mean fewer look-backs per byte, more registers fewer waves per SIMD,
// and more serial work per workgroup. Large inputs: UTF-8 is fastest at 6
// (68 registers, seven waves per SIMD; 5 fits eight waves but leaves one- and
// two-byte text 5 % slower, 7 and 8 slow down three- and four-byte text),
// UTF-16 at 6 (64 registers; 8 and 10 are far slower). Smaller inputs take
// smaller tiles, which spread them over more of the chip and shorten each
// workgroup's serial part. Size classes by input bytes, from the measured
// crossovers on mixed text (1..63 MiB, tiles of 1, 2, 5 / 6 sub-tiles):
// UTF-8 1 MiB 7.8 us at 1 sub-tile against 13.7 at 5, 16 MiB 24.9 us at 2
// against 27.3 at 5, 5 ahead from 24 MiB on; UTF-16 1 MiB 8.9 against 23.8
// at 6, 32 MiB 41.3 at 2 against 45.1 at 6, 6 ahead from 48 MiB on.
struct TileClass {
    unsigned long long below;   // inputs of fewer bytes than this (and more than the class before)
    int sub_tiles;
};
constexpr TileClass kConvert8Classes[] = {
    {4ull << 20, 1}, {24ull << 20, 2}, {64ull << 20, 5}, {~0ull, 6}};
constexpr TileClass kConvert16Classes[] = {{8ull << 20, 1}, {48ull << 20, 2}, {~0ull, 6}};

template <int N>
constexpr int class_sub_tiles(const TileClass (&c)[N], unsigned long long n_bytes)
{
    for (int i = 0; i < N; ++i)
        if (n_bytes < c[i].below)
            return c[i].sub_tiles;
    return c[N - 1].sub_tiles;
}

// Largest tile count any input of at most n_bytes takes (15 bytes of source
// alignment offset at most): the status words a workspace for such inputs
// must hold.
template <int N>
constexpr unsigned long long class_max_tiles(const TileClass (&c)[N], unsigned long long n_bytes,
                                             unsigned long long sub_bytes)
{
    unsigned long long lo = 0, most = 0;
    for (int i = 0; i < N && lo <= n_bytes; ++i) {
        const unsigned long long top = (c[i].below - 1 < n_bytes ? c[i].below - 1 : n_bytes) + 15;
        const unsigned long long tb = (unsigned long long)c[i].sub_tiles * sub_bytes;
        const unsigned long long t = (top + tb - 1) / tb;
        most = t > most ? t : most;
        lo = c[i].below;
    }
    return most;
}

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
    unsigned int groups_per_cu = 0;   // persistent kernels: resident workgroups per CU at most (0: no limit)
};

// The length kernels run at most this many workgroups (waves per SIMD) per
// CU: each measured faster there than at the one more its registers allow
// (UTF-8 length of UTF-16 input: three-byte text by 5-7 %; UTF-16 length of
// UTF-8 input: Latin and Cyrillic by 6-8 %).
constexpr unsigned int kLength16GroupsPerCu = 5;
constexpr unsigned int kLength8GroupsPerCu = 6;

// An op with flags (variants.hip): false when the combination has no kernel.
bool choose_variant(int op, unsigned long long n_bytes, KernelChoice &kc);

}  // namespace hu
