// Single-pass and four-step pass instances with split LDS exchanges (real
// parts, then imaginary parts): half the LDS of the complex tile, so lengths
// whose tile otherwise leaves one or two workgroups per CU get twice as
// many.  Kept in a translation unit of their own so they do not share
// inlined code with the other instances.
#include "fsinst.hpp"
#include "spinst.hpp"

namespace fftseg {

SinglePassDesc split_desc(int config, int variant, int grid_mult)
{
    using namespace sp;
    //                       N      T   S  PS  F                             radices
    switch (config) {
    case 0:
        // twiddles read in pairs: 10 table reads per radix-32 butterfly
        // instead of 31 (3.2-3.3 ms per 8 GiB against 4.6 with direct reads)
        return SpInst<16384, 512, 1, 4, kSplit | kNT | kNoHoist | kW4 | kTwPair | kFrames, 16, 32,
                      32>::desc(variant, grid_mult);
    case 1:
        return SpInst<16384, 512, 1, 4, kSplit | kNT | kNoHoist | kW4, 32, 32, 16>::desc(
            variant, grid_mult);
    case 2:
        return SpInst<16384, 512, 1, 4, kSplit | kNT | kNoHoist | kW4, 16, 16, 16, 4>::desc(
            variant, grid_mult);
    case 3:
        return SpInst<16384, 512, 1, 4, kSplit | kPrefetch | kNT | kNoHoist | kW2, 32, 32,
                      16>::desc(variant, grid_mult);
    case 4:
        // 1024 threads, 16 values each: two workgroups per CU give 32 waves
        // (8 per SIMD, 64 VGPRs) instead of 16
        return SpInst<16384, 1024, 1, 4, kSplit | kNT | kNoHoist | kW8, 16, 16, 16, 4>::desc(
            variant, grid_mult);
    case 5:
        return SpInst<16384, 512, 1, 4, kSplit | kNT | kNoHoist | kW4, 16, 32, 32>::desc(
            variant, grid_mult);
    case 6:
        return SpInst<8192, 512, 1, 4, kSplit | kNT | kNoHoist | kW4 | kTwPair, 16, 16, 32>::desc(
            variant, grid_mult);
    default:
        return SinglePassDesc{};
    }
}

ColumnDesc split_column_desc(int config, int variant)
{
    using namespace fs;
    //                        M     T   C  PS  F                                  radices
    switch (config) {
    case 0:
        return ColInst<1024, 32, 16, 4, kSplit | kNoHoist | kXcd | kW4, 16, 16, 4>::desc(variant);
    case 1:
        return ColInst<2048, 128, 8, 4, kSplit | kNoHoist | kXcd | kW8, 16, 16, 8>::desc(variant);
    case 2:
        return ColInst<1024, 32, 16, 4, kSplit | kNoHoist | kXcd | kW4, 32, 32>::desc(variant);
    case 3:
        return ColInst<1024, 32, 16, 4, kSplit | kNoHoist | kXcd | kW4 | kLdsTw | kTwPair, 32,
                       32>::desc(variant);
    case 4:
        return ColInst<512, 16, 16, 4, kSplit | kNoHoist | kXcd | kW4 | kLdsTw | kTwPair, 32,
                       16>::desc(variant);
    case 5:
        return ColInst<2048, 64, 16, 4, kSplit | kNoHoist | kXcd | kW4 | kLdsTw | kTwPair, 16, 16,
                       8>::desc(variant);
    default:
        return ColumnDesc{};
    }
}

RowDesc split_row_desc(int config, int variant)
{
    using namespace fs;
    switch (config) {
    case 0:
        return RowInst<1024, 32, 16, 4, kSplit | kNoHoist | kXcd | kW4, 16, 16, 4>::desc(variant);
    case 1:
        return RowInst<2048, 128, 8, 4, kSplit | kNoHoist | kXcd | kW8, 16, 16, 8>::desc(variant);
    case 2:
        return RowInst<1024, 32, 16, 4, kSplit | kNoHoist | kXcd | kW4, 32, 32>::desc(variant);
    case 3:
        return RowInst<1024, 32, 16, 4, kSplit | kNoHoist | kXcd | kW4 | kTwPair, 32, 32>::desc(
            variant);
    case 4:
        return RowInst<512, 16, 16, 4, kSplit | kNoHoist | kXcd | kW4 | kTwPair, 32, 16>::desc(
            variant);
    case 5:
        // 16 rows per tile (whole 128-byte lines in the transposed store) fit
        // the 2048-point row tile's LDS only with split exchanges
        return RowInst<2048, 64, 16, 4, kSplit | kNoHoist | kXcd | kW4 | kShifted | kTwPair, 16,
                       16, 8>::desc(variant);
    default:
        return RowDesc{};
    }
}

}  // namespace fftseg
