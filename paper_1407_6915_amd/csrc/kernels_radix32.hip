// Four-step tiles with radix-32 stages: 1024 = 32 x 32 and 512 = 32 x 16
// take two Stockham stages, so one LDS exchange (two barriers) per tile
// instead of two or three, for 32 values per thread.  The default tiles
// (configs 0 and 1) read the second stage's twiddles in pairs (kTwPair),
// and the column tiles split W_N^{n2 k1} through LDS (kLdsTw); the column
// configs 3 / 4 are those tiles with neither, 5 / 6 without the pairs, and
// the row configs 3 / 4 without the pairs.  (The same radices in
// one-pass kernels of 512 and 1024 points measured no faster than the
// table's defaults.)  Kept in a translation unit of their own so they do not
// share inlined code with the other instances.
#include "fsinst.hpp"

namespace fftseg {

ColumnDesc radix32_column_desc(int config, int variant)
{
    using namespace fs;
    //                        M     T   C  PS  F                        radices
    switch (config) {
    case 0:
        return ColInst<1024, 32, 16, 4,
                       kNoHoist | kXcd | kW2 | kFrames | kShifted | kLdsTw | kTwPair, 32,
                       32>::desc(variant);
    case 1:
        // streamed (non-temporal) access: 5.84-5.87 ms per 8 GiB of 2^18-point
        // segments with the row tile's against 6.13 cached (at 1024 points the
        // streamed forms, configs 7 here and 5 below, are 3-10 % slower)
        return ColInst<512, 16, 16, 4,
                       kNT | kNoHoist | kXcd | kW2 | kFrames | kShifted | kLdsTw | kTwPair |
                           kYBlocked,
                       32, 16>::desc(variant);
    case 2:
        return ColInst<512, 32, 16, 4, kXcd | kW2, 16, 32>::desc(variant);
    case 3:
        return ColInst<1024, 32, 16, 4, kNoHoist | kXcd | kW2, 32, 32>::desc(variant);
    case 4:
        return ColInst<512, 16, 16, 4, kNoHoist | kXcd | kW2, 32, 16>::desc(variant);
    case 5:
        return ColInst<1024, 32, 16, 4, kNoHoist | kXcd | kW2 | kLdsTw, 32, 32>::desc(variant);
    case 6:
        return ColInst<512, 16, 16, 4, kNoHoist | kXcd | kW2 | kLdsTw, 32, 16>::desc(variant);
    case 7:
        return ColInst<1024, 32, 16, 4, kNT | kNoHoist | kXcd | kW2 | kLdsTw | kTwPair, 32,
                       32>::desc(variant);
    case 8:
        return ColInst<512, 16, 16, 4, kNoHoist | kXcd | kW2 | kLdsTw | kTwPair, 32, 16>::desc(
            variant);
    default:
        return ColumnDesc{};
    }
}

RowDesc radix32_row_desc(int config, int variant)
{
    using namespace fs;
    switch (config) {
    case 0:
        return RowInst<1024, 32, 16, 4, kNoHoist | kXcd | kW2 | kShifted | kTwPair, 32, 32>::desc(
            variant);
    case 1:
        return RowInst<512, 16, 16, 4,
                       kNT | kNoHoist | kXcd | kW2 | kShifted | kTwPair | kYBlocked, 32,
                       16>::desc(variant);
    case 2:
        return RowInst<512, 32, 16, 4, kXcd | kW2, 16, 32>::desc(variant);
    case 3:
        return RowInst<1024, 32, 16, 4, kNoHoist | kXcd | kW2, 32, 32>::desc(variant);
    case 4:
        return RowInst<512, 16, 16, 4, kNoHoist | kXcd | kW2, 32, 16>::desc(variant);
    case 5:
        return RowInst<1024, 32, 16, 4, kNT | kNoHoist | kXcd | kW2 | kTwPair, 32, 32>::desc(
            variant);
    case 6:
        return RowInst<512, 16, 16, 4, kNoHoist | kXcd | kW2 | kTwPair, 32, 16>::desc(variant);
    default:
        return RowDesc{};
    }
}

}  // namespace fftseg
