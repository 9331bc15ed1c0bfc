// One-pass kernels over segments at listed offsets, for the work list's
// one-pass lengths: the same shapes and tiles as the dense defaults of each
// length (and a few alternatives the tuner may pick), so a length's
// segments, wherever they sit in the list, run at that length's plain rate.
// Kept in a translation unit of their own so they do not share inlined code
// with the dense instances.
#include "fsinst.hpp"
#include "spinst.hpp"

namespace fftseg {
namespace {

using namespace sp;

// Candidate 0 of each length is the default; grid_mult as in the dense table.
//                 N      T    S  PS  F                                  radices   cand, grid_mult
const SinglePassDesc kIdx256[] = {
    SpInst<256, 16, 8, 4, kPlain | kIndexed, 16, 16>::desc(0, 0),
    SpInst<256, 16, 8, 4, kNT | kPlain | kIndexed, 16, 16>::desc(1, 32),
    SpInst<256, 16, 8, 4, kClassic | kNT | kIndexed, 16, 16>::desc(2, 64),
};
const SinglePassDesc kIdx1000[] = {
    SpInst<1000, 100, 2, 4, kClassic | kIndexed, 10, 10, 10>::desc(0, 64),
    SpInst<1000, 100, 2, 4, kClassic | kNT | kIndexed, 10, 10, 10>::desc(1, 64),
};
const SinglePassDesc kIdx1024[] = {
    SpInst<1024, 64, 2, 4, kNT | kPlain | kIndexed, 16, 16, 4>::desc(0, 64),
    SpInst<1024, 64, 4, 4, kClassic | kIndexed, 16, 16, 4>::desc(1, 32),
};
const SinglePassDesc kIdx1536[] = {
    SpInst<1536, 96, 2, 4, kNT | kPlain | kIndexed, 16, 16, 6>::desc(0, 64),
    SpInst<1536, 96, 2, 4, kClassic | kNT | kIndexed, 16, 16, 6>::desc(1, 64),
};
const SinglePassDesc kIdx4096[] = {
    SpInst<4096, 128, 2, 4, kClassic | kNT | kIndexed, 16, 16, 16>::desc(0, 32),
    SpInst<4096, 128, 2, 4, kClassic | kIndexed, 16, 16, 16>::desc(1, 32),
};
const SinglePassDesc kIdx6000[] = {
    SpInst<6000, 400, 1, 4, kNT | kNoHoist | kTwPair | kW4 | kIndexed, 16, 15, 25>::desc(0, 0),
    SpInst<6000, 400, 1, 4, kClassic | kNT | kIndexed, 16, 15, 25>::desc(1, 32),
    SpInst<6000, 400, 1, 4, kClassic | kIndexed, 16, 15, 25>::desc(2, 32),
};
const SinglePassDesc kIdx16384[] = {
    SpInst<16384, 512, 1, 4, kSplit | kNT | kNoHoist | kW4 | kTwPair | kIndexed, 16, 32, 32>::desc(
        0, 0),
};

// the 65536-point two-pass tiles (256 x 256), as the plan's defaults
const ColumnDesc kIdxCol65536 =
    fs::ColInst<256, 16, 16, 4, fs::kNT | fs::kXcd | fs::kHoistLast | fs::kIndexed | fs::kLdsTw,
                16, 16>::desc(0);
const RowDesc kIdxRow65536 =
    fs::RowInst<256, 16, 16, 4, fs::kNT | fs::kXcd | fs::kHoistLast | fs::kIndexed, 16,
                16>::desc(0);

}  // namespace

bool indexed_four_step(uint32_t n, const ColumnDesc **col, const RowDesc **row)
{
    if (n != 65536)
        return false;
    *col = &kIdxCol65536;
    *row = &kIdxRow65536;
    return true;
}

const SinglePassDesc *indexed_table(uint32_t n, int *count)
{
#define FFTSEG_IDX(N, T)                                   \
    case N:                                                \
        *count = (int)(sizeof(T) / sizeof(T[0]));          \
        return T;
    switch (n) {
        FFTSEG_IDX(256, kIdx256)
        FFTSEG_IDX(1000, kIdx1000)
        FFTSEG_IDX(1024, kIdx1024)
        FFTSEG_IDX(1536, kIdx1536)
        FFTSEG_IDX(4096, kIdx4096)
        FFTSEG_IDX(6000, kIdx6000)
        FFTSEG_IDX(16384, kIdx16384)
    default:
        *count = 0;
        return nullptr;
    }
#undef FFTSEG_IDX
}

}  // namespace fftseg
