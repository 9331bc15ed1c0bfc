// Four-step pass kernels (column pass A, row pass B) and the global-memory
// radix-stage fallback.
#include "fsinst.hpp"

namespace fftseg {
namespace {

using namespace fs;

// Variant 0 of each length is the default; the tuner tries the others.  The
// default column tiles split W_N^{n2 k1} through LDS (kLdsTw), and the 512-
// and 1024-point tiles (kernels_radix32.hip) also read their second stage's
// twiddles in pairs (kTwPair); the forms without these stay as variants.
// The default 128-, 256- and 512-point tiles also come in the form with Y
// in blocks of 16 columns (kYBlocked): plans of two such tiles take it
// (65536 points: 5.71-5.73 ms per 8 GiB against 5.94-6.13; at 1024 points
// the blocked form was 2-3 % slower).  The default 2048-point row tile has
// 16 rows and split exchanges (kernels_split.hip): its transposed store
// writes whole lines (2^22 points: 8.37 ms per 8 GiB against 9.35 with 8
// rows); the 16-column split column tile spills and stays a variant.
//                          M     T    C  PS  F                   radices       variant
const ColumnDesc kColumns[] = {
    ColInst<128, 8, 16, 4, kFrames | kShifted | kLdsTw | kYBlocked, 16, 8>::desc(0),
    ColInst<128, 8, 32, 4, kXcd, 16, 8>::desc(1),
    ColInst<128, 8, 32, 4, kXcd | kPlainLane, 16, 8>::desc(2),
    ColInst<128, 8, 16, 4, 0, 16, 8>::desc(3),
    ColInst<256, 16, 16, 4, kNT | kXcd | kHoistLast | kFrames | kShifted | kLdsTw | kYBlocked, 16,
            16>::desc(0),
    ColInst<256, 16, 16, 4, kXcd, 16, 16>::desc(1),
    ColInst<256, 16, 32, 4, kNT | kXcd, 16, 16>::desc(2),
    ColInst<256, 16, 16, 4, kNT | kXcd, 16, 16>::desc(3),
    ColInst<256, 16, 16, 4, 0, 16, 16>::desc(4),
    ColInst<256, 16, 16, 4, kXcd | kPlainLane, 16, 16>::desc(5),
    ColInst<256, 16, 16, 4, kNT | kXcd | kPlainLane, 16, 16>::desc(6),
    ColInst<256, 16, 32, 4, kNT | kXcd | kPlainLane, 16, 16>::desc(7),
    ColInst<256, 16, 16, 4, kNT | kXcd | kHoistLast, 16, 16>::desc(8),
    radix32_column_desc(1, 0),
    ColInst<512, 64, 8, 4, 0, 8, 8, 8>::desc(1),
    ColInst<512, 64, 8, 4, kXcd, 8, 8, 8>::desc(2),
    ColInst<512, 64, 8, 4, kXcd | kPlainLane, 8, 8, 8>::desc(3),
    radix32_column_desc(2, 4),
    radix32_column_desc(4, 5),
    radix32_column_desc(6, 6),
    split_column_desc(4, 7),
    radix32_column_desc(8, 8),
    radix32_column_desc(0, 0),
    ColInst<1024, 64, 16, 4, kNoHoist | kXcd, 16, 16, 4>::desc(1),
    ColInst<1024, 64, 8, 4, kXcd, 16, 16, 4>::desc(2),
    ColInst<1024, 64, 8, 4, kNT | kXcd, 16, 16, 4>::desc(3),
    ColInst<1024, 64, 8, 4, 0, 16, 16, 4>::desc(4),
    ColInst<1024, 64, 4, 4, kXcd, 16, 16, 4>::desc(5),
    ColInst<1024, 64, 8, 4, kNT | kXcd | kHoistLast | kW2, 16, 16, 4>::desc(6),
    ColInst<1024, 64, 8, 4, kNT | kXcd | kNoHoist | kW2, 16, 16, 4>::desc(7),
    ColInst<1024, 64, 8, 4, kXcd | kPlainLane, 16, 16, 4>::desc(8),
    ColInst<1024, 64, 8, 4, kNT | kXcd | kPlainLane, 16, 16, 4>::desc(9),
    ColInst<1024, 64, 16, 4, kNoHoist | kXcd | kPlainLane, 16, 16, 4>::desc(10),
    split_column_desc(0, 11),
    split_column_desc(2, 12),
    radix32_column_desc(3, 13),
    radix32_column_desc(5, 14),
    split_column_desc(3, 15),
    radix32_column_desc(7, 16),
    ColInst<2048, 128, 8, 4, kNoHoist | kXcd | kPlainLane | kFrames | kShifted | kLdsTw, 16, 16,
            8>::desc(0),
    ColInst<2048, 128, 8, 4, kNoHoist, 16, 16, 8>::desc(1),
    ColInst<2048, 128, 8, 4, kNoHoist | kXcd, 16, 16, 8>::desc(2),
    split_column_desc(1, 3),
    ColInst<2048, 128, 8, 4, kNoHoist | kXcd | kPlainLane, 16, 16, 8>::desc(4),
    ColInst<2048, 128, 8, 4, kNoHoist | kXcd | kPlainLane | kLdsTw | kTwPair, 16, 16, 8>::desc(5),
    split_column_desc(5, 6),
};

const RowDesc kRows[] = {
    RowInst<128, 8, 16, 4, kShifted | kYBlocked, 16, 8>::desc(0),
    RowInst<128, 8, 32, 4, kXcd, 16, 8>::desc(1),
    RowInst<128, 8, 32, 4, kXcd | kPlainLane, 16, 8>::desc(2),
    RowInst<256, 16, 16, 4, kNT | kXcd | kHoistLast | kShifted | kYBlocked, 16, 16>::desc(0),
    RowInst<256, 16, 16, 4, kXcd, 16, 16>::desc(1),
    RowInst<256, 16, 32, 4, kNT | kXcd, 16, 16>::desc(2),
    RowInst<256, 16, 16, 4, kNT | kXcd, 16, 16>::desc(3),
    RowInst<256, 16, 16, 4, 0, 16, 16>::desc(4),
    RowInst<256, 16, 16, 4, kXcd | kPlainLane, 16, 16>::desc(5),
    RowInst<256, 16, 16, 4, kNT | kXcd | kPlainLane, 16, 16>::desc(6),
    RowInst<256, 16, 32, 4, kNT | kXcd | kPlainLane, 16, 16>::desc(7),
    radix32_row_desc(1, 0),
    RowInst<512, 64, 8, 4, 0, 8, 8, 8>::desc(1),
    RowInst<512, 64, 8, 4, kXcd, 8, 8, 8>::desc(2),
    RowInst<512, 64, 8, 4, kXcd | kPlainLane, 8, 8, 8>::desc(3),
    radix32_row_desc(2, 4),
    radix32_row_desc(4, 5),
    split_row_desc(4, 6),
    radix32_row_desc(6, 7),
    radix32_row_desc(0, 0),
    RowInst<1024, 64, 16, 4, kNoHoist | kXcd, 16, 16, 4>::desc(1),
    RowInst<1024, 64, 8, 4, kXcd, 16, 16, 4>::desc(2),
    RowInst<1024, 64, 8, 4, kNT | kXcd, 16, 16, 4>::desc(3),
    RowInst<1024, 64, 8, 4, 0, 16, 16, 4>::desc(4),
    RowInst<1024, 64, 4, 4, kXcd, 16, 16, 4>::desc(5),
    RowInst<1024, 64, 8, 4, kNT | kXcd | kHoistLast | kW2, 16, 16, 4>::desc(6),
    RowInst<1024, 64, 8, 4, kNT | kXcd | kNoHoist | kW2, 16, 16, 4>::desc(7),
    RowInst<1024, 64, 8, 4, kXcd | kPlainLane, 16, 16, 4>::desc(8),
    RowInst<1024, 64, 8, 4, kNT | kXcd | kPlainLane, 16, 16, 4>::desc(9),
    RowInst<1024, 64, 16, 4, kNoHoist | kXcd | kPlainLane, 16, 16, 4>::desc(10),
    split_row_desc(0, 11),
    split_row_desc(2, 12),
    radix32_row_desc(3, 13),
    split_row_desc(3, 14),
    radix32_row_desc(5, 15),
    split_row_desc(5, 0),
    RowInst<2048, 128, 8, 4, kNoHoist | kXcd, 16, 16, 8>::desc(1),
    RowInst<2048, 128, 8, 4, kNoHoist | kXcd | kPlainLane, 16, 16, 8>::desc(2),
    split_row_desc(1, 3),
    RowInst<2048, 128, 8, 4, kNoHoist | kXcd | kPlainLane | kTwPair, 16, 16, 8>::desc(4),
    RowInst<2048, 128, 8, 4, kNoHoist | kShifted, 16, 16, 8>::desc(5),
};

template <int R>
void launch_stage(int dir, const void *in, void *out, const void *tl, const void *th,
                  int sh, uint64_t n, uint64_t l, uint64_t batch, unsigned grid,
                  hipStream_t s)
{
    if (dir < 0)
        hipLaunchKernelGGL((stockham_global_stage_kernel<R, -1>), dim3(grid), dim3(256),
                           0, s, (const c32 *)in, (c32 *)out, (const c32 *)tl,
                           (const c32 *)th, sh, n, l, batch);
    else
        hipLaunchKernelGGL((stockham_global_stage_kernel<R, 1>), dim3(grid), dim3(256),
                           0, s, (const c32 *)in, (c32 *)out, (const c32 *)tl,
                           (const c32 *)th, sh, n, l, batch);
}

}  // namespace

const ColumnDesc *column_table(int *count)
{
    *count = (int)(sizeof(kColumns) / sizeof(kColumns[0]));
    return kColumns;
}

const RowDesc *row_table(int *count)
{
    *count = (int)(sizeof(kRows) / sizeof(kRows[0]));
    return kRows;
}

bool generic_radix_supported(int radix)
{
    switch (radix) {
    case 2: case 3: case 4: case 5: case 8: case 16:
        return true;
    default:
        return false;
    }
}

void launch_generic_stage(int radix, int dir, const void *in, void *out, const void *tl,
                          const void *th, int sh, uint64_t n, uint64_t l, uint64_t batch,
                          unsigned grid, hipStream_t s)
{
    switch (radix) {
    case 2: launch_stage<2>(dir, in, out, tl, th, sh, n, l, batch, grid, s); break;
    case 3: launch_stage<3>(dir, in, out, tl, th, sh, n, l, batch, grid, s); break;
    case 4: launch_stage<4>(dir, in, out, tl, th, sh, n, l, batch, grid, s); break;
    case 5: launch_stage<5>(dir, in, out, tl, th, sh, n, l, batch, grid, s); break;
    case 8: launch_stage<8>(dir, in, out, tl, th, sh, n, l, batch, grid, s); break;
    case 16: launch_stage<16>(dir, in, out, tl, th, sh, n, l, batch, grid, s); break;
    default: break;
    }
}

}  // namespace fftseg
