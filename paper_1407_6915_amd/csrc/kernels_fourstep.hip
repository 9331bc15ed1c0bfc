// Four-step pass kernels (column pass A, row pass B) and the global-memory
// radix-stage fallback.
#include "registry.hpp"
#include "tile.hpp"

namespace fftseg {
namespace {

// flag bits: streamed global access; twiddles reloaded per tile (all
// stages, or all but the last); XCD-aware tile order; register allocation
// for 2 waves per SIMD; lane index kept across the tiles of the persistent
// loop
constexpr int kNT = 1, kNoHoist = 2, kXcd = 4, kHoistLast = 8, kW2 = 16, kPlainLane = 32;

template <int NS, int F>
constexpr int hoist_mask()
{
    return (F & kNoHoist) ? 0 : (F & kHoistLast) ? (1 << (NS - 1)) : -1;
}

template <int M, int T, int C, int PS, int F, int... Rs>
struct ColInst {
    using Sh = Shape<M, T, Radices<Rs...>>;
    using Pol = ColumnPolicy<Sh, C, PS, (F & kNT) != 0, hoist_mask<sizeof...(Rs), F>(),
                             (F & kXcd) != 0, (F & kW2) ? 2 : 1, (F & kPlainLane) != 0>;
    static void launch(int dir, const void *in, void *ybuf, const void *tw,
                       const void *tl, const void *th, int sh, int n2,
                       uint64_t batch, unsigned grid, hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL((four_step_columns_kernel<Sh, Pol, -1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)ybuf, (const c32 *)tw,
                               (const c32 *)tl, (const c32 *)th, sh, n2, batch);
        else
            hipLaunchKernelGGL((four_step_columns_kernel<Sh, Pol, 1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)ybuf, (const c32 *)tw,
                               (const c32 *)tl, (const c32 *)th, sh, n2, batch);
    }
    static ColumnDesc desc(int variant)
    {
        ColumnDesc d{};
        d.n1 = M;
        d.variant = variant;
        d.flags = F;
        d.cols = C;
        d.threads = T;
        d.lds_bytes = Pol::kLdsElems * (int)sizeof(c32);
        d.nrad = (int)sizeof...(Rs);
        const int r[] = {Rs...};
        for (int i = 0; i < d.nrad; ++i)
            d.radices[i] = r[i];
        d.launch = &launch;
        d.kernel[0] = (const void *)&four_step_columns_kernel<Sh, Pol, -1>;
        d.kernel[1] = (const void *)&four_step_columns_kernel<Sh, Pol, 1>;
        return d;
    }
};

template <int M, int T, int C, int PS, int F, int... Rs>
struct RowInst {
    using Sh = Shape<M, T, Radices<Rs...>>;
    using Pol = RowPolicy<Sh, C, PS, (F & kNT) != 0, hoist_mask<sizeof...(Rs), F>(),
                          (F & kXcd) != 0, (F & kW2) ? 2 : 1, (F & kPlainLane) != 0>;
    static void launch(int dir, const void *ybuf, void *out, const void *tw, int n1,
                       uint64_t batch, unsigned grid, hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL((four_step_rows_kernel<Sh, Pol, -1>), g, b, 0, s,
                               (const c32 *)ybuf, (c32 *)out, (const c32 *)tw, n1, batch);
        else
            hipLaunchKernelGGL((four_step_rows_kernel<Sh, Pol, 1>), g, b, 0, s,
                               (const c32 *)ybuf, (c32 *)out, (const c32 *)tw, n1, batch);
    }
    static RowDesc desc(int variant)
    {
        RowDesc d{};
        d.n2 = M;
        d.variant = variant;
        d.flags = F;
        d.rows = C;
        d.threads = T;
        d.lds_bytes = Pol::kLdsElems * (int)sizeof(c32);
        d.nrad = (int)sizeof...(Rs);
        const int r[] = {Rs...};
        for (int i = 0; i < d.nrad; ++i)
            d.radices[i] = r[i];
        d.launch = &launch;
        d.kernel[0] = (const void *)&four_step_rows_kernel<Sh, Pol, -1>;
        d.kernel[1] = (const void *)&four_step_rows_kernel<Sh, Pol, 1>;
        return d;
    }
};

// Variant 0 of each length is the default; the tuner tries the others.
//                          M     T    C  PS  F                   radices       variant
const ColumnDesc kColumns[] = {
    ColInst<128, 8, 16, 4, 0, 16, 8>::desc(0),
    ColInst<128, 8, 32, 4, kXcd, 16, 8>::desc(1),
    ColInst<128, 8, 32, 4, kXcd | kPlainLane, 16, 8>::desc(2),
    ColInst<256, 16, 16, 4, kNT | kXcd | kHoistLast, 16, 16>::desc(0),
    ColInst<256, 16, 16, 4, kXcd, 16, 16>::desc(1),
    ColInst<256, 16, 32, 4, kNT | kXcd, 16, 16>::desc(2),
    ColInst<256, 16, 16, 4, kNT | kXcd, 16, 16>::desc(3),
    ColInst<256, 16, 16, 4, 0, 16, 16>::desc(4),
    ColInst<256, 16, 16, 4, kXcd | kPlainLane, 16, 16>::desc(5),
    ColInst<256, 16, 16, 4, kNT | kXcd | kPlainLane, 16, 16>::desc(6),
    ColInst<256, 16, 32, 4, kNT | kXcd | kPlainLane, 16, 16>::desc(7),
    ColInst<512, 64, 8, 4, 0, 8, 8, 8>::desc(0),
    ColInst<512, 64, 8, 4, kXcd, 8, 8, 8>::desc(1),
    ColInst<512, 64, 8, 4, kXcd | kPlainLane, 8, 8, 8>::desc(2),
    ColInst<1024, 64, 16, 4, kNoHoist | kXcd, 16, 16, 4>::desc(0),
    ColInst<1024, 64, 8, 4, kXcd, 16, 16, 4>::desc(1),
    ColInst<1024, 64, 8, 4, kNT | kXcd, 16, 16, 4>::desc(2),
    ColInst<1024, 64, 8, 4, 0, 16, 16, 4>::desc(3),
    ColInst<1024, 64, 4, 4, kXcd, 16, 16, 4>::desc(4),
    ColInst<1024, 64, 8, 4, kNT | kXcd | kHoistLast | kW2, 16, 16, 4>::desc(5),
    ColInst<1024, 64, 8, 4, kNT | kXcd | kNoHoist | kW2, 16, 16, 4>::desc(6),
    ColInst<1024, 64, 8, 4, kXcd | kPlainLane, 16, 16, 4>::desc(7),
    ColInst<1024, 64, 8, 4, kNT | kXcd | kPlainLane, 16, 16, 4>::desc(8),
    ColInst<1024, 64, 16, 4, kNoHoist | kXcd | kPlainLane, 16, 16, 4>::desc(9),
    ColInst<2048, 128, 8, 4, kNoHoist, 16, 16, 8>::desc(0),
    ColInst<2048, 128, 8, 4, kNoHoist | kXcd, 16, 16, 8>::desc(1),
    ColInst<2048, 128, 8, 4, kNoHoist | kXcd | kPlainLane, 16, 16, 8>::desc(2),
};

const RowDesc kRows[] = {
    RowInst<128, 8, 16, 4, 0, 16, 8>::desc(0),
    RowInst<128, 8, 32, 4, kXcd, 16, 8>::desc(1),
    RowInst<128, 8, 32, 4, kXcd | kPlainLane, 16, 8>::desc(2),
    RowInst<256, 16, 16, 4, kNT | kXcd | kHoistLast, 16, 16>::desc(0),
    RowInst<256, 16, 16, 4, kXcd, 16, 16>::desc(1),
    RowInst<256, 16, 32, 4, kNT | kXcd, 16, 16>::desc(2),
    RowInst<256, 16, 16, 4, kNT | kXcd, 16, 16>::desc(3),
    RowInst<256, 16, 16, 4, 0, 16, 16>::desc(4),
    RowInst<256, 16, 16, 4, kXcd | kPlainLane, 16, 16>::desc(5),
    RowInst<256, 16, 16, 4, kNT | kXcd | kPlainLane, 16, 16>::desc(6),
    RowInst<256, 16, 32, 4, kNT | kXcd | kPlainLane, 16, 16>::desc(7),
    RowInst<512, 64, 8, 4, 0, 8, 8, 8>::desc(0),
    RowInst<512, 64, 8, 4, kXcd, 8, 8, 8>::desc(1),
    RowInst<512, 64, 8, 4, kXcd | kPlainLane, 8, 8, 8>::desc(2),
    RowInst<1024, 64, 16, 4, kNoHoist | kXcd, 16, 16, 4>::desc(0),
    RowInst<1024, 64, 8, 4, kXcd, 16, 16, 4>::desc(1),
    RowInst<1024, 64, 8, 4, kNT | kXcd, 16, 16, 4>::desc(2),
    RowInst<1024, 64, 8, 4, 0, 16, 16, 4>::desc(3),
    RowInst<1024, 64, 4, 4, kXcd, 16, 16, 4>::desc(4),
    RowInst<1024, 64, 8, 4, kNT | kXcd | kHoistLast | kW2, 16, 16, 4>::desc(5),
    RowInst<1024, 64, 8, 4, kNT | kXcd | kNoHoist | kW2, 16, 16, 4>::desc(6),
    RowInst<1024, 64, 8, 4, kXcd | kPlainLane, 16, 16, 4>::desc(7),
    RowInst<1024, 64, 8, 4, kNT | kXcd | kPlainLane, 16, 16, 4>::desc(8),
    RowInst<1024, 64, 16, 4, kNoHoist | kXcd | kPlainLane, 16, 16, 4>::desc(9),
    RowInst<2048, 128, 8, 4, kNoHoist, 16, 16, 8>::desc(0),
    RowInst<2048, 128, 8, 4, kNoHoist | kXcd, 16, 16, 8>::desc(1),
    RowInst<2048, 128, 8, 4, kNoHoist | kXcd | kPlainLane, 16, 16, 8>::desc(2),
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
