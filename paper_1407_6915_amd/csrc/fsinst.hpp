// Compile-time description of the four-step pass instances (column pass A,
// row pass B) and the descriptors the planner sees for them.
#pragma once

#include "registry.hpp"
#include "tile.hpp"

namespace fftseg {
namespace fs {

// flag bits: streamed global access; twiddles reloaded per tile (all
// stages, or all but the last); XCD-aware tile order; register allocation
// for 2 waves per SIMD; lane index kept across the tiles of the persistent
// loop; split (real, then imaginary) LDS exchanges; register allocation for
// 4 / 8 waves per SIMD; the column pass also comes in a form that reads
// overlapping, windowed frames; both passes also come in a form whose blocks
// start at any column / row and wrap round (for segments off a line
// boundary); both passes also come in a form over segments at listed
// offsets (kIndexed); one row per length carries each of these forms;
// the column pass splits W_N^{n2 k1} into a per-butterfly lookup and a
// per-tile LDS table (kLdsTw, ColumnPolicy); stages that reload their
// twiddles read them as pairs (kTwPair, tw_pair_low); both passes also come
// in a form with Y in blocks of 16 columns (kYBlocked, see kYBlock), which a
// plan takes when its column and row tiles both have it
constexpr int kNT = 1, kNoHoist = 2, kXcd = 4, kHoistLast = 8, kW2 = 16, kPlainLane = 32,
              kSplit = 64, kW4 = 128, kW8 = 256, kFrames = 1024, kShifted = 2048,
              kIndexed = 4096, kLdsTw = 8192, kTwPair = 16384, kYBlocked = 32768;

template <int NS, int F>
constexpr int hoist_mask()
{
    return (F & kNoHoist) ? 0 : (F & kHoistLast) ? (1 << (NS - 1)) : -1;
}

template <int F>
constexpr int waves()
{
    return (F & kW8) ? 8 : (F & kW4) ? 4 : (F & kW2) ? 2 : 1;
}
template <int F>
constexpr int elem_bytes()
{
    return (F & kSplit) ? (int)sizeof(float) : (int)sizeof(c32);
}

template <int M, int T, int C, int PS, int F, int... Rs>
struct ColInst {
    using Sh = Shape<M, T, Radices<Rs...>>;
    using Pol = ColumnPolicy<Sh, C, PS, (F & kNT) != 0, hoist_mask<sizeof...(Rs), F>(),
                             (F & kXcd) != 0, waves<F>(), (F & kPlainLane) != 0,
                             (F & kSplit) != 0, false, (F & kLdsTw) != 0,
                             (F & kTwPair) != 0>;
    using PolW = ColumnPolicy<Sh, C, PS, (F & kNT) != 0, hoist_mask<sizeof...(Rs), F>(),
                              (F & kXcd) != 0, waves<F>(), (F & kPlainLane) != 0,
                              (F & kSplit) != 0, true, (F & kLdsTw) != 0,
                              (F & kTwPair) != 0>;
    using PolB = ColumnPolicy<Sh, C, PS, (F & kNT) != 0, hoist_mask<sizeof...(Rs), F>(),
                              (F & kXcd) != 0, waves<F>(), (F & kPlainLane) != 0,
                              (F & kSplit) != 0, false, (F & kLdsTw) != 0,
                              (F & kTwPair) != 0, true>;
    static void launch_yblocked(int dir, const void *in, void *ybuf, const void *tw,
                                const void *tl, const void *th, int sh, int n2,
                                uint64_t batch, unsigned grid, hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL((four_step_columns_kernel<Sh, PolB, -1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)ybuf, (const c32 *)tw,
                               (const c32 *)tl, (const c32 *)th, sh, n2, batch);
        else
            hipLaunchKernelGGL((four_step_columns_kernel<Sh, PolB, 1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)ybuf, (const c32 *)tw,
                               (const c32 *)tl, (const c32 *)th, sh, n2, batch);
    }
    static void launch_shifted(int dir, const void *in, void *ybuf, const void *tw,
                               const void *tl, const void *th, int sh, int n2, uint64_t batch,
                               int shift, unsigned grid, hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL((four_step_columns_shifted_kernel<Sh, PolW, -1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)ybuf, (const c32 *)tw, (const c32 *)tl,
                               (const c32 *)th, sh, n2, batch, shift);
        else
            hipLaunchKernelGGL((four_step_columns_shifted_kernel<Sh, PolW, 1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)ybuf, (const c32 *)tw, (const c32 *)tl,
                               (const c32 *)th, sh, n2, batch, shift);
    }
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
    static void launch_frames(int dir, const void *in, void *ybuf, const void *tw,
                              const void *tl, const void *th, int sh, int n2, uint64_t batch,
                              uint64_t hop, const float *window, unsigned grid, hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL((four_step_columns_frames_kernel<Sh, Pol, -1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)ybuf, (const c32 *)tw, (const c32 *)tl,
                               (const c32 *)th, sh, n2, batch, hop, window);
        else
            hipLaunchKernelGGL((four_step_columns_frames_kernel<Sh, Pol, 1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)ybuf, (const c32 *)tw, (const c32 *)tl,
                               (const c32 *)th, sh, n2, batch, hop, window);
    }
    static void launch_frames_yblocked(int dir, const void *in, void *ybuf, const void *tw,
                                       const void *tl, const void *th, int sh, int n2,
                                       uint64_t batch, uint64_t hop, const float *window,
                                       unsigned grid, hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL((four_step_columns_frames_kernel<Sh, PolB, -1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)ybuf, (const c32 *)tw, (const c32 *)tl,
                               (const c32 *)th, sh, n2, batch, hop, window);
        else
            hipLaunchKernelGGL((four_step_columns_frames_kernel<Sh, PolB, 1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)ybuf, (const c32 *)tw, (const c32 *)tl,
                               (const c32 *)th, sh, n2, batch, hop, window);
    }
    static void launch_indexed(int dir, const void *in, void *ybuf, const void *tw,
                               const void *tl, const void *th, int sh, int n2,
                               const uint64_t *offs, uint64_t batch, unsigned grid,
                               hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL((four_step_columns_indexed_kernel<Sh, PolW, -1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)ybuf, (const c32 *)tw, (const c32 *)tl,
                               (const c32 *)th, sh, n2, offs, batch);
        else
            hipLaunchKernelGGL((four_step_columns_indexed_kernel<Sh, PolW, 1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)ybuf, (const c32 *)tw, (const c32 *)tl,
                               (const c32 *)th, sh, n2, offs, batch);
    }
    static ColumnDesc desc(int variant)
    {
        ColumnDesc d{};
        d.n1 = M;
        d.variant = variant;
        d.flags = F;
        d.cols = C;
        d.threads = T;
        d.lds_bytes = Pol::kLdsElems * elem_bytes<F>();
        d.nrad = (int)sizeof...(Rs);
        const int r[] = {Rs...};
        for (int i = 0; i < d.nrad; ++i)
            d.radices[i] = r[i];
        d.launch = &launch;
        d.kernel[0] = (const void *)&four_step_columns_kernel<Sh, Pol, -1>;
        d.kernel[1] = (const void *)&four_step_columns_kernel<Sh, Pol, 1>;
        if constexpr ((F & kFrames) != 0) {
            d.launch_frames = &launch_frames;
            d.kernel_frames[0] = (const void *)&four_step_columns_frames_kernel<Sh, Pol, -1>;
            d.kernel_frames[1] = (const void *)&four_step_columns_frames_kernel<Sh, Pol, 1>;
        }
        if constexpr ((F & kShifted) != 0) {
            d.launch_shifted = &launch_shifted;
            d.kernel_shifted[0] = (const void *)&four_step_columns_shifted_kernel<Sh, PolW, -1>;
            d.kernel_shifted[1] = (const void *)&four_step_columns_shifted_kernel<Sh, PolW, 1>;
        }
        if constexpr ((F & kIndexed) != 0) {
            d.launch_indexed = &launch_indexed;
            d.kernel_indexed[0] = (const void *)&four_step_columns_indexed_kernel<Sh, PolW, -1>;
            d.kernel_indexed[1] = (const void *)&four_step_columns_indexed_kernel<Sh, PolW, 1>;
        }
        if constexpr ((F & kYBlocked) != 0) {
            d.launch_yblocked = &launch_yblocked;
            d.kernel_yblocked[0] = (const void *)&four_step_columns_kernel<Sh, PolB, -1>;
            d.kernel_yblocked[1] = (const void *)&four_step_columns_kernel<Sh, PolB, 1>;
        }
        if constexpr ((F & kYBlocked) != 0 && (F & kFrames) != 0) {
            d.launch_frames_yblocked = &launch_frames_yblocked;
            d.kernel_frames_yblocked[0] =
                (const void *)&four_step_columns_frames_kernel<Sh, PolB, -1>;
            d.kernel_frames_yblocked[1] =
                (const void *)&four_step_columns_frames_kernel<Sh, PolB, 1>;
        }
        return d;
    }
};

template <int M, int T, int C, int PS, int F, int... Rs>
struct RowInst {
    using Sh = Shape<M, T, Radices<Rs...>>;
    using Pol = RowPolicy<Sh, C, PS, (F & kNT) != 0, hoist_mask<sizeof...(Rs), F>(),
                          (F & kXcd) != 0, waves<F>(), (F & kPlainLane) != 0,
                          (F & kSplit) != 0, false, (F & kTwPair) != 0>;
    using PolW = RowPolicy<Sh, C, PS, (F & kNT) != 0, hoist_mask<sizeof...(Rs), F>(),
                           (F & kXcd) != 0, waves<F>(), (F & kPlainLane) != 0,
                           (F & kSplit) != 0, true, (F & kTwPair) != 0>;
    using PolB = RowPolicy<Sh, C, PS, (F & kNT) != 0, hoist_mask<sizeof...(Rs), F>(),
                           (F & kXcd) != 0, waves<F>(), (F & kPlainLane) != 0,
                           (F & kSplit) != 0, false, (F & kTwPair) != 0, true>;
    static void launch_yblocked(int dir, const void *ybuf, void *out, const void *tw, int n1,
                                uint64_t batch, unsigned grid, hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL((four_step_rows_kernel<Sh, PolB, -1>), g, b, 0, s,
                               (const c32 *)ybuf, (c32 *)out, (const c32 *)tw, n1, batch);
        else
            hipLaunchKernelGGL((four_step_rows_kernel<Sh, PolB, 1>), g, b, 0, s,
                               (const c32 *)ybuf, (c32 *)out, (const c32 *)tw, n1, batch);
    }
    static void launch_shifted(int dir, const void *ybuf, void *out, const void *tw, int n1,
                               uint64_t batch, int shift, unsigned grid, hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL((four_step_rows_shifted_kernel<Sh, PolW, -1>), g, b, 0, s,
                               (const c32 *)ybuf, (c32 *)out, (const c32 *)tw, n1, batch, shift);
        else
            hipLaunchKernelGGL((four_step_rows_shifted_kernel<Sh, PolW, 1>), g, b, 0, s,
                               (const c32 *)ybuf, (c32 *)out, (const c32 *)tw, n1, batch, shift);
    }
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
    static void launch_indexed(int dir, const void *in, const void *ybuf, void *out,
                               const void *tw, int n1, const uint64_t *offs, uint64_t batch,
                               unsigned grid, hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL((four_step_rows_indexed_kernel<Sh, PolW, -1>), g, b, 0, s,
                               (const c32 *)in, (const c32 *)ybuf, (c32 *)out,
                               (const c32 *)tw, n1, offs, batch);
        else
            hipLaunchKernelGGL((four_step_rows_indexed_kernel<Sh, PolW, 1>), g, b, 0, s,
                               (const c32 *)in, (const c32 *)ybuf, (c32 *)out,
                               (const c32 *)tw, n1, offs, batch);
    }
    static RowDesc desc(int variant)
    {
        RowDesc d{};
        d.n2 = M;
        d.variant = variant;
        d.flags = F;
        d.rows = C;
        d.threads = T;
        d.lds_bytes = Pol::kLdsElems * elem_bytes<F>();
        d.nrad = (int)sizeof...(Rs);
        const int r[] = {Rs...};
        for (int i = 0; i < d.nrad; ++i)
            d.radices[i] = r[i];
        d.launch = &launch;
        d.kernel[0] = (const void *)&four_step_rows_kernel<Sh, Pol, -1>;
        d.kernel[1] = (const void *)&four_step_rows_kernel<Sh, Pol, 1>;
        if constexpr ((F & kShifted) != 0) {
            d.launch_shifted = &launch_shifted;
            d.kernel_shifted[0] = (const void *)&four_step_rows_shifted_kernel<Sh, PolW, -1>;
            d.kernel_shifted[1] = (const void *)&four_step_rows_shifted_kernel<Sh, PolW, 1>;
        }
        if constexpr ((F & kIndexed) != 0) {
            d.launch_indexed = &launch_indexed;
            d.kernel_indexed[0] = (const void *)&four_step_rows_indexed_kernel<Sh, PolW, -1>;
            d.kernel_indexed[1] = (const void *)&four_step_rows_indexed_kernel<Sh, PolW, 1>;
        }
        if constexpr ((F & kYBlocked) != 0) {
            d.launch_yblocked = &launch_yblocked;
            d.kernel_yblocked[0] = (const void *)&four_step_rows_kernel<Sh, PolB, -1>;
            d.kernel_yblocked[1] = (const void *)&four_step_rows_kernel<Sh, PolB, 1>;
        }
        return d;
    }
};

}  // namespace fs
}  // namespace fftseg
