// Compile-time description of one single-pass kernel instance (length,
// threads per segment, segments per workgroup, LDS padding, flags, radix
// list) and the descriptor the planner sees for it.
#pragma once

#include "registry.hpp"
#include "tile.hpp"

namespace fftseg {
namespace sp {

// F: flag bits.  kNT = streamed (non-temporal) global access; kNoHoist =
// every stage reloads its twiddles per segment; kHoistLast = only the last
// stage keeps its twiddles in registers across segments (default: all
// stages do); kW2 / kW3 = the register allocation must allow 2 / 3 waves
// per SIMD; kPlainLane / kPlainLds = the lane index is kept across the
// segments of the persistent loop / LDS addresses are computed per access;
// kClassic = the plainly written kernel (see SinglePassPolicy); kAux = this
// row also provides the length's frame (overlapping segment) and
// real-input kernels (one row per length); kPrefetch = the plainly written
// kernel with the next segment's loads issued ahead (implies the classic
// policy); kSplit = the kernel with split (real, then imaginary) LDS
// exchanges; kW4 / kW8 = 4 / 8 waves per SIMD; kIndexed = the row also
// provides the kernel over segments at listed offsets; kTwPair = stages that
// reload their twiddles read them as pairs (tw_pair_low); kFrames = the row
// also provides a frame kernel (not the real-input ones); kXcdFrames = its
// frame kernel deals the frames to the XCDs in contiguous runs.  Frame
// kernels read overlapping frames through the cache
// (single_pass_strided_kernel).  kSmallBatch = the planner's choice for
// batches too small to give the default kernel two workgroups per CU.
constexpr int kNT = 1, kNoHoist = 2, kHoistLast = 4, kW2 = 8, kW3 = 16, kPlainLane = 32,
              kPlainLds = 64, kPlain = kPlainLane | kPlainLds, kClassic = 128, kAux = 256,
              kPrefetch = 512, kSplit = 1024, kW4 = 2048, kW8 = 4096, kIndexed = 8192,
              kTwPair = 16384, kFrames = 32768, kXcdFrames = 65536, kSmallBatch = 131072;

template <int NS, int F>
constexpr int hoist_mask()
{
    return (F & kNoHoist) ? 0 : (F & kHoistLast) ? (1 << (NS - 1)) : -1;
}
template <int F>
constexpr int waves()
{
    return (F & kW8) ? 8 : (F & kW4) ? 4 : (F & kW3) ? 3 : (F & kW2) ? 2 : 1;
}

template <int N, int T, int S, int PS, int F, int... Rs>
struct SpInst {
    using Sh = Shape<N, T, Radices<Rs...>>;
    using Pol = SinglePassPolicy<Sh, S, PS, (F & kNT) != 0, hoist_mask<sizeof...(Rs), F>(),
                                 false, waves<F>(), (F & kPlainLane) != 0,
                                 (F & kPlainLds) != 0, (F & (kClassic | kPrefetch)) != 0,
                                 (F & kSplit) != 0, (F & kTwPair) != 0>;
    static_assert(!((F & kSplit) && (F & (kAux | kClassic))),
                  "split exchanges: transform and frame kernels only");

    using kernel_fn = void (*)(const c32 *, c32 *, const c32 *, uint64_t);
    template <int D>
    static constexpr kernel_fn kernel()
    {
        if constexpr ((F & kSplit) != 0 && (F & kPrefetch) != 0)
            return &single_pass_split_prefetch_kernel<Sh, Pol, D>;
        else if constexpr ((F & kSplit) != 0)
            return &single_pass_split_kernel<Sh, Pol, D>;
        else if constexpr ((F & kPrefetch) != 0)
            return &single_pass_prefetch_kernel<Sh, Pol, D>;
        else if constexpr ((F & kClassic) != 0)
            return &single_pass_plain_kernel<Sh, Pol, D>;
        else
            return &single_pass_kernel<Sh, Pol, D>;
    }
    static void launch(int dir, const void *in, void *out, const void *tw,
                       uint64_t batch, unsigned grid, hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL(kernel<-1>(), g, b, 0, s, (const c32 *)in, (c32 *)out,
                               (const c32 *)tw, batch);
        else
            hipLaunchKernelGGL(kernel<1>(), g, b, 0, s, (const c32 *)in, (c32 *)out,
                               (const c32 *)tw, batch);
    }
    static constexpr int kFrameMode = (F & kXcdFrames) ? 3 : 1;
    static void launch_strided(int dir, const void *in, void *out, const void *tw,
                               uint64_t batch, uint64_t in_stride, uint64_t out_stride,
                               const float *window, unsigned grid, hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL((single_pass_strided_kernel<Sh, Pol, -1, kFrameMode>), g, b, 0,
                               s, (const c32 *)in, (c32 *)out, (const c32 *)tw, batch,
                               in_stride, out_stride, window);
        else
            hipLaunchKernelGGL((single_pass_strided_kernel<Sh, Pol, 1, kFrameMode>), g, b, 0,
                               s, (const c32 *)in, (c32 *)out, (const c32 *)tw, batch,
                               in_stride, out_stride, window);
    }
    static void launch_real(int dir, const void *in, void *out, const void *tw, const void *hw,
                            uint64_t batch, unsigned grid, hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL((real_forward_kernel<Sh, Pol>), g, b, 0, s, (const c32 *)in,
                               (c32 *)out, (const c32 *)tw, (const c32 *)hw, batch);
        else
            hipLaunchKernelGGL((real_inverse_kernel<Sh, Pol>), g, b, 0, s, (const c32 *)in,
                               (c32 *)out, (const c32 *)tw, (const c32 *)hw, batch);
    }
    static void launch_indexed(int dir, const void *in, void *out, const void *tw,
                               const uint64_t *offs, uint64_t batch, unsigned grid,
                               hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL((single_pass_indexed_kernel<Sh, Pol, -1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)out, (const c32 *)tw, offs, batch);
        else
            hipLaunchKernelGGL((single_pass_indexed_kernel<Sh, Pol, 1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)out, (const c32 *)tw, offs, batch);
    }
    static SinglePassDesc desc(int variant, int grid_mult)
    {
        SinglePassDesc d{};
        d.grid_mult = grid_mult;
        d.n = N;
        d.variant = variant;
        d.threads = T;
        d.segs_per_wg = S;
        d.pad_shift = PS;
        d.nontemporal = (F & kNT) != 0;
        d.small_batch = (F & kSmallBatch) != 0;
        d.hoist = hoist_mask<sizeof...(Rs), F>();
        d.lds_bytes = Pol::kLdsElems * (int)((F & kSplit) ? sizeof(float) : sizeof(c32));
        d.nrad = (int)sizeof...(Rs);
        const int r[] = {Rs...};
        for (int i = 0; i < d.nrad; ++i)
            d.radices[i] = r[i];
        d.launch = &launch;
        d.kernel[0] = (const void *)kernel<-1>();
        d.kernel[1] = (const void *)kernel<1>();
        if constexpr ((F & kIndexed) != 0) {
            d.launch_indexed = &launch_indexed;
            d.kernel_indexed[0] = (const void *)&single_pass_indexed_kernel<Sh, Pol, -1>;
            d.kernel_indexed[1] = (const void *)&single_pass_indexed_kernel<Sh, Pol, 1>;
        }
        if constexpr ((F & (kAux | kFrames | kXcdFrames)) != 0) {
            d.launch_strided = &launch_strided;
            d.kernel_strided[0] =
                (const void *)&single_pass_strided_kernel<Sh, Pol, -1, kFrameMode>;
            d.kernel_strided[1] =
                (const void *)&single_pass_strided_kernel<Sh, Pol, 1, kFrameMode>;
        }
        if constexpr ((F & kAux) != 0) {
            d.launch_real = &launch_real;
            d.kernel_real[0] = (const void *)&real_forward_kernel<Sh, Pol>;
            d.kernel_real[1] = (const void *)&real_inverse_kernel<Sh, Pol>;
        }
        return d;
    }
};

}  // namespace sp
}  // namespace fftseg
