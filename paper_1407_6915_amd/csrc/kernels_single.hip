// Single-pass (LDS-resident) kernel variants per segment length.
//
// Variant 0 of each length is the planner's default; the others are the
// autotuner's candidates (different radix orders, threads per segment,
// segments per workgroup and LDS padding).
#include "registry.hpp"
#include "tile.hpp"

namespace fftseg {
namespace {

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
// policy).
constexpr int kNT = 1, kNoHoist = 2, kHoistLast = 4, kW2 = 8, kW3 = 16, kPlainLane = 32,
              kPlainLds = 64, kPlain = kPlainLane | kPlainLds, kClassic = 128, kAux = 256,
              kPrefetch = 512;

template <int NS, int F>
constexpr int hoist_mask()
{
    return (F & kNoHoist) ? 0 : (F & kHoistLast) ? (1 << (NS - 1)) : -1;
}
template <int F>
constexpr int waves()
{
    return (F & kW3) ? 3 : (F & kW2) ? 2 : 1;
}

template <int N, int T, int S, int PS, int F, int... Rs>
struct SpInst {
    using Sh = Shape<N, T, Radices<Rs...>>;
    using Pol = SinglePassPolicy<Sh, S, PS, (F & kNT) != 0, hoist_mask<sizeof...(Rs), F>(),
                                 false, waves<F>(), (F & kPlainLane) != 0,
                                 (F & kPlainLds) != 0, (F & (kClassic | kPrefetch)) != 0>;

    using kernel_fn = void (*)(const c32 *, c32 *, const c32 *, uint64_t);
    template <int D>
    static constexpr kernel_fn kernel()
    {
        if constexpr ((F & kPrefetch) != 0)
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
    static void launch_strided(int dir, const void *in, void *out, const void *tw,
                               uint64_t batch, uint64_t in_stride, uint64_t out_stride,
                               const float *window, unsigned grid, hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL((single_pass_strided_kernel<Sh, Pol, -1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)out, (const c32 *)tw, batch, in_stride,
                               out_stride, window);
        else
            hipLaunchKernelGGL((single_pass_strided_kernel<Sh, Pol, 1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)out, (const c32 *)tw, batch, in_stride,
                               out_stride, window);
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
        d.hoist = hoist_mask<sizeof...(Rs), F>();
        d.lds_bytes = Pol::kLdsElems * (int)sizeof(c32);
        d.nrad = (int)sizeof...(Rs);
        const int r[] = {Rs...};
        for (int i = 0; i < d.nrad; ++i)
            d.radices[i] = r[i];
        d.launch = &launch;
        d.kernel[0] = (const void *)kernel<-1>();
        d.kernel[1] = (const void *)kernel<1>();
        if constexpr ((F & kAux) != 0) {
            d.launch_strided = &launch_strided;
            d.kernel_strided[0] = (const void *)&single_pass_strided_kernel<Sh, Pol, -1>;
            d.kernel_strided[1] = (const void *)&single_pass_strided_kernel<Sh, Pol, 1>;
            d.launch_real = &launch_real;
            d.kernel_real[0] = (const void *)&real_forward_kernel<Sh, Pol>;
            d.kernel_real[1] = (const void *)&real_inverse_kernel<Sh, Pol>;
        }
        return d;
    }
};

// Variant 0 is the measured best of each length on MI355X (GB/s at 8 GiB
// batches); grid_mult = resident workgroup waves per CU of the persistent
// grid (0: one workgroup per tile).
//                 N      T    S  PS  F              radices     variant, grid_mult
const SinglePassDesc kTable[] = {
    SpInst<2, 1, 64, 0, kNT | kPlain | kAux, 2>::desc(0, 0),
    SpInst<4, 1, 64, 0, kNT | kPlain | kAux, 4>::desc(0, 0),
    SpInst<8, 1, 64, 0, kNT | kPlain | kAux, 8>::desc(0, 0),
    SpInst<16, 1, 64, 0, kNT | kPlain | kAux, 16>::desc(0, 0),
    SpInst<32, 4, 32, 4, kNT | kPlain | kAux, 8, 4>::desc(0, 0),
    SpInst<64, 8, 32, 4, kNT | kPlain | kAux, 8, 8>::desc(0, 0),
    SpInst<128, 8, 32, 4, kNT | kPlain | kAux, 16, 8>::desc(0, 0),
    SpInst<256, 16, 8, 4, kPlain | kAux, 16, 16>::desc(0, 0),
    SpInst<256, 16, 8, 4, kNT | kPlain, 16, 16>::desc(1, 32),
    SpInst<256, 16, 8, 4, kNT, 16, 16>::desc(2, 32),
    SpInst<256, 16, 8, 4, kClassic | kNT, 16, 16>::desc(3, 64),
    SpInst<512, 64, 4, 4, kNT | kPlain, 8, 8, 8>::desc(0, 0),
    SpInst<512, 64, 4, 4, kPlain, 8, 8, 8>::desc(1, 32),
    SpInst<512, 32, 8, 4, kNT | kPlain, 16, 16, 2>::desc(2, 64),
    SpInst<512, 64, 4, 4, kClassic | kNT | kAux, 8, 8, 8>::desc(3, 32),
    SpInst<1024, 64, 2, 4, kNT | kPlain | kAux, 16, 16, 4>::desc(0, 64),
    SpInst<1024, 64, 4, 4, kNT | kPlain, 16, 16, 4>::desc(1, 64),
    SpInst<1024, 64, 4, 4, kPlain, 16, 16, 4>::desc(2, 32),
    SpInst<1024, 64, 4, 4, kNT, 16, 16, 4>::desc(3, 32),
    SpInst<1024, 64, 4, 4, kClassic, 16, 16, 4>::desc(4, 32),
    SpInst<2048, 128, 1, 4, kNT | kPlain | kAux, 16, 16, 8>::desc(0, 64),
    SpInst<2048, 128, 2, 4, kNT | kPlain, 16, 16, 8>::desc(1, 64),
    SpInst<2048, 128, 2, 4, kPlain, 16, 16, 8>::desc(2, 32),
    SpInst<2048, 128, 2, 4, kClassic, 16, 16, 8>::desc(3, 32),
    SpInst<4096, 128, 2, 4, kClassic | kNT, 16, 16, 16>::desc(0, 64),
    SpInst<4096, 128, 2, 4, kClassic, 16, 16, 16>::desc(1, 64),
    SpInst<4096, 512, 1, 4, kNT | kPlain | kAux, 8, 8, 8, 8>::desc(2, 64),
    SpInst<4096, 256, 1, 0, kNT | kPlain, 16, 16, 16>::desc(3, 32),
    SpInst<4096, 128, 2, 0, kNT | kPlain, 16, 16, 16>::desc(4, 32),
    SpInst<4096, 256, 1, 4, kPlain, 16, 16, 16>::desc(5, 32),
    SpInst<4096, 256, 1, 0, kClassic | kNT, 16, 16, 16>::desc(6, 32),
    SpInst<4096, 512, 1, 4, kClassic | kNT, 8, 8, 8, 8>::desc(7, 32),
    shuffle4096_desc(8, 64, 2),
    shuffle4096_desc(9, 64, 0),
    shuffle4096_desc(10, 32, 2),
    SpInst<4096, 256, 1, 0, kPrefetch | kNT, 16, 16, 16>::desc(11, 32),
    SpInst<4096, 512, 1, 4, kPrefetch | kNT, 8, 8, 8, 8>::desc(12, 32),
    SpInst<8192, 512, 1, 4, kPrefetch, 16, 16, 16, 2>::desc(0, 32),
    SpInst<8192, 512, 1, 4, kClassic, 16, 16, 16, 2>::desc(1, 32),
    SpInst<8192, 512, 1, 4, kPlain, 16, 16, 16, 2>::desc(2, 32),
    SpInst<8192, 512, 1, 4, kNT | kPlain | kAux, 16, 16, 16, 2>::desc(3, 32),
    SpInst<8192, 256, 1, 4, kNT | kNoHoist, 32, 16, 16>::desc(4, 32),
    SpInst<8192, 512, 1, 4, kPrefetch | kNT, 16, 16, 16, 2>::desc(5, 32),
    SpInst<16384, 1024, 1, 4, kNT | kNoHoist | kPlain | kAux, 16, 16, 16, 4>::desc(0, 32),
    SpInst<16384, 1024, 1, 4, kNT | kNoHoist, 16, 16, 16, 4>::desc(1, 32),
    SpInst<16384, 512, 1, 4, kNT | kNoHoist, 16, 16, 16, 4>::desc(2, 32),
    // mixed radix 2/3/5
    SpInst<1000, 100, 2, 4, kClassic, 10, 10, 10>::desc(0, 64),
    SpInst<1000, 100, 2, 4, kPlain, 10, 10, 10>::desc(1, 64),
    SpInst<1000, 100, 2, 4, kNT | kPlain | kAux, 10, 10, 10>::desc(2, 32),
    SpInst<1000, 125, 2, 4, kNT | kPlain, 8, 5, 5, 5>::desc(3, 32),
    SpInst<1536, 96, 2, 4, kNT | kPlain | kAux, 16, 16, 6>::desc(0, 64),
    SpInst<1536, 96, 2, 4, kPlain, 16, 16, 6>::desc(1, 32),
    SpInst<1536, 96, 2, 4, kNT, 16, 16, 6>::desc(2, 32),
    SpInst<1536, 96, 2, 4, kClassic | kNT, 16, 16, 6>::desc(3, 64),
    SpInst<6000, 400, 1, 4, kClassic | kNT, 16, 15, 25>::desc(0, 32),
    SpInst<6000, 400, 1, 4, kNT | kNoHoist, 16, 15, 25>::desc(1, 0),
    SpInst<6000, 300, 1, 4, kNT | kNoHoist | kAux, 20, 20, 15>::desc(2, 32),
    SpInst<6000, 400, 1, 4, kNT | kNoHoist | kPlain, 16, 15, 25>::desc(3, 32),
    SpInst<6000, 400, 1, 4, kPrefetch | kNT, 16, 15, 25>::desc(4, 32),
};

}  // namespace

const SinglePassDesc *single_pass_table(int *count)
{
    *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace fftseg
