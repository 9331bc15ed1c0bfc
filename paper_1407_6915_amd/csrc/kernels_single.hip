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
// per SIMD.
constexpr int kNT = 1, kNoHoist = 2, kHoistLast = 4, kW2 = 8, kW3 = 16;

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
                                 false, waves<F>()>;

    static void launch(int dir, const void *in, void *out, const void *tw,
                       uint64_t batch, unsigned grid, hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL((single_pass_kernel<Sh, Pol, -1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)out, (const c32 *)tw, batch);
        else
            hipLaunchKernelGGL((single_pass_kernel<Sh, Pol, 1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)out, (const c32 *)tw, batch);
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
        d.kernel[0] = (const void *)&single_pass_kernel<Sh, Pol, -1>;
        d.kernel[1] = (const void *)&single_pass_kernel<Sh, Pol, 1>;
        return d;
    }
};

// Variant 0 is the measured best of each length on MI355X (GB/s at 8 GiB
// batches); grid_mult = resident workgroup waves per CU of the persistent
// grid (0: one workgroup per tile).
//                 N      T    S  PS  F              radices     variant, grid_mult
const SinglePassDesc kTable[] = {
    SpInst<2, 1, 64, 0, kNT, 2>::desc(0, 0),
    SpInst<4, 1, 64, 0, kNT, 4>::desc(0, 0),
    SpInst<8, 1, 64, 0, kNT, 8>::desc(0, 0),
    SpInst<16, 1, 64, 0, kNT, 16>::desc(0, 0),
    SpInst<32, 4, 32, 4, kNT, 8, 4>::desc(0, 0),
    SpInst<64, 8, 32, 4, kNT, 8, 8>::desc(0, 0),
    SpInst<128, 8, 32, 4, kNT, 16, 8>::desc(0, 0),
    SpInst<256, 16, 8, 4, kNT, 16, 16>::desc(0, 32),
    SpInst<256, 16, 8, 4, 0, 16, 16>::desc(1, 0),
    SpInst<256, 16, 16, 4, 0, 16, 16>::desc(2, 0),
    SpInst<512, 64, 4, 4, kNT, 8, 8, 8>::desc(0, 16),
    SpInst<512, 32, 8, 4, kNT, 16, 16, 2>::desc(1, 16),
    SpInst<1024, 64, 4, 4, kNT, 16, 16, 4>::desc(0, 0),
    SpInst<1024, 64, 4, 4, 0, 16, 16, 4>::desc(1, 0),
    SpInst<1024, 64, 4, 4, 0, 4, 16, 16>::desc(2, 32),
    SpInst<1024, 128, 2, 4, 0, 8, 8, 16>::desc(3, 32),
    SpInst<1024, 64, 2, 4, kNT, 16, 16, 4>::desc(4, 32),
    SpInst<2048, 128, 2, 4, kNT, 16, 16, 8>::desc(0, 16),
    SpInst<2048, 128, 1, 4, kNT, 16, 16, 8>::desc(1, 16),
    SpInst<2048, 64, 2, 4, kNT, 16, 16, 8>::desc(2, 16),
    SpInst<4096, 128, 2, 4, kNT | kHoistLast | kW2, 16, 16, 16>::desc(0, 32),
    SpInst<4096, 128, 2, 4, kNT | kNoHoist | kW2, 16, 16, 16>::desc(1, 32),
    SpInst<4096, 128, 2, 4, kNT | kW2, 16, 16, 16>::desc(2, 32),
    SpInst<4096, 128, 2, 4, kNT, 16, 16, 16>::desc(3, 32),
    SpInst<4096, 256, 1, 4, kNT, 16, 16, 16>::desc(4, 32),
    SpInst<4096, 256, 1, 0, kNT, 16, 16, 16>::desc(5, 32),
    SpInst<4096, 512, 1, 4, kNT, 8, 8, 8, 8>::desc(6, 32),
    SpInst<4096, 256, 1, 4, kNT | kHoistLast | kW3, 16, 16, 16>::desc(7, 32),
    SpInst<8192, 512, 1, 4, kNT, 16, 16, 16, 2>::desc(0, 4),
    SpInst<8192, 256, 1, 4, kNT | kNoHoist, 32, 16, 16>::desc(1, 4),
    SpInst<8192, 512, 1, 4, kNT | kNoHoist, 16, 16, 16, 2>::desc(2, 4),
    SpInst<8192, 512, 1, 4, kNT | kHoistLast | kW2, 16, 16, 16, 2>::desc(3, 8),
    SpInst<16384, 1024, 1, 4, kNT | kNoHoist, 16, 16, 16, 4>::desc(0, 8),
    SpInst<16384, 512, 1, 4, kNT | kNoHoist, 16, 16, 16, 4>::desc(1, 8),
    SpInst<16384, 1024, 1, 4, kNoHoist, 16, 16, 16, 4>::desc(2, 8),
    SpInst<16384, 1024, 1, 0, kNT | kNoHoist, 16, 16, 16, 4>::desc(3, 8),
    // mixed radix 2/3/5
    SpInst<1000, 100, 2, 4, kNT, 10, 10, 10>::desc(0, 32),
    SpInst<1000, 100, 2, 4, 0, 10, 10, 10>::desc(1, 32),
    SpInst<1000, 125, 2, 4, kNT, 8, 5, 5, 5>::desc(2, 32),
    SpInst<1000, 200, 1, 4, kNT, 5, 5, 5, 8>::desc(3, 32),
    SpInst<1536, 96, 2, 4, kNT, 16, 16, 6>::desc(0, 32),
    SpInst<1536, 96, 2, 4, 0, 16, 16, 6>::desc(1, 32),
    SpInst<1536, 192, 1, 4, kNT, 8, 8, 8, 3>::desc(2, 32),
    SpInst<6000, 400, 1, 4, kNT, 16, 15, 25>::desc(0, 16),
    SpInst<6000, 400, 1, 4, 0, 16, 15, 25>::desc(1, 16),
    SpInst<6000, 400, 1, 4, kNT | kNoHoist, 16, 15, 25>::desc(2, 0),
    SpInst<6000, 300, 1, 4, kNT | kNoHoist, 20, 20, 15>::desc(3, 0),
    SpInst<6000, 400, 1, 4, kNT | kHoistLast | kW2, 16, 15, 25>::desc(4, 16),
};

}  // namespace

const SinglePassDesc *single_pass_table(int *count)
{
    *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace fftseg
