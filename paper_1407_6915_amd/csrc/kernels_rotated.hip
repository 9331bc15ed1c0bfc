// One-pass kernels with the thread -> butterfly assignment rotated, for
// outputs whose base pointer sits inside a 128-byte line: the rotation puts
// each wave's stores back on line boundaries.  The same shape, radices,
// padding and access flags as the length's default variant.  Kept in a
// translation unit of their own so they do not share inlined code with the
// table's instances.
#include "registry.hpp"
#include "tile.hpp"

namespace fftseg {
namespace {

template <int N, int T, int S, int PS, int... Rs>
struct RotInst {
    using Sh = Shape<N, T, Radices<Rs...>>;
    // streamed access, all twiddles held in registers, the plainly written
    // kernel: the policy of the 4096-point default
    using Pol = SinglePassPolicy<Sh, S, PS, true, -1, false, 1, false, false, true>;
    static void launch(int dir, const void *in, void *out, const void *tw, uint64_t batch,
                       int rot, unsigned grid, hipStream_t s)
    {
        const dim3 g(grid), b(Pol::kThreads);
        if (dir < 0)
            hipLaunchKernelGGL((single_pass_rotated_kernel<Sh, Pol, -1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)out, (const c32 *)tw, batch, rot);
        else
            hipLaunchKernelGGL((single_pass_rotated_kernel<Sh, Pol, 1>), g, b, 0, s,
                               (const c32 *)in, (c32 *)out, (const c32 *)tw, batch, rot);
    }
    static const void *kernel(int i)
    {
        return i ? (const void *)&single_pass_rotated_kernel<Sh, Pol, 1>
                 : (const void *)&single_pass_rotated_kernel<Sh, Pol, -1>;
    }
};

}  // namespace

sp_rotated_launch_fn rotated_launcher(uint64_t n, int *variant, const void **kernels)
{
    using R4096 = RotInst<4096, 128, 2, 4, 16, 16, 16>;
    if (n == 4096) {
        *variant = 0;
        kernels[0] = R4096::kernel(0);
        kernels[1] = R4096::kernel(1);
        return &R4096::launch;
    }
    return nullptr;
}

}  // namespace fftseg
