// Single-pass instances with one LDS pad element every 32 (instead of every
// 16), or with the XOR-swizzled layout (kLdsXor), for the autotuner: fewer
// padding bytes, a different bank pattern.
// Kept in a translation unit of their own so they do not share inlined code
// with the other instances of the same shapes.
#include "spinst.hpp"

namespace fftseg {

SinglePassDesc pad32_desc(int config, int variant, int grid_mult)
{
    using namespace sp;
    //                       N      T   S  PS  F                    radices
    switch (config) {
    case 0:
        return SpInst<4096, 128, 2, 5, kClassic | kNT, 16, 16, 16>::desc(variant, grid_mult);
    case 1:
        return SpInst<1024, 64, 2, 5, kNT | kPlain, 16, 16, 4>::desc(variant, grid_mult);
    case 2:
        return SpInst<8192, 512, 1, 5, kPrefetch, 16, 16, 16, 2>::desc(variant, grid_mult);
    case 3:
        return SpInst<2048, 128, 1, 5, kNT | kPlain, 16, 16, 8>::desc(variant, grid_mult);
    case 4:
        return SpInst<4096, 128, 2, kLdsXor, kClassic | kNT | kW2, 16, 16, 16>::desc(variant,
                                                                              grid_mult);
    default:
        return SinglePassDesc{};
    }
}

}  // namespace fftseg
