// Single-pass (LDS-resident) kernel variants per segment length.
//
// Variant 0 of each length is the planner's default; the others are the
// autotuner's candidates (different radix orders, threads per segment,
// segments per workgroup and LDS padding).
#include "spinst.hpp"

namespace fftseg {
namespace {

using namespace sp;

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
    SpInst<512, 16, 16, 4, kClassic | kNT, 32, 16>::desc(4, 32),
    SpInst<1024, 64, 2, 4, kNT | kPlain | kAux | kSmallBatch, 16, 16, 4>::desc(7, 64),
    SpInst<1024, 64, 4, 4, kNT | kPlain, 16, 16, 4>::desc(1, 64),
    SpInst<1024, 64, 4, 4, kPlain, 16, 16, 4>::desc(2, 32),
    SpInst<1024, 64, 4, 4, kNT, 16, 16, 4>::desc(3, 32),
    SpInst<1024, 64, 4, 4, kClassic, 16, 16, 4>::desc(4, 32),
    pad32_desc(1, 5, 64),
    SpInst<1024, 64, 4, 4, kClassic | kNT, 16, 16, 4>::desc(6, 32),
    // radix 32, eight segments per workgroup: 2.83-2.85 ms per 8 GiB against
    // 3.03-3.04 for the radix-16 kernel of variant 7, which small batches take
    // (1024 segments: 128 workgroups of this kernel)
    SpInst<1024, 32, 8, 4, kClassic | kNT, 32, 32>::desc(0, 32),
    SpInst<1024, 32, 4, 4, kClassic | kNT, 32, 32>::desc(8, 32),
    SpInst<1024, 32, 16, 4, kClassic | kNT, 32, 32>::desc(9, 32),
    SpInst<2048, 128, 1, 4, kNT | kPlain | kAux | kSmallBatch, 16, 16, 8>::desc(6, 64),
    SpInst<2048, 128, 2, 4, kNT | kPlain, 16, 16, 8>::desc(1, 64),
    SpInst<2048, 128, 2, 4, kPlain, 16, 16, 8>::desc(2, 32),
    SpInst<2048, 128, 2, 4, kClassic, 16, 16, 8>::desc(3, 32),
    pad32_desc(3, 4, 64),
    SpInst<2048, 128, 2, 4, kClassic | kNT, 16, 16, 8>::desc(5, 32),
    // 2.86-2.87 ms per 8 GiB against 2.99-3.04 for the 16-16-8 kernel of variant 6
    // (small batches)
    SpInst<2048, 64, 4, 4, kClassic | kNT, 32, 8, 8>::desc(0, 32),
    SpInst<4096, 128, 2, 4, kClassic | kNT, 16, 16, 16>::desc(0, 32),
    SpInst<4096, 128, 2, 4, kClassic, 16, 16, 16>::desc(1, 64),
    // (variant 3 first: the length's frame and real-input kernels are the
    // first row with them; the frame kernel takes 2.89 ms per 2^18 frames
    // every 1024 samples at this grid of 16, 2.92-2.98 at 32)
    SpInst<4096, 256, 1, 0, kNT | kPlain | kAux, 16, 16, 16>::desc(3, 16),
    SpInst<4096, 512, 1, 4, kNT | kPlain | kAux, 8, 8, 8, 8>::desc(2, 64),
    SpInst<4096, 128, 2, 0, kNT | kPlain, 16, 16, 16>::desc(4, 32),
    SpInst<4096, 256, 1, 4, kPlain, 16, 16, 16>::desc(5, 32),
    SpInst<4096, 256, 1, 0, kClassic | kNT, 16, 16, 16>::desc(6, 32),
    SpInst<4096, 512, 1, 4, kClassic | kNT, 8, 8, 8, 8>::desc(7, 32),
    shuffle4096_desc(8, 64, 2),
    shuffle4096_desc(9, 64, 0),
    shuffle4096_desc(10, 32, 2),
    SpInst<4096, 256, 1, 0, kPrefetch | kNT, 16, 16, 16>::desc(11, 32),
    SpInst<4096, 512, 1, 4, kPrefetch | kNT, 8, 8, 8, 8>::desc(12, 32),
    pad32_desc(0, 13, 64),
    pad32_desc(4, 14, 32),
    SpInst<4096, 256, 1, 0, kNT | kPlain | kXcdFrames, 16, 16, 16>::desc(15, 32),
    pad32_desc(2, 8, 16),
    SpInst<8192, 512, 1, 4, kClassic, 16, 16, 16, 2>::desc(1, 32),
    SpInst<8192, 512, 1, 4, kPlain, 16, 16, 16, 2>::desc(2, 32),
    // the length's frame kernel (the first row with one): one workgroup per
    // frame, 3.05 ms per 2^17 frames every 2048 samples against 4.06 through
    // the real-input row below
    SpInst<8192, 512, 1, 4, kNT | kNoHoist | kTwPair | kW4 | kFrames, 16, 16, 16, 2>::desc(7, 0),
    SpInst<8192, 512, 1, 4, kNT | kPlain | kAux, 16, 16, 16, 2>::desc(3, 32),
    SpInst<8192, 256, 1, 4, kNT | kNoHoist, 32, 16, 16>::desc(4, 32),
    SpInst<8192, 512, 1, 4, kPrefetch | kNT, 16, 16, 16, 2>::desc(5, 32),
    SpInst<8192, 512, 1, 4, kPrefetch, 16, 16, 16, 2>::desc(6, 16),
    // split exchanges, paired twiddle reads, one workgroup per segment: 2.99-3.01
    // ms per 8 GiB against 3.20-3.28 for the prefetch kernel (variant 8)
    split_desc(6, 0, 0),
    split_desc(0, 0, 0),  // one workgroup per segment: 2.95-2.97 ms against 3.19-3.20 at 32
    SpInst<16384, 1024, 1, 4, kNT | kNoHoist | kPlain | kAux, 16, 16, 16, 4>::desc(1, 32),
    SpInst<16384, 1024, 1, 4, kNT | kNoHoist, 16, 16, 16, 4>::desc(2, 32),
    SpInst<16384, 512, 1, 4, kNT | kNoHoist, 16, 16, 16, 4>::desc(3, 32),
    split_desc(1, 4, 32),
    split_desc(2, 5, 32),
    split_desc(3, 6, 32),
    split_desc(4, 7, 32),
    split_desc(5, 8, 32),
    // mixed radix 2/3/5
    SpInst<1000, 100, 2, 4, kClassic, 10, 10, 10>::desc(0, 64),
    SpInst<1000, 100, 2, 4, kPlain, 10, 10, 10>::desc(1, 64),
    SpInst<1000, 100, 2, 4, kNT | kPlain | kAux, 10, 10, 10>::desc(2, 32),
    SpInst<1000, 125, 2, 4, kNT | kPlain, 8, 5, 5, 5>::desc(3, 32),
    SpInst<1536, 96, 2, 4, kNT | kPlain | kAux, 16, 16, 6>::desc(0, 64),
    SpInst<1536, 96, 2, 4, kPlain, 16, 16, 6>::desc(1, 32),
    SpInst<1536, 96, 2, 4, kNT, 16, 16, 6>::desc(2, 32),
    SpInst<1536, 96, 2, 4, kClassic | kNT, 16, 16, 6>::desc(3, 64),
    // twiddles reloaded per segment and read in pairs, registers for two
    // workgroups per CU (79 VGPRs, three workgroups fit the LDS): 4.8-4.9
    // TB/s against 4.1-4.2 for the plainly written kernel (variant 7); one
    // workgroup per segment, as nothing stays in registers across segments
    // (3.21 ms per 8 GiB against 3.41-3.46 on a persistent grid of 32)
    SpInst<6000, 400, 1, 4, kNT | kNoHoist | kTwPair | kW4, 16, 15, 25>::desc(0, 0),
    SpInst<6000, 400, 1, 4, kNT | kNoHoist, 16, 15, 25>::desc(1, 0),
    SpInst<6000, 300, 1, 4, kNT | kNoHoist | kAux, 20, 20, 15>::desc(2, 32),
    SpInst<6000, 400, 1, 4, kNT | kNoHoist | kPlain, 16, 15, 25>::desc(3, 32),
    SpInst<6000, 400, 1, 4, kPrefetch | kNT, 16, 15, 25>::desc(4, 32),
    // cached loads and stores (stage 0 reads 375-sample runs that straddle
    // lines; streamed loads fetch the shared lines twice)
    SpInst<6000, 400, 1, 4, kClassic, 16, 15, 25>::desc(5, 32),
    // radix 25 first: stage 0 reads at a stride of 240 samples, whole lines
    SpInst<6000, 400, 1, 4, kClassic | kNT, 25, 15, 16>::desc(6, 32),
    SpInst<6000, 400, 1, 4, kClassic | kNT, 16, 15, 25>::desc(7, 32),
    SpInst<6000, 300, 1, 4, kNT | kNoHoist | kTwPair | kW4, 20, 20, 15>::desc(8, 32),
};

}  // namespace

const SinglePassDesc *single_pass_table(int *count)
{
    *count = (int)(sizeof(kTable) / sizeof(kTable[0]));
    return kTable;
}

}  // namespace fftseg
