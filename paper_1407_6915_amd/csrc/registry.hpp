// Compiled kernel variants and their launch shapes, as seen by the planner.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fftseg {

constexpr int kMaxRadices = 12;

using sp_launch_fn = void (*)(int dir, const void *in, void *out, const void *tw,
                              uint64_t batch, unsigned grid, hipStream_t s);
using sp_strided_launch_fn = void (*)(int dir, const void *in, void *out, const void *tw,
                                      uint64_t batch, uint64_t in_stride, uint64_t out_stride,
                                      const float *window, unsigned grid, hipStream_t s);
using sp_rotated_launch_fn = void (*)(int dir, const void *in, void *out, const void *tw,
                                      uint64_t batch, int rot, unsigned grid, hipStream_t s);
using sp_indexed_launch_fn = void (*)(int dir, const void *in, void *out, const void *tw,
                                      const uint64_t *offs, uint64_t batch, unsigned grid,
                                      hipStream_t s);
using sp_real_launch_fn = void (*)(int dir, const void *in, void *out, const void *tw,
                                   const void *hw, uint64_t batch, unsigned grid,
                                   hipStream_t s);
using col_launch_fn = void (*)(int dir, const void *in, void *ybuf, const void *tw,
                               const void *tl, const void *th, int sh, int n2,
                               uint64_t batch, unsigned grid, hipStream_t s);
using row_launch_fn = void (*)(int dir, const void *ybuf, void *out, const void *tw,
                               int n1, uint64_t batch, unsigned grid, hipStream_t s);
using col_shifted_launch_fn = void (*)(int dir, const void *in, void *ybuf, const void *tw,
                                       const void *tl, const void *th, int sh, int n2,
                                       uint64_t batch, int shift, unsigned grid, hipStream_t s);
using row_shifted_launch_fn = void (*)(int dir, const void *ybuf, void *out, const void *tw,
                                       int n1, uint64_t batch, int shift, unsigned grid,
                                       hipStream_t s);
using col_indexed_launch_fn = void (*)(int dir, const void *in, void *ybuf, const void *tw,
                                       const void *tl, const void *th, int sh, int n2,
                                       const uint64_t *offs, uint64_t batch, unsigned grid,
                                       hipStream_t s);
using row_indexed_launch_fn = void (*)(int dir, const void *in, const void *ybuf, void *out,
                                       const void *tw, int n1, const uint64_t *offs,
                                       uint64_t batch, unsigned grid, hipStream_t s);
using col_frames_launch_fn = void (*)(int dir, const void *in, void *ybuf, const void *tw,
                                      const void *tl, const void *th, int sh, int n2,
                                      uint64_t batch, uint64_t hop, const float *window,
                                      unsigned grid, hipStream_t s);

// One LDS-resident pass over whole segments.
struct SinglePassDesc {
    int n;              // segment length
    int variant;        // 0 = default for this length
    int threads;        // threads per segment (T)
    int segs_per_wg;    // segments per workgroup (S)
    int pad_shift;      // one LDS pad element every 2^pad_shift (0: none)
    int nontemporal;    // streamed (non-temporal) global loads and stores
    int hoist;          // bit i: stage i keeps its twiddles in registers across segments
    int grid_mult;      // default persistent grid: resident waves of workgroups
    int lds_bytes;
    int shuffle;        // 1: an exchange between stages runs through lane shuffles
    int small_batch;    // 1: the length's kernel for batches that give the default
                        //    fewer than two workgroups per CU
    int nrad;
    int radices[kMaxRadices];
    sp_launch_fn launch;
    const void *kernel[2];  // [0] forward, [1] inverse (occupancy queries)
    sp_strided_launch_fn launch_strided;  // overlapping/windowed segments (variant 0)
    const void *kernel_strided[2];
    sp_real_launch_fn launch_real;  // real segments of length 2n (variant 0)
    const void *kernel_real[2];     // [0] forward (real in), [1] inverse (real out)
    sp_indexed_launch_fn launch_indexed;  // segments at listed offsets
    const void *kernel_indexed[2];
};

// Four-step pass A: N1-point column transforms, C columns per workgroup.
struct ColumnDesc {
    int n1, variant, cols, threads, lds_bytes, flags, nrad;
    int radices[kMaxRadices];
    col_launch_fn launch;
    const void *kernel[2];
    col_frames_launch_fn launch_frames;  // overlapping/windowed frames as input
    const void *kernel_frames[2];
    col_shifted_launch_fn launch_shifted;  // blocks from a column offset, wrapping
    const void *kernel_shifted[2];
    col_indexed_launch_fn launch_indexed;  // segments at listed offsets
    const void *kernel_indexed[2];
    col_launch_fn launch_yblocked;  // as launch, Y in blocks of 16 columns
    const void *kernel_yblocked[2];
    col_frames_launch_fn launch_frames_yblocked;  // as launch_frames, Y blocked
    const void *kernel_frames_yblocked[2];
};

// Four-step pass B: N2-point row transforms, C rows per workgroup.
struct RowDesc {
    int n2, variant, rows, threads, lds_bytes, flags, nrad;
    int radices[kMaxRadices];
    row_launch_fn launch;
    const void *kernel[2];
    row_shifted_launch_fn launch_shifted;  // blocks from a row offset, wrapping
    const void *kernel_shifted[2];
    row_indexed_launch_fn launch_indexed;  // segments at listed offsets
    const void *kernel_indexed[2];
    row_launch_fn launch_yblocked;  // as launch, Y in blocks of 16 columns
    const void *kernel_yblocked[2];
};

const SinglePassDesc *single_pass_table(int *count);
// the 4096-point pass with a lane-shuffle exchange (kernels_shuffle.hip)
SinglePassDesc shuffle4096_desc(int variant, int grid_mult, int nontemporal);
// single-pass and four-step instances with split LDS exchanges
// (kernels_split.hip)
SinglePassDesc split_desc(int config, int variant, int grid_mult);
ColumnDesc split_column_desc(int config, int variant);
RowDesc split_row_desc(int config, int variant);
// The one-pass kernel of length n with rotated lanes (kernels_rotated.hip),
// for outputs off a 128-byte line; null launcher if the length has none.
// `variant` receives the table variant whose kernel it mirrors.
sp_rotated_launch_fn rotated_launcher(uint64_t n, int *variant, const void **kernels);
// One-pass kernels over segments at listed offsets (kernels_indexed.hip):
// the work list's candidates for each of its one-pass lengths, `count`
// receives how many there are (0 for other lengths); null if none.
const SinglePassDesc *indexed_table(uint32_t n, int *count);
// The two passes over segments at listed offsets for the work list's
// two-pass length n (kernels_indexed.hip); false if n has none.  Each
// segment's Y takes n + 16 samples of scratch.
bool indexed_four_step(uint32_t n, const ColumnDesc **col, const RowDesc **row);
// single-pass instances with one LDS pad element every 32 (kernels_pad.hip)
SinglePassDesc pad32_desc(int config, int variant, int grid_mult);
// four-step tiles with radix-32 stages (kernels_radix32.hip)
ColumnDesc radix32_column_desc(int config, int variant);
RowDesc radix32_row_desc(int config, int variant);
const ColumnDesc *column_table(int *count);
const RowDesc *row_table(int *count);

// Fallback radix stage over global memory (radix in {2,3,4,5,8,16}).
bool generic_radix_supported(int radix);
void launch_generic_stage(int radix, int dir, const void *in, void *out,
                          const void *tl, const void *th, int sh, uint64_t n,
                          uint64_t l, uint64_t batch, unsigned grid, hipStream_t s);

}  // namespace fftseg
