// 4096-point single pass whose first data exchange runs through lane
// shuffles instead of LDS.
//
// The transform is the radix-16 x 16 x 16 Stockham pass of tile.hpp (stage
// i reads a[b + 256 r], writes a'[(b / L) 16 L + b % L + r L]).  With 256
// threads per segment, split into 16 rows of 16 lanes (row e = t / 16, lane
// p = t % 16):
//   stage 0: lane p of row e owns butterfly e + 16 p, whose output r'
//            belongs at a1[16 (e + 16 p) + r'];
//   stage 1: lane p of row e owns butterfly 16 e + p, which needs
//            a1[16 e + p + 256 r] = output p of stage-0 lane r of the same
//            row, for r = 0..15.
// So the exchange between stages 0 and 1 is a 16 x 16 transpose inside each
// 16-lane row (lane index <-> element index).  It is done in four steps: at
// step s (s = 1, 2, 4, 8) lanes p and p ^ s swap the halves of their element
// pairs (r, r | s) that the other one needs.  Lanes exchange 32-bit words
// with DPP moves (wavefront shuffles on the vector ALU): no LDS space, no LDS
// instruction and no barrier.  Stage 1 then exchanges through LDS as usual
// and stage 2 (butterfly t) reads and stores with unit stride across lanes.
// Stage 0 reads 32-byte runs (4 rows of a wave take 4 consecutive
// butterflies); the other waves of the workgroup read the rest of each line.
#include "registry.hpp"
#include "tile.hpp"

namespace fftseg {
namespace {

// 32-bit word of lane (lane ^ S), S in {1, 2, 4, 8}, within 16-lane rows,
// all through DPP (VALU lane moves, no LDS instruction): quad permutes for
// 1 and 2; a rotation of the 16-lane row by 8 for 8; for 4, rotations by 4
// and by 12 (row_ror:k gives lane i the word of lane (i - k) mod 16), the
// one that reaches lane i ^ 4 chosen by bit 2 of the lane.
template <int S>
__device__ __forceinline__ float lane_xor(float v, int lane)
{
    const int x = __builtin_bit_cast(int, v);
    int y;
    if constexpr (S == 1) {
        y = __builtin_amdgcn_mov_dpp(x, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    } else if constexpr (S == 2) {
        y = __builtin_amdgcn_mov_dpp(x, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    } else if constexpr (S == 8) {
        y = __builtin_amdgcn_mov_dpp(x, 0x128, 0xF, 0xF, false);  // row_ror:8
    } else {
        const int from_below = __builtin_amdgcn_mov_dpp(x, 0x124, 0xF, 0xF, false);  // ror:4
        const int from_above = __builtin_amdgcn_mov_dpp(x, 0x12C, 0xF, 0xF, false);  // ror:12
        y = (lane & 4) ? from_below : from_above;
    }
    return __builtin_bit_cast(float, y);
}

template <int S>
__device__ __forceinline__ void transpose_step(c32 *v, int lane)
{
    // value selects only: every index into v stays a compile-time constant,
    // so the array lives in registers
    const bool hi = (lane & S) != 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        if (r & S)
            continue;
        const c32 a = v[r], b = v[r | S];
        const c32 send = {hi ? a.x : b.x, hi ? a.y : b.y};
        const c32 recv = {lane_xor<S>(send.x, lane), lane_xor<S>(send.y, lane)};
        v[r] = hi ? recv : a;
        v[r | S] = hi ? b : recv;
    }
}

// v[r] of lane p becomes v[p] of lane r, within each 16-lane row
__device__ __forceinline__ void transpose16(c32 *v, int p)
{
    transpose_step<1>(v, p);
    transpose_step<2>(v, p);
    transpose_step<4>(v, p);
    transpose_step<8>(v, p);
}

constexpr int kM = 4096, kT = 256, kPad = 4;
__device__ __forceinline__ int pad(int i) { return i + (i >> kPad); }

// The twiddles of stages 1 and 2 stay in registers across the segments of
// the persistent loop (about 140 VGPRs: 2 waves per SIMD).
// LoadNT / StoreNT: non-temporal global loads / stores.  The 32-byte runs of
// stage 0 are better read through the cache, whose lines the other waves of
// the workgroup then hit.
template <int D, bool LoadNT, bool StoreNT>
__global__ void __launch_bounds__(kT) __attribute__((amdgpu_waves_per_eu(1, 2)))
    shuffle4096_kernel(const c32 *in, c32 *out, const c32 *__restrict__ tw, uint64_t batch)
{
    __shared__ c32 lds[kM + (kM >> kPad)];
    const int t = threadIdx.x;
    const int p = t & 15, e = t >> 4;
    const int b0 = e + 16 * p;  // stage-0 butterfly
    const int b1 = 16 * e + p;  // stage-1 butterfly (after the transpose)
    for (uint64_t seg = blockIdx.x; seg < batch; seg += gridDim.x) {
        const c32 *x = in + seg * kM;
        c32 *y = out + seg * kM;
        c32 v[16];
        // stage 0: butterfly b0 reads x[b0 + 256 r]
#pragma unroll
        for (int r = 0; r < 16; ++r)
            v[r] = gload<LoadNT>(x + b0 + 256 * r);
        dft<16, D>(v);
        // exchange inside the 16-lane row: v[r] = a1[b1 + 256 r]
        transpose16(v, p);
        // stage 1: butterfly b1, twiddle W_256^{r (b1 % 16)}, writes
        // a2[(b1 / 16) 256 + b1 % 16 + 16 r]
#pragma unroll
        for (int r = 1; r < 16; ++r)
            v[r] = twiddle<D>(v[r], tw[r * p * 16]);
        dft<16, D>(v);
#pragma unroll
        for (int r = 0; r < 16; ++r)
            lds[pad(256 * e + p + 16 * r)] = v[r];
        __syncthreads();
        // stage 2: butterfly t reads a2[t + 256 r], twiddle W_4096^{r t},
        // writes X[t + 256 r]
#pragma unroll
        for (int r = 0; r < 16; ++r)
            v[r] = lds[pad(t + 256 * r)];
        __syncthreads();  // the next segment's stage 1 reuses the LDS
#pragma unroll
        for (int r = 1; r < 16; ++r)
            v[r] = twiddle<D>(v[r], tw[r * t]);
        dft<16, D>(v);
#pragma unroll
        for (int r = 0; r < 16; ++r)
            gstore<StoreNT>(y + t + 256 * r, v[r]);
    }
}

template <bool LoadNT, bool StoreNT>
void launch(int dir, const void *in, void *out, const void *tw, uint64_t batch, unsigned grid,
            hipStream_t s)
{
    if (dir < 0)
        hipLaunchKernelGGL((shuffle4096_kernel<-1, LoadNT, StoreNT>), dim3(grid), dim3(kT), 0,
                           s, (const c32 *)in, (c32 *)out, (const c32 *)tw, batch);
    else
        hipLaunchKernelGGL((shuffle4096_kernel<1, LoadNT, StoreNT>), dim3(grid), dim3(kT), 0,
                           s, (const c32 *)in, (c32 *)out, (const c32 *)tw, batch);
}

template <bool LoadNT, bool StoreNT>
void set_kernels(SinglePassDesc &d)
{
    d.launch = &launch<LoadNT, StoreNT>;
    d.kernel[0] = (const void *)&shuffle4096_kernel<-1, LoadNT, StoreNT>;
    d.kernel[1] = (const void *)&shuffle4096_kernel<1, LoadNT, StoreNT>;
}

}  // namespace

// nontemporal: bit 0 loads, bit 1 stores
SinglePassDesc shuffle4096_desc(int variant, int grid_mult, int nontemporal)
{
    SinglePassDesc d{};
    d.n = kM;
    d.variant = variant;
    d.threads = kT;
    d.segs_per_wg = 1;
    d.pad_shift = kPad;
    d.nontemporal = nontemporal;
    d.hoist = -1;
    d.grid_mult = grid_mult;
    d.lds_bytes = (int)sizeof(c32) * (kM + (kM >> kPad));
    d.nrad = 3;
    d.radices[0] = d.radices[1] = d.radices[2] = 16;
    d.shuffle = 1;
    switch (nontemporal & 3) {
    case 0: set_kernels<false, false>(d); break;
    case 1: set_kernels<true, false>(d); break;
    case 2: set_kernels<false, true>(d); break;
    default: set_kernels<true, true>(d); break;
    }
    return d;
}

}  // namespace fftseg
