// Stockham (self-sorting) Cooley-Tukey stages for a tile of G independent
// transforms of length M held by one workgroup, T threads per transform.
//
// With radices R_0 .. R_{s-1} (product M) and L = R_0 * .. * R_{i-1}, stage i
// does M/R_i butterflies; butterfly b reads
//     a[b + r * M/R_i],  r = 0..R_i-1,
// multiplies element r by W_{L R_i}^{r (b mod L)}, takes the R_i-point DFT
// in registers and writes element r to
//     a'[(b / L) * L R_i + (b mod L) + r * L].
// After the last stage a holds the DFT in natural order: the digit-reversal
// permutation of the textbook Cooley-Tukey form is folded into the write
// index of every stage.  Stage 0 (L = 1, no twiddles) reads a[b + r M/R_0]
// and the last stage (L R = M) writes a'[b + r M/R_last]: both are unit
// stride across consecutive butterflies, so with consecutive lanes on
// consecutive butterflies the global loads and stores coalesce.  The stages
// in between exchange data through LDS.
//
// Twiddles W_{L R}^{m'} = W_M^{m' M/(L R)} come from a table of the forward
// roots W_M^m = exp(-2 pi i m / M), m < M, evaluated in FP64 and rounded
// once to float32 on the host; the inverse conjugates them.
#pragma once

#include "radix.hpp"

namespace fftseg {

template <int... Rs>
struct Radices {
    static constexpr int count = sizeof...(Rs);
    static constexpr int at(int i)
    {
        constexpr int a[] = {Rs...};
        return a[i];
    }
    static constexpr long long product() { return (1LL * ... * Rs); }
    static constexpr int max_radix()
    {
        int m = 0;
        for (int i = 0; i < count; ++i)
            m = at(i) > m ? at(i) : m;
        return m;
    }
};

// Global memory access: plain, or non-temporal (streamed data that is not
// re-read soon, so it need not displace cached lines).
typedef float f2v __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ c32 gload(const c32 *p)
{
    if constexpr (NT) {
        const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v *>(p));
        return c32{v.x, v.y};
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ void gstore(c32 *p, c32 v)
{
    if constexpr (NT) {
        const f2v w = {v.x, v.y};
        __builtin_nontemporal_store(w, reinterpret_cast<f2v *>(p));
    } else {
        *p = v;
    }
}

// Transform shape: length M, T threads per transform, radix list.
template <int M_, int T_, class Rad_>
struct Shape {
    static constexpr int M = M_;
    static constexpr int T = T_;
    using Rad = Rad_;
    static constexpr int NS = Rad::count;
    static_assert(Rad::product() == M, "radices must multiply to M");
    static constexpr int units(int r) { return (M / r + T - 1) / T; }
    static constexpr int max_e()
    {
        int m = 1;
        for (int i = 0; i < NS; ++i) {
            int e = units(Rad::at(i)) * Rad::at(i);
            m = e > m ? e : m;
        }
        return m;
    }
    static constexpr int kMaxE = max_e();  // complex values per thread
};

template <class Sh, int I, int L>
struct Stage {
    static constexpr int R = Sh::Rad::at(I);
    static constexpr int NB = Sh::M / R;           // butterflies
    static constexpr int U = (NB + Sh::T - 1) / Sh::T;  // per thread
    static constexpr bool kFull = NB % Sh::T == 0;
    static constexpr bool kLast = I + 1 == Sh::NS;
    static constexpr int kTwStride = Sh::M / (L * R);
};

// v[u*R + r] <- get(b + r*NB) for this thread's butterflies b = t + u*T
template <class St, class Sh, class Get>
__device__ __forceinline__ void st_gather(c32 *v, int t, Get &&get)
{
#pragma unroll
    for (int u = 0; u < St::U; ++u) {
        const int b = t + u * Sh::T;
        if (St::kFull || b < St::NB) {
#pragma unroll
            for (int r = 0; r < St::R; ++r)
                v[u * St::R + r] = get(b + r * St::NB);
        }
    }
}

// twiddle + R-point DFT of this thread's butterflies
// (Hoist = false keeps the twiddle loads inside a persistent loop: the
// index is made opaque to the compiler so the loads are not lifted out and
// held in registers across segments.)
// Paired twiddles: for a radix R = R1 R2 with R1 the smallest divisor whose
// square reaches R (R >= 12), W^{(q R1 + j) e} = W^{q R1 e} W^{j e}, so a
// butterfly reads R1 - 1 + R2 - 1 table entries instead of R - 1 and forms
// the rest with one complex product each (0: direct reads).
constexpr int tw_pair_low(int r)
{
    if (r < 12)
        return 0;
    for (int d = 2; d < r; ++d)
        if (r % d == 0 && d * d >= r)
            return d;
    return 0;
}

template <class St, class Sh, int L, int D, bool Hoist = true, bool TwPair = false>
__device__ __forceinline__ void st_compute(c32 *v, int t,
                                           const c32 *__restrict__ tw)
{
    constexpr int R1 = (TwPair && !Hoist) ? tw_pair_low(St::R) : 0;
#pragma unroll
    for (int u = 0; u < St::U; ++u) {
        const int b = t + u * Sh::T;
        if (St::kFull || b < St::NB) {
            if constexpr (L > 1 && R1 > 0) {
                int k = b % L;
                asm volatile("" : "+v"(k));
                c32 *x = v + u * St::R;
                c32 wl[R1];
#pragma unroll
                for (int j = 1; j < R1; ++j) {
                    wl[j] = tw[j * k * St::kTwStride];
                    x[j] = twiddle<D>(x[j], wl[j]);
                }
#pragma unroll
                for (int q = 1; q < St::R / R1; ++q) {
                    const c32 wq = tw[q * R1 * k * St::kTwStride];
                    x[q * R1] = twiddle<D>(x[q * R1], wq);
#pragma unroll
                    for (int j = 1; j < R1; ++j)
                        x[q * R1 + j] = twiddle<D>(x[q * R1 + j], cmul(wq, wl[j]));
                }
            } else if constexpr (L > 1) {
                int k = b % L;
                if constexpr (!Hoist)
                    asm volatile("" : "+v"(k));
#pragma unroll
                for (int r = 1; r < St::R; ++r)
                    v[u * St::R + r] = twiddle<D>(
                        v[u * St::R + r], tw[r * k * St::kTwStride]);
            }
            dft<St::R, D>(v + u * St::R);
        }
    }
}

// put(index, value) for the stage outputs a'[(b/L) L R + b%L + r L]
template <class St, class Sh, int L, class Put>
__device__ __forceinline__ void st_scatter(const c32 *v, int t, Put &&put)
{
#pragma unroll
    for (int u = 0; u < St::U; ++u) {
        const int b = t + u * Sh::T;
        if (St::kFull || b < St::NB) {
            const int base = (b / L) * (L * St::R) + (b % L);
#pragma unroll
            for (int r = 0; r < St::R; ++r)
                put(base + r * L, v[u * St::R + r]);
        }
    }
}

// LDS exchange.  Pol::lds(c, i) is the padded LDS slot of element i of tile
// column c; when a stride of `step` elements keeps its padding pattern
// (step a multiple of the padding period, or one run of R unit steps
// starting on a period boundary) the R accesses of a butterfly are one base
// address plus compile-time offsets, so no per-element address registers
// are needed.
template <class Pol, int STEP, int R>
struct LdsRun {
    static constexpr bool kStrided = Pol::template strided<STEP>();
    static constexpr bool kUnitRun = (STEP == 1) && Pol::template unit_run<R>();
    static constexpr bool kSep = (kStrided || kUnitRun) && !Pol::kPlainLds;
    static constexpr int kStride = kStrided ? Pol::template stride<STEP>() : Pol::template stride<1>();
};

template <class St, class Sh, class Pol, int L>
__device__ __forceinline__ void lds_scatter(const c32 *v, int t, int c, c32 *lds)
{
    using Run = LdsRun<Pol, L, St::R>;
#pragma unroll
    for (int u = 0; u < St::U; ++u) {
        const int b = t + u * Sh::T;
        if (St::kFull || b < St::NB) {
            const int base = (b / L) * (L * St::R) + (b % L);
            if constexpr (Run::kSep) {
                c32 *p = lds + Pol::lds(c, base);
#pragma unroll
                for (int r = 0; r < St::R; ++r)
                    p[r * Run::kStride] = v[u * St::R + r];
            } else {
#pragma unroll
                for (int r = 0; r < St::R; ++r)
                    lds[Pol::lds(c, base + r * L)] = v[u * St::R + r];
            }
        }
    }
}

template <class St, class Sh, class Pol>
__device__ __forceinline__ void lds_gather(c32 *v, int t, int c, const c32 *lds)
{
    using Run = LdsRun<Pol, St::NB, St::R>;
#pragma unroll
    for (int u = 0; u < St::U; ++u) {
        const int b = t + u * Sh::T;
        if (St::kFull || b < St::NB) {
            if constexpr (Run::kStrided && !Pol::kPlainLds) {
                const c32 *p = lds + Pol::lds(c, b);
#pragma unroll
                for (int r = 0; r < St::R; ++r)
                    v[u * St::R + r] = p[r * Run::kStride];
            } else {
#pragma unroll
                for (int r = 0; r < St::R; ++r)
                    v[u * St::R + r] = lds[Pol::lds(c, b + r * St::NB)];
            }
        }
    }
}

// Run stages I.. of a tile.  Pol supplies the lane mapping per stage
// (col<I>, thr<I>), the LDS address of element i of tile column c, and the
// final store (which sees the last stage's outputs at b + r*NB).
// `tid` drives addressing and `tid_tw` the twiddle indices: the caller may
// make `tid` opaque per loop iteration so lane-derived addresses are
// recomputed (cheap) instead of held in registers across a persistent
// loop, while twiddles indexed by `tid_tw` can still stay in registers.
template <class Sh, class Pol, int D, int I, int L>
__device__ __forceinline__ void tile_run(c32 *v, c32 *lds,
                                         const c32 *__restrict__ tw, int tid, int tid_tw,
                                         const typename Pol::Ctx &ctx)
{
    using St = Stage<Sh, I, L>;
    const int c = Pol::template col<I>(tid);
    const int t = Pol::template thr<I>(tid);
    const bool act = Pol::active(tid);
    if (act)
        st_compute<St, Sh, L, D, Pol::hoists(I), Pol::kTwPair>(v, Pol::template thr<I>(tid_tw),
                                                              tw);
    if constexpr (St::kLast) {
        if (act)
            Pol::template store<St, D>(v, t, c, ctx);
    } else {
        if (act)
            lds_scatter<St, Sh, Pol, L>(v, t, c, lds);
        __syncthreads();
        using Nx = Stage<Sh, I + 1, L * St::R>;
        const int c2 = Pol::template col<I + 1>(tid);
        const int t2 = Pol::template thr<I + 1>(tid);
        if (act)
            lds_gather<Nx, Sh, Pol>(v, t2, c2, lds);
        __syncthreads();
        tile_run<Sh, Pol, D, I + 1, L * St::R>(v, lds, tw, tid, tid_tw, ctx);
    }
}

// The same stages written plainly: every LDS access computes its own padded
// address and the compiler is left to keep whatever it hoists in registers
// (single_pass_plain_kernel also computes the lane mapping once, outside
// its persistent loop).
template <class Sh, class Pol, int D, int I, int L>
__device__ __forceinline__ void tile_run_plain(c32 *v, c32 *lds, const c32 *__restrict__ tw,
                                               int tid, const typename Pol::Ctx &ctx)
{
    using St = Stage<Sh, I, L>;
    const int c = Pol::template col<I>(tid);
    const int t = Pol::template thr<I>(tid);
    st_compute<St, Sh, L, D>(v, t, tw);
    if constexpr (St::kLast) {
        Pol::template store<St, D>(v, t, c, ctx);
    } else {
        st_scatter<St, Sh, L>(v, t, [&](int i, c32 a) { lds[Pol::lds(c, i)] = a; });
        __syncthreads();
        using Nx = Stage<Sh, I + 1, L * St::R>;
        const int c2 = Pol::template col<I + 1>(tid);
        const int t2 = Pol::template thr<I + 1>(tid);
        st_gather<Nx, Sh>(v, t2, [&](int i) { return lds[Pol::lds(c2, i)]; });
        __syncthreads();
        tile_run_plain<Sh, Pol, D, I + 1, L * St::R>(v, lds, tw, tid, ctx);
    }
}

// One half (F = 0: real parts, F = 1: imaginary parts) of an LDS exchange
// through a float array indexed like the complex one (see lds_scatter and
// lds_gather).
template <int F>
__device__ __forceinline__ float &part(c32 &a)
{
    if constexpr (F == 0)
        return a.x;
    else
        return a.y;
}
template <int F>
__device__ __forceinline__ float part(const c32 &a)
{
    if constexpr (F == 0)
        return a.x;
    else
        return a.y;
}

template <class St, class Sh, class Pol, int L, int F>
__device__ __forceinline__ void lds_scatter_part(const c32 *v, int t, int c, float *lds)
{
    using Run = LdsRun<Pol, L, St::R>;
#pragma unroll
    for (int u = 0; u < St::U; ++u) {
        const int b = t + u * Sh::T;
        if (St::kFull || b < St::NB) {
            const int base = (b / L) * (L * St::R) + (b % L);
            if constexpr (Run::kSep) {
                float *p = lds + Pol::lds(c, base);
#pragma unroll
                for (int r = 0; r < St::R; ++r)
                    p[r * Run::kStride] = part<F>(v[u * St::R + r]);
            } else {
#pragma unroll
                for (int r = 0; r < St::R; ++r)
                    lds[Pol::lds(c, base + r * L)] = part<F>(v[u * St::R + r]);
            }
        }
    }
}

template <class St, class Sh, class Pol, int F>
__device__ __forceinline__ void lds_gather_part(c32 *v, int t, int c, const float *lds)
{
    using Run = LdsRun<Pol, St::NB, St::R>;
#pragma unroll
    for (int u = 0; u < St::U; ++u) {
        const int b = t + u * Sh::T;
        if (St::kFull || b < St::NB) {
            if constexpr (Run::kStrided && !Pol::kPlainLds) {
                const float *p = lds + Pol::lds(c, b);
#pragma unroll
                for (int r = 0; r < St::R; ++r)
                    part<F>(v[u * St::R + r]) = p[r * Run::kStride];
            } else {
#pragma unroll
                for (int r = 0; r < St::R; ++r)
                    part<F>(v[u * St::R + r]) = lds[Pol::lds(c, b + r * St::NB)];
            }
        }
    }
}

// tile_run with every LDS exchange split in two: the real parts go through
// LDS first, then the imaginary parts, through a float array with the same
// (padded) indexing as the complex one.  The tile then needs half the LDS,
// so twice as many workgroups fit a CU, for two more barriers per exchange.
// Between the halves a register slot holds the next stage's real part and
// this stage's imaginary part.
template <class Sh, class Pol, int D, int I, int L>
__device__ __forceinline__ void tile_run_split(c32 *v, float *lds, const c32 *__restrict__ tw,
                                               int tid, int tid_tw,
                                               const typename Pol::Ctx &ctx)
{
    using St = Stage<Sh, I, L>;
    const int c = Pol::template col<I>(tid);
    const int t = Pol::template thr<I>(tid);
    const bool act = Pol::active(tid);
    if (act)
        st_compute<St, Sh, L, D, Pol::hoists(I), Pol::kTwPair>(v, Pol::template thr<I>(tid_tw),
                                                              tw);
    if constexpr (St::kLast) {
        if (act)
            Pol::template store<St, D>(v, t, c, ctx);
    } else {
        using Nx = Stage<Sh, I + 1, L * St::R>;
        const int c2 = Pol::template col<I + 1>(tid);
        const int t2 = Pol::template thr<I + 1>(tid);
        if (act)
            lds_scatter_part<St, Sh, Pol, L, 0>(v, t, c, lds);
        __syncthreads();
        if (act)
            lds_gather_part<Nx, Sh, Pol, 0>(v, t2, c2, lds);
        __syncthreads();
        if (act)
            lds_scatter_part<St, Sh, Pol, L, 1>(v, t, c, lds);
        __syncthreads();
        if (act)
            lds_gather_part<Nx, Sh, Pol, 1>(v, t2, c2, lds);
        __syncthreads();
        tile_run_split<Sh, Pol, D, I + 1, L * St::R>(v, lds, tw, tid, tid_tw, ctx);
    }
}

// LDS of a tile in complex elements: Elems complex values, or Elems floats
// (rounded up) when the exchanges are split
template <int Elems, bool Split>
constexpr int lds_c32() { return Split ? (Elems + 1) / 2 : Elems; }

// a copy of the lane index the compiler cannot treat as loop-invariant
__device__ __forceinline__ int opaque_lane()
{
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// LDS layout code for an XOR swizzle instead of a pad shift (SinglePassPolicy)
constexpr int kLdsXor = -1;

// ---------------------------------------------------------------------------
// Single pass: S whole segments per workgroup, each owned by T threads.
//   lane mapping: segment slot = tid / T, thread t = tid % T (all stages);
//   LDS: slot * SegStride + i + (i >> PS) (one pad element every 2^PS).
// (Partial = the workgroup may have more threads than S*T; the extra
// threads only take part in barriers.  HoistMask bit i lets stage i keep its
// twiddles in registers across the segments of a persistent loop.  Waves =
// the waves per SIMD the register allocation must allow.)
template <class Sh, int S_, int PS_, bool NT_ = false, int HoistMask_ = -1,
          bool Partial_ = false, int Waves_ = 1, bool PlainLane_ = false,
          bool PlainLds_ = false, bool Classic_ = false, bool Split_ = false,
          bool TwPair_ = false>
struct SinglePassPolicy {
    static constexpr int S = S_;
    static constexpr int PS = PS_;
    // TwPair: stages that reload their twiddles per segment read them as
    // pairs (tw_pair_low)
    static constexpr bool kTwPair = TwPair_;
    // PlainLane: the persistent loop keeps the lane index (and what the
    // compiler derives from it) across segments instead of recomputing it;
    // PlainLds: every LDS access computes its padded address on its own;
    // Classic: the stages run through tile_run_plain (both of the above,
    // and no per-stage choices left to the policy); Split: the exchanges
    // run through tile_run_split (real and imaginary halves)
    static constexpr bool kPlainLane = PlainLane_ || Classic_;
    static constexpr bool kSplit = Split_;
    static constexpr bool kPlainLds = PlainLds_;
    static constexpr bool kClassic = Classic_;
    static constexpr bool kNT = NT_;
    static constexpr int kHoistMask = HoistMask_;
    static constexpr bool kPartial = Partial_;
    static constexpr int kWaves = Waves_;
    static constexpr bool hoists(int stage) { return (kHoistMask >> stage) & 1; }
    // LDS layout of a segment: one pad element every 2^PS (PS > 0), none
    // (PS = 0), or (PS = kLdsXor) an XOR swizzle that permutes each run of
    // 32 elements by the bits above it, i ^ ((i >> 5) mod 32): strides of 16
    // and 256 elements then spread over all 32 eight-byte bank slots, with no
    // gaps in the layout.  The swizzle needs per-element addresses (the
    // plainly written stages), not the base-plus-offset runs of LdsRun.
    static constexpr int pad(int i)
    {
        return PS > 0 ? i + (i >> PS) : PS == kLdsXor ? (i ^ ((i >> 5) & 31)) : i;
    }
    static_assert(PS != kLdsXor || kClassic || kPlainLds, "the swizzle needs per-element addresses");
    static_assert(PS != kLdsXor || Sh::M % 32 == 0, "the swizzle permutes whole runs of 32");
    // the swizzle is not monotone: its last element is not its largest
    static constexpr int kSegStride = PS == kLdsXor ? Sh::M : pad(Sh::M - 1) + 1;
    static constexpr int kLdsElems = Sh::NS > 1 ? S * kSegStride : 1;
    static constexpr int kThreads = Sh::T * S;

    struct Ctx {
        c32 *y;       // output segment base of this thread's slot
        bool valid;   // the slot holds a real segment
    };
    template <int I>
    static __device__ __forceinline__ int col(int tid) { return S == 1 ? 0 : tid / Sh::T; }
    template <int I>
    static __device__ __forceinline__ int thr(int tid) { return S == 1 ? tid : tid % Sh::T; }
    static __device__ __forceinline__ int lds(int c, int i) { return c * kSegStride + pad(i); }
    static __device__ __forceinline__ bool active(int tid)
    {
        return !kPartial || tid < kThreads;
    }
    // padding-aware strides (see LdsRun)
    template <int STEP>
    static constexpr bool strided() { return PS <= 0 || STEP % (1 << PS) == 0; }
    template <int STEP>
    static constexpr int stride() { return PS > 0 ? STEP + (STEP >> PS) : STEP; }
    template <int R>
    static constexpr bool unit_run() { return PS > 0 && R == (1 << PS); }

    template <class St, int D>
    static __device__ __forceinline__ void store(const c32 *v, int t, int, const Ctx &ctx)
    {
        if (!ctx.valid)
            return;
#pragma unroll
        for (int u = 0; u < St::U; ++u) {
            const int b = t + u * Sh::T;
            if (St::kFull || b < St::NB) {
#pragma unroll
                for (int r = 0; r < St::R; ++r)
                    gstore<kNT>(ctx.y + b + r * St::NB, v[u * St::R + r]);
            }
        }
    }
};

// One tile of up to S whole segments: slot c of the tile reads x_c and
// writes y_c (valid_c false for an empty slot).
template <class Sh, class Pol, int D>
__device__ __forceinline__ void single_tile(c32 *lds, const c32 *__restrict__ tw, int tid,
                                            int tid_tw, const c32 *x, c32 *y, bool valid)
{
    const int t = Pol::template thr<0>(tid);
    typename Pol::Ctx ctx{y, valid && Pol::active(tid)};
    c32 v[Sh::kMaxE];
    using S0 = Stage<Sh, 0, 1>;
    if (ctx.valid)
        st_gather<S0, Sh>(v, t, [&](int i) { return gload<Pol::kNT>(x + i); });
    // lds holds lds_c32<kLdsElems, kSplit>() complex elements
    if constexpr (Pol::kSplit)
        tile_run_split<Sh, Pol, D, 0, 1>(v, reinterpret_cast<float *>(lds), tw, tid, tid_tw,
                                         ctx);
    else
        tile_run<Sh, Pol, D, 0, 1>(v, lds, tw, tid, tid_tw, ctx);
}

// Tile order of a persistent grid.  Workgroups are dispatched round-robin
// over the 8 XCDs (workgroup w on XCD w % 8); with Xcd the tiles of one
// sweep are dealt so that the workgroups of one XCD take consecutive tiles,
// so adjacent column blocks -- the two halves of the same cache lines --
// are read through the same L2 at about the same time.
template <bool Xcd>
__device__ __forceinline__ uint64_t tile_of(uint64_t sweep_base, unsigned w, unsigned grid)
{
    if constexpr (Xcd) {
        if ((grid & 7u) == 0)
            return sweep_base + (uint64_t)(w & 7u) * (grid >> 3) + (w >> 3);
    }
    return sweep_base + w;
}

// Overlapping, windowed segments (short-time transform): segment s reads
// x_s[n] = in[s * in_stride + n] * window[n] (window may be null) and writes
// its spectrum at out + s * out_stride.
template <class Sh, class Pol, int D>
__device__ __forceinline__ void windowed_tile(c32 *lds, const c32 *__restrict__ tw, int tid,
                                              int tid_tw, const c32 *x, c32 *y, bool valid,
                                              const float *__restrict__ window, bool cached)
{
    const int t = Pol::template thr<0>(tid);
    typename Pol::Ctx ctx{y, valid && Pol::active(tid)};
    c32 v[Sh::kMaxE];
    using S0 = Stage<Sh, 0, 1>;
    if (ctx.valid) {
        if (cached) {
            // overlapping frames: the samples a frame shares with the next
            // ones stay in L2 for them
            if (window) {
                st_gather<S0, Sh>(v, t, [&](int i) {
                    const c32 a = gload<false>(x + i);
                    const float w = window[i];
                    return c32{a.x * w, a.y * w};
                });
            } else {
                st_gather<S0, Sh>(v, t, [&](int i) { return gload<false>(x + i); });
            }
        } else if (window) {
            st_gather<S0, Sh>(v, t, [&](int i) {
                const c32 a = gload<Pol::kNT>(x + i);
                const float w = window[i];
                return c32{a.x * w, a.y * w};
            });
        } else {
            st_gather<S0, Sh>(v, t, [&](int i) { return gload<Pol::kNT>(x + i); });
        }
    }
    // lds holds lds_c32<kLdsElems, kSplit>() complex elements
    if constexpr (Pol::kSplit)
        tile_run_split<Sh, Pol, D, 0, 1>(v, reinterpret_cast<float *>(lds), tw, tid, tid_tw,
                                         ctx);
    else if constexpr (Pol::kClassic)
        tile_run_plain<Sh, Pol, D, 0, 1>(v, lds, tw, tid, ctx);
    else
        tile_run<Sh, Pol, D, 0, 1>(v, lds, tw, tid, tid_tw, ctx);
}

// Mode bit 0: frames that overlap (in_stride < M) are read through the
// cache even where the policy streams (4096-point frames every 1024
// samples: 2.89 ms per 2^18 frames against 3.19 streamed); bit 1: each XCD
// takes a contiguous run of frame groups per sweep of the grid (tile_of),
// so the frames that share samples are read through the same L2 (a quarter
// of the HBM reads, but 2.99 ms).  These forms ask for at least two waves
// per SIMD, so the window and stride registers cannot push a kernel down to
// one.
template <class Sh, class Pol, int D, int Mode = 0>
__global__ void __launch_bounds__(Pol::kThreads)
    __attribute__((amdgpu_waves_per_eu(Mode != 0 && Pol::kWaves < 2 ? 2 : Pol::kWaves)))
    single_pass_strided_kernel(const c32 *in, c32 *out, const c32 *__restrict__ tw,
                               uint64_t batch, uint64_t in_stride, uint64_t out_stride,
                               const float *__restrict__ window)
{
    __shared__ c32 lds[lds_c32<Pol::kLdsElems, Pol::kSplit>()];
    const int tid_tw = threadIdx.x;
    const uint64_t groups = (batch + Pol::S - 1) / Pol::S;
    const bool cached = (Mode & 1) && in_stride < (uint64_t)Sh::M;
    // tile_of(base, w, grid) is base plus a permutation of the workgroups
    for (uint64_t g = tile_of<(Mode & 2) != 0>(0, blockIdx.x, gridDim.x); g < groups;
         g += gridDim.x) {
        const int tid = Pol::kPlainLane ? tid_tw : opaque_lane();
        const uint64_t seg = g * Pol::S + Pol::template col<0>(tid);
        windowed_tile<Sh, Pol, D>(lds, tw, tid, tid_tw, in + seg * in_stride,
                                  out + seg * out_stride, seg < batch, window, cached);
    }
}

template <class Sh, class Pol, int D>
__global__ void __launch_bounds__(Pol::kThreads) __attribute__((amdgpu_waves_per_eu(Pol::kWaves)))
    single_pass_plain_kernel(const c32 *in, c32 *out, const c32 *__restrict__ tw,
                             uint64_t batch)
{
    __shared__ c32 lds[Pol::kLdsElems];
    const int tid = threadIdx.x;
    const int slot = Pol::template col<0>(tid);
    const int t = Pol::template thr<0>(tid);
    const uint64_t groups = (batch + Pol::S - 1) / Pol::S;
    for (uint64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const uint64_t seg = g * Pol::S + slot;
        typename Pol::Ctx ctx{out + seg * Sh::M, seg < batch};
        const c32 *x = in + seg * Sh::M;
        c32 v[Sh::kMaxE];
        using S0 = Stage<Sh, 0, 1>;
        if (ctx.valid)
            st_gather<S0, Sh>(v, t, [&](int i) { return gload<Pol::kNT>(x + i); });
        tile_run_plain<Sh, Pol, D, 0, 1>(v, lds, tw, tid, ctx);
    }
}

// single_pass_plain_kernel with the thread -> butterfly assignment rotated
// by `rot` (thread t of a segment takes the butterflies of t' = (t + rot)
// mod T in every stage; any bijection is a valid Stockham schedule, since
// the LDS exchange is addressed by element).  With rot = -(out offset
// within a 128-byte line) the last stage's stores of each wave start on a
// line boundary again when the output base pointer does not.
template <class Sh, class Pol, int D>
__global__ void __launch_bounds__(Pol::kThreads) __attribute__((amdgpu_waves_per_eu(2)))
    single_pass_rotated_kernel(const c32 *in, c32 *out, const c32 *__restrict__ tw,
                               uint64_t batch, int rot)
{
    static_assert(!Pol::kPartial, "every thread of the workgroup owns butterflies");
    static_assert((Sh::T & (Sh::T - 1)) == 0, "rotation by mask");
    __shared__ c32 lds[Pol::kLdsElems];
    const int slot = Pol::template col<0>((int)threadIdx.x);
    const int t = (int)(((unsigned)Pol::template thr<0>((int)threadIdx.x) + (unsigned)rot) &
                        (unsigned)(Sh::T - 1));
    const int tid = slot * Sh::T + t;
    const uint64_t groups = (batch + Pol::S - 1) / Pol::S;
    for (uint64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const uint64_t seg = g * Pol::S + slot;
        typename Pol::Ctx ctx{out + seg * Sh::M, seg < batch};
        const c32 *x = in + seg * Sh::M;
        c32 v[Sh::kMaxE];
        using S0 = Stage<Sh, 0, 1>;
        if (ctx.valid)
            st_gather<S0, Sh>(v, t, [&](int i) { return gload<Pol::kNT>(x + i); });
        tile_run_plain<Sh, Pol, D, 0, 1>(v, lds, tw, tid, ctx);
    }
}

// single_pass_plain_kernel with the next segment's stage-0 loads issued
// before the current segment's stages (software pipelining in registers):
// for lengths whose LDS footprint leaves few workgroups per CU, the loads of
// segment g + grid are in flight while segment g is transformed and stored.
template <class Sh, class Pol, int D>
__global__ void __launch_bounds__(Pol::kThreads)
    single_pass_prefetch_kernel(const c32 *in, c32 *out, const c32 *__restrict__ tw,
                                uint64_t batch)
{
    __shared__ c32 lds[Pol::kLdsElems];
    using S0 = Stage<Sh, 0, 1>;
    const int tid = threadIdx.x;
    const int slot = Pol::template col<0>(tid);
    const int t = Pol::template thr<0>(tid);
    const uint64_t groups = (batch + Pol::S - 1) / Pol::S;
    c32 nx[Sh::kMaxE];
    uint64_t g = blockIdx.x;
    {
        const uint64_t seg = g * Pol::S + slot;
        if (g < groups && seg < batch) {
            const c32 *x = in + seg * Sh::M;
            st_gather<S0, Sh>(nx, t, [&](int i) { return gload<Pol::kNT>(x + i); });
        }
    }
    for (; g < groups; g += gridDim.x) {
        const uint64_t seg = g * Pol::S + slot;
        typename Pol::Ctx ctx{out + seg * Sh::M, seg < batch};
        c32 v[Sh::kMaxE];
#pragma unroll
        for (int i = 0; i < Sh::kMaxE; ++i)
            v[i] = nx[i];
        const uint64_t gn = g + gridDim.x, segn = gn * Pol::S + slot;
        if (gn < groups && segn < batch) {
            const c32 *x = in + segn * Sh::M;
            st_gather<S0, Sh>(nx, t, [&](int i) { return gload<Pol::kNT>(x + i); });
        }
        tile_run_plain<Sh, Pol, D, 0, 1>(v, lds, tw, tid, ctx);
    }
}

// single_pass_kernel with split exchanges (tile_run_split): for lengths
// whose complex LDS tile leaves one or two workgroups per CU.
template <class Sh, class Pol, int D>
__global__ void __launch_bounds__(Pol::kThreads) __attribute__((amdgpu_waves_per_eu(Pol::kWaves)))
    single_pass_split_kernel(const c32 *in, c32 *out, const c32 *__restrict__ tw,
                             uint64_t batch)
{
    static_assert(Pol::kSplit, "split exchanges only");
    __shared__ float lds[Pol::kLdsElems];
    const int tid_tw = threadIdx.x;
    const uint64_t groups = (batch + Pol::S - 1) / Pol::S;
    for (uint64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int tid = Pol::kPlainLane ? tid_tw : opaque_lane();
        const int t = Pol::template thr<0>(tid);
        const uint64_t seg = g * Pol::S + Pol::template col<0>(tid);
        typename Pol::Ctx ctx{out + seg * Sh::M, seg < batch && Pol::active(tid)};
        const c32 *x = in + seg * Sh::M;
        c32 v[Sh::kMaxE];
        using S0 = Stage<Sh, 0, 1>;
        if (ctx.valid)
            st_gather<S0, Sh>(v, t, [&](int i) { return gload<Pol::kNT>(x + i); });
        tile_run_split<Sh, Pol, D, 0, 1>(v, lds, tw, tid, tid_tw, ctx);
    }
}

// single_pass_split_kernel with the next segment's stage-0 loads issued
// before the current segment's stages, as in single_pass_prefetch_kernel.
template <class Sh, class Pol, int D>
__global__ void __launch_bounds__(Pol::kThreads) __attribute__((amdgpu_waves_per_eu(Pol::kWaves)))
    single_pass_split_prefetch_kernel(const c32 *in, c32 *out, const c32 *__restrict__ tw,
                                      uint64_t batch)
{
    static_assert(Pol::kSplit, "split exchanges only");
    __shared__ float lds[Pol::kLdsElems];
    using S0 = Stage<Sh, 0, 1>;
    const int tid = threadIdx.x;
    const int slot = Pol::template col<0>(tid);
    const int t = Pol::template thr<0>(tid);
    const uint64_t groups = (batch + Pol::S - 1) / Pol::S;
    c32 nx[Sh::kMaxE];
    uint64_t g = blockIdx.x;
    {
        const uint64_t seg = g * Pol::S + slot;
        if (g < groups && seg < batch) {
            const c32 *x = in + seg * Sh::M;
            st_gather<S0, Sh>(nx, t, [&](int i) { return gload<Pol::kNT>(x + i); });
        }
    }
    for (; g < groups; g += gridDim.x) {
        const uint64_t seg = g * Pol::S + slot;
        typename Pol::Ctx ctx{out + seg * Sh::M, seg < batch && Pol::active(tid)};
        c32 v[Sh::kMaxE];
#pragma unroll
        for (int i = 0; i < Sh::kMaxE; ++i)
            v[i] = nx[i];
        const uint64_t gn = g + gridDim.x, segn = gn * Pol::S + slot;
        if (gn < groups && segn < batch) {
            const c32 *x = in + segn * Sh::M;
            st_gather<S0, Sh>(nx, t, [&](int i) { return gload<Pol::kNT>(x + i); });
        }
        tile_run_split<Sh, Pol, D, 0, 1>(v, lds, tw, tid, tid, ctx);
    }
}

template <class Sh, class Pol, int D>
__global__ void __launch_bounds__(Pol::kThreads) __attribute__((amdgpu_waves_per_eu(Pol::kWaves)))
    single_pass_kernel(const c32 *in, c32 *out, const c32 *__restrict__ tw,
                       uint64_t batch)
{
    __shared__ c32 lds[Pol::kLdsElems];
    const int tid_tw = threadIdx.x;
    const uint64_t groups = (batch + Pol::S - 1) / Pol::S;
    for (uint64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int tid = Pol::kPlainLane ? tid_tw : opaque_lane();
        const uint64_t seg = g * Pol::S + Pol::template col<0>(tid);
        single_tile<Sh, Pol, D>(lds, tw, tid, tid_tw, in + seg * Sh::M, out + seg * Sh::M,
                                seg < batch);
    }
}

// Indexed segments: segment s of the launch reads in + offs[3s] and writes
// out + offs[3s + 1] (sample offsets; offs holds records of three words, the
// third unused here), so a batch of one length whose segments sit anywhere
// runs through the same tile as the dense kernel of that length: the
// plainly written tile (Pol::kClassic), split exchanges (Pol::kSplit) or the
// policy-driven tile.
template <class Sh, class Pol, int D>
__global__ void __launch_bounds__(Pol::kThreads) __attribute__((amdgpu_waves_per_eu(Pol::kWaves)))
    single_pass_indexed_kernel(const c32 *in, c32 *out, const c32 *__restrict__ tw,
                               const uint64_t *__restrict__ offs, uint64_t batch)
{
    using S0 = Stage<Sh, 0, 1>;
    const int tid_tw = threadIdx.x;
    const uint64_t groups = (batch + Pol::S - 1) / Pol::S;
    if constexpr (Pol::kSplit) {
        __shared__ float lds[Pol::kLdsElems];
        for (uint64_t g = blockIdx.x; g < groups; g += gridDim.x) {
            const int tid = Pol::kPlainLane ? tid_tw : opaque_lane();
            const int t = Pol::template thr<0>(tid);
            const uint64_t seg = g * Pol::S + Pol::template col<0>(tid);
            const bool valid = seg < batch && Pol::active(tid);
            const uint64_t io = valid ? offs[3 * seg] : 0, oo = valid ? offs[3 * seg + 1] : 0;
            typename Pol::Ctx ctx{out + oo, valid};
            const c32 *x = in + io;
            c32 v[Sh::kMaxE];
            if (ctx.valid)
                st_gather<S0, Sh>(v, t, [&](int i) { return gload<Pol::kNT>(x + i); });
            tile_run_split<Sh, Pol, D, 0, 1>(v, lds, tw, tid, tid_tw, ctx);
        }
    } else if constexpr (Pol::kClassic) {
        __shared__ c32 lds[Pol::kLdsElems];
        const int slot = Pol::template col<0>(tid_tw);
        const int t = Pol::template thr<0>(tid_tw);
        for (uint64_t g = blockIdx.x; g < groups; g += gridDim.x) {
            const uint64_t seg = g * Pol::S + slot;
            const bool valid = seg < batch;
            const uint64_t io = valid ? offs[3 * seg] : 0, oo = valid ? offs[3 * seg + 1] : 0;
            typename Pol::Ctx ctx{out + oo, valid};
            const c32 *x = in + io;
            c32 v[Sh::kMaxE];
            if (ctx.valid)
                st_gather<S0, Sh>(v, t, [&](int i) { return gload<Pol::kNT>(x + i); });
            tile_run_plain<Sh, Pol, D, 0, 1>(v, lds, tw, tid_tw, ctx);
        }
    } else {
        __shared__ c32 lds[Pol::kLdsElems];
        for (uint64_t g = blockIdx.x; g < groups; g += gridDim.x) {
            const int tid = Pol::kPlainLane ? tid_tw : opaque_lane();
            const uint64_t seg = g * Pol::S + Pol::template col<0>(tid);
            const bool valid = seg < batch && Pol::active(tid);
            const uint64_t io = valid ? offs[3 * seg] : 0, oo = valid ? offs[3 * seg + 1] : 0;
            single_tile<Sh, Pol, D>(lds, tw, tid, tid_tw, in + io, out + oo, valid);
        }
    }
}

// ---------------------------------------------------------------------------
// Real-input segments of even length N = 2M through one M-point complex
// transform.
// Forward: the N real samples are read as M complex values
// z[m] = x[2m] + i x[2m+1]; Z = DFT_M(z); with A = Z[k] and
// B = conj Z[(M-k) mod M], the half spectrum is
//     X[k] = (A + B)/2 - i W_N^k (A - B)/2,   0 <= k <= M,
// stored as M+1 complex values per segment.  Z[k] and Z[M-k] sit in
// different threads, so the last stage writes Z to LDS and the twist
// reads it back.
// Inverse (bins 0..M in; bins 0 and M of a real signal are real, their
// imaginary parts are dropped): with A = X[k] and B = conj X[M-k],
//     Z[k] = (A + B) + i W_N^{-k} (A - B),   0 <= k < M,
// and the unnormalised inverse M-point DFT of Z is x[2m] + i x[2m+1]:
// the N real outputs, written as M complex values.
// hw holds W_N^k = exp(-2 pi i k / N) for k = 0..M.

// the tile's last stage writes its natural-order outputs to LDS
template <class Base>
struct LdsStorePolicy : Base {
    struct Ctx {
        c32 *lds;
        bool valid;
    };
    template <class St, int D>
    static __device__ __forceinline__ void store(const c32 *v, int t, int c, const Ctx &ctx)
    {
        if (!ctx.valid)
            return;
#pragma unroll
        for (int u = 0; u < St::U; ++u) {
            const int b = t + u * Base::kThreads / Base::S;
            if (St::kFull || b < St::NB) {
#pragma unroll
                for (int r = 0; r < St::R; ++r)
                    ctx.lds[Base::lds(c, b + r * St::NB)] = v[u * St::R + r];
            }
        }
    }
};

template <class Sh, class Pol>
__global__ void __launch_bounds__(Pol::kThreads) __attribute__((amdgpu_waves_per_eu(Pol::kWaves)))
    real_forward_kernel(const c32 *in, c32 *out, const c32 *__restrict__ tw,
                        const c32 *__restrict__ hw, uint64_t batch)
{
    constexpr int M = Sh::M;
    __shared__ c32 lds[Pol::S * Pol::kSegStride];
    using LP = LdsStorePolicy<Pol>;
    using S0 = Stage<Sh, 0, 1>;
    const int tid_tw = threadIdx.x;
    const uint64_t groups = (batch + Pol::S - 1) / Pol::S;
    for (uint64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int tid = Pol::kPlainLane ? tid_tw : opaque_lane();
        const int c = Pol::template col<0>(tid);
        const int t = Pol::template thr<0>(tid);
        const uint64_t seg = g * Pol::S + c;
        const bool valid = seg < batch && Pol::active(tid);
        c32 v[Sh::kMaxE];
        const c32 *x = in + seg * M;
        if (valid)
            st_gather<S0, Sh>(v, t, [&](int i) { return gload<Pol::kNT>(x + i); });
        const typename LP::Ctx ctx{lds, valid};
        if constexpr (Pol::kClassic)
            tile_run_plain<Sh, LP, -1, 0, 1>(v, lds, tw, tid, ctx);
        else
            tile_run<Sh, LP, -1, 0, 1>(v, lds, tw, tid, tid_tw, ctx);
        __syncthreads();
        if (valid) {
            // rows of M + 1 values are not line-aligned: cached stores let the
            // L2 merge the partial lines that neighbouring rows share
            // (streaming stores of those partial lines measured 15-20 % slower)
            c32 *y = out + seg * (uint64_t)(M + 1);
            for (int k = t; k <= M; k += Sh::T) {
                const c32 a = lds[Pol::lds(c, k == M ? 0 : k)];
                const c32 z = lds[Pol::lds(c, k == 0 ? 0 : M - k)];
                const c32 e = {0.5f * (a.x + z.x), 0.5f * (a.y - z.y)};
                const c32 d = {0.5f * (a.x - z.x), 0.5f * (a.y + z.y)};  // (A - B) / 2
                gstore<false>(y + k, cadd(e, cmul(mul_di<-1>(d), hw[k])));
            }
        }
        __syncthreads();
    }
}

template <class Sh, class Pol>
__global__ void __launch_bounds__(Pol::kThreads) __attribute__((amdgpu_waves_per_eu(Pol::kWaves)))
    real_inverse_kernel(const c32 *in, c32 *out, const c32 *__restrict__ tw,
                        const c32 *__restrict__ hw, uint64_t batch)
{
    constexpr int M = Sh::M;
    __shared__ c32 lds[Pol::kLdsElems];
    using S0 = Stage<Sh, 0, 1>;
    const int tid_tw = threadIdx.x;
    const uint64_t groups = (batch + Pol::S - 1) / Pol::S;
    for (uint64_t g = blockIdx.x; g < groups; g += gridDim.x) {
        const int tid = Pol::kPlainLane ? tid_tw : opaque_lane();
        const int t = Pol::template thr<0>(tid);
        const uint64_t seg = g * Pol::S + Pol::template col<0>(tid);
        const typename Pol::Ctx ctx{out + seg * M, seg < batch && Pol::active(tid)};
        c32 v[Sh::kMaxE];
        // bins k and M-k of one segment are read by different lanes: plain
        // loads keep the lines cached for the second read
        const c32 *x = in + seg * (uint64_t)(M + 1);
        if (ctx.valid)
            st_gather<S0, Sh>(v, t, [&](int i) {
                c32 a = x[i];
                const c32 z = x[M - i];
                c32 b = {z.x, -z.y};
                if (i == 0) {
                    a.y = 0.f;
                    b.y = 0.f;
                }
                const c32 d = cmulc(csub(a, b), hw[i]);  // (A - B) W_N^{-k}
                return cadd(cadd(a, b), mul_di<1>(d));
            });
        if constexpr (Pol::kClassic)
            tile_run_plain<Sh, Pol, 1, 0, 1>(v, lds, tw, tid, ctx);
        else
            tile_run<Sh, Pol, 1, 0, 1>(v, lds, tw, tid, tid_tw, ctx);
    }
}

// ---------------------------------------------------------------------------
// Four-step split N = N1 * N2 for segments longer than one LDS tile.
// With n = n1*N2 + n2 and k = k1 + N1*k2:
//   X[k1 + N1 k2] = sum_{n2} W_{N2}^{n2 k2} [ W_N^{n2 k1} sum_{n1} x[n1 N2 + n2] W_{N1}^{n1 k1} ]
// Pass A: for every column n2, the N1-point DFT over n1 (stride N2), times
//         W_N^{n2 k1}, stored as Y[k1 N2 + n2] (same layout as the input).
// Pass B: for every row k1 of Y, the N2-point DFT over n2 (contiguous),
//         stored transposed as X[k1 + N1 k2].
// A workgroup owns C adjacent columns (pass A) or C adjacent rows (pass B)
// of one segment, so every global access moves runs of C*8 contiguous bytes.
// W_N^m (m = n2*k1 < N) is the product of two table entries
// th[m >> sh] * tl[m & (2^sh - 1)], each evaluated in FP64 and rounded once.

// Y between the two passes: in the input's layout, Y[k1][n2] at k1 N2 + n2,
// or (policies with YBlk) in blocks of kYBlock columns, at
// ((n2 / kYBlock) N1 + k1) kYBlock + n2 mod kYBlock.  Blocked, a column tile
// of 16 columns writes whole runs of 16 N1 samples instead of 128-byte
// pieces N2 samples apart, and a row tile of 16 rows reads runs of 256
// samples instead of whole rows; the plan pairs blocked column and row
// tiles only (the forms that wrap round keep the input's layout).
constexpr int kYBlock = 16;

struct FourStepCtx {
    const c32 *x;   // pass A: segment input;     pass B: segment of Y
    c32 *y;         // pass A: segment of Y;      pass B: segment output
    int first;      // first column (A) / row (B) of the tile
    int n1, n2;
    const c32 *__restrict__ tl;
    const c32 *__restrict__ th;
    int sh;
    bool valid;
    // pass A with the twiddle factors split in LDS: W_N^{n2 r NB} for the
    // tile's columns and the last stage's outputs r (column-fastest)
    const c32 *ltw = nullptr;
};

// Pass A: lanes column-fastest (c = tid % C, t = tid / C) in every stage.
//
// LdsTw: the factor W_N^{n2 k1} of output k1 = b + r NB of the last stage
// (NB butterflies of radix R) is formed as W_N^{n2 b} W_N^{n2 r NB}.  The
// first is one table lookup per butterfly b a thread owns; the second,
// shared by every thread of a column, is looked up once per tile into LDS
// (R x C values, two buffers alternating between consecutive tiles), so an
// output costs one LDS read instead of two table reads.
template <class Sh, int C_, int PS_, bool NT_ = false, int HoistMask_ = -1,
          bool Xcd_ = false, int Waves_ = 1, bool PlainLane_ = false, bool Split_ = false,
          bool Wrap_ = false, bool LdsTw_ = false, bool TwPair_ = false, bool YBlk_ = false>
struct ColumnPolicy {
    static constexpr int C = C_;
    static constexpr bool kYBlk = YBlk_ && !Wrap_;  // Y in blocks of kYBlock columns
    static constexpr bool kTwPair = TwPair_;  // as in SinglePassPolicy
    static constexpr bool kSplit = Split_;  // as in SinglePassPolicy
    // Wrap: tile columns are first + c modulo the (power-of-two) column
    // count, so blocks may start at any column and the last one wraps
    static constexpr bool kWrap = Wrap_;
    static constexpr bool kLdsTw = LdsTw_;
    static_assert(!kLdsTw || Sh::NS > 1, "the LDS twiddles are ordered by the exchange barriers");
    static constexpr int PS = PS_;
    static constexpr bool kPlainLds = false;
    static constexpr bool kPlainLane = PlainLane_;  // as in SinglePassPolicy
    static constexpr bool kNT = NT_;
    static constexpr int kHoistMask = HoistMask_;
    static constexpr bool kXcd = Xcd_;
    static constexpr int kWaves = Waves_;
    static constexpr bool hoists(int stage) { return (kHoistMask >> stage) & 1; }
    static constexpr int pad(int i) { return PS > 0 ? i + (i >> PS) : i; }
    static constexpr int kLastR = Sh::Rad::at(Sh::NS - 1);
    static constexpr int kLastNB = Sh::M / kLastR;
    // exchange elements: complex values, or floats with split exchanges
    static constexpr int kExchElems = (pad(Sh::M - 1) + 1) * C;
    static constexpr int kTwElems = kLdsTw ? kLastR * C : 0;
    // the two twiddle buffers follow the exchange area (offset in complex
    // values from the LDS base); kLdsElems counts in the exchange's units
    static constexpr int kTwOffset = kSplit ? (kExchElems + 1) / 2 : kExchElems;
    static constexpr int kLdsElems = kSplit ? 2 * kTwOffset + 4 * kTwElems
                                            : kExchElems + 2 * kTwElems;
    static constexpr int kThreads = Sh::T * C;
    using Ctx = FourStepCtx;
    // index of Y[k1][n2] (see kYBlock)
    static __device__ __forceinline__ size_t y_at(unsigned k1, unsigned n2, const Ctx &ctx)
    {
        if constexpr (kYBlk)
            return ((size_t)(n2 / kYBlock) * (unsigned)Sh::M + k1) * kYBlock + n2 % kYBlock;
        else
            return (size_t)k1 * ctx.n2 + n2;
    }
    template <int I>
    static __device__ __forceinline__ int col(int tid) { return tid % C; }
    template <int I>
    static __device__ __forceinline__ int thr(int tid) { return tid / C; }
    static __device__ __forceinline__ int lds(int c, int i) { return pad(i) * C + c; }
    static __device__ __forceinline__ bool active(int) { return true; }
    template <int STEP>
    static constexpr bool strided() { return PS <= 0 || STEP % (1 << PS) == 0; }
    template <int STEP>
    static constexpr int stride() { return (PS > 0 ? STEP + (STEP >> PS) : STEP) * C; }
    template <int R>
    static constexpr bool unit_run() { return PS > 0 && R == (1 << PS); }

    template <class St, int D>
    static __device__ __forceinline__ void store(const c32 *v, int t, int c, const Ctx &ctx)
    {
        if (!ctx.valid)
            return;
        const unsigned n2 = kWrap ? (unsigned)((ctx.first + c) & (ctx.n2 - 1))
                                  : (unsigned)(ctx.first + c);
        const unsigned mask = (1u << ctx.sh) - 1u;
        if constexpr (kLdsTw) {
            static_assert(St::R == kLastR, "the store sees the last stage");
            const c32 *bw = ctx.ltw + c;
#pragma unroll
            for (int u = 0; u < St::U; ++u) {
                const int b = t + u * Sh::T;
                if (St::kFull || b < St::NB) {
                    const unsigned m = n2 * (unsigned)b;
                    const c32 a = cmul(ctx.th[m >> ctx.sh], ctx.tl[m & mask]);
#pragma unroll
                    for (int r = 0; r < St::R; ++r) {
                        const unsigned k1 = (unsigned)(b + r * St::NB);
                        gstore<kNT>(ctx.y + y_at(k1, n2, ctx),
                                    twiddle<D>(v[u * St::R + r], cmul(a, bw[r * C])));
                    }
                }
            }
            return;
        }
#pragma unroll
        for (int u = 0; u < St::U; ++u) {
            const int b = t + u * Sh::T;
            if (St::kFull || b < St::NB) {
#pragma unroll
                for (int r = 0; r < St::R; ++r) {
                    const unsigned k1 = (unsigned)(b + r * St::NB);
                    const unsigned m = n2 * k1;
                    const c32 w = cmul(ctx.th[m >> ctx.sh], ctx.tl[m & mask]);
                    gstore<kNT>(ctx.y + y_at(k1, n2, ctx), twiddle<D>(v[u * St::R + r], w));
                }
            }
        }
    }
};

// Pol::kLdsTw: the tile's W_N^{n2 r NB} into the LDS buffer of parity
// `par` (consecutive tiles of a workgroup alternate).  Written before the
// tile's first exchange barrier and read after it; a workgroup reaches the
// next tile's write to the same buffer only after the barriers of the tile
// between, which every thread enters after its store.
template <class Sh, class Pol>
__device__ __forceinline__ void column_lds_twiddles(c32 *lds, FourStepCtx &ctx, int par,
                                                    int tid)
{
    if constexpr (Pol::kLdsTw) {
        c32 *ltw = lds + Pol::kTwOffset + (par & 1) * Pol::kTwElems;
        const unsigned mask = (1u << ctx.sh) - 1u;
        for (int e = tid; e < Pol::kTwElems; e += Pol::kThreads) {
            const int r = e / Pol::C, c = e - (e / Pol::C) * Pol::C;
            const unsigned n2 = Pol::kWrap ? (unsigned)((ctx.first + c) & (ctx.n2 - 1))
                                           : (unsigned)(ctx.first + c);
            const unsigned m = n2 * (unsigned)(r * Pol::kLastNB);  // < N1 N2
            ltw[e] = cmul(ctx.th[m >> ctx.sh], ctx.tl[m & mask]);
        }
        ctx.ltw = ltw;
    }
}

// One pass-A tile: columns first..first+C-1 of one segment (x: segment
// input, y: the segment's Y buffer, n2 columns); par: the tile's parity in
// the workgroup's sequence (LDS twiddle buffer).
template <class Sh, class Pol, int D>
__device__ __forceinline__ void column_tile(c32 *lds, const c32 *__restrict__ tw,
                                            const c32 *__restrict__ tl,
                                            const c32 *__restrict__ th, int sh, int tid,
                                            int tid_tw, const c32 *x, c32 *y, int first, int n2,
                                            int par)
{
    FourStepCtx ctx{x, y, first, Sh::M, n2, tl, th, sh, true};
    column_lds_twiddles<Sh, Pol>(lds, ctx, par, tid);
    const int c = Pol::template col<0>(tid);
    const int t = Pol::template thr<0>(tid);
    c32 v[Sh::kMaxE];
    using S0 = Stage<Sh, 0, 1>;
    const c32 *xc = x + (Pol::kWrap ? ((first + c) & (n2 - 1)) : (first + c));
    st_gather<S0, Sh>(v, t, [&](int i) { return gload<Pol::kNT>(xc + (size_t)i * n2); });
    if constexpr (Pol::kSplit)
        tile_run_split<Sh, Pol, D, 0, 1>(v, reinterpret_cast<float *>(lds), tw, tid, tid_tw,
                                         ctx);
    else
        tile_run<Sh, Pol, D, 0, 1>(v, lds, tw, tid, tid_tw, ctx);
}

template <class Sh, class Pol, int D>
__global__ void __launch_bounds__(Pol::kThreads) __attribute__((amdgpu_waves_per_eu(Pol::kWaves)))
    four_step_columns_kernel(const c32 *in, c32 *ybuf, const c32 *__restrict__ tw,
                             const c32 *__restrict__ tl, const c32 *__restrict__ th,
                             int sh, int n2, uint64_t batch)
{
    __shared__ c32 lds[lds_c32<Pol::kLdsElems, Pol::kSplit>()];
    const uint64_t nseg = (uint64_t)Sh::M * (uint64_t)n2;
    const uint64_t blocks = (uint64_t)(n2 / Pol::C);
    const uint64_t tiles = batch * blocks;
    int par = 0;
    for (uint64_t base = 0; base < tiles; base += gridDim.x, par ^= 1) {
        const uint64_t g = tile_of<Pol::kXcd>(base, blockIdx.x, gridDim.x);
        if (g >= tiles)
            continue;
        const uint64_t seg = g / blocks;
        const int first = (int)(g - seg * blocks) * Pol::C;
        column_tile<Sh, Pol, D>(lds, tw, tl, th, sh,
                                Pol::kPlainLane ? (int)threadIdx.x : opaque_lane(), threadIdx.x,
                                in + seg * nseg, ybuf + seg * nseg, first, n2, par);
    }
}

// Pass A of segments that start anywhere in a 128-byte line: column blocks
// start at column `shift`, the first whose address is line-aligned, and the
// last block wraps round to the columns before it (Pol::kWrap), so every
// block reads and writes whole lines when ybuf has the input's offset
// within a line.
template <class Sh, class Pol, int D>
__global__ void __launch_bounds__(Pol::kThreads) __attribute__((amdgpu_waves_per_eu(Pol::kWaves)))
    four_step_columns_shifted_kernel(const c32 *in, c32 *ybuf, const c32 *__restrict__ tw,
                                     const c32 *__restrict__ tl, const c32 *__restrict__ th,
                                     int sh, int n2, uint64_t batch, int shift)
{
    static_assert(Pol::kWrap, "shifted blocks wrap round");
    __shared__ c32 lds[lds_c32<Pol::kLdsElems, Pol::kSplit>()];
    const uint64_t nseg = (uint64_t)Sh::M * (uint64_t)n2;
    const uint64_t blocks = (uint64_t)(n2 / Pol::C);
    const uint64_t tiles = batch * blocks;
    int par = 0;
    for (uint64_t base = 0; base < tiles; base += gridDim.x, par ^= 1) {
        const uint64_t g = tile_of<Pol::kXcd>(base, blockIdx.x, gridDim.x);
        if (g >= tiles)
            continue;
        const uint64_t seg = g / blocks;
        const int first = (int)(g - seg * blocks) * Pol::C + shift;
        column_tile<Sh, Pol, D>(lds, tw, tl, th, sh,
                                Pol::kPlainLane ? (int)threadIdx.x : opaque_lane(), threadIdx.x,
                                in + seg * nseg, ybuf + seg * nseg, first, n2, par);
    }
}

// Pass A over overlapping, windowed frames (short-time transform): frame s
// starts at in + s * hop and its sample n is multiplied by window[n] (window
// may be null) as the column loads read it; otherwise as
// four_step_columns_kernel.  Y keeps one N1 x N2 block per frame.
template <class Sh, class Pol, int D>
__global__ void __launch_bounds__(Pol::kThreads) __attribute__((amdgpu_waves_per_eu(Pol::kWaves)))
    four_step_columns_frames_kernel(const c32 *in, c32 *ybuf, const c32 *__restrict__ tw,
                                    const c32 *__restrict__ tl, const c32 *__restrict__ th,
                                    int sh, int n2, uint64_t batch, uint64_t hop,
                                    const float *__restrict__ window)
{
    __shared__ c32 lds[lds_c32<Pol::kLdsElems, Pol::kSplit>()];
    using S0 = Stage<Sh, 0, 1>;
    const uint64_t nseg = (uint64_t)Sh::M * (uint64_t)n2;
    const uint64_t blocks = (uint64_t)(n2 / Pol::C);
    const uint64_t tiles = batch * blocks;
    int par = 0;
    for (uint64_t base = 0; base < tiles; base += gridDim.x, par ^= 1) {
        const uint64_t g = tile_of<Pol::kXcd>(base, blockIdx.x, gridDim.x);
        if (g >= tiles)
            continue;
        const uint64_t seg = g / blocks;
        const int first = (int)(g - seg * blocks) * Pol::C;
        const int tid = Pol::kPlainLane ? (int)threadIdx.x : opaque_lane();
        const int c = Pol::template col<0>(tid);
        const int t = Pol::template thr<0>(tid);
        FourStepCtx ctx{nullptr, ybuf + seg * nseg, first, Sh::M, n2, tl, th, sh, true};
        column_lds_twiddles<Sh, Pol>(lds, ctx, par, tid);
        c32 v[Sh::kMaxE];
        const c32 *xc = in + seg * hop + first + c;
        // overlapping frames are loaded through the cache (as in
        // single_pass_strided_kernel)
        auto gather = [&](auto load) {
            if (window) {
                const float *wc = window + first + c;
                st_gather<S0, Sh>(v, t, [&](int i) {
                    const c32 a = load(xc + (size_t)i * n2);
                    const float w = wc[(size_t)i * n2];
                    return c32{a.x * w, a.y * w};
                });
            } else {
                st_gather<S0, Sh>(v, t, [&](int i) { return load(xc + (size_t)i * n2); });
            }
        };
        if (hop < nseg)
            gather([](const c32 *p) { return gload<false>(p); });
        else
            gather([](const c32 *p) { return gload<Pol::kNT>(p); });
        if constexpr (Pol::kSplit)
            tile_run_split<Sh, Pol, D, 0, 1>(v, reinterpret_cast<float *>(lds), tw, tid,
                                             threadIdx.x, ctx);
        else
            tile_run<Sh, Pol, D, 0, 1>(v, lds, tw, tid, threadIdx.x, ctx);
    }
}

// Pass B: lanes row-major (c = tid / T, t = tid % T) up to the last stage,
// row-fastest (c = tid % C, t = tid / C) in the last stage so the
// transposed store X[k1 + N1 k2] writes C consecutive k1 per k2.
template <class Sh, int C_, int PS_, bool NT_ = false, int HoistMask_ = -1,
          bool Xcd_ = false, int Waves_ = 1, bool PlainLane_ = false, bool Split_ = false,
          bool Wrap_ = false, bool TwPair_ = false, bool YBlk_ = false>
struct RowPolicy {
    static constexpr int C = C_;
    static constexpr bool kYBlk = YBlk_ && !Wrap_;  // as in ColumnPolicy
    static constexpr bool kTwPair = TwPair_;  // as in SinglePassPolicy
    static constexpr bool kSplit = Split_;  // as in SinglePassPolicy
    static constexpr bool kWrap = Wrap_;    // as in ColumnPolicy (rows modulo n1)
    static constexpr int PS = PS_;
    static constexpr bool kPlainLds = false;
    static constexpr bool kPlainLane = PlainLane_;  // as in SinglePassPolicy
    static constexpr bool kNT = NT_;
    static constexpr int kHoistMask = HoistMask_;
    static constexpr bool kXcd = Xcd_;
    static constexpr int kWaves = Waves_;
    static constexpr bool hoists(int stage) { return (kHoistMask >> stage) & 1; }
    static constexpr int pad(int i) { return PS > 0 ? i + (i >> PS) : i; }
    static constexpr int kRow = (pad(Sh::M - 1) + 1) | 1;  // odd row stride
    static constexpr int kLdsElems = kRow * C;
    static constexpr int kThreads = Sh::T * C;
    using Ctx = FourStepCtx;
    template <int I>
    static __device__ __forceinline__ int col(int tid)
    {
        return (I + 1 == Sh::NS) ? tid % C : tid / Sh::T;
    }
    template <int I>
    static __device__ __forceinline__ int thr(int tid)
    {
        return (I + 1 == Sh::NS) ? tid / C : tid % Sh::T;
    }
    static __device__ __forceinline__ int lds(int c, int i) { return c * kRow + pad(i); }
    static __device__ __forceinline__ bool active(int) { return true; }
    template <int STEP>
    static constexpr bool strided() { return PS <= 0 || STEP % (1 << PS) == 0; }
    template <int STEP>
    static constexpr int stride() { return PS > 0 ? STEP + (STEP >> PS) : STEP; }
    template <int R>
    static constexpr bool unit_run() { return PS > 0 && R == (1 << PS); }

    template <class St, int D>
    static __device__ __forceinline__ void store(const c32 *v, int t, int c, const Ctx &ctx)
    {
        if (!ctx.valid)
            return;
        c32 *y = ctx.y + (kWrap ? ((ctx.first + c) & (ctx.n1 - 1)) : (ctx.first + c));
#pragma unroll
        for (int u = 0; u < St::U; ++u) {
            const int b = t + u * Sh::T;
            if (St::kFull || b < St::NB) {
#pragma unroll
                for (int r = 0; r < St::R; ++r)
                    gstore<kNT>(y + (size_t)(b + r * St::NB) * ctx.n1, v[u * St::R + r]);
            }
        }
    }
};

// One pass-B tile: rows first..first+C-1 of one segment's Y (y: Y of the
// segment, x: segment output, n1 rows).
template <class Sh, class Pol, int D>
__device__ __forceinline__ void row_tile(c32 *lds, const c32 *__restrict__ tw, int tid,
                                         int tid_tw, const c32 *y, c32 *x, int first, int n1)
{
    static_assert(Sh::NS > 1, "the row pass changes lane mapping through LDS");
    FourStepCtx ctx{y, x, first, n1, Sh::M, nullptr, nullptr, 0, true};
    const int c = Pol::template col<0>(tid);
    const int t = Pol::template thr<0>(tid);
    c32 v[Sh::kMaxE];
    using S0 = Stage<Sh, 0, 1>;
    if constexpr (Pol::kYBlk) {
        // Y in blocks of kYBlock columns (row k1 = first + c)
        const c32 *yr = y + (size_t)(first + c) * kYBlock;
        const size_t blk = (size_t)n1 * kYBlock;
        st_gather<S0, Sh>(v, t, [&](int i) {
            return gload<Pol::kNT>(yr + (size_t)(i / kYBlock) * blk + i % kYBlock);
        });
    } else {
        const c32 *yr =
            y + (size_t)(Pol::kWrap ? ((first + c) & (n1 - 1)) : (first + c)) * Sh::M;
        st_gather<S0, Sh>(v, t, [&](int i) { return gload<Pol::kNT>(yr + i); });
    }
    if constexpr (Pol::kSplit)
        tile_run_split<Sh, Pol, D, 0, 1>(v, reinterpret_cast<float *>(lds), tw, tid, tid_tw,
                                         ctx);
    else
        tile_run<Sh, Pol, D, 0, 1>(v, lds, tw, tid, tid_tw, ctx);
}

template <class Sh, class Pol, int D>
__global__ void __launch_bounds__(Pol::kThreads) __attribute__((amdgpu_waves_per_eu(Pol::kWaves)))
    four_step_rows_kernel(const c32 *ybuf, c32 *out, const c32 *__restrict__ tw,
                          int n1, uint64_t batch)
{
    __shared__ c32 lds[lds_c32<Pol::kLdsElems, Pol::kSplit>()];
    const uint64_t nseg = (uint64_t)Sh::M * (uint64_t)n1;
    const uint64_t blocks = (uint64_t)(n1 / Pol::C);
    const uint64_t tiles = batch * blocks;
    for (uint64_t base = 0; base < tiles; base += gridDim.x) {
        const uint64_t g = tile_of<Pol::kXcd>(base, blockIdx.x, gridDim.x);
        if (g >= tiles)
            continue;
        const uint64_t seg = g / blocks;
        const int first = (int)(g - seg * blocks) * Pol::C;
        row_tile<Sh, Pol, D>(lds, tw, Pol::kPlainLane ? (int)threadIdx.x : opaque_lane(),
                             threadIdx.x, ybuf + seg * nseg,
                             out + seg * nseg, first, n1);
    }
}

// Pass B with row blocks starting at row `shift` (the first whose transposed
// store is line-aligned in out) and the last one wrapping round (Pol::kWrap).
template <class Sh, class Pol, int D>
__global__ void __launch_bounds__(Pol::kThreads) __attribute__((amdgpu_waves_per_eu(Pol::kWaves)))
    four_step_rows_shifted_kernel(const c32 *ybuf, c32 *out, const c32 *__restrict__ tw,
                                  int n1, uint64_t batch, int shift)
{
    static_assert(Pol::kWrap, "shifted blocks wrap round");
    __shared__ c32 lds[lds_c32<Pol::kLdsElems, Pol::kSplit>()];
    const uint64_t nseg = (uint64_t)Sh::M * (uint64_t)n1;
    const uint64_t blocks = (uint64_t)(n1 / Pol::C);
    const uint64_t tiles = batch * blocks;
    for (uint64_t base = 0; base < tiles; base += gridDim.x) {
        const uint64_t g = tile_of<Pol::kXcd>(base, blockIdx.x, gridDim.x);
        if (g >= tiles)
            continue;
        const uint64_t seg = g / blocks;
        const int first = (int)(g - seg * blocks) * Pol::C + shift;
        row_tile<Sh, Pol, D>(lds, tw, Pol::kPlainLane ? (int)threadIdx.x : opaque_lane(),
                             threadIdx.x, ybuf + seg * nseg, out + seg * nseg, first, n1);
    }
}

// Both passes over segments at listed offsets (offs holds records of three
// words per segment: input offset, output offset, unused; sample units).
// Segment s keeps its Y at ybuf + s * (N + 16), plus the input's offset
// within a 128-byte line (16 samples), and each pass starts its blocks at
// the first column (row) whose address in x (out) is line-aligned, wrapping
// round, as the shifted kernels do for a whole batch: every block then
// reads and writes whole lines wherever the caller's segments start.
constexpr int kIdxLine = 16;

__device__ __forceinline__ int line_offset(const c32 *p)
{
    return (int)(((uintptr_t)p / sizeof(c32)) & (kIdxLine - 1));
}

template <class Sh, class Pol, int D>
__global__ void __launch_bounds__(Pol::kThreads) __attribute__((amdgpu_waves_per_eu(Pol::kWaves)))
    four_step_columns_indexed_kernel(const c32 *in, c32 *ybuf, const c32 *__restrict__ tw,
                                     const c32 *__restrict__ tl, const c32 *__restrict__ th,
                                     int sh, int n2, const uint64_t *__restrict__ offs,
                                     uint64_t batch)
{
    static_assert(Pol::kWrap, "blocks wrap round");
    __shared__ c32 lds[lds_c32<Pol::kLdsElems, Pol::kSplit>()];
    const uint64_t nseg = (uint64_t)Sh::M * (uint64_t)n2;
    const uint64_t blocks = (uint64_t)(n2 / Pol::C);
    const uint64_t tiles = batch * blocks;
    int par = 0;
    for (uint64_t base = 0; base < tiles; base += gridDim.x, par ^= 1) {
        const uint64_t g = tile_of<Pol::kXcd>(base, blockIdx.x, gridDim.x);
        if (g >= tiles)
            continue;
        const uint64_t seg = g / blocks;
        const c32 *x = in + offs[3 * seg];
        const int in_m = line_offset(x);
        const int first = (int)(g - seg * blocks) * Pol::C + ((kIdxLine - in_m) & (kIdxLine - 1));
        column_tile<Sh, Pol, D>(lds, tw, tl, th, sh,
                                Pol::kPlainLane ? (int)threadIdx.x : opaque_lane(), threadIdx.x,
                                x, ybuf + seg * (nseg + kIdxLine) + in_m, first, n2, par);
    }
}

template <class Sh, class Pol, int D>
__global__ void __launch_bounds__(Pol::kThreads) __attribute__((amdgpu_waves_per_eu(Pol::kWaves)))
    four_step_rows_indexed_kernel(const c32 *in, const c32 *ybuf, c32 *out,
                                  const c32 *__restrict__ tw, int n1,
                                  const uint64_t *__restrict__ offs, uint64_t batch)
{
    static_assert(Pol::kWrap, "blocks wrap round");
    __shared__ c32 lds[lds_c32<Pol::kLdsElems, Pol::kSplit>()];
    const uint64_t nseg = (uint64_t)Sh::M * (uint64_t)n1;
    const uint64_t blocks = (uint64_t)(n1 / Pol::C);
    const uint64_t tiles = batch * blocks;
    for (uint64_t base = 0; base < tiles; base += gridDim.x) {
        const uint64_t g = tile_of<Pol::kXcd>(base, blockIdx.x, gridDim.x);
        if (g >= tiles)
            continue;
        const uint64_t seg = g / blocks;
        const int in_m = line_offset(in + offs[3 * seg]);
        c32 *y = out + offs[3 * seg + 1];
        const int first =
            (int)(g - seg * blocks) * Pol::C + ((kIdxLine - line_offset(y)) & (kIdxLine - 1));
        row_tile<Sh, Pol, D>(lds, tw, Pol::kPlainLane ? (int)threadIdx.x : opaque_lane(),
                             threadIdx.x, ybuf + seg * (nseg + kIdxLine) + in_m, y, first, n1);
    }
}

// ---------------------------------------------------------------------------
// Fallback for lengths without a compiled tile: one launch per Stockham
// stage over global memory, one thread per butterfly, radix R at run-time
// stride L.  Twiddle W_N^m = th[m >> sh] * tl[m & mask] as in pass A.
template <int R, int D>
__global__ void __launch_bounds__(256)
    stockham_global_stage_kernel(const c32 *in, c32 *out, const c32 *__restrict__ tl,
                                 const c32 *__restrict__ th, int sh,
                                 uint64_t n, uint64_t l, uint64_t batch)
{
    const uint64_t nb = n / R;
    const uint64_t total = nb * batch;
    const uint64_t tw_stride = n / (l * R);
    const unsigned mask = (1u << sh) - 1u;
    for (uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; gid < total;
         gid += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t seg = gid / nb;
        const uint64_t b = gid - seg * nb;
        const c32 *x = in + seg * n;
        c32 *y = out + seg * n;
        c32 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r)
            v[r] = x[b + r * nb];
        const uint64_t k = b % l;
        if (l > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                const unsigned m = (unsigned)(r * k * tw_stride);
                v[r] = twiddle<D>(v[r], cmul(th[m >> sh], tl[m & mask]));
            }
        }
        dft<R, D>(v);
        const uint64_t base = (b / l) * (l * R) + k;
#pragma unroll
        for (int r = 0; r < R; ++r)
            y[base + r * l] = v[r];
    }
}

}  // namespace fftseg
