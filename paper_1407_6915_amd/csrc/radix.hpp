// In-register small DFT butterflies for the Cooley-Tukey stages.
//
// dft<R, D>(v) replaces v[0..R) by its R-point DFT
//     v'[k] = sum_j v[j] * exp(D * 2*pi*i * j*k / R),   D = -1 forward, +1 inverse,
// with no scaling.  Radices 2, 3, 4 and 5 are written out; every other
// radix R = P * Q is built in registers by one decimation-in-time step
// (P sub-sequences v[p + P*t] of length Q, twiddles W_R^{p*kq}, then
// P-point DFTs), so all constants are compile-time.
//
// Constant twiddles come from a constexpr cos/sin of 2*pi*j/n that reduces
// the angle to the first octant in exact integer arithmetic and sums a
// Taylor series there in double, then rounds once to float.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fftseg {

struct alignas(8) c32 {
    float x, y;
};

__device__ __forceinline__ c32 cadd(c32 a, c32 b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ c32 csub(c32 a, c32 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ c32 cmul(c32 a, c32 b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
__device__ __forceinline__ c32 cmulc(c32 a, c32 b)
{
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// a * (D * i):  D = +1 -> multiply by i, D = -1 -> by -i
template <int D>
__device__ __forceinline__ c32 mul_di(c32 a)
{
    if constexpr (D > 0)
        return {-a.y, a.x};
    else
        return {a.y, -a.x};
}
// multiply by a forward-table twiddle w = exp(-2 pi i m / N) in direction D
template <int D>
__device__ __forceinline__ c32 twiddle(c32 a, c32 w)
{
    if constexpr (D < 0)
        return cmul(a, w);
    else
        return cmulc(a, w);
}

// ---------------------------------------------------------------------------
// constexpr trigonometry for compile-time twiddles
namespace ct {
constexpr double kHalfPi = 1.57079632679489661923132169163975144;

constexpr double sin_series(double x)
{
    double t = x, s = x;
    for (int k = 1; k < 14; ++k) {
        t *= -x * x / double((2 * k) * (2 * k + 1));
        s += t;
    }
    return s;
}
constexpr double cos_series(double x)
{
    double t = 1.0, s = 1.0;
    for (int k = 1; k < 14; ++k) {
        t *= -x * x / double((2 * k - 1) * (2 * k));
        s += t;
    }
    return s;
}
// (cos, sin) of 2*pi*j/n.  4j = q*n + r -> quadrant q, angle (pi/2)(r/n);
// r > n/2 is folded to the complementary angle so |x| <= pi/4.
struct cs {
    double c, s;
};
constexpr cs cossin2pi(long long j, long long n)
{
    j %= n;
    if (j < 0)
        j += n;
    long long q = (4 * j) / n;
    long long r = 4 * j - q * n;  // in [0, n)
    double c = 0, s = 0;
    if (2 * r <= n) {
        double x = kHalfPi * double(r) / double(n);
        c = cos_series(x);
        s = sin_series(x);
    } else {
        double x = kHalfPi * double(n - r) / double(n);
        c = sin_series(x);
        s = cos_series(x);
    }
    switch (q & 3) {
    case 0: return {c, s};
    case 1: return {-s, c};
    case 2: return {-c, -s};
    default: return {s, -c};
    }
}
constexpr float wre(long long j, long long n, int d) { return float(cossin2pi(j, n).c); }
constexpr float wim(long long j, long long n, int d) { return float(d * cossin2pi(j, n).s); }

constexpr int smallest_factor(int r)
{
    for (int p = 2; p * p <= r; ++p)
        if (r % p == 0)
            return p;
    return r;
}
// split of a composite radix R into P * Q for the in-register step
constexpr int split_p(int r)
{
    if (r % 4 == 0 && r > 4 && r != 8)
        return 4;
    return smallest_factor(r);
}
}  // namespace ct

// v * exp(D 2 pi i j / n) with compile-time j, n; exact for multiples of pi/2
template <long long J, long long NN, int D>
__device__ __forceinline__ c32 cmul_const(c32 v)
{
    constexpr long long j = ((J % NN) + NN) % NN;
    if constexpr (j == 0) {
        return v;
    } else if constexpr ((4 * j) % NN == 0) {
        constexpr long long q = (4 * j) / NN;
        if constexpr (q == 1)
            return mul_di<D>(v);
        else if constexpr (q == 2)
            return {-v.x, -v.y};
        else
            return mul_di<-D>(v);
    } else if constexpr ((8 * j) % NN == 0) {
        // odd multiple of pi/4: (+-1 +- i) / sqrt(2)
        constexpr float h = 0.70710678118654752440f;
        constexpr float c = ct::wre(j, NN, D) > 0 ? h : -h;
        constexpr float s = ct::wim(j, NN, D) > 0 ? h : -h;
        return {c * v.x - s * v.y, c * v.y + s * v.x};
    } else {
        constexpr float c = ct::wre(j, NN, D);
        constexpr float s = ct::wim(j, NN, D);
        return {c * v.x - s * v.y, c * v.y + s * v.x};
    }
}

// ---------------------------------------------------------------------------
// DFT kernels on v[0], v[S], v[2S], ... (stride S in the register array)
template <int R, int D, int S = 1>
struct Dft;

template <int D, int S>
struct Dft<1, D, S> {
    static __device__ __forceinline__ void run(c32 *) {}
};

template <int D, int S>
struct Dft<2, D, S> {
    static __device__ __forceinline__ void run(c32 *v)
    {
        c32 a = v[0], b = v[S];
        v[0] = cadd(a, b);
        v[S] = csub(a, b);
    }
};

template <int D, int S>
struct Dft<3, D, S> {
    static __device__ __forceinline__ void run(c32 *v)
    {
        // W3 = -1/2 + i D sqrt(3)/2
        constexpr float h = 0.86602540378443864676f;
        c32 a = v[0], b = v[S], c = v[2 * S];
        c32 s = cadd(b, c);
        c32 d = csub(b, c);
        c32 m = {a.x - 0.5f * s.x, a.y - 0.5f * s.y};
        c32 r = mul_di<D>(c32{h * d.x, h * d.y});
        v[0] = cadd(a, s);
        v[S] = cadd(m, r);
        v[2 * S] = csub(m, r);
    }
};

template <int D, int S>
struct Dft<4, D, S> {
    static __device__ __forceinline__ void run(c32 *v)
    {
        c32 a = v[0], b = v[S], c = v[2 * S], d = v[3 * S];
        c32 s0 = cadd(a, c), d0 = csub(a, c);
        c32 s1 = cadd(b, d), d1 = mul_di<D>(csub(b, d));
        v[0] = cadd(s0, s1);
        v[2 * S] = csub(s0, s1);
        v[S] = cadd(d0, d1);
        v[3 * S] = csub(d0, d1);
    }
};

template <int D, int S>
struct Dft<5, D, S> {
    static __device__ __forceinline__ void run(c32 *v)
    {
        constexpr float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
        constexpr float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
        constexpr float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
        constexpr float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
        c32 x0 = v[0];
        c32 a1 = cadd(v[S], v[4 * S]), b1 = csub(v[S], v[4 * S]);
        c32 a2 = cadd(v[2 * S], v[3 * S]), b2 = csub(v[2 * S], v[3 * S]);
        c32 p1 = {x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y};
        c32 p2 = {x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y};
        c32 q1 = mul_di<D>(c32{s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y});
        c32 q2 = mul_di<D>(c32{s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y});
        v[0] = {x0.x + a1.x + a2.x, x0.y + a1.y + a2.y};
        v[S] = cadd(p1, q1);
        v[4 * S] = csub(p1, q1);
        v[2 * S] = cadd(p2, q2);
        v[3 * S] = csub(p2, q2);
    }
};

// Composite radix R = P*Q by one in-register decimation-in-time step:
//   Y_p = DFT_Q(v[p + P t]),  X[kq + Q kp] = DFT_P_p(W_R^{p kq} Y_p[kq]).
template <int R, int D, int S>
struct Dft {
    static constexpr int P = ct::split_p(R);
    static constexpr int Q = R / P;
    static_assert(P > 1 && Q > 1, "composite radix expected");

    template <int p>
    static __device__ __forceinline__ void sub_q(c32 *v)
    {
        if constexpr (p < P) {
            Dft<Q, D, S * P>::run(v + p * S);
            sub_q<p + 1>(v);
        }
    }
    template <int p, int kq>
    static __device__ __forceinline__ void tw(c32 *t)
    {
        if constexpr (p < P) {
            if constexpr (kq < Q) {
                t[p * Q + kq] = cmul_const<(long long)p * kq, R, D>(t[p * Q + kq]);
                tw<p, kq + 1>(t);
            } else {
                tw<p + 1, 0>(t);
            }
        }
    }
    static __device__ __forceinline__ void run(c32 *v)
    {
        // Y_p[kq] lands at v[(p + P*kq) * S] after the strided Q-point DFTs
        sub_q<0>(v);
        c32 t[R];
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int kq = 0; kq < Q; ++kq)
                t[p * Q + kq] = v[(p + P * kq) * S];
        tw<0, 0>(t);
#pragma unroll
        for (int kq = 0; kq < Q; ++kq)
            Dft<P, D, Q>::run(t + kq);
        // X[kq + Q kp] = t[kp * Q + kq]
#pragma unroll
        for (int k = 0; k < R; ++k)
            v[k * S] = t[k];
    }
};

template <int R, int D>
__device__ __forceinline__ void dft(c32 *v)
{
    Dft<R, D, 1>::run(v);
}

}  // namespace fftseg
