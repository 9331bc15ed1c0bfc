/*
 * Seeded synthetic signal generator.
 *
 * Serves both the FP64 oracle's tests and the GPU library's tests and
 * benchmark, and holds none of the transform's arithmetic: it only draws
 * random numbers, synthesises test signals (noise, tones, a chirp) and sums
 * the energy of segments (for Parseval checks of streamed runs).
 *
 * Random numbers come from Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
 * "Parallel random numbers: as easy as 1, 2, 3", SC'11), written here from
 * its published definition: a 4 x 32-bit counter, a 2 x 32-bit key, ten
 * rounds of two 32x32->64 multiplies (multipliers 0xD2511F53, 0xCD9E8D57)
 * with the key bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85)
 * between rounds.  Being counter based, sample g of a signal is a pure
 * function of (seed, stream, g): any chunk or segment can be regenerated on
 * its own, in any order, by any number of threads.
 *
 * Counter layout: ctr = (lo32(index), hi32(index), stream, purpose),
 * key = (lo32(seed), hi32(seed)); purpose separates noise samples,
 * uniform draws and normal draws.  One noise draw at index j serves the two
 * samples 2j (words 0, 1) and 2j + 1 (words 2, 3).
 *
 * Transcendentals are computed here, not by libm, so that every host and
 * every instruction-set clone below gives the same bits: the natural log by
 * splitting off the binary exponent and summing the atanh series of
 * (m - 1) / (m + 1); cosine and sine by reducing the angle, given as an
 * exact integer ratio of quarter turns, to |x| <= pi/4 in integers, then
 * their Taylor series (truncation error below 5e-17).  Products and sums
 * are written out with fma(), and the file is compiled without
 * floating-point contraction, so no compiler choice changes a result.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define SG_PURPOSE_NOISE 0u
#define SG_PURPOSE_UNIFORM 1u
#define SG_PURPOSE_NORMAL 2u

#define SG_M0 0xD2511F53u
#define SG_M1 0xCD9E8D57u
#define SG_W0 0x9E3779B9u
#define SG_W1 0xBB67AE85u

/* The hot loops are compiled three times (AVX-512, AVX2 + FMA, baseline
 * x86-64) and one is chosen at run time from the CPU's features; every
 * version computes the same bits (fma() is exact in all of them). */
#if defined(__x86_64__) && defined(__GNUC__)
#define SG_X86_DISPATCH 1
#define SG_T512 __attribute__((target("avx512f,avx512dq,avx512vl,avx512bw,avx2,fma,bmi,bmi2")))
#define SG_T256 __attribute__((target("avx2,fma,bmi,bmi2")))
#endif

static const double SG_HALF_PI = 1.5707963267948966192313216916398;
static const double SG_LN2 = 0.69314718055994530941723212145818;
static const double SG_SQRT2 = 1.4142135623730950488016887242097;

void sg_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                      uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += SG_W0;
            k1 += SG_W1;
        }
        uint64_t p0 = (uint64_t)SG_M0 * c0;
        uint64_t p1 = (uint64_t)SG_M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

static inline void draw(uint64_t seed, uint32_t stream, uint32_t purpose,
                        uint64_t index, uint32_t r[4])
{
    uint32_t ctr[4] = {(uint32_t)index, (uint32_t)(index >> 32), stream,
                       purpose};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    sg_philox4x32_10(ctr, key, r);
}

/* (0,1) with 53 bits from two words. */
static inline double u53_open(uint32_t a, uint32_t b)
{
    uint64_t m = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return ((double)m + 0.5) * (1.0 / 9007199254740992.0);
}

#define SG_INLINE static inline __attribute__((always_inline))

/* ln x for a normal, positive x. */
SG_INLINE double sg_ln(double x)
{
    uint64_t b;
    memcpy(&b, &x, sizeof b);
    double e = (double)((int64_t)(b >> 52) - 1023);
    uint64_t mb = (b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull;
    double m;
    memcpy(&m, &mb, sizeof m);           /* [1, 2) */
    const int fold = m > SG_SQRT2;       /* fold to [sqrt(1/2), sqrt(2)) */
    m = fold ? m * 0.5 : m;
    e = fold ? e + 1.0 : e;
    double s = (m - 1.0) / (m + 1.0);    /* |s| < 0.1716 */
    double z = s * s;
    /* ln m = 2 atanh s = 2 s (1 + z/3 + z^2/5 + ... + z^10/21) */
    double p = 1.0 / 21.0;
    p = fma(p, z, 1.0 / 19.0);
    p = fma(p, z, 1.0 / 17.0);
    p = fma(p, z, 1.0 / 15.0);
    p = fma(p, z, 1.0 / 13.0);
    p = fma(p, z, 1.0 / 11.0);
    p = fma(p, z, 1.0 / 9.0);
    p = fma(p, z, 1.0 / 7.0);
    p = fma(p, z, 1.0 / 5.0);
    p = fma(p, z, 1.0 / 3.0);
    p = fma(p, z, 1.0);
    return fma(e, SG_LN2, 2.0 * s * p);
}

/* (cos, sin) of (pi/2) (k + t) for an integer k and |t| <= 1/2. */
SG_INLINE void sg_quarter(int64_t k, double t, double *co, double *si)
{
    double x = t * SG_HALF_PI;
    double z = x * x;
    double sp = -1.0 / 1307674368000.0;             /* -1/15! */
    sp = fma(sp, z, 1.0 / 6227020800.0);
    sp = fma(sp, z, -1.0 / 39916800.0);
    sp = fma(sp, z, 1.0 / 362880.0);
    sp = fma(sp, z, -1.0 / 5040.0);
    sp = fma(sp, z, 1.0 / 120.0);
    sp = fma(sp, z, -1.0 / 6.0);
    sp = fma(sp * z, x, x);
    double cp = 1.0 / 20922789888000.0;             /* 1/16! */
    cp = fma(cp, z, -1.0 / 87178291200.0);
    cp = fma(cp, z, 1.0 / 479001600.0);
    cp = fma(cp, z, -1.0 / 3628800.0);
    cp = fma(cp, z, 1.0 / 40320.0);
    cp = fma(cp, z, -1.0 / 720.0);
    cp = fma(cp, z, 1.0 / 24.0);
    cp = fma(cp, z, -0.5);
    cp = fma(cp, z, 1.0);
    const int64_t q = k & 3;
    const double c = (q & 1) ? sp : cp;
    const double s = (q & 1) ? cp : sp;
    const double cneg = ((q + 1) & 2) ? -1.0 : 1.0;   /* q = 1, 2 */
    const double sneg = (q & 2) ? -1.0 : 1.0;         /* q = 2, 3 */
    *co = c * cneg;
    *si = s * sneg;
}

/* (cos, sin) of (pi/2) * num / den for integers num >= 0, den > 0,
 * with num * 2 + den < 2^63: the quarter-turn count is rounded in
 * integers and only the remainder ratio is rounded to double. */
static inline void sg_quarter_ratio(uint64_t num, uint64_t den, double *co,
                                    double *si)
{
    uint64_t k = (2 * num + den) / (2 * den);
    int64_t rem = (int64_t)num - (int64_t)(k * den);   /* in [-den/2, den/2) */
    sg_quarter((int64_t)k, (double)rem / (double)den, co, si);
}

typedef struct {
    uint64_t seed;
    uint32_t stream;
    uint32_t n_tones;
    double sigma;         /* noise std-dev per I and per Q component   */
    uint64_t seg_len;     /* tones and chirp restart every seg_len     */
    const int64_t *tone_bin;   /* integer bins in [0, seg_len)         */
    const double *tone_amp;
    const double *tone_phase;  /* radians                              */
    double chirp_amp;     /* amplitude of exp(i*pi*n^2/seg_len), n = g mod seg_len */
} sg_signal;

/* Tables and constants one fill call shares between its threads. */
typedef struct fill_ctx_s {
    const sg_signal *s;
    uint64_t n;
    int pow2;             /* n is a power of two            */
    int lg;               /* log2 n when pow2               */
    double *root;         /* (cos, sin)(2 pi j / n), j < n  */
    double *tone_c;       /* A e^{i phi} per tone           */
    double (*block)(const struct fill_ctx_s *, uint64_t, float *);
} fill_ctx;

/* noise + tones + chirp of one sample, given its noise words (ra, rb) */
static inline void sample_value(const fill_ctx *F, uint64_t g, uint32_t ra,
                                uint32_t rb, double *re, double *im)
{
    const sg_signal *s = F->s;
    double xr = 0.0, xi = 0.0;
    if (s->sigma != 0.0) {
        double u1 = ((double)ra + 0.5) * (1.0 / 4294967296.0);
        double rad = s->sigma * sqrt(-2.0 * sg_ln(u1));
        double c, si;
        /* angle 2 pi (rb + 1/2) / 2^32 = (pi/2) (2 rb + 1) / 2^31 */
        uint64_t num = 2 * (uint64_t)rb + 1;
        int64_t k = (int64_t)((num + (1ull << 30)) >> 31);
        sg_quarter(k, (double)((int64_t)num - (k << 31)) * (1.0 / 2147483648.0), &c, &si);
        xr = rad * c;
        xi = rad * si;
    }
    if (F->root || s->chirp_amp != 0.0) {
        uint64_t ph = F->pow2 ? (g & (F->n - 1)) : g % F->n;
        for (uint32_t t = 0; t < s->n_tones; ++t) {
            uint64_t j = ((uint64_t)s->tone_bin[t] * ph) % F->n;
            double cr = F->root[2 * j], ci = F->root[2 * j + 1];
            double ar = F->tone_c[2 * t], ai = F->tone_c[2 * t + 1];
            xr += fma(ar, cr, -ai * ci);
            xi += fma(ar, ci, ai * cr);
        }
        if (s->chirp_amp != 0.0) {
            /* e^{i pi c / n}, c = ph^2 mod 2n: (pi/2) * (2c) / n */
            uint64_t c2 = F->pow2 ? ((ph * ph) & (2 * F->n - 1)) : (ph * ph) % (2 * F->n);
            double c, si;
            if (F->pow2) {
                uint64_t num = 2 * c2;
                int64_t k = (int64_t)((num + (F->n >> 1)) >> F->lg);
                sg_quarter(k, (double)((int64_t)num - (k << F->lg)) / (double)F->n, &c, &si);
            } else {
                sg_quarter_ratio(2 * c2, F->n, &c, &si);
            }
            xr = fma(s->chirp_amp, c, xr);
            xi = fma(s->chirp_amp, si, xi);
        }
    }
    *re = xr;
    *im = xi;
}

/* energy sum |x|^2 (FP64) of 8 * n8 complex64 values, over 16 fixed lanes
 * summed in a fixed order */
SG_INLINE double energy_body(const float *x, uint64_t n8)
{
    double acc[16];
    for (int l = 0; l < 16; ++l)
        acc[l] = 0.0;
    for (uint64_t i = 0; i < n8; ++i)
        for (int l = 0; l < 16; ++l) {
            double v = (double)x[16 * i + l];
            acc[l] = fma(v, v, acc[l]);
        }
    for (int l = 0; l < 8; ++l)
        acc[l] += acc[l + 8];
    return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

#define SG_BLK 512   /* samples per block: 256 noise draws */

/*
 * Samples g0 .. g0 + SG_BLK - 1 (g0 even) into dst; returns their energy
 * sum |x|^2 of the stored float values, accumulated over 8 fixed lanes.
 */
SG_INLINE double fill_block_body(const fill_ctx *F, uint64_t g0, float *dst)
{
    const sg_signal *s = F->s;
    uint32_t ra[SG_BLK], rb[SG_BLK];   /* the two words of each sample */
    if (s->sigma != 0.0) {
        const uint64_t j0 = g0 >> 1;
        const uint32_t key0 = (uint32_t)s->seed, key1 = (uint32_t)(s->seed >> 32);
        for (int i = 0; i < SG_BLK / 2; ++i) {
            uint64_t j = j0 + (uint64_t)i;
            uint32_t c0 = (uint32_t)j, c1 = (uint32_t)(j >> 32), c2 = s->stream,
                     c3 = SG_PURPOSE_NOISE;
            uint32_t k0 = key0, k1 = key1;
            for (int rr = 0; rr < 10; ++rr) {
                uint64_t p0 = (uint64_t)SG_M0 * c0;
                uint64_t p1 = (uint64_t)SG_M1 * c2;
                uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
                uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
                c1 = (uint32_t)p1;
                c3 = (uint32_t)p0;
                c0 = n0;
                c2 = n2;
                k0 += SG_W0;
                k1 += SG_W1;
            }
            ra[2 * i] = c0;
            rb[2 * i] = c1;
            ra[2 * i + 1] = c2;
            rb[2 * i + 1] = c3;
        }
    }
    double vr[SG_BLK], vi[SG_BLK];
    if (s->sigma != 0.0) {
        const double sigma = s->sigma;
        for (int i = 0; i < SG_BLK; ++i) {
            double u1 = ((double)ra[i] + 0.5) * (1.0 / 4294967296.0);
            double rad = sigma * sqrt(-2.0 * sg_ln(u1));
            uint64_t num = 2 * (uint64_t)rb[i] + 1;
            int64_t k = (int64_t)((num + (1ull << 30)) >> 31);
            double c, si;
            sg_quarter(k, (double)((int64_t)num - (k << 31)) * (1.0 / 2147483648.0), &c, &si);
            vr[i] = rad * c;
            vi[i] = rad * si;
        }
    } else {
        for (int i = 0; i < SG_BLK; ++i)
            vr[i] = vi[i] = 0.0;
    }
    if (F->root) {
        for (int i = 0; i < SG_BLK; ++i) {
            uint64_t g = g0 + (uint64_t)i;
            uint64_t ph = F->pow2 ? (g & (F->n - 1)) : g % F->n;
            double xr = vr[i], xi = vi[i];
            for (uint32_t t = 0; t < s->n_tones; ++t) {
                uint64_t j = ((uint64_t)s->tone_bin[t] * ph) % F->n;
                double cr = F->root[2 * j], ci = F->root[2 * j + 1];
                double ar = F->tone_c[2 * t], ai = F->tone_c[2 * t + 1];
                xr += fma(ar, cr, -ai * ci);
                xi += fma(ar, ci, ai * cr);
            }
            vr[i] = xr;
            vi[i] = xi;
        }
    }
    if (s->chirp_amp != 0.0) {
        const double amp = s->chirp_amp;
        if (F->pow2) {
            const uint64_t mask = F->n - 1, mask2 = 2 * F->n - 1, half = F->n >> 1;
            const int lg = F->lg;
            const double inv = 1.0 / (double)F->n;   /* a power of two: exact */
            for (int i = 0; i < SG_BLK; ++i) {
                uint64_t ph = (g0 + (uint64_t)i) & mask;
                uint64_t num = 2 * ((ph * ph) & mask2);
                int64_t k = (int64_t)((num + half) >> lg);
                double c, si;
                sg_quarter(k, (double)((int64_t)num - (k << lg)) * inv, &c, &si);
                vr[i] = fma(amp, c, vr[i]);
                vi[i] = fma(amp, si, vi[i]);
            }
        } else {
            for (int i = 0; i < SG_BLK; ++i) {
                uint64_t ph = (g0 + (uint64_t)i) % F->n;
                double c, si;
                sg_quarter_ratio(2 * ((ph * ph) % (2 * F->n)), F->n, &c, &si);
                vr[i] = fma(amp, c, vr[i]);
                vi[i] = fma(amp, si, vi[i]);
            }
        }
    }
    float fo[2 * SG_BLK];
    for (int i = 0; i < SG_BLK; ++i) {
        fo[2 * i] = (float)vr[i];
        fo[2 * i + 1] = (float)vi[i];
    }
    memcpy(dst, fo, sizeof fo);
    return energy_body(fo, SG_BLK / 8);
}

typedef double (*fill_block_fn)(const fill_ctx *, uint64_t, float *);

static double fill_block_base(const fill_ctx *F, uint64_t g0, float *dst)
{
    return fill_block_body(F, g0, dst);
}
#ifdef SG_X86_DISPATCH
SG_T512 static double fill_block_512(const fill_ctx *F, uint64_t g0, float *dst)
{
    return fill_block_body(F, g0, dst);
}
SG_T256 static double fill_block_256(const fill_ctx *F, uint64_t g0, float *dst)
{
    return fill_block_body(F, g0, dst);
}
#endif

/* 2 = AVX-512, 1 = AVX2 + FMA, 0 = baseline; a cap set by sg_set_isa
 * (tests compare the versions bit for bit) */
static int g_isa_cap = 2;

static int isa_level(void)
{
    if (g_isa_cap <= 0)
        return 0;
#ifdef SG_X86_DISPATCH
    __builtin_cpu_init();
    if (g_isa_cap >= 2 && __builtin_cpu_supports("avx512f") &&
        __builtin_cpu_supports("avx512dq") && __builtin_cpu_supports("avx512vl") &&
        __builtin_cpu_supports("avx512bw") && __builtin_cpu_supports("fma") &&
        __builtin_cpu_supports("bmi2"))
        return 2;
    if (__builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma") &&
        __builtin_cpu_supports("bmi2"))
        return 1;
#endif
    return 0;
}

static fill_block_fn pick_fill_block(void)
{
#ifdef SG_X86_DISPATCH
    switch (isa_level()) {
    case 2:
        return fill_block_512;
    case 1:
        return fill_block_256;
    }
#endif
    return fill_block_base;
}

/* one sample outside the block grid (an odd first index, or a tail) */
static double fill_one(const fill_ctx *F, uint64_t g, float *dst)
{
    uint32_t r[4] = {0, 0, 0, 0};
    if (F->s->sigma != 0.0)
        draw(F->s->seed, F->s->stream, SG_PURPOSE_NOISE, g >> 1, r);
    const int w = (int)(g & 1) * 2;
    double re, im;
    sample_value(F, g, r[w], r[w + 1], &re, &im);
    float fr = (float)re, fi = (float)im;
    dst[0] = fr;
    dst[1] = fi;
    return fma((double)fr, (double)fr, (double)fi * (double)fi);
}

static int ctx_init(fill_ctx *F, const sg_signal *s, int threads)
{
    memset(F, 0, sizeof *F);
    F->s = s;
    F->block = pick_fill_block();
    uint64_t n = s->seg_len;
    int need_tab = (s->n_tones > 0 || s->chirp_amp != 0.0);
    if (need_tab && (n == 0 || n > (1ull << 30)))
        return -1;
    F->n = n ? n : 1;
    F->pow2 = (F->n & (F->n - 1)) == 0;
    while ((1ull << F->lg) < F->n)
        ++F->lg;
    if (s->n_tones > 0) {
        F->root = (double *)malloc(2 * (size_t)n * sizeof(double));
        F->tone_c = (double *)malloc(2 * (size_t)s->n_tones * sizeof(double));
        if (!F->root || !F->tone_c)
            return -2;
        for (uint32_t t = 0; t < s->n_tones; ++t) {
            if (s->tone_bin[t] < 0 || (uint64_t)s->tone_bin[t] >= n)
                return -1;
            F->tone_c[2 * t] = s->tone_amp[t] * cos(s->tone_phase[t]);
            F->tone_c[2 * t + 1] = s->tone_amp[t] * sin(s->tone_phase[t]);
        }
        long long nn = (long long)n;
        double *root = F->root;
#pragma omp parallel for num_threads(threads) schedule(static)
        for (long long j = 0; j < nn; ++j)   /* 2 pi j / n = (pi/2) (4j) / n */
            sg_quarter_ratio(4 * (uint64_t)j, n, &root[2 * j], &root[2 * j + 1]);
    }
    return 0;
}

static void ctx_free(fill_ctx *F)
{
    free(F->root);
    free(F->tone_c);
}

static int default_threads(int threads)
{
    if (threads > 0)
        return threads;
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* samples [a, b) of the signal into dst (dst[0] is sample a); energy sum */
static double fill_range(const fill_ctx *F, uint64_t a, uint64_t b, float *dst)
{
    double e = 0.0;
    uint64_t g = a;
    if ((g & 1) && g < b) {
        e += fill_one(F, g, dst);
        ++g;
    }
    for (; g + SG_BLK <= b; g += SG_BLK)
        e += F->block(F, g, dst + 2 * (g - a));
    for (; g < b; ++g)
        e += fill_one(F, g, dst + 2 * (g - a));
    return e;
}

/*
 * Sample g (global index, counted from the start of the signal):
 *   noise:  Box-Muller on the two words of its draw: sigma * sqrt(-2 ln u1)
 *           * (cos 2 pi u2, sin 2 pi u2), u = (word + 1/2) / 2^32;
 *   tones:  sum_t (A_t e^{i phi_t}) * e^{2 pi i j_t / N},
 *           j_t = (bin_t * (g mod N)) mod N  (exact integers);
 *   chirp:  chirp_amp * e^{i pi c / N}, c = (n*n) mod 2N, n = g mod N.
 * All terms in double, summed, rounded once to float.
 * dst receives 2*count floats (interleaved re, im).
 */
int sg_fill(const sg_signal *s, uint64_t first, uint64_t count, float *dst,
            int threads)
{
    if (!s || !dst)
        return -1;
    threads = default_threads(threads);
    fill_ctx F;
    int rc = ctx_init(&F, s, threads);
    if (rc != 0) {
        ctx_free(&F);
        return rc;
    }
    /* contiguous spans of whole blocks per thread, aligned to the global
     * block grid so every thread but the edges takes the vector path */
    const uint64_t span = 64 * SG_BLK;
    const uint64_t a0 = first, b0 = first + count;
    const uint64_t base = a0 / span * span;
    const long long n_span = (long long)((b0 + span - 1 - base) / span);
#pragma omp parallel for num_threads(threads) schedule(dynamic, 4)
    for (long long i = 0; i < n_span; ++i) {
        uint64_t a = base + (uint64_t)i * span, b = a + span;
        if (a < a0)
            a = a0;
        if (b > b0)
            b = b0;
        if (a < b)
            (void)fill_range(&F, a, b, dst + 2 * (a - a0));
    }
    ctx_free(&F);
    return 0;
}

/*
 * Segments first_seg .. first_seg + n_seg - 1 of length s->seg_len into
 * dst, and each segment's energy sum |x|^2 of the stored floats (FP64)
 * into energy[0 .. n_seg - 1] when energy is not NULL.
 */
int sg_fill_segments(const sg_signal *s, uint64_t first_seg, uint64_t n_seg,
                     float *dst, double *energy, int threads)
{
    if (!s || !dst || s->seg_len == 0)
        return -1;
    threads = default_threads(threads);
    fill_ctx F;
    int rc = ctx_init(&F, s, threads);
    if (rc != 0) {
        ctx_free(&F);
        return rc;
    }
    const uint64_t n = s->seg_len;
    /* a segment is split into parts when there are too few segments to
     * keep every thread busy; parts are summed in a fixed order */
    uint64_t parts = 1;
    while (n_seg * parts < 4 * (uint64_t)threads && n / (parts * 2) >= 4 * SG_BLK)
        parts *= 2;
    const uint64_t plen = (n + parts - 1) / parts;
    double *pe = (double *)malloc((size_t)(n_seg * parts) * sizeof(double));
    if (!pe) {
        ctx_free(&F);
        return -2;
    }
    const long long tasks = (long long)(n_seg * parts);
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
    for (long long t = 0; t < tasks; ++t) {
        const uint64_t sgi = (uint64_t)t / parts, part = (uint64_t)t % parts;
        uint64_t a = part * plen, b = a + plen;
        if (b > n)
            b = n;
        const uint64_t g0 = (first_seg + sgi) * n;
        pe[t] = a < b ? fill_range(&F, g0 + a, g0 + b, dst + 2 * (sgi * n + a)) : 0.0;
    }
    if (energy)
        for (uint64_t i = 0; i < n_seg; ++i) {
            double e = 0.0;
            for (uint64_t p = 0; p < parts; ++p)
                e += pe[i * parts + p];
            energy[i] = e;
        }
    free(pe);
    ctx_free(&F);
    return 0;
}

typedef double (*energy_fn)(const float *, uint64_t);

static double energy_base(const float *x, uint64_t n8) { return energy_body(x, n8); }
#ifdef SG_X86_DISPATCH
SG_T512 static double energy_512(const float *x, uint64_t n8) { return energy_body(x, n8); }
SG_T256 static double energy_256(const float *x, uint64_t n8) { return energy_body(x, n8); }
#endif

static energy_fn pick_energy(void)
{
#ifdef SG_X86_DISPATCH
    switch (isa_level()) {
    case 2:
        return energy_512;
    case 1:
        return energy_256;
    }
#endif
    return energy_base;
}

int sg_energy(const float *x, uint64_t n_seg, uint64_t seg_len, double *out,
              int threads)
{
    if ((!x || !out) && n_seg)
        return -1;
    threads = default_threads(threads);
    uint64_t parts = 1;
    while (n_seg * parts < 4 * (uint64_t)threads && seg_len / (parts * 2) >= 4096)
        parts *= 2;
    const uint64_t plen = (seg_len + parts - 1) / parts;
    const energy_fn energy_span = pick_energy();
    double *pe = (double *)malloc((size_t)(n_seg * parts + 1) * sizeof(double));
    if (!pe)
        return -2;
    const long long tasks = (long long)(n_seg * parts);
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
    for (long long t = 0; t < tasks; ++t) {
        const uint64_t sgi = (uint64_t)t / parts, part = (uint64_t)t % parts;
        uint64_t a = part * plen, b = a + plen;
        if (b > seg_len)
            b = seg_len;
        double e = 0.0;
        if (a < b) {
            const float *p = x + 2 * (sgi * seg_len + a);
            const uint64_t n8 = (b - a) / 8;
            e = energy_span(p, n8);
            for (uint64_t i = 8 * n8; i < b - a; ++i)
                e = fma((double)p[2 * i], (double)p[2 * i],
                        fma((double)p[2 * i + 1], (double)p[2 * i + 1], e));
        }
        pe[t] = e;
    }
    for (uint64_t i = 0; i < n_seg; ++i) {
        double e = 0.0;
        for (uint64_t p = 0; p < parts; ++p)
            e += pe[i * parts + p];
        out[i] = e;
    }
    free(pe);
    return 0;
}

/* count uniform doubles in (0,1), 53-bit, draw index first..first+count-1. */
int sg_uniform(uint64_t seed, uint32_t stream, uint64_t first, uint64_t count,
               double *out)
{
    if (!out)
        return -1;
    for (uint64_t i = 0; i < count; ++i) {
        uint32_t r[4];
        draw(seed, stream, SG_PURPOSE_UNIFORM, first + i, r);
        out[i] = u53_open(r[0], r[1]);
    }
    return 0;
}

/* count standard normal doubles (Box-Muller on 53-bit uniforms). */
int sg_normal(uint64_t seed, uint32_t stream, uint64_t first, uint64_t count,
              double *out)
{
    if (!out)
        return -1;
    for (uint64_t i = 0; i < count; ++i) {
        uint32_t r[4];
        draw(seed, stream, SG_PURPOSE_NORMAL, first + i, r);
        double u1 = u53_open(r[0], r[1]);
        /* 2 pi u2 = (pi/2) (2m + 1) / 2^52 for u2 = (m + 1/2) / 2^53 */
        uint64_t m = ((uint64_t)(r[2] >> 5) << 26) | (uint64_t)(r[3] >> 6);
        double c, s;
        sg_quarter_ratio(2 * m + 1, 1ull << 52, &c, &s);
        out[i] = sqrt(-2.0 * sg_ln(u1)) * c;
    }
    return 0;
}

/* Cap the instruction-set version used by later calls (0 baseline, 1 AVX2,
 * 2 AVX-512; not thread-safe against running fills); returns the version
 * that is then in use. */
int sg_set_isa(int cap)
{
    g_isa_cap = cap < 0 ? 0 : cap > 2 ? 2 : cap;
    return isa_level();
}

/* ln and (cos, sin)(2 pi num / den) as the generator computes them, for
 * the tests that hold them against libm */
double sg_test_ln(double x) { return sg_ln(x); }

void sg_test_turn(uint64_t num, uint64_t den, double out[2])
{
    sg_quarter_ratio(4 * num, den, &out[0], &out[1]);
}

/*
 * Producer and consumer callbacks for streamed chunks: chunk c of
 * chunk_samples samples starts at global sample first_sample + c *
 * chunk_samples.  The signatures match (user, chunk, buffer, bytes)
 * callbacks.  With check_seg_len set (chunks hold whole segments of that
 * length), the producer records each segment's input energy and the
 * consumer each segment's output energy, for a Parseval check of every
 * segment, and the consumer keeps a copy of the first and last segment of
 * every chunk (saved_out: 2 segments per chunk) for spot checks.  A
 * streaming library may call the consumer on another thread while the
 * producer fills later chunks: the two write disjoint parts of the arrays,
 * and drain_threads keeps the consumer's memory-bound sums from taking
 * every core from the producer.
 */
typedef struct {
    sg_signal sig;
    uint64_t first_sample;
    uint64_t chunk_samples;
    int threads;
    uint64_t check_seg_len;
    uint64_t n_chunks;        /* bound on chunk indices for the arrays  */
    double *energy_in;        /* [n_chunks * segs per chunk] or NULL    */
    double *energy_out;       /* [n_chunks * segs per chunk] or NULL    */
    float *saved_out;         /* [n_chunks * 2 * check_seg_len * 2] or NULL */
    int drain_threads;        /* threads of the consumer's sums (<= 0: threads) */
} sg_chunk_source;

int sg_fill_chunk(void *user, uint64_t chunk, void *dst, uint64_t bytes)
{
    const sg_chunk_source *src = (const sg_chunk_source *)user;
    if (!src || bytes != src->chunk_samples * 8ull)
        return -1;
    const uint64_t first = src->first_sample + chunk * src->chunk_samples;
    const uint64_t L = src->check_seg_len;
    if (L && src->energy_in) {
        if (chunk >= src->n_chunks || src->chunk_samples % L || first % L ||
            src->sig.seg_len != L)
            return -1;
        const uint64_t spc = src->chunk_samples / L;
        return sg_fill_segments(&src->sig, first / L, spc, (float *)dst,
                                src->energy_in + chunk * spc, src->threads);
    }
    return sg_fill(&src->sig, first, src->chunk_samples, (float *)dst, src->threads);
}

int sg_drain_chunk(void *user, uint64_t chunk, const void *src_buf, uint64_t bytes)
{
    const sg_chunk_source *src = (const sg_chunk_source *)user;
    if (!src || bytes != src->chunk_samples * 8ull)
        return -1;
    const uint64_t L = src->check_seg_len;
    if (!L)
        return 0;
    if (chunk >= src->n_chunks || src->chunk_samples % L)
        return -1;
    const uint64_t spc = src->chunk_samples / L;
    const float *y = (const float *)src_buf;
    if (src->energy_out &&
        sg_energy(y, spc, L, src->energy_out + chunk * spc,
                  src->drain_threads > 0 ? src->drain_threads : src->threads) != 0)
        return -2;
    if (src->saved_out) {
        float *keep = src->saved_out + chunk * 2 * L * 2;
        memcpy(keep, y, L * 8);
        memcpy(keep + 2 * L, y + 2 * (spc - 1) * L, L * 8);
    }
    return 0;
}
