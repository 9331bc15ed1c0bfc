/*
 * Seeded synthetic signal generator.
 *
 * Serves both the FP64 oracle's tests and the GPU library's tests and
 * benchmark, and holds none of the transform's arithmetic: it only draws
 * random numbers and synthesises test signals (noise, tones, a chirp).
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
 * uniform draws and normal draws.
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

static const double SG_TWO_PI = 6.283185307179586476925286766559;
static const double SG_PI = 3.1415926535897932384626433832795;

void sg_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                      uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
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

/* (0,1) from 32 bits: never 0, never 1. */
static inline double u32_open(uint32_t x)
{
    return ((double)x + 0.5) * (1.0 / 4294967296.0);
}

/* (0,1) with 53 bits from two words. */
static inline double u53_open(uint32_t a, uint32_t b)
{
    uint64_t m = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return ((double)m + 0.5) * (1.0 / 9007199254740992.0);
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

/*
 * Sample g (global index, counted from the start of the signal):
 *   noise:  Box-Muller on two Philox words, sigma * sqrt(-2 ln u1) *
 *           (cos 2 pi u2, sin 2 pi u2);
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
    uint64_t n = s->seg_len;
    int need_tab = (s->n_tones > 0 || s->chirp_amp != 0.0);
    if (need_tab && (n == 0 || n > (1ull << 30)))
        return -1;
    double *root = NULL, *chirp = NULL, *tone_c = NULL;
    if (s->n_tones > 0) {
        root = (double *)malloc(2 * (size_t)n * sizeof(double));
        tone_c = (double *)malloc(2 * (size_t)s->n_tones * sizeof(double));
        if (!root || !tone_c)
            goto oom;
        for (uint32_t t = 0; t < s->n_tones; ++t) {
            if (s->tone_bin[t] < 0 || (uint64_t)s->tone_bin[t] >= n)
                goto bad;
            tone_c[2 * t] = s->tone_amp[t] * cos(s->tone_phase[t]);
            tone_c[2 * t + 1] = s->tone_amp[t] * sin(s->tone_phase[t]);
        }
    }
    if (s->chirp_amp != 0.0) {
        chirp = (double *)malloc(4 * (size_t)n * sizeof(double));
        if (!chirp)
            goto oom;
    }
    if (threads <= 0) {
#ifdef _OPENMP
        threads = omp_get_max_threads();
#else
        threads = 1;
#endif
    }
    if (root) {
        long long nn = (long long)n;
#pragma omp parallel for num_threads(threads) schedule(static)
        for (long long j = 0; j < nn; ++j) {
            double a = SG_TWO_PI * (double)j / (double)n;
            root[2 * j] = cos(a);
            root[2 * j + 1] = sin(a);
        }
    }
    if (chirp) {
        long long n2 = 2 * (long long)n;
#pragma omp parallel for num_threads(threads) schedule(static)
        for (long long j = 0; j < n2; ++j) {
            double a = SG_PI * (double)j / (double)n;
            chirp[2 * j] = s->chirp_amp * cos(a);
            chirp[2 * j + 1] = s->chirp_amp * sin(a);
        }
    }
    {
        long long cnt = (long long)count;
        const double sigma = s->sigma;
#pragma omp parallel for num_threads(threads) schedule(static, 65536)
        for (long long i = 0; i < cnt; ++i) {
            uint64_t g = first + (uint64_t)i;
            double re = 0.0, im = 0.0;
            if (sigma != 0.0) {
                uint32_t r[4];
                draw(s->seed, s->stream, SG_PURPOSE_NOISE, g, r);
                double rad = sigma * sqrt(-2.0 * log(u32_open(r[0])));
                double a = SG_TWO_PI * u32_open(r[1]);
                re = rad * cos(a);
                im = rad * sin(a);
            }
            if (need_tab) {
                uint64_t ph = g % n;
                for (uint32_t t = 0; t < s->n_tones; ++t) {
                    uint64_t j = ((uint64_t)s->tone_bin[t] * ph) % n;
                    double cr = root[2 * j], ci = root[2 * j + 1];
                    double ar = tone_c[2 * t], ai = tone_c[2 * t + 1];
                    re += ar * cr - ai * ci;
                    im += ar * ci + ai * cr;
                }
                if (chirp) {
                    uint64_t c = (ph * ph) % (2 * n);
                    re += chirp[2 * c];
                    im += chirp[2 * c + 1];
                }
            }
            dst[2 * i] = (float)re;
            dst[2 * i + 1] = (float)im;
        }
    }
    free(root);
    free(chirp);
    free(tone_c);
    return 0;
bad:
    free(root);
    free(chirp);
    free(tone_c);
    return -1;
oom:
    free(root);
    free(chirp);
    free(tone_c);
    return -2;
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
        double u2 = u53_open(r[2], r[3]);
        out[i] = sqrt(-2.0 * log(u1)) * cos(SG_TWO_PI * u2);
    }
    return 0;
}

/*
 * Fill-callback adapter for streamed chunks: chunk c of chunk_samples
 * samples starts at global sample first_sample + c * chunk_samples.  The
 * signature matches a (user, chunk, dst, bytes) producer callback.
 */
typedef struct {
    sg_signal sig;
    uint64_t first_sample;
    uint64_t chunk_samples;
    int threads;
} sg_chunk_source;

int sg_fill_chunk(void *user, uint64_t chunk, void *dst, uint64_t bytes)
{
    const sg_chunk_source *src = (const sg_chunk_source *)user;
    if (!src || bytes != src->chunk_samples * 8ull)
        return -1;
    return sg_fill(&src->sig, src->first_sample + chunk * src->chunk_samples,
                   src->chunk_samples, (float *)dst, src->threads);
}
