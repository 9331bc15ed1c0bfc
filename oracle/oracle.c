/*
 * FP64 CPU oracle for batched 1-D complex DFTs over fixed-length segments.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the GPU library.
 *
 * What it computes (the paper, Sec. I-II: the Cooley-Tukey FFT is an exact
 * refactoring of the discrete Fourier transform, so the result the method
 * must reach is the plain DFT of every segment; Sec. III: the signal is cut
 * into consecutive fixed-length segments, each transformed on its own):
 *
 *     X_s[k] = sum_{n=0}^{N-1} x_s[n] * exp(d * 2*pi*i * n*k / N),
 *
 * d = -1 for the forward and +1 for the inverse transform, no scaling, for
 * every segment s of a row-major [batch][N] array of complex numbers stored
 * as interleaved (re, im) doubles.
 *
 * Two independent routines:
 *   orc_dft_direct     O(N^2) definition, angle index (n*k) mod N taken in
 *                      exact 64-bit integer arithmetic.
 *   orc_fft_recursive  decimation-in-time Cooley-Tukey: N = p*m with p the
 *                      smallest of {2,3,5} dividing N; the p sub-sequences
 *                      x[q + p*t] are transformed recursively and combined as
 *                      X[k] = sum_q W_N^{(q*k) mod N} * Y_q[k mod m].
 *                      A length with no factor in {2,3,5} (a prime > 5) is
 *                      done by the direct definition.
 *
 * Twiddles: W_n^j = exp(d*2*pi*i*j/n) evaluated with libm cos/sin in double
 * from the exact integer j.  Within one call every sub-length n' divides the
 * top length N, so W_{n'}^j is read as W_N^{j*N/n'} from one table of N
 * entries built once per call (same value, exact integer index).
 *
 * Segments are independent; OpenMP spreads them over host threads.
 * Built with gcc -O2, no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double re, im;
} cplx;

/* Errors returned to the caller (never abort). */
#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

static const double TWO_PI = 6.283185307179586476925286766559;

/* Table w[j] = exp(d*2*pi*i*j/n), j in [0, n). */
static cplx *root_table(uint64_t n, int d)
{
    cplx *w = (cplx *)malloc((size_t)n * sizeof(cplx));
    if (!w)
        return NULL;
    for (uint64_t j = 0; j < n; ++j) {
        double a = TWO_PI * (double)j / (double)n;
        w[j].re = cos(a);
        w[j].im = (double)d * sin(a);
    }
    return w;
}

static inline cplx cmul(cplx a, cplx b)
{
    cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}

/* ------------------------------------------------------------------ */
/* Direct O(N^2) DFT of one segment read with element stride `is`.      */
/* w is the table of the top length `ntop`; this length n divides ntop. */
static void dft_one(const cplx *x, uint64_t is, uint64_t n, cplx *X,
                    const cplx *w, uint64_t ntop)
{
    uint64_t scale = ntop / n;
    for (uint64_t k = 0; k < n; ++k) {
        double re = 0.0, im = 0.0;
        for (uint64_t t = 0; t < n; ++t) {
            cplx tw = w[((t * k) % n) * scale];
            cplx xv = x[t * is];
            re += xv.re * tw.re - xv.im * tw.im;
            im += xv.re * tw.im + xv.im * tw.re;
        }
        X[k].re = re;
        X[k].im = im;
    }
}

int orc_dft_direct(const double *in, double *out, uint64_t batch, uint64_t n,
                   int dir)
{
    if (n == 0 || (dir != 1 && dir != -1) || !in || !out || in == out)
        return ORC_EINVAL;
    if (n > (1ull << 26))
        return ORC_EINVAL; /* (n-1)^2 must fit in 64 bits with room */
    cplx *w = root_table(n, dir);
    if (!w)
        return ORC_ENOMEM;
    const cplx *x = (const cplx *)in;
    cplx *X = (cplx *)out;
    long long b = (long long)batch;
#pragma omp parallel for schedule(dynamic, 1)
    for (long long s = 0; s < b; ++s)
        dft_one(x + (uint64_t)s * n, 1, n, X + (uint64_t)s * n, w, n);
    free(w);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
static uint64_t smallest_factor_235(uint64_t n)
{
    if (n % 2 == 0)
        return 2;
    if (n % 3 == 0)
        return 3;
    if (n % 5 == 0)
        return 5;
    return 0;
}

/*
 * Recursive decimation-in-time FFT of x (stride is, length n) into X
 * (contiguous).  work holds at least 2*n entries: the first n receive the
 * p sub-transforms Y_q (Y_q at work + q*m), the rest is scratch for the
 * recursion one level down (which needs 2*m <= n entries).
 */
static void fft_rec(const cplx *x, uint64_t is, uint64_t n, cplx *X,
                    cplx *work, const cplx *w, uint64_t ntop)
{
    if (n == 1) {
        X[0] = x[0];
        return;
    }
    uint64_t p = smallest_factor_235(n);
    if (p == 0) {
        dft_one(x, is, n, X, w, ntop);
        return;
    }
    uint64_t m = n / p;
    cplx *Y = work;
    for (uint64_t q = 0; q < p; ++q)
        fft_rec(x + q * is, is * p, m, Y + q * m, work + n, w, ntop);
    uint64_t scale = ntop / n; /* W_n^j = W_ntop^{j*scale} */
    for (uint64_t k = 0; k < n; ++k) {
        cplx acc = {0.0, 0.0};
        uint64_t km = k % m;
        for (uint64_t q = 0; q < p; ++q) {
            cplx t = cmul(w[((q * k) % n) * scale], Y[q * m + km]);
            acc.re += t.re;
            acc.im += t.im;
        }
        X[k] = acc;
    }
}

int orc_fft_recursive(const double *in, double *out, uint64_t batch,
                      uint64_t n, int dir)
{
    if (n == 0 || (dir != 1 && dir != -1) || !in || !out || in == out)
        return ORC_EINVAL;
    if (n > (1ull << 26))
        return ORC_EINVAL;
    cplx *w = root_table(n, dir);
    if (!w)
        return ORC_ENOMEM;
    const cplx *x = (const cplx *)in;
    cplx *X = (cplx *)out;
    long long b = (long long)batch;
    int err = 0;
#pragma omp parallel
    {
        cplx *work = (cplx *)malloc(2 * (size_t)n * sizeof(cplx));
        if (!work) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (long long s = 0; s < b; ++s)
            if (work)
                fft_rec(x + (uint64_t)s * n, 1, n, X + (uint64_t)s * n, work,
                        w, n);
        free(work);
    }
    free(w);
    return err ? ORC_ENOMEM : ORC_OK;
}

/* Threads an OpenMP parallel region of this library would use. */
int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
