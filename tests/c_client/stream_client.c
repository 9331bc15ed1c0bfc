/*
 * A C client of libfftseg's streaming entry points (no Python, no torch, no
 * OpenMP): a pool of pinned host chunks from fft_host_alloc is streamed
 * through the pipeline (host-to-device copy, transform, device-to-host copy
 * on three streams), the per-chunk timeline is printed, and everything the
 * program created is released before main returns.
 *
 * Each segment is an impulse at sample 0 scaled by the segment's global
 * index (x_s[n] = (s + 1) * [n == 0]), whose spectrum is the constant
 * s + 1 at every bin (the DFT of an impulse); the program checks the first
 * and last segment of every chunk against that and exits non-zero on a
 * mismatch or a library error.
 *
 * usage: stream_client <segment_len> <segments_per_chunk> <chunks> <pool>
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "fftseg.h"

static int check_segment(const float *y, size_t n, double want)
{
    for (size_t k = 0; k < n; ++k) {
        const double re = y[2 * k], im = y[2 * k + 1];
        if (re < want * (1 - 1e-6) || re > want * (1 + 1e-6) || im < -1e-3 || im > 1e-3)
            return -1;
    }
    return 0;
}

int main(int argc, char **argv)
{
    if (argc != 5) {
        fprintf(stderr, "usage: %s segment_len segments_per_chunk chunks pool\n", argv[0]);
        return 2;
    }
    const size_t n = strtoull(argv[1], NULL, 10), b = strtoull(argv[2], NULL, 10);
    const uint64_t chunks = strtoull(argv[3], NULL, 10);
    const int pool = atoi(argv[4]);
    if (!n || !b || !chunks || pool < 1 || pool > 16 || (uint64_t)pool > chunks) {
        fprintf(stderr, "bad arguments\n");
        return 2;
    }
    const size_t bytes = n * b * 8;
    int rc = 1;
    void *in[16] = {0}, *out[16] = {0};
    fft_chunk_times_t *tl = NULL;
    fft_plan_t plan = fft_plan_create(n, b, FFT_FORWARD);
    if (!plan) {
        fprintf(stderr, "plan: %s\n", fft_last_error());
        return 1;
    }
    for (int i = 0; i < pool; ++i) {
        in[i] = fft_host_alloc(bytes);
        out[i] = fft_host_alloc(bytes);
        if (!in[i] || !out[i]) {
            fprintf(stderr, "pinned: %s\n", fft_last_error());
            goto done;
        }
        /* chunk i of the pool: segment s of the signal is (s + 1) * impulse */
        memset(in[i], 0, bytes);
        for (size_t s = 0; s < b; ++s)
            ((float *)in[i])[2 * s * n] = (float)((uint64_t)i * b + s + 1);
    }
    fft_stream_stats_t st;
    if (fft_exec_stream_pinned(plan, chunks, in, pool, out, pool, 3, &st) != FFT_OK) {
        fprintf(stderr, "stream: %s\n", fft_last_error());
        goto done;
    }
    /* chunk c read pool slot c % pool; the last round of the pool holds the
     * spectra of chunks chunks - pool .. chunks - 1 */
    for (int i = 0; i < pool; ++i)
        for (size_t s = 0; s < b; s += b - 1) {
            const double want = (double)((uint64_t)i * b + s + 1);
            if (check_segment((const float *)out[i] + 2 * s * n, n, want) != 0) {
                fprintf(stderr, "spectrum mismatch: pool slot %d segment %zu\n", i, s);
                goto done;
            }
            if (b == 1)
                break;
        }
    const int k = fft_stream_last_timeline(plan, NULL, 0);
    if (k < 0 || !(tl = (fft_chunk_times_t *)calloc((size_t)k + 1, sizeof(*tl))) ||
        fft_stream_last_timeline(plan, tl, (size_t)k) != k) {
        fprintf(stderr, "timeline: %s\n", fft_last_error());
        goto done;
    }
    printf("{\"segment_len\": %zu, \"segments_per_chunk\": %zu, \"chunks\": %llu, "
           "\"wall_s\": %.4f, \"host_link_GBps_each_way\": %.2f, \"timeline_ms\": [",
           n, b, (unsigned long long)chunks, st.wall_s,
           st.bytes_h2d / st.wall_s / 1e9);
    for (int i = 0; i < k; ++i)
        printf("%s[%llu, %.3f, %.3f, %.3f, %.3f, %.3f, %.3f]", i ? ", " : "",
               (unsigned long long)tl[i].chunk, tl[i].h2d_start_ms, tl[i].h2d_end_ms,
               tl[i].compute_start_ms, tl[i].compute_end_ms, tl[i].d2h_start_ms,
               tl[i].d2h_end_ms);
    printf("]}\n");
    rc = 0;
done:
    free(tl);
    for (int i = 0; i < pool; ++i) {
        fft_host_free(in[i]);
        fft_host_free(out[i]);
    }
    fft_plan_destroy(plan);
    return rc;
}
