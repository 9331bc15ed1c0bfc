/*
 * fftseg -- batched 1-D complex FFTs over the fixed-length segments of a
 * long signal, on one AMD Instinct MI355X (gfx950).
 *
 * The method (Tsiomenko & Rees, "Accelerating Fast Fourier Transforms Using
 * Hadoop and CUDA", arXiv:1407.6915):
 *   Sec. III   a very large signal is cut into consecutive fixed-length FFT
 *              segments, each an <offset, FFT segment> record whose offset
 *              is the byte offset from the start of the signal; a whole block
 *              of such segments moves to the GPU in one allocate+copy pair
 *              and one batched plan transforms every segment of the block;
 *              the transform may run in place; outputs are kept in the
 *              order (position) of their inputs.
 *   Sec. I-II  the transform is the Cooley-Tukey FFT, i.e. exactly the DFT
 *                 X_s[k] = sum_{n<N} x_s[n] exp(d 2 pi i n k / N),
 *              d = -1 forward, +1 inverse, no normalisation.
 *   Sec. II, III  data larger than device memory is moved between host and
 *              device in few, large transfers (streaming entry point below).
 *
 * Data layout: a batch is `batch` consecutive segments of `segment_len`
 * complex64 samples (interleaved float32 re, im; 8 bytes per sample), row
 * major [batch][segment_len].  The record at byte offset s*segment_len*8 of
 * the input yields its spectrum at the same byte offset of the output, in
 * natural frequency order k = 0..segment_len-1.
 *
 * Conventions shared by every entry point:
 *  - Pointers named in/out/base are DEVICE pointers (hipMalloc'd memory or
 *    a sub-range of it) and stay owned by the caller; they must stay valid
 *    until the work enqueued on `stream` has run.  They must be 8-byte
 *    aligned; 16-byte alignment is not required.
 *  - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *    Exec calls only enqueue work and return.
 *  - Every call returns an fft_status_t (or NULL for constructors) and never
 *    aborts.  On failure fft_last_status()/fft_last_error() of the calling
 *    thread hold the status and a message (with hipGetErrorString text for
 *    FFT_ERR_HIP).  All argument checks happen before any device work.
 *  - Supported lengths: 1 <= segment_len <= 2^24 whose prime factors are
 *    2, 3 and 5.  Other lengths give FFT_ERR_UNSUPPORTED_LENGTH.
 *  - A plan may be used from one thread at a time and has at most one exec
 *    in flight (long-segment plans own a scratch buffer); create one plan
 *    per concurrent stream.
 */
#ifndef FFTSEG_H
#define FFTSEG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FFT_FORWARD (-1) /* exp(-2 pi i n k / N) */
#define FFT_INVERSE (+1) /* exp(+2 pi i n k / N), unnormalised */

typedef enum {
    FFT_OK = 0,
    FFT_ERR_INVALID_ARG = -1,        /* zero/overflowing size, bad direction, NULL */
    FFT_ERR_UNSUPPORTED_LENGTH = -2, /* prime factor > 5, or length > 2^24     */
    FFT_ERR_OUT_OF_MEMORY = -3,      /* device or pinned allocation failed      */
    FFT_ERR_ALIGNMENT = -4,          /* pointer not 8-byte aligned              */
    FFT_ERR_OVERLAP = -5,            /* in and out partially overlap            */
    FFT_ERR_HIP = -6,                /* a HIP runtime call failed               */
    FFT_ERR_CALLBACK = -7,           /* a user fill/drain callback failed       */
    FFT_ERR_BOUNDS = -8,             /* buffer smaller than the work needs      */
    FFT_ERR_TIMEOUT = -9             /* a bounded device wait gave up           */
} fft_status_t;

typedef struct fftseg_plan *fft_plan_t;

/* ------------------------------------------------------------------------
 * Plain batched path (Sec. III: one batched plan over a block of segments).
 * ------------------------------------------------------------------------ */

/* Build a plan for `batch` segments of `segment_len` samples in direction
 * FFT_FORWARD or FFT_INVERSE.  Factorises the length, picks the kernel (one
 * LDS-resident pass up to 16384 samples, a two-pass "four-step" split
 * N = N1*N2 above, a radix-by-radix fallback otherwise; a tuned choice
 * first, and for a batch that would give the length's default one-pass
 * kernel fewer than two workgroups per CU, the length's small-batch
 * kernel where it has one), uploads the
 * twiddle tables (evaluated in FP64, rounded once to float32) and allocates
 * the scratch of two-pass plans.  Returns NULL on error.  Validation:
 * segment_len == 0, batch == 0, batch*segment_len*8 overflowing size_t or
 * direction not +-1 -> FFT_ERR_INVALID_ARG; unsupported length ->
 * FFT_ERR_UNSUPPORTED_LENGTH. */
fft_plan_t fft_plan_create(size_t segment_len, size_t batch, int direction);

/* Plan for real-input segments (the float32 samples of Sec. III, 4 bytes
 * each).  segment_len = N must be even, at least 4, and a supported length
 * (prime factors 2, 3, 5; at most 2^24); otherwise
 * FFT_ERR_UNSUPPORTED_LENGTH.  Executed by fft_exec_segments /
 * fft_exec_segments_n, always out of place (in and out must not overlap,
 * else FFT_ERR_OVERLAP):
 *   FFT_FORWARD  in:  batch x N float32 (row s at byte offset s*N*4)
 *                out: batch x (N/2+1) complex64, bins k = 0..N/2 of
 *                     X_s[k] = sum_n x_s[n] exp(-2 pi i n k / N)
 *                     (row s at byte offset s*(N/2+1)*8)
 *   FFT_INVERSE  in:  batch x (N/2+1) complex64 bins 0..N/2
 *                out: batch x N float32,
 *                     x_s[n] = sum_{k<N} X_s[k] exp(+2 pi i n k / N)
 *                     with X_s[N-k] = conj X_s[k], unnormalised; the
 *                     imaginary parts of bins 0 and N/2 are ignored.
 * Both buffers must be 8-byte aligned.  The N reals are transformed as
 * N/2 complex values z[m] = x[2m] + i x[2m+1].  Where N/2 has a one-pass
 * kernel the split into even and odd parts is fused into its store
 * (forward) or load (inverse), so each byte crosses HBM once.  Other even
 * lengths run the N/2-point complex plan (two passes or radix stages) and
 * the split as a separate pass through a buffer of up to 2 GiB of N/2-point
 * rows (plus that plan's own scratch; fft_plan_scratch_bytes reports both).
 * Streaming, frames, graph and work-list entry points take complex plans
 * only. */
fft_plan_t fft_plan_create_real(size_t segment_len, size_t batch, int direction);

/* Transform every segment: the record at byte offset s*segment_len*8 of
 * `in` yields its spectrum at the same offset of `out`.  in == out (in
 * place) is allowed; any other overlap gives FFT_ERR_OVERLAP.  Each buffer
 * must lie inside one device allocation of at least batch*segment_len*8
 * bytes from the pointer on (else FFT_ERR_BOUNDS).  Pointers need 8-byte
 * alignment only; two-pass plans start their tiles where the buffers'
 * 128-byte lines do, so bases off a line boundary cost them little. */
int fft_exec_segments(fft_plan_t plan, const void *in, void *out, void *stream);

/* Same as fft_exec_segments for the first `batch` segments only
 * (1 <= batch <= the plan's batch). */
int fft_exec_segments_n(fft_plan_t plan, const void *in, void *out,
                        size_t batch, void *stream);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): the
 * transform of fft_exec_segments without a plan, allocating nothing.
 * `batch` segments of `segment_len` samples in direction FFT_FORWARD or
 * FFT_INVERSE go from `in` to `out` (same layout, aliasing, alignment and
 * bounds rules and the same kernels as a plan's).  The twiddle tables are
 * computed on the device by each call, and the buffer between the two
 * passes of long segments is used in sub-batches; both live in one static
 * device array of the library, 2^15 + 2^24 + 32 complex64 samples (about
 * 128 MiB) per GPU, allocated when the library's code first runs on that
 * GPU and held until the process ends.  Supported: every length of
 * fft_plan_create up to 2^23 (lengths without a two-pass split need two
 * buffers of N samples); 2^24 gives FFT_ERR_UNSUPPORTED_LENGTH.  Every call
 * on one GPU uses the same array: calls that overlap in time on one GPU
 * (other streams, other threads) race and give wrong results.  Asynchronous
 * on stream. */
int fft_exec_segments_noalloc(size_t segment_len, size_t batch, int direction,
                              const void *in, void *out, void *stream);

/* Synchronise the plan's last stream, then free the plan.  NULL is a no-op. */
int fft_plan_destroy(fft_plan_t plan);

/* Status and message of the calling thread's most recent call (FFT_OK and
 * an empty message after a success). */
int fft_last_status(void);
const char *fft_last_error(void);

/* ------------------------------------------------------------------------
 * Introspection (host only, no device work).
 * ------------------------------------------------------------------------ */

/* Factorise n into the radices the planner would use for one pass of up to
 * 16384 samples (or for the fallback path).  Writes up to `max` radices to
 * `radices` and returns their count, or a negative fft_status_t. */
int fft_plan_factorize(size_t n, int *radices, int max);

/* Describe the plan as a JSON object (kind, kernels, radices, split,
 * threads, LDS bytes, scratch bytes; for two-pass plans also the sub-batch
 * and whether the intermediate array is kept in blocks of 16 columns,
 * "y_blocked") into buf (NUL terminated, truncated to len).  Returns the
 * full length needed, or a negative fft_status_t. */
int fft_plan_describe(fft_plan_t plan, char *buf, size_t len);

/* Bytes of device scratch the plan owns (0 for single-pass plans). */
size_t fft_plan_scratch_bytes(fft_plan_t plan);

/* ------------------------------------------------------------------------
 * Streaming of signals larger than device memory (Sec. II-III: move data
 * between host and device in few large transfers).
 * ------------------------------------------------------------------------ */

/* Producer: write chunk `chunk` (bytes = plan batch * segment_len * 8) into
 * the library's pinned host slot `dst`.  Return 0 on success.  Called from
 * the thread that called fft_exec_stream, in chunk order. */
typedef int (*fft_fill_fn)(void *user, uint64_t chunk, void *dst, uint64_t bytes);
/* Consumer: read the spectra of chunk `chunk` from pinned slot `src`.
 * Called in chunk order from a worker thread of the library, at the same
 * time as fill works on later chunks: `user` state that both touch must
 * allow that. */
typedef int (*fft_drain_fn)(void *user, uint64_t chunk, const void *src,
                            uint64_t bytes);

typedef struct {
    double wall_s;          /* whole call                                  */
    double fill_s;          /* time inside fill callbacks                  */
    double drain_s;         /* time inside drain callbacks                 */
    double h2d_s;           /* sum of host->device copy durations          */
    double d2h_s;           /* sum of device->host copy durations          */
    double compute_s;       /* sum of transform durations                  */
    uint64_t bytes_h2d;
    uint64_t bytes_d2h;
    uint64_t chunks_done;   /* chunks fully drained                        */
} fft_stream_stats_t;

/* Transform n_chunks chunks of `batch` segments each (the plan's batch):
 * chunk c is the signal's samples [c*batch*N, (c+1)*batch*N).  Pinned host
 * ring of `n_slots` (>= 2) slots per direction; host->device copies run on
 * one side stream, transforms on another, device->host copies on a third,
 * ordered by events, so copies of chunk c+1 and c-1 overlap the transform
 * of chunk c.  If a callback fails, the call stops, returns
 * FFT_ERR_CALLBACK and stores the failing chunk index in *failed_chunk
 * (chunks below it were fully drained: a caller may resume from there).
 * drain may be NULL (results discarded).  stats may be NULL. */
int fft_exec_stream(fft_plan_t plan, uint64_t n_chunks, fft_fill_fn fill,
                    fft_drain_fn drain, void *user, int n_slots,
                    uint64_t *failed_chunk, fft_stream_stats_t *stats);

/* Same pipeline with caller-owned pinned buffers: chunk c is read from
 * host_in[c % n_in] and its spectra written to host_out[c % n_out]; each
 * must hold batch*segment_len*8 bytes of hipHostMalloc'd memory. */
int fft_exec_stream_pinned(fft_plan_t plan, uint64_t n_chunks,
                           void *const *host_in, int n_in,
                           void *const *host_out, int n_out, int n_slots,
                           fft_stream_stats_t *stats);

/* Per-chunk timeline of a streamed call, on the GPU clock, in ms from the
 * start of chunk 0's host->device copy: when each chunk's copy in, its
 * transform and its copy out started and ended.  It is how the overlap of
 * copies and transforms (Sec. III's concern that host transfers dominate)
 * is measured from inside the pipeline. */
typedef struct {
    uint64_t chunk;
    float h2d_start_ms, h2d_end_ms;
    float compute_start_ms, compute_end_ms;
    float d2h_start_ms, d2h_end_ms;
} fft_chunk_times_t;

/* Copy up to `max` entries of the timeline of the plan's last
 * fft_exec_stream, fft_exec_stream_pinned or fft_exec_file call (one per
 * chunk that completed, in chunk order) into out; returns the number of
 * entries the timeline holds (0 before any streamed call).  NULL plan, or
 * NULL out with max > 0 -> FFT_ERR_INVALID_ARG. */
int fft_stream_last_timeline(fft_plan_t plan, fft_chunk_times_t *out, size_t max);

/* Pinned (page-locked) host memory for fft_exec_stream_pinned, for callers
 * with no pinned allocator of their own (Sec. III's large host transfers
 * run at the link's full rate only from pinned memory).  fft_host_alloc
 * returns NULL on failure (bytes == 0 -> FFT_ERR_INVALID_ARG, allocation
 * failure -> FFT_ERR_OUT_OF_MEMORY; fft_last_error says why).  The caller
 * owns the memory and releases it with fft_host_free before the process
 * ends: no library destructor frees it.  fft_host_free(NULL) is a no-op;
 * a pointer not from fft_host_alloc -> FFT_ERR_HIP. */
void *fft_host_alloc(size_t bytes);
int fft_host_free(void *ptr);

/* Overlapping, optionally windowed segments: a short-time transform, the
 * overlapping FFTs named as future work in Sec. VI.  Frame s
 * (0 <= s < n_frames) is
 *     x_s[j] = in[s*hop + j] * window[j],   0 <= j < segment_len,
 * (window == NULL: all ones) and its spectrum is written at
 * out + s*segment_len, natural order, same direction and scaling as
 * fft_exec_segments.  hop < segment_len overlaps consecutive frames,
 * hop == segment_len with no window is fft_exec_segments_n.
 *   in      device, in_len complex64 samples; the frames read
 *           (n_frames-1)*hop + segment_len of them (more -> FFT_ERR_BOUNDS)
 *   out     device, n_frames*segment_len complex64; must not overlap in
 *           (FFT_ERR_OVERLAP)
 *   window  device, segment_len float32 values, 4-byte aligned, or NULL
 * 1 <= n_frames <= the plan's batch and hop >= 1, else
 * FFT_ERR_INVALID_ARG.  Lengths with a one-pass kernel read the frames in
 * place (with the plan's own kernel variant when it has a frame form, else
 * the length's default frame kernel; overlapping frames are loaded through
 * the cache), two-pass lengths in their first pass; other lengths gather
 * the windowed frames into out first and transform out in place. */
int fft_exec_frames(fft_plan_t plan, const void *in, size_t in_len, void *out,
                    size_t n_frames, size_t hop, const float *window, void *stream);

/* File-backed streaming (Sec. III-IV: the signal lives in a file, the
 * outputs are kept in input order).  Chunk c (c = first_chunk ..
 * first_chunk + n_chunks - 1, each batch*segment_len*8 bytes) is read from
 * byte in_offset + c*chunk_bytes of in_path and its spectra are written at
 * byte out_offset + c*chunk_bytes of out_path (created if missing, never
 * truncated), so every record keeps its offset and no merge step is needed.
 * Reads and writes use io_threads parallel pread/pwrite calls per chunk,
 * through the pipeline of fft_exec_stream.  A file shorter than the range
 * gives FFT_ERR_BOUNDS before any device work; an I/O failure gives
 * FFT_ERR_CALLBACK with *failed_chunk = the absolute chunk index (chunks
 * below it are complete in out_path: rerun with first_chunk = that index to
 * resume). */
int fft_exec_file(fft_plan_t plan, const char *in_path, uint64_t in_offset,
                  const char *out_path, uint64_t out_offset, uint64_t first_chunk,
                  uint64_t n_chunks, int n_slots, int io_threads, uint64_t *failed_chunk,
                  fft_stream_stats_t *stats);

/* ------------------------------------------------------------------------
 * Uneven batches: a persistent kernel over a work list (Sec. III batches
 * the segments of a block into one plan; here segments of several lengths,
 * at any offsets, share one kernel).
 * ------------------------------------------------------------------------ */

typedef struct {
    uint64_t in_off;      /* sample offset (not bytes) of the segment in in_base */
    uint64_t out_off;     /* sample offset of its spectrum in out_base          */
    uint32_t segment_len; /* a length fft_worklist_supported() accepts          */
    uint32_t job;         /* caller's tag; not used by the library              */
} fft_work_t;

typedef struct fftseg_worklist *fft_worklist_t;

/* 1 if segment_len has a work-list routine (256, 1000, 1024, 1536, 4096,
 * 6000 and 16384 in one pass; 65536 in two passes; 2^20 through a
 * four-step plan the work list keeps), else 0. */
int fft_worklist_supported(uint32_t segment_len);

/* Number of indexed kernels a work list can send segments of this length
 * through: launches of their own over the segments' listed offsets,
 * instead of the work-list kernel's tiles.  One-pass lengths: the indexed
 * one-pass kernels; 65536: 1, its two passes as launches of their own; 0
 * for 16384, 2^20 and unsupported lengths.  Route 0 is the tiles, route
 * 1 + k the k-th indexed kernel; fft_autotune picks one per length,
 * untuned one-pass lengths take route 1, untuned 65536 route 0. */
int fft_worklist_indexed_count(uint32_t segment_len);

/* Compile n entries into workgroup tasks: segments are grouped by length,
 * packed S per tile for short lengths, split into column/row tiles for the
 * two-pass lengths; 16384-point segments become "wide" tiles of their own
 * launch (one 512-thread workgroup per segment).  2^20-point entries get no
 * tasks: each run of consecutive ones whose input and output offsets both
 * advance by 2^20 goes through a four-step plan of that length, which the
 * work list builds (or rebuilds, after a device-wide synchronisation) for
 * the longest run seen.  The task list, per-length twiddle tables and the
 * two-pass scratch (one Y buffer per 65536-point segment) are uploaded
 * once.  Output ranges must not overlap
 * (FFT_ERR_OVERLAP); an unsupported length gives FFT_ERR_UNSUPPORTED_LENGTH.
 * n may be 0 (an empty list to fill later with fft_worklist_reset).  All
 * entry checks run before any device work.  NULL on error. */
fft_worklist_t fft_worklist_create(const fft_work_t *items, size_t n, int direction);

/* Replace the entries of an existing work list (same rules as create),
 * keeping its twiddle tables and device arrays (grown, after a device-wide
 * synchronisation, only when too small).  The new task list is uploaded
 * from pinned staging on `stream`, so it is ordered after earlier launches
 * and before later ones on that stream.  For continuous batching: one work
 * list is re-filled with whatever segments are ready.  Entries that fail the
 * checks leave the previous ones in force; a reset that fails after them
 * (device memory for the grown arrays or the 2^20-point plan) leaves the
 * work list unable to run (FFT_ERR_INVALID_ARG from the exec calls) until a
 * reset succeeds. */
int fft_worklist_reset(fft_worklist_t wl, const fft_work_t *items, size_t n, void *stream);

/* One call per uneven batch: transform the n entries of `items` (direction
 * FFT_FORWARD or FFT_INVERSE) from in_base to out_base on `stream`, as
 * fft_worklist_create + fft_worklist_exec would, with the same entry and
 * buffer rules and errors.  The work list behind the call is kept by the
 * library, one per (device, direction, stream), and re-filled on each call
 * (fft_worklist_reset): calls on one stream are ordered by it and may
 * share that work list's device arrays and scratch; calls on different
 * streams use different ones.  `items` is read before the call returns.
 * The kept work lists hold their device memory until
 * fft_worklist_cache_clear. */
int fft_exec_worklist(const fft_work_t *items, size_t n, int direction,
                      const void *in_base, void *out_base, void *stream);

/* Synchronise the device and free the work lists kept by
 * fft_exec_worklist (a later call builds them again). */
int fft_worklist_cache_clear(void);

/* Run every entry of a work list made by fft_worklist_create: the planned
 * 2^20-point runs (their plan's two passes per run, in sub-batches), a
 * cursor-clearing kernel, then the persistent kernel
 * twice (workgroups claim tasks through an atomic cursor): first over the
 * first-pass tiles of the two-pass segments and the one-pass tiles, then
 * over the second-pass tiles, which the launch boundary orders after their
 * first passes.  The wide tiles run between the two, as a persistent
 * grid-stride launch over the 16384-point segments.  in_base and
 * out_base are device pointers; every entry's range must lie in its
 * buffer's allocation (FFT_ERR_BOUNDS).  in_base == out_base is allowed
 * when each entry's output range either equals its input range or overlaps
 * no input range (FFT_ERR_OVERLAP otherwise).  Asynchronous on stream. */
int fft_worklist_exec(fft_worklist_t wl, const void *in_base, void *out_base, void *stream);

/* Same work, launched as a hipGraph captured on first use.  The captured
 * launches hold the bases, task counts and splits, grids, device arrays and
 * planned runs as fixed arguments; the graph is captured again whenever any
 * of them differs from the capture (new bases, or a reset that changes
 * them). */
int fft_worklist_exec_graph(fft_worklist_t wl, const void *in_base, void *out_base,
                            void *stream);

/* Synchronise `stream` and report whether the last run on it completed:
 * FFT_ERR_HIP if the stream reports an error or a launch left tasks
 * unclaimed.  (No work-list kernel waits on another workgroup, so
 * FFT_ERR_TIMEOUT is not returned here.) */
int fft_worklist_status(fft_worklist_t wl, void *stream);

/* JSON summary (items, tasks, wide segments, planned runs, per-length
 * counts, scratch bytes, grids). */
int fft_worklist_describe(fft_worklist_t wl, char *buf, size_t len);

/* Synchronise the device, then free the work list.  NULL is a no-op. */
int fft_worklist_destroy(fft_worklist_t wl);

/* ------------------------------------------------------------------------
 * HIP graphs.
 * ------------------------------------------------------------------------ */

/* fft_exec_segments through a hipGraph: the plan's launch sequence for
 * (in, out) is captured on the first call and replayed afterwards
 * (re-captured when in or out change).  Same checks as fft_exec_segments. */
int fft_exec_segments_graph(fft_plan_t plan, const void *in, void *out, void *stream);

/* ------------------------------------------------------------------------
 * Autotuning and kernel variants.
 * ------------------------------------------------------------------------ */

/* Time every compiled single-pass variant of segment_len (radix order,
 * threads per segment, segments per workgroup, LDS padding, streamed or
 * cached global access) at persistent-grid sizes {0, 4, 8, 16, 32, 64}
 * resident workgroup waves per CU (two-pass lengths: every column-tile x
 * row-tile variant of the planner's split n1 x n2, columns/rows per
 * workgroup, tile order, streamed access, and the default tiles of every
 * other split n1' x n/n1' with compiled tiles, at each grid size), on
 * device buffers of batch segments it allocates and frees.  The fastest
 * choice goes into the process-wide tuning table used by later plans and,
 * if path != NULL, is merged into that JSON cache file.  For a one-pass
 * length that work lists support it also picks the work-list route (Sec.
 * III's batching of a block into one launch): the work-list kernel's tiles,
 * or a launch of its own through each indexed one-pass kernel of the length
 * at each grid size, timed on `batch` segments packed at odd offsets; work
 * lists built later use the winner.  Returns the number
 * of configurations timed (negative status on error); *best_us (may be
 * NULL) receives the winner's time per exec in microseconds. */
int fft_autotune(size_t segment_len, size_t batch, int direction, const char *path,
                 double *best_us);

/* Load a cache written by fft_autotune for this device's architecture;
 * entries naming variants or splits the library lacks are skipped.  Returns
 * the number of entries loaded. */
int fft_tune_load(const char *path);

/* Forget every tuned choice (plans use the built-in defaults again). */
int fft_tune_clear(void);

/* Number of single-pass kernel variants compiled in for length n. */
int fft_variant_count(size_t n);

/* fft_plan_create, forcing single-pass variant `variant` (0 = default). */
fft_plan_t fft_plan_create_variant(size_t segment_len, size_t batch, int direction,
                                   int variant);

/* For a two-pass length: the split N = n1 * n2 the planner uses and the
 * number of compiled column-tile and row-tile variants for it.  Returns 1,
 * or 0 if n is not a two-pass length (outputs set to 0). */
int fft_split_info(size_t n, size_t *n1, size_t *n2, int *n_column_variants,
                   int *n_row_variants);

/* fft_plan_create for a two-pass length, forcing its column-tile and
 * row-tile variants.  NULL (FFT_ERR_INVALID_ARG) if n is not two-pass or a
 * variant does not exist. */
fft_plan_t fft_plan_create_split(size_t segment_len, size_t batch, int direction,
                                 int column_variant, int row_variant);

#ifdef __cplusplus
}
#endif

#endif /* FFTSEG_H */
