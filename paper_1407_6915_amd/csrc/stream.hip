// Streaming of signals larger than device memory (fft_exec_stream*).
//
// The paper moves each block of segments to the GPU in one large transfer
// because the host link is slow next to device memory (Sec. II-III).  Here
// chunk c of `batch` segments goes host -> device on one stream, is
// transformed in place on a second and comes back on a third; events order
// the three, so the copies of chunks c+1 and c-1 overlap the transform of
// chunk c.  Host slots live in pinned memory allocated with hipHostMalloc.
#include "fftseg.h"
#include "runtime.hpp"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace fftseg {
namespace {

constexpr int kDevSlots = 3;  // device buffers: copy-in, transform, copy-out

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct ChunkEvents {
    hipEvent_t h2d0 = nullptr, h2d1 = nullptr, c0 = nullptr, c1 = nullptr,
               d2h0 = nullptr, d2h1 = nullptr;
};

struct Pipeline {
    Plan *plan = nullptr;
    uint64_t bytes = 0;
    hipStream_t s_in = nullptr, s_comp = nullptr, s_out = nullptr;
    void *dev[kDevSlots] = {nullptr, nullptr, nullptr};
    std::vector<ChunkEvents> ev;  // one set per chunk in flight ring
    int ring = 0;
    hipEvent_t ref = nullptr;     // time origin of the per-chunk timeline
    std::vector<fft_chunk_times_t> *times = nullptr;

    int init(Plan *p, int ring_len, std::vector<fft_chunk_times_t> *timeline)
    {
        plan = p;
        ring = ring_len;
        times = timeline;
        if (times)
            times->clear();
        bytes = p->batch * p->n * sizeof(c32);
        hipError_t e;
        if ((e = hipEventCreate(&ref)) != hipSuccess) {
            ref = nullptr;
            return hip_error(e, "hipEventCreate");
        }
        for (hipStream_t *s : {&s_in, &s_comp, &s_out})
            if ((e = hipStreamCreateWithFlags(s, hipStreamNonBlocking)) != hipSuccess)
                return hip_error(e, "hipStreamCreate");
        for (int i = 0; i < kDevSlots; ++i)
            if ((e = hipMalloc(&dev[i], bytes)) != hipSuccess) {
                dev[i] = nullptr;
                (void)hipGetLastError();
                return set_error(FFT_ERR_OUT_OF_MEMORY, "device chunk buffer of %llu bytes",
                                 (unsigned long long)bytes);
            }
        ev.resize(ring);
        for (auto &c : ev)
            for (hipEvent_t *q : {&c.h2d0, &c.h2d1, &c.c0, &c.c1, &c.d2h0, &c.d2h1})
                if ((e = hipEventCreate(q)) != hipSuccess)
                    return hip_error(e, "hipEventCreate");
        return FFT_OK;
    }

    ~Pipeline()
    {
        for (hipStream_t s : {s_in, s_comp, s_out})
            if (s)
                (void)hipStreamSynchronize(s);
        for (auto &c : ev)
            for (hipEvent_t q : {c.h2d0, c.h2d1, c.c0, c.c1, c.d2h0, c.d2h1})
                if (q)
                    (void)hipEventDestroy(q);
        if (ref)
            (void)hipEventDestroy(ref);
        for (void *d : dev)
            if (d)
                (void)hipFree(d);
        for (hipStream_t s : {s_in, s_comp, s_out})
            if (s)
                (void)hipStreamDestroy(s);
    }

    // enqueue chunk c: host src -> device slot -> transform -> host dst
    int issue(uint64_t c, const void *src, void *dst)
    {
        ChunkEvents &E = ev[c % ring];
        void *d = dev[c % kDevSlots];
        hipError_t e;
        if (c >= (uint64_t)kDevSlots) {
            // device slot free once the copy-out of chunk c - kDevSlots is done
            ChunkEvents &P = ev[(c - kDevSlots) % ring];
            if ((e = hipStreamWaitEvent(s_in, P.d2h1, 0)) != hipSuccess)
                return hip_error(e, "hipStreamWaitEvent");
        }
        if (c == 0)
            (void)hipEventRecord(ref, s_in);
        (void)hipEventRecord(E.h2d0, s_in);
        if ((e = hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, s_in)) != hipSuccess)
            return hip_error(e, "host-to-device copy");
        (void)hipEventRecord(E.h2d1, s_in);
        (void)hipStreamWaitEvent(s_comp, E.h2d1, 0);
        (void)hipEventRecord(E.c0, s_comp);
        int st = plan_enqueue(plan, d, d, plan->batch, s_comp);
        if (st != FFT_OK)
            return st;
        (void)hipEventRecord(E.c1, s_comp);
        (void)hipStreamWaitEvent(s_out, E.c1, 0);
        (void)hipEventRecord(E.d2h0, s_out);
        if ((e = hipMemcpyAsync(dst, d, bytes, hipMemcpyDeviceToHost, s_out)) != hipSuccess)
            return hip_error(e, "device-to-host copy");
        (void)hipEventRecord(E.d2h1, s_out);
        return FFT_OK;
    }

    // block until chunk c is back on the host; add its GPU times to stats
    int wait_chunk(uint64_t c, fft_stream_stats_t *st)
    {
        ChunkEvents &E = ev[c % ring];
        hipError_t e = hipEventSynchronize(E.d2h1);
        if (e != hipSuccess)
            return hip_error(e, "hipEventSynchronize");
        float a = 0, b = 0, d = 0;
        (void)hipEventElapsedTime(&a, E.h2d0, E.h2d1);
        (void)hipEventElapsedTime(&b, E.c0, E.c1);
        (void)hipEventElapsedTime(&d, E.d2h0, E.d2h1);
        if (times) {
            // every event of chunk c on the GPU clock, from the first copy
            float t[6] = {0, 0, 0, 0, 0, 0};
            const hipEvent_t q[6] = {E.h2d0, E.h2d1, E.c0, E.c1, E.d2h0, E.d2h1};
            for (int i = 0; i < 6; ++i)
                (void)hipEventElapsedTime(&t[i], ref, q[i]);
            times->push_back({c, t[0], t[1], t[2], t[3], t[4], t[5]});
        }
        if (st) {
            st->h2d_s += a * 1e-3;
            st->compute_s += b * 1e-3;
            st->d2h_s += d * 1e-3;
            st->bytes_h2d += bytes;
            st->bytes_d2h += bytes;
        }
        return FFT_OK;
    }

    // block until chunk c's input has left host slot memory
    int wait_input_consumed(uint64_t c)
    {
        hipError_t e = hipEventSynchronize(ev[c % ring].h2d1);
        return e == hipSuccess ? FFT_OK : hip_error(e, "hipEventSynchronize");
    }
};

struct PinnedRing {
    std::vector<void *> in, out;
    uint64_t bytes = 0;
    ~PinnedRing() { release(); }
    void release()
    {
        for (void *p : in)
            if (p)
                (void)hipHostFree(p);
        for (void *p : out)
            if (p)
                (void)hipHostFree(p);
        in.clear();
        out.clear();
    }
    int reserve(int slots, uint64_t b)
    {
        if ((int)in.size() == slots && bytes == b)
            return FFT_OK;
        release();
        bytes = b;
        in.assign(slots, nullptr);
        out.assign(slots, nullptr);
        for (int i = 0; i < slots; ++i) {
            if (hipHostMalloc(&in[i], b, hipHostMallocDefault) != hipSuccess ||
                hipHostMalloc(&out[i], b, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                release();
                return set_error(FFT_ERR_OUT_OF_MEMORY, "pinned host slot of %llu bytes",
                                 (unsigned long long)b);
            }
        }
        return FFT_OK;
    }
};

}  // namespace

// pinned ring kept with the plan between calls (freed with the plan), and
// the per-chunk timeline of the plan's last streamed call
struct StreamState {
    PinnedRing ring;
    std::vector<fft_chunk_times_t> timeline;
};

StreamState *stream_state(Plan *p)
{
    if (!p->stream_state)
        p->stream_state = new StreamState();
    return static_cast<StreamState *>(p->stream_state);
}

void stream_state_free(Plan *p)
{
    delete static_cast<StreamState *>(p->stream_state);
    p->stream_state = nullptr;
}

}  // namespace fftseg

using namespace fftseg;

extern "C" int fft_exec_stream(fft_plan_t plan, uint64_t n_chunks, fft_fill_fn fill,
                               fft_drain_fn drain, void *user, int n_slots,
                               uint64_t *failed_chunk, fft_stream_stats_t *stats)
{
    try {
        Plan *p = reinterpret_cast<Plan *>(plan);
        if (!p)
            return set_error(FFT_ERR_INVALID_ARG, "plan is NULL");
        if (reject_real(p, "fft_exec_stream") != FFT_OK)
            return last_status();
        if (!fill)
            return set_error(FFT_ERR_INVALID_ARG, "fill callback is NULL");
        if (n_slots < 2 || n_slots > 64)
            return set_error(FFT_ERR_INVALID_ARG, "n_slots must be in [2, 64]");
        if (failed_chunk)
            *failed_chunk = UINT64_MAX;
        if (stats)
            std::memset(stats, 0, sizeof(*stats));
        if (n_chunks == 0)
            return set_ok();
        const double t_start = now_s();
        StreamState *S = stream_state(p);
        const uint64_t bytes = p->batch * p->n * sizeof(c32);
        int st = S->ring.reserve(n_slots, bytes);
        if (st != FFT_OK)
            return st;
        Pipeline pl;
        if ((st = pl.init(p, std::max(n_slots, kDevSlots) + 1, &S->timeline)) != FFT_OK)
            return st;
        // The drain side runs on a worker thread: it waits for each chunk's
        // copy out, hands the chunk to drain and frees its output slot, in
        // chunk order, while this thread fills and issues later chunks, so
        // host work on both sides overlaps.  Chunk c reuses the slots of
        // chunk c - n_slots once that chunk's input has left host memory
        // and its output has been drained.
        struct Shared {
            std::mutex mu;
            std::condition_variable cv;
            uint64_t issued = 0, drained = 0;
            bool done_issuing = false;
            bool failed = false;  // the worker stopped at fail_at
            uint64_t fail_at = UINT64_MAX;
            int code = FFT_OK;
            std::string msg;
        } sh;
        std::thread worker([&] {
            uint64_t c = 0;
            try {
                for (;; ++c) {
                    {
                        std::unique_lock<std::mutex> lk(sh.mu);
                        sh.cv.wait(lk, [&] { return c < sh.issued || sh.done_issuing; });
                        if (c >= sh.issued)
                            return;
                    }
                    int s2 = pl.wait_chunk(c, stats);
                    if (s2 == FFT_OK && drain) {
                        const double t0 = now_s();
                        const int rc = drain(user, c, S->ring.out[c % n_slots], bytes);
                        if (stats)
                            stats->drain_s += now_s() - t0;
                        if (rc != 0)
                            s2 = set_error(FFT_ERR_CALLBACK,
                                           "drain callback returned %d at chunk %llu", rc,
                                           (unsigned long long)c);
                    }
                    std::lock_guard<std::mutex> lk(sh.mu);
                    if (s2 != FFT_OK) {
                        // status and message are thread-local: carry them over
                        sh.failed = true;
                        sh.fail_at = c;
                        sh.code = last_status();
                        sh.msg = last_message();
                        sh.cv.notify_all();
                        return;
                    }
                    sh.drained = c + 1;
                    if (stats)
                        stats->chunks_done = c + 1;
                    sh.cv.notify_all();
                }
            } catch (...) {
                std::lock_guard<std::mutex> lk(sh.mu);
                sh.failed = true;
                sh.fail_at = c;
                sh.code = FFT_ERR_OUT_OF_MEMORY;
                sh.msg = "host allocation failed";
                sh.cv.notify_all();
            }
        });
        // whatever way this function leaves, the worker is told that no
        // more chunks come and is joined first
        struct Joiner {
            std::thread &t;
            Shared &sh;
            ~Joiner()
            {
                {
                    std::lock_guard<std::mutex> lk(sh.mu);
                    sh.done_issuing = true;
                    sh.cv.notify_all();
                }
                if (t.joinable())
                    t.join();
            }
        } joiner{worker, sh};
        int fail = FFT_OK;
        uint64_t fail_at = UINT64_MAX;
        std::string fail_msg;
        for (uint64_t c = 0; c < n_chunks; ++c) {
            if (c >= (uint64_t)n_slots) {
                if ((st = pl.wait_input_consumed(c - n_slots)) != FFT_OK) {
                    fail = st;
                    fail_at = c;
                    fail_msg = last_message();
                    break;
                }
                std::unique_lock<std::mutex> lk(sh.mu);
                sh.cv.wait(lk, [&] { return sh.drained > c - n_slots || sh.failed; });
            }
            {
                std::lock_guard<std::mutex> lk(sh.mu);
                if (sh.failed)
                    break;
            }
            const double t0 = now_s();
            const int rc = fill(user, c, S->ring.in[c % n_slots], bytes);
            if (stats)
                stats->fill_s += now_s() - t0;
            if (rc != 0) {
                fail = set_error(FFT_ERR_CALLBACK, "fill callback returned %d at chunk %llu", rc,
                                 (unsigned long long)c);
                fail_at = c;
                fail_msg = last_message();
                break;
            }
            if ((st = pl.issue(c, S->ring.in[c % n_slots], S->ring.out[c % n_slots])) != FFT_OK) {
                fail = st;
                fail_at = c;
                fail_msg = last_message();
                break;
            }
            std::lock_guard<std::mutex> lk(sh.mu);
            sh.issued = c + 1;
            sh.cv.notify_all();
        }
        {
            // the worker drains every chunk issued (or stops at a failure)
            std::lock_guard<std::mutex> lk(sh.mu);
            sh.done_issuing = true;
            sh.cv.notify_all();
        }
        worker.join();  // (the joiner then finds it joined)
        (void)hipStreamSynchronize(pl.s_in);
        (void)hipStreamSynchronize(pl.s_comp);
        (void)hipStreamSynchronize(pl.s_out);
        if (stats)
            stats->wall_s = now_s() - t_start;
        // a drain that failed below the chunk this thread stopped at is the
        // reported failure; chunks below the reported one were handed out
        if (sh.failed && sh.fail_at < fail_at) {
            fail = sh.code;
            fail_at = sh.fail_at;
            fail_msg = sh.msg;
        }
        if (fail != FFT_OK) {
            if (failed_chunk)
                *failed_chunk = fail_at;
            return set_error(fail, "%s", fail_msg.c_str());
        }
        return set_ok();
    } catch (...) {
        return set_error(FFT_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

extern "C" int fft_exec_stream_pinned(fft_plan_t plan, uint64_t n_chunks,
                                      void *const *host_in, int n_in,
                                      void *const *host_out, int n_out, int n_slots,
                                      fft_stream_stats_t *stats)
{
    try {
        Plan *p = reinterpret_cast<Plan *>(plan);
        if (!p)
            return set_error(FFT_ERR_INVALID_ARG, "plan is NULL");
        if (reject_real(p, "fft_exec_stream_pinned") != FFT_OK)
            return last_status();
        if (!host_in || !host_out || n_in < 1 || n_out < 1)
            return set_error(FFT_ERR_INVALID_ARG, "host buffer lists are empty");
        if (n_slots < 2 || n_slots > 64)
            return set_error(FFT_ERR_INVALID_ARG, "n_slots must be in [2, 64]");
        for (int i = 0; i < n_in; ++i)
            if (!host_in[i])
                return set_error(FFT_ERR_INVALID_ARG, "host_in[%d] is NULL", i);
        for (int i = 0; i < n_out; ++i)
            if (!host_out[i])
                return set_error(FFT_ERR_INVALID_ARG, "host_out[%d] is NULL", i);
        if (stats)
            std::memset(stats, 0, sizeof(*stats));
        if (n_chunks == 0)
            return set_ok();
        const double t_start = now_s();
        Pipeline pl;
        int st = pl.init(p, n_slots + kDevSlots, &stream_state(p)->timeline);
        if (st != FFT_OK)
            return st;
        const uint64_t lag = (uint64_t)n_slots - 1;
        uint64_t waited = 0;
        for (uint64_t c = 0; c < n_chunks; ++c) {
            if ((st = pl.issue(c, host_in[c % n_in], host_out[c % n_out])) != FFT_OK)
                return st;
            if (c >= lag) {
                if ((st = pl.wait_chunk(waited, stats)) != FFT_OK)
                    return st;
                ++waited;
                if (stats)
                    stats->chunks_done = waited;
            }
        }
        while (waited < n_chunks) {
            if ((st = pl.wait_chunk(waited, stats)) != FFT_OK)
                return st;
            ++waited;
            if (stats)
                stats->chunks_done = waited;
        }
        if (stats)
            stats->wall_s = now_s() - t_start;
        return set_ok();
    } catch (...) {
        return set_error(FFT_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

// ---------------------------------------------------------------------------
// File-backed streaming.  The paper's measured bottleneck is reading and
// writing the signal file (Sec. IV); its outputs are written per block and
// named by position so that concatenation restores the order (Sec. III).
// Here chunk c is read from byte in_offset + c * chunk_bytes of the input
// file and its spectra are written at out_offset + c * chunk_bytes of the
// output file: every record keeps its offset, no merge step is needed, and
// a failed run can resume from the failing chunk.
#include <fcntl.h>
#include <sys/stat.h>
#include <unistd.h>

#include <atomic>
#include <thread>

namespace fftseg {
namespace {

struct FileIo {
    int in_fd = -1, out_fd = -1;
    uint64_t in_offset = 0, out_offset = 0, first_chunk = 0;
    int threads = 1;
};

// transfer `bytes` at file offset `off` with `threads` parallel pread or
// pwrite calls over disjoint parts; 0 on success
int parallel_io(int fd, bool write, void *buf, uint64_t bytes, uint64_t off, int threads)
{
    const uint64_t part = (bytes + threads - 1) / threads;
    std::atomic<int> failed{0};
    auto work = [&](int i) {
        const uint64_t a = (uint64_t)i * part;
        if (a >= bytes)
            return;
        uint64_t left = std::min(part, bytes - a);
        char *p = (char *)buf + a;
        uint64_t o = off + a;
        while (left > 0) {
            const ssize_t k = write ? pwrite(fd, p, left, (off_t)o) : pread(fd, p, left, (off_t)o);
            if (k <= 0) {
                failed = 1;
                return;
            }
            p += k;
            o += (uint64_t)k;
            left -= (uint64_t)k;
        }
    };
    if (threads <= 1) {
        work(0);
    } else {
        std::vector<std::thread> pool;
        for (int i = 0; i < threads; ++i)
            pool.emplace_back(work, i);
        for (auto &t : pool)
            t.join();
    }
    return failed ? -1 : 0;
}

int file_fill(void *user, uint64_t chunk, void *dst, uint64_t bytes)
{
    const FileIo *f = (const FileIo *)user;
    return parallel_io(f->in_fd, false, dst, bytes,
                       f->in_offset + (f->first_chunk + chunk) * bytes, f->threads);
}

int file_drain(void *user, uint64_t chunk, const void *src, uint64_t bytes)
{
    const FileIo *f = (const FileIo *)user;
    return parallel_io(f->out_fd, true, const_cast<void *>(src), bytes,
                       f->out_offset + (f->first_chunk + chunk) * bytes, f->threads);
}

}  // namespace
}  // namespace fftseg

extern "C" int fft_exec_file(fft_plan_t plan, const char *in_path, uint64_t in_offset,
                             const char *out_path, uint64_t out_offset, uint64_t first_chunk,
                             uint64_t n_chunks, int n_slots, int io_threads,
                             uint64_t *failed_chunk, fft_stream_stats_t *stats)
{
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p)
        return set_error(FFT_ERR_INVALID_ARG, "plan is NULL");
    if (reject_real(p, "fft_exec_file") != FFT_OK)
        return last_status();
    if (!in_path || !out_path)
        return set_error(FFT_ERR_INVALID_ARG, "file paths must not be NULL");
    if (io_threads < 1 || io_threads > 64)
        return set_error(FFT_ERR_INVALID_ARG, "io_threads must be in [1, 64]");
    const uint64_t chunk_bytes = p->batch * p->n * sizeof(c32);
    if (first_chunk > UINT64_MAX / chunk_bytes || n_chunks > UINT64_MAX / chunk_bytes ||
        (first_chunk + n_chunks) > UINT64_MAX / chunk_bytes ||
        in_offset > UINT64_MAX - (first_chunk + n_chunks) * chunk_bytes ||
        out_offset > UINT64_MAX - (first_chunk + n_chunks) * chunk_bytes)
        return set_error(FFT_ERR_INVALID_ARG, "file range overflows");
    FileIo f;
    f.in_offset = in_offset;
    f.out_offset = out_offset;
    f.first_chunk = first_chunk;
    f.threads = io_threads;
    f.in_fd = open(in_path, O_RDONLY);
    if (f.in_fd < 0)
        return set_error(FFT_ERR_INVALID_ARG, "cannot open %s for reading", in_path);
    struct stat sb;
    const uint64_t need = in_offset + (first_chunk + n_chunks) * chunk_bytes;
    if (fstat(f.in_fd, &sb) != 0 || (uint64_t)sb.st_size < need) {
        close(f.in_fd);
        return set_error(FFT_ERR_BOUNDS, "%s holds %lld bytes, %llu needed", in_path,
                         (long long)sb.st_size, (unsigned long long)need);
    }
    f.out_fd = open(out_path, O_WRONLY | O_CREAT, 0644);
    if (f.out_fd < 0) {
        close(f.in_fd);
        return set_error(FFT_ERR_INVALID_ARG, "cannot open %s for writing", out_path);
    }
    uint64_t failed = UINT64_MAX;
    const int st = fft_exec_stream(plan, n_chunks, &file_fill, &file_drain, &f, n_slots,
                                   &failed, stats);
    const int code = last_status();
    std::string msg = last_message();
    close(f.in_fd);
    if (close(f.out_fd) != 0 && st == FFT_OK)
        return set_error(FFT_ERR_CALLBACK, "closing %s failed", out_path);
    if (failed_chunk)
        *failed_chunk = failed == UINT64_MAX ? UINT64_MAX : first_chunk + failed;
    if (st != FFT_OK)
        return set_error(code, "%s", msg.c_str());
    return set_ok();
}

extern "C" void *fft_host_alloc(size_t bytes)
{
    if (bytes == 0) {
        set_error(FFT_ERR_INVALID_ARG, "fft_host_alloc: 0 bytes");
        return nullptr;
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        set_error(FFT_ERR_OUT_OF_MEMORY, "pinned host allocation of %llu bytes",
                  (unsigned long long)bytes);
        return nullptr;
    }
    set_ok();
    return p;
}

extern "C" int fft_host_free(void *ptr)
{
    if (!ptr)
        return set_ok();
    hipError_t e = hipHostFree(ptr);
    if (e != hipSuccess)
        return hip_error(e, "hipHostFree");
    return set_ok();
}

extern "C" int fft_stream_last_timeline(fft_plan_t plan, fft_chunk_times_t *out, size_t max)
{
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p)
        return set_error(FFT_ERR_INVALID_ARG, "plan is NULL");
    if (!out && max)
        return set_error(FFT_ERR_INVALID_ARG, "out is NULL");
    const StreamState *S = static_cast<const StreamState *>(p->stream_state);
    const size_t have = S ? S->timeline.size() : 0;
    const size_t n = std::min(have, max);
    for (size_t i = 0; i < n; ++i)
        out[i] = S->timeline[i];
    set_ok();
    return (int)std::min<size_t>(have, (size_t)INT32_MAX);
}
