// Autotuner and plan graphs.
//
// fft_autotune times every compiled single-pass variant of a length (radix
// order, threads per segment, segments per workgroup, LDS padding,
// streamed or cached global access) at several persistent-grid sizes and
// keeps the fastest; two-pass lengths tune their column-tile and row-tile
// variants and grid size.  Choices live
// in a process-wide table that later plans consult, and can be merged into
// a JSON cache file keyed by device architecture and length.
#include "fftseg.h"
#include "runtime.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace fftseg {
namespace {

const int kMults[] = {0, 4, 8, 16, 32, 64};

std::string arch_name()
{
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    std::string a = p.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// time one configuration: warm-up, then `reps` execs between events
int time_plan(Plan *p, void *in, void *out, hipStream_t s, int reps, double *us)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return hip_error(hipGetLastError(), "hipEventCreate");
    int st = FFT_OK;
    for (int i = 0; i < 2 && st == FFT_OK; ++i)
        st = plan_enqueue(p, in, out, p->batch, s);
    (void)hipEventRecord(e0, s);
    for (int i = 0; i < reps && st == FFT_OK; ++i)
        st = plan_enqueue(p, in, out, p->batch, s);
    (void)hipEventRecord(e1, s);
    hipError_t e = hipEventSynchronize(e1);
    float ms = 0;
    if (st == FFT_OK && e == hipSuccess)
        e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FFT_OK)
        return st;
    if (e != hipSuccess)
        return hip_error(e, "event timing");
    *us = ms * 1e3 / reps;
    return FFT_OK;
}

// Work-list route of a length with indexed kernels: batch segments at sample offsets
// s * (n + 3), so they start at every position within a cache line as in
// a packed mixed list, through the work-list kernel's tiles (route 0) and
// through each indexed one-pass kernel of the length (route 1 + k) at each
// grid size; the fastest goes into *route, *grid, *us.  Returns the number
// of configurations timed (0 if the length has no work-list tiles or no
// indexed kernel), or a negative status.
int tune_worklist_route(uint64_t n, uint64_t batch, int dir, hipStream_t s, int *route,
                        int *grid, double *us_best)
{
    const int cnt = fft_worklist_indexed_count((uint32_t)n);
    if (cnt == 0)
        return 0;
    const uint64_t stride = n + 3, total = batch * stride;
    void *in = nullptr, *out = nullptr;
    if (hipMalloc(&in, total * sizeof(c32)) != hipSuccess ||
        hipMalloc(&out, total * sizeof(c32)) != hipSuccess) {
        (void)hipGetLastError();
        if (in)
            (void)hipFree(in);
        return set_error(FFT_ERR_OUT_OF_MEMORY, "work-list tuning buffers");
    }
    (void)hipMemset(in, 0, total * sizeof(c32));
    std::vector<fft_work_t> items(batch);
    for (uint64_t i = 0; i < batch; ++i)
        items[i] = {i * stride, i * stride, (uint32_t)n, 0};
    // the route in the table while tuning is restored afterwards
    int keep_grid = 0;
    const int keep_route = tuned_wl_route(n, &keep_grid);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    int timed = 0, st = FFT_OK;
    double best = 1e300;
    for (int r = 0; r <= cnt && st == FFT_OK; ++r) {
        for (int m : kMults) {
            if (r == 0 && m != kMults[0])
                break;  // the tiles' grid is the work list's own
            set_tuned_wl_route(n, r, m, 0);
            fft_worklist_t w = fft_worklist_create(items.data(), batch, dir);
            if (!w) {
                st = last_status();
                break;
            }
            for (int i = 0; i < 2 && st == FFT_OK; ++i)
                st = fft_worklist_exec(w, in, out, s);
            (void)hipEventRecord(e0, s);
            for (int i = 0; i < 5 && st == FFT_OK; ++i)
                st = fft_worklist_exec(w, in, out, s);
            (void)hipEventRecord(e1, s);
            float ms = 0;
            if (st == FFT_OK && hipEventSynchronize(e1) == hipSuccess &&
                hipEventElapsedTime(&ms, e0, e1) == hipSuccess) {
                const double us = ms * 1e3 / 5;
                ++timed;
                if (us < best) {
                    best = us;
                    *route = r;
                    *grid = r == 0 ? 0 : m;
                }
            }
            fft_worklist_destroy(w);
        }
    }
    set_tuned_wl_route(n, keep_route, keep_grid, 0);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(in);
    (void)hipFree(out);
    if (st != FFT_OK)
        return st;
    *us_best = best;
    return timed;
}

// minimal reader of the cache written below: entries of integer/float keys
bool read_number(const std::string &obj, const char *key, double *v)
{
    const std::string k = std::string("\"") + key + "\"";
    size_t p = obj.find(k);
    if (p == std::string::npos)
        return false;
    p = obj.find(':', p + k.size());
    if (p == std::string::npos)
        return false;
    char *end = nullptr;
    *v = strtod(obj.c_str() + p + 1, &end);
    return end != obj.c_str() + p + 1;
}

std::vector<std::string> entry_objects(const std::string &js)
{
    std::vector<std::string> out;
    size_t p = js.find("\"entries\"");
    if (p == std::string::npos)
        return out;
    p = js.find('[', p);
    if (p == std::string::npos)
        return out;
    const size_t close = js.find(']', p);
    while (true) {
        const size_t a = js.find('{', p);
        if (a == std::string::npos || (close != std::string::npos && a > close))
            break;
        const size_t b = js.find('}', a);
        if (b == std::string::npos)
            break;
        out.push_back(js.substr(a, b - a + 1));
        p = b + 1;
    }
    return out;
}

bool read_file(const char *path, std::string &s)
{
    FILE *f = fopen(path, "rb");
    if (!f)
        return false;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof buf, f)) > 0)
        s.append(buf, k);
    fclose(f);
    return true;
}

std::string arch_of(const std::string &js)
{
    const size_t p = js.find("\"arch\"");
    if (p == std::string::npos)
        return "";
    const size_t a = js.find('"', js.find(':', p) + 1);
    const size_t b = a == std::string::npos ? a : js.find('"', a + 1);
    return (a == std::string::npos || b == std::string::npos) ? "" : js.substr(a + 1, b - a - 1);
}

int write_cache(const char *path)
{
    // merge: entries already in the file for other lengths are kept
    std::vector<TunedChoice> merged = tuned_snapshot();
    std::string old;
    const std::string arch = arch_name();
    if (read_file(path, old) && arch_of(old) == arch) {
        for (const std::string &o : entry_objects(old)) {
            double n = 0, v = 0, g = 0, us = 0, b = 0, cv = 0, rv = 0, n1 = 0;
            double wr = -1, wg = 0, wus = 0;
            if (!read_number(o, "n", &n) || !read_number(o, "variant", &v) ||
                !read_number(o, "grid_mult", &g))
                continue;
            read_number(o, "us", &us);
            read_number(o, "batch", &b);
            read_number(o, "column_variant", &cv);
            read_number(o, "row_variant", &rv);
            read_number(o, "n1", &n1);
            read_number(o, "wl_route", &wr);
            read_number(o, "wl_grid", &wg);
            read_number(o, "wl_us", &wus);
            bool have = false;
            for (auto &m : merged)
                have |= m.n == (uint64_t)n;
            if (!have) {
                TunedChoice c{(uint64_t)n, (int)v, (int)g, us, (uint64_t)b, (int)cv, (int)rv,
                              (uint64_t)n1};
                c.wl_route = (int)wr;
                c.wl_grid = (int)wg;
                c.wl_us = wus;
                merged.push_back(c);
            }
        }
    }
    std::sort(merged.begin(), merged.end(),
              [](const TunedChoice &a, const TunedChoice &b) { return a.n < b.n; });
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f)
        return set_error(FFT_ERR_INVALID_ARG, "cannot write tuning cache %s", path);
    fprintf(f, "{\n  \"arch\": \"%s\",\n  \"entries\": [\n", arch.c_str());
    for (size_t i = 0; i < merged.size(); ++i)
        fprintf(f,
                "    {\"n\": %llu, \"variant\": %d, \"grid_mult\": %d, \"us\": %.3f, "
                "\"batch\": %llu, \"column_variant\": %d, \"row_variant\": %d, "
                "\"n1\": %llu, \"wl_route\": %d, \"wl_grid\": %d, \"wl_us\": %.3f}%s\n",
                (unsigned long long)merged[i].n, merged[i].variant, merged[i].grid_mult,
                merged[i].us, (unsigned long long)merged[i].batch, merged[i].col_variant,
                merged[i].row_variant, (unsigned long long)merged[i].n1, merged[i].wl_route,
                merged[i].wl_grid, merged[i].wl_us, i + 1 < merged.size() ? "," : "");
    fprintf(f, "  ]\n}\n");
    fclose(f);
    if (rename(tmp.c_str(), path) != 0)
        return set_error(FFT_ERR_INVALID_ARG, "cannot replace tuning cache %s", path);
    return FFT_OK;
}

}  // namespace
}  // namespace fftseg

using namespace fftseg;

extern "C" int fft_autotune(size_t segment_len, size_t batch, int direction, const char *path,
                            double *best_us)
{
    try {
        if (validate_create(segment_len, batch, direction) != FFT_OK)
            return last_status();
        const uint64_t bytes = (uint64_t)segment_len * batch * sizeof(c32);
        void *in = nullptr, *out = nullptr;
        hipError_t e;
        if ((e = hipMalloc(&in, bytes)) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(FFT_ERR_OUT_OF_MEMORY, "autotune input of %llu bytes",
                             (unsigned long long)bytes);
        }
        if ((e = hipMalloc(&out, bytes)) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(in);
            return set_error(FFT_ERR_OUT_OF_MEMORY, "autotune output");
        }
        (void)hipMemset(in, 0, bytes);
        hipStream_t s = nullptr;
        (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        const int nv = variant_count(segment_len);
        int ncol = 0, nrow = 0;
        if (nv == 0)
            split_variant_counts(segment_len, &ncol, &nrow);
        // candidates: single-pass variants; or, for two-pass lengths, every
        // column x row tile variant of the planner's split and the default
        // tiles of every other split n1 x n/n1 with compiled tiles
        struct Cand {
            int first, second;
            uint64_t n1;  // 0: the planner's split
        };
        std::vector<Cand> cand;
        if (nv > 0) {
            for (int v = 0; v < nv; ++v)
                cand.push_back({v, -1, 0});
        } else if (ncol > 0) {
            for (int c = 0; c < ncol; ++c)
                for (int r = 0; r < nrow; ++r)
                    cand.push_back({c, r, 0});
            const ColumnDesc *dc = nullptr;
            const RowDesc *dr = nullptr;
            find_split(segment_len, &dc, &dr, 0, 0);
            for (uint64_t n1 : split_candidates(segment_len))
                if (n1 != (uint64_t)dc->n1)
                    cand.push_back({0, 0, n1});
        } else {
            cand.push_back({-1, -1, 0});
        }
        double best = 1e300;
        TunedChoice choice{segment_len, nv > 0 ? 0 : -1, 0, 0, batch, 0, 0};
        int timed = 0, st = FFT_OK;
        for (const auto &cv : cand) {
            if (st != FFT_OK)
                break;
            for (int m : kMults) {
                Plan p;
                if (nv > 0)
                    st = plan_build(&p, segment_len, batch, direction, cv.first, -1);
                else
                    st = plan_build(&p, segment_len, batch, direction, -1,
                                    ncol > 0 ? (cv.first | (cv.second << 8)) : -1, cv.n1);
                if (st != FFT_OK) {
                    plan_free(&p);
                    break;
                }
                p.grid_mult = m;
                const uint64_t plan_n1 = p.kind == Plan::FOURSTEP ? p.n1 : 0;
                double us = 0;
                st = time_plan(&p, in, out, s, 5, &us);
                plan_free(&p);
                if (st != FFT_OK)
                    break;
                ++timed;
                if (us < best) {
                    best = us;
                    choice.variant = nv > 0 ? cv.first : -1;
                    choice.col_variant = nv > 0 ? 0 : std::max(cv.first, 0);
                    choice.row_variant = nv > 0 ? 0 : std::max(cv.second, 0);
                    choice.n1 = plan_n1;
                    choice.grid_mult = m;
                    choice.us = us;
                }
            }
        }
        (void)hipStreamSynchronize(s);
        (void)hipFree(in);
        (void)hipFree(out);
        if (st == FFT_OK) {
            // lengths with indexed work-list kernels: the work-list route too
            int r = -1, g = 0;
            double wus = 0;
            const int k = tune_worklist_route(segment_len, batch, direction, s, &r, &g, &wus);
            if (k < 0)
                st = k;
            else if (k > 0) {
                choice.wl_route = r;
                choice.wl_grid = g;
                choice.wl_us = wus;
                timed += k;
            }
        }
        (void)hipStreamDestroy(s);
        if (st != FFT_OK)
            return st;
        set_tuned(choice);
        if (best_us)
            *best_us = best;
        if (path && (st = write_cache(path)) != FFT_OK)
            return st;
        set_ok();
        return timed;
    } catch (...) {
        return set_error(FFT_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

extern "C" int fft_tune_load(const char *path)
{
    try {
        if (!path)
            return set_error(FFT_ERR_INVALID_ARG, "path is NULL");
        std::string js;
        if (!read_file(path, js))
            return set_error(FFT_ERR_INVALID_ARG, "cannot read %s", path);
        const std::string arch = arch_of(js);
        const std::string mine = arch_name();
        if (arch != mine)
            return set_error(FFT_ERR_INVALID_ARG, "cache is for %s, device is %s", arch.c_str(),
                             mine.c_str());
        int k = 0;
        for (const std::string &o : entry_objects(js)) {
            double n = 0, v = 0, g = 0, us = 0, b = 0, cv = 0, rv = 0, n1 = 0;
            double wr = -1, wg = 0, wus = 0;
            if (!read_number(o, "n", &n) || !read_number(o, "variant", &v) ||
                !read_number(o, "grid_mult", &g))
                continue;
            read_number(o, "column_variant", &cv);
            read_number(o, "row_variant", &rv);
            read_number(o, "n1", &n1);
            read_number(o, "wl_route", &wr);
            read_number(o, "wl_grid", &wg);
            read_number(o, "wl_us", &wus);
            int ncol = 0, nrow = 0;
            if (v < 0)
                split_variant_counts((uint64_t)n, &ncol, &nrow);
            const ColumnDesc *sc = nullptr;
            const RowDesc *sr = nullptr;
            if (n < 1 || v < -2 || (v >= 0 && v >= variant_count((uint64_t)n)) || g < 0 ||
                g > 1024 ||
                (v < 0 && (cv < 0 || rv < 0 || (ncol && cv >= ncol) || (nrow && rv >= nrow))) ||
                n1 < 0 || (n1 > 0 && !find_split((uint64_t)n, &sc, &sr, 0, 0, (uint64_t)n1)))
                continue;  // stale entry for variants the library does not have
            const int n_idx = fft_worklist_indexed_count((uint32_t)n);
            if (wr < -1 || wr > n_idx || wg < 0 || wg > 1024)
                wr = -1, wg = 0;  // a work-list route the library does not have
            read_number(o, "us", &us);
            read_number(o, "batch", &b);
            TunedChoice c{(uint64_t)n, (int)v, (int)g, us, (uint64_t)b, (int)cv, (int)rv,
                          (uint64_t)n1};
            c.wl_route = (int)wr;
            c.wl_grid = (int)wg;
            c.wl_us = wus;
            set_tuned(c);
            ++k;
        }
        set_ok();
        return k;
    } catch (...) {
        return set_error(FFT_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

extern "C" int fft_tune_clear(void)
{
    clear_tuned();
    return set_ok();
}

// ---------------------------------------------------------------------------
// plan graphs
extern "C" int fft_exec_segments_graph(fft_plan_t plan, const void *in, void *out, void *stream)
{
    try {
        Plan *p = reinterpret_cast<Plan *>(plan);
        if (!p)
            return set_error(FFT_ERR_INVALID_ARG, "plan is NULL");
        if (reject_real(p, "fft_exec_segments_graph") != FFT_OK)
            return last_status();
        const uint64_t bytes = p->batch * p->n * sizeof(c32);
        int st = check_io(in, out, bytes);
        if (st != FFT_OK)
            return st;
        hipError_t e;
        if (!p->graph_exec || p->graph_in != in || p->graph_out != out) {
            if (p->graph_exec) {
                (void)hipGraphExecDestroy(p->graph_exec);
                p->graph_exec = nullptr;
            }
            if (p->graph) {
                (void)hipGraphDestroy(p->graph);
                p->graph = nullptr;
            }
            if (!p->capture_stream &&
                (e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking)) !=
                    hipSuccess)
                return hip_error(e, "hipStreamCreate");
            if ((e = hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal)) !=
                hipSuccess)
                return hip_error(e, "hipStreamBeginCapture");
            st = plan_enqueue(p, in, out, p->batch, p->capture_stream);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(p->capture_stream, &g);
            if (st != FFT_OK) {
                if (g)
                    (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess)
                return hip_error(e, "hipStreamEndCapture");
            p->graph = g;
            if ((e = hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0)) != hipSuccess) {
                p->graph_exec = nullptr;
                return hip_error(e, "hipGraphInstantiate");
            }
            p->graph_in = in;
            p->graph_out = out;
        }
        if ((e = hipGraphLaunch(p->graph_exec, (hipStream_t)stream)) != hipSuccess)
            return hip_error(e, "hipGraphLaunch");
        p->used = true;
        p->last_stream = (hipStream_t)stream;
        p->last_stream_valid = true;
        return set_ok();
    } catch (...) {
        return set_error(FFT_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}
