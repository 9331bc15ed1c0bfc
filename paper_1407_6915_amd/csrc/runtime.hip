// Planner, twiddle tables, argument checks and the C entry points of the
// batched segment FFT (declared in fftseg.h).
#include "fftseg.h"
#include "runtime.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

namespace fftseg {

// ---------------------------------------------------------------------------
// per-thread status
namespace {
thread_local int t_status = FFT_OK;
thread_local char t_msg[512] = "";
}  // namespace

int set_ok()
{
    t_status = FFT_OK;
    t_msg[0] = 0;
    return FFT_OK;
}

int set_error(int status, const char *fmt, ...)
{
    t_status = status;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_msg, sizeof(t_msg), fmt, ap);
    va_end(ap);
    return status;
}

int hip_error(hipError_t e, const char *what)
{
    return set_error(FFT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

int last_status() { return t_status; }
const char *last_message() { return t_msg; }

// ---------------------------------------------------------------------------
// twiddles: exp(-2 pi i m / n) in FP64 with the angle folded to the first
// octant in exact integer arithmetic, rounded once to float32
c32 root_forward(uint64_t m, uint64_t n)
{
    m %= n;
    // angle 2 pi m / n = (pi/4) (o + r/n) with 8m = o*n + r; quadrant
    // j = floor((o + 1) / 2) and x = (pi/4) (o - 2j + r/n) in [-pi/4, pi/4)
    const unsigned __int128 m8 = (unsigned __int128)m * 8u;
    const uint64_t o = (uint64_t)(m8 / n);
    const uint64_t r = (uint64_t)(m8 - (unsigned __int128)o * n);
    const uint64_t j = (o + 1) / 2;
    const double quarter_pi = 0.78539816339744830961566084581987572;
    const double x = ((double)((long long)o - 2 * (long long)j) + (double)r / (double)n) *
                     quarter_pi;
    const double cx = std::cos(x), sx = std::sin(x);
    double c, s;
    switch (j & 3) {
    case 0: c = cx; s = sx; break;
    case 1: c = -sx; s = cx; break;
    case 2: c = -cx; s = -sx; break;
    default: c = sx; s = -cx; break;
    }
    return c32{(float)c, (float)(-s)};
}

namespace {

std::vector<c32> root_table(uint64_t n)
{
    std::vector<c32> t(n);
    for (uint64_t m = 0; m < n; ++m)
        t[m] = root_forward(m, n);
    return t;
}

int ilog2_ceil(uint64_t v)
{
    int k = 0;
    while ((1ull << k) < v)
        ++k;
    return k;
}

bool is_pow2(uint64_t v) { return v && !(v & (v - 1)); }

bool smooth235(uint64_t n)
{
    if (n == 0)
        return false;
    for (uint64_t p : {2ull, 3ull, 5ull})
        while (n % p == 0)
            n /= p;
    return n == 1;
}

// greedy radix list for the global-memory fallback
std::vector<int> generic_radices(uint64_t n)
{
    std::vector<int> r;
    for (int p : {16, 8, 4, 2, 5, 3}) {
        while (n % p == 0 && n > 1) {
            r.push_back(p);
            n /= p;
        }
    }
    return r;
}

hipError_t upload(const std::vector<c32> &h, void **d)
{
    *d = nullptr;
    hipError_t e = hipMalloc(d, h.size() * sizeof(c32));
    if (e != hipSuccess) {
        *d = nullptr;
        return e;
    }
    e = hipMemcpy(*d, h.data(), h.size() * sizeof(c32), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(*d);
        *d = nullptr;
    }
    return e;
}

// the tuning table: preferred single-pass variant and grid per length
std::mutex g_tune_mu;
std::vector<TunedChoice> g_tuned;

}  // namespace

int tuned_variant(uint64_t n)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto &p : g_tuned)
        if (p.n == n)
            return p.variant;
    return -1;
}

int tuned_grid_mult(uint64_t n, int variant, int fallback)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto &p : g_tuned)
        if (p.n == n && p.variant == variant)
            return p.grid_mult;
    return fallback;
}

void tuned_split_variants(uint64_t n, int *col_variant, int *row_variant, uint64_t *n1)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto &p : g_tuned)
        if (p.n == n && p.variant < 0) {
            *col_variant = p.col_variant;
            *row_variant = p.row_variant;
            *n1 = p.n1;
            return;
        }
}

int tuned_wl_route(uint64_t n, int *grid)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto &p : g_tuned)
        if (p.n == n) {
            if (grid)
                *grid = p.wl_grid;
            return p.wl_route;
        }
    return -1;
}

void set_tuned(const TunedChoice &c)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto &p : g_tuned)
        if (p.n == c.n) {
            p = c;
            return;
        }
    g_tuned.push_back(c);
}

void set_tuned_wl_route(uint64_t n, int route, int grid, double us)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto &p : g_tuned)
        if (p.n == n) {
            p.wl_route = route;
            p.wl_grid = grid;
            p.wl_us = us;
            return;
        }
    TunedChoice c{n, -2, 0, 0, 0, 0, 0};  // variant -2: no plan choice
    c.wl_route = route;
    c.wl_grid = grid;
    c.wl_us = us;
    g_tuned.push_back(c);
}

void clear_tuned()
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned.clear();
}

std::vector<TunedChoice> tuned_snapshot()
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tuned;
}

const SinglePassDesc *find_single(uint64_t n, int variant)
{
    int cnt = 0;
    const SinglePassDesc *t = single_pass_table(&cnt);
    for (int i = 0; i < cnt; ++i)
        if ((uint64_t)t[i].n == n && t[i].variant == variant)
            return &t[i];
    return nullptr;
}

// the variant of length n that carries the frame and real-input kernels
static const SinglePassDesc *find_small_batch(uint64_t n)
{
    int cnt = 0;
    const SinglePassDesc *t = single_pass_table(&cnt);
    for (int i = 0; i < cnt; ++i)
        if ((uint64_t)t[i].n == n && t[i].small_batch)
            return &t[i];
    return nullptr;
}

const SinglePassDesc *find_frames(uint64_t n)
{
    int cnt = 0;
    const SinglePassDesc *t = single_pass_table(&cnt);
    for (int i = 0; i < cnt; ++i)
        if ((uint64_t)t[i].n == n && t[i].launch_strided)
            return &t[i];
    return nullptr;
}

const SinglePassDesc *find_aux(uint64_t n)
{
    int cnt = 0;
    const SinglePassDesc *t = single_pass_table(&cnt);
    for (int i = 0; i < cnt; ++i)
        if ((uint64_t)t[i].n == n && t[i].launch_strided && t[i].launch_real)
            return &t[i];
    return nullptr;
}

int variant_count(uint64_t n)
{
    int cnt = 0, k = 0;
    const SinglePassDesc *t = single_pass_table(&cnt);
    for (int i = 0; i < cnt; ++i)
        k += (uint64_t)t[i].n == n;
    return k;
}

// best four-step split n = n1 * n2 with compiled column and row tiles;
// the split is chosen on the default tiles, then the requested variants of
// those lengths are used (default where a variant does not exist)
bool find_split(uint64_t n, const ColumnDesc **col, const RowDesc **row, int col_variant,
                int row_variant, uint64_t want_n1)
{
    int nc = 0, nr = 0;
    const ColumnDesc *ct = column_table(&nc);
    const RowDesc *rt = row_table(&nr);
    double best = 1e30;
    *col = nullptr;
    *row = nullptr;
    for (int i = 0; i < nc; ++i) {
        if (ct[i].variant != 0 || n % (uint64_t)ct[i].n1 ||
            (want_n1 && (uint64_t)ct[i].n1 != want_n1))
            continue;
        const uint64_t n2 = n / (uint64_t)ct[i].n1;
        for (int j = 0; j < nr; ++j) {
            if (rt[j].variant != 0 || (uint64_t)rt[j].n2 != n2)
                continue;
            // prefer balanced splits, then the smaller column length
            const double score =
                std::fabs(std::log2((double)ct[i].n1) - std::log2((double)n2)) * 2.0 +
                (ct[i].n1 > (int)n2 ? 1.0 : 0.0);
            if (score < best) {
                best = score;
                *col = &ct[i];
                *row = &rt[j];
            }
        }
    }
    if (!*col)
        return false;
    const uint64_t n1 = (uint64_t)(*col)->n1, n2 = n / n1;
    auto fits = [&](const ColumnDesc &c, const RowDesc &r) {
        return n2 % (uint64_t)c.cols == 0 && n1 % (uint64_t)r.rows == 0;
    };
    for (int i = 0; i < nc; ++i)
        if ((uint64_t)ct[i].n1 == n1 && ct[i].variant == col_variant && fits(ct[i], **row))
            *col = &ct[i];
    for (int j = 0; j < nr; ++j)
        if ((uint64_t)rt[j].n2 == n2 && rt[j].variant == row_variant && fits(**col, rt[j]))
            *row = &rt[j];
    return fits(**col, **row);
}

std::vector<uint64_t> split_candidates(uint64_t n)
{
    std::vector<uint64_t> out;
    int nc = 0;
    const ColumnDesc *ct = column_table(&nc);
    for (int i = 0; i < nc; ++i) {
        const ColumnDesc *c = nullptr;
        const RowDesc *r = nullptr;
        if (ct[i].variant == 0 && n % (uint64_t)ct[i].n1 == 0 &&
            find_split(n, &c, &r, 0, 0, (uint64_t)ct[i].n1))
            out.push_back((uint64_t)ct[i].n1);
    }
    return out;
}

const ColumnDesc *find_column_shifted(uint64_t n1)
{
    int nc = 0;
    const ColumnDesc *ct = column_table(&nc);
    for (int i = 0; i < nc; ++i)
        if ((uint64_t)ct[i].n1 == n1 && ct[i].launch_shifted)
            return &ct[i];
    return nullptr;
}

const RowDesc *find_row_shifted(uint64_t n2)
{
    int nr = 0;
    const RowDesc *rt = row_table(&nr);
    for (int j = 0; j < nr; ++j)
        if ((uint64_t)rt[j].n2 == n2 && rt[j].launch_shifted)
            return &rt[j];
    return nullptr;
}

int split_variant_counts(uint64_t n, int *ncol, int *nrow)
{
    const ColumnDesc *c = nullptr;
    const RowDesc *r = nullptr;
    *ncol = *nrow = 0;
    if (!find_split(n, &c, &r, 0, 0))
        return 0;
    int nc = 0, nr = 0;
    const ColumnDesc *ct = column_table(&nc);
    const RowDesc *rt = row_table(&nr);
    for (int i = 0; i < nc; ++i)
        *ncol += ct[i].n1 == c->n1;
    for (int j = 0; j < nr; ++j)
        *nrow += rt[j].n2 == r->n2;
    return 1;
}

// CU count per device and resident workgroups per CU per kernel, cached:
// both are fixed for the life of the process and the queries are slow.
namespace {
std::mutex g_occ_mu;
std::vector<std::pair<int, int>> g_cus;                      // (device, CUs)
std::vector<std::pair<std::pair<const void *, int>, int>> g_occ;  // ((kernel, dev), per CU)
}  // namespace

static int device_cus(int dev)
{
    std::lock_guard<std::mutex> lk(g_occ_mu);
    for (auto &c : g_cus)
        if (c.first == dev)
            return c.second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0) {
        (void)hipGetLastError();
        n = 256;
    }
    g_cus.emplace_back(dev, n);
    return n;
}

static int resident_per_cu(const void *kernel, int threads, int dev)
{
    {
        std::lock_guard<std::mutex> lk(g_occ_mu);
        for (auto &o : g_occ)
            if (o.first.first == kernel && o.first.second == dev)
                return o.second;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
        per_cu <= 0) {
        (void)hipGetLastError();
        per_cu = 1;
    }
    std::lock_guard<std::mutex> lk(g_occ_mu);
    g_occ.push_back({{kernel, dev}, per_cu});
    return per_cu;
}

unsigned grid_for(const void *kernel, int threads, uint64_t work_groups, int dev,
                  int grid_mult)
{
    uint64_t g = work_groups;
    if (grid_mult > 0) {
        const uint64_t cap = (uint64_t)resident_per_cu(kernel, threads, dev) *
                             (uint64_t)device_cus(dev) * (uint64_t)grid_mult;
        g = std::min<uint64_t>(g, cap);
    }
    g = std::min<uint64_t>(g, 0x7fffffffull);
    return (unsigned)std::max<uint64_t>(g, 1);
}

// Persistent grid: this many resident workgroup waves per CU (each
// workgroup walks tiles with a grid-stride loop, so twiddles loaded once
// stay in registers); FFTSEG_GRID_MULT=0 gives one workgroup per tile.
constexpr int kDefaultGridMult = 8;
constexpr int kTwoPassGridMult = 32;  // four-step passes without a measured choice

// Four-step passes: the measured best grid by column-tile length (sweeps at
// 8 GiB; 128 resident waves per CU is one workgroup per tile of a 4 GiB
// sub-batch from 128- to 2048-point columns, which beat the persistent
// grids of 16-64 once the tiles' twiddle reads were cut: 2^15 points
// 6.21 ms against 6.45 at 32, 2^20 6.42-6.44 against 6.50-6.78 at 64,
// 2^22 9.40 against 9.63 at 32)
int two_pass_grid_mult(uint64_t n1)
{
    switch (n1) {
    case 128:
    case 256:
    case 512:
    case 1024:
    case 2048:
        return 128;
    default:
        return kTwoPassGridMult;
    }
}

int env_grid_mult()
{
    const char *e = getenv("FFTSEG_GRID_MULT");
    return e ? atoi(e) : kDefaultGridMult;
}

// ---------------------------------------------------------------------------
// plan construction: the choice of kernels, split and sub-batch (host only),
// then the device tables and scratch
int plan_choose(Plan *p, uint64_t n, uint64_t batch, int dir, int forced_variant,
                int forced_split_variants, uint64_t forced_n1, uint64_t max_sub_samples)
{
    p->n = n;
    p->batch = batch;
    p->dir = dir;
    if (hipGetDevice(&p->device) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(FFT_ERR_HIP, "no HIP device available");
    }
    p->grid_mult = env_grid_mult();
    if (n == 1) {
        p->kind = Plan::COPY;
        return set_ok();
    }
    const int tuned = forced_variant >= 0 ? -1 : tuned_variant(n);
    int variant = forced_variant >= 0 ? forced_variant : tuned;
    if (variant < 0)
        variant = 0;
    p->sp = find_single(n, variant);
    if (!p->sp && forced_variant < 0)
        p->sp = find_single(n, 0);
    if (p->sp && forced_variant < 0 && tuned < 0) {
        // a batch that gives the default kernel fewer than two workgroups
        // per CU takes the length's small-batch kernel, if it has one
        const SinglePassDesc *alt = find_small_batch(n);
        const uint64_t groups =
            (batch + (uint64_t)p->sp->segs_per_wg - 1) / (uint64_t)p->sp->segs_per_wg;
        if (alt && groups < 2 * (uint64_t)device_cus(p->device))
            p->sp = alt;
    }
    if (forced_variant >= 0 && !p->sp)
        return set_error(FFT_ERR_INVALID_ARG, "length %llu has no variant %d",
                         (unsigned long long)n, forced_variant);
    if (p->sp) {
        p->kind = Plan::SINGLE;
        if (!getenv("FFTSEG_GRID_MULT"))
            p->grid_mult = tuned_grid_mult(n, p->sp->variant, p->sp->grid_mult);
        return set_ok();
    }
    p->sh = ilog2_ceil(n) / 2 + (ilog2_ceil(n) & 1);
    int cv = 0, rv = 0;
    uint64_t n1 = forced_n1;
    if (forced_split_variants >= 0) {
        cv = forced_split_variants & 0xff;
        rv = (forced_split_variants >> 8) & 0xff;
    } else if (!forced_n1) {
        tuned_split_variants(n, &cv, &rv, &n1);
    }
    bool split = find_split(n, &p->col, &p->row, cv, rv, n1);
    if (!split && n1 && !forced_n1)
        split = find_split(n, &p->col, &p->row, 0, 0, 0);  // a tuned split the library lacks
    if (!split && forced_n1)
        return set_error(FFT_ERR_INVALID_ARG, "length %llu has no split with %llu columns",
                         (unsigned long long)n, (unsigned long long)forced_n1);
    if (!getenv("FFTSEG_GRID_MULT"))
        p->grid_mult = tuned_grid_mult(n, -1,
                                       split ? two_pass_grid_mult((uint64_t)p->col->n1)
                                             : kTwoPassGridMult);
    if (split) {
        p->kind = Plan::FOURSTEP;
        p->n1 = (uint64_t)p->col->n1;
        p->n2 = (uint64_t)p->row->n2;
        // Y in blocks of 16 columns where both tiles have that form
        // (FFTSEG_Y_LAYOUT=plain keeps the input's layout, for comparison)
        const char *yl = getenv("FFTSEG_Y_LAYOUT");
        p->y_blocked = p->col->launch_yblocked && p->row->launch_yblocked &&
                       !(yl && strcmp(yl, "plain") == 0);
        // (one line more: Y may start at the input's offset within a line)
        p->sub_batch = std::min<uint64_t>(batch, max_sub_samples / n);
        p->scratch_bytes = (p->sub_batch * n + kLineSamples) * sizeof(c32);
    } else {
        p->kind = Plan::GENERIC;
        p->radices = generic_radices(n);
        p->sub_batch = std::min<uint64_t>(batch, max_sub_samples / n);
        p->scratch_bytes = 2 * p->sub_batch * n * sizeof(c32);
    }
    if (p->sub_batch == 0)
        return set_error(FFT_ERR_INVALID_ARG,
                         "one %llu-point segment needs more scratch than %llu samples",
                         (unsigned long long)n, (unsigned long long)max_sub_samples);
    return set_ok();
}

int plan_build(Plan *p, uint64_t n, uint64_t batch, int dir, int forced_variant,
               int forced_split_variants, uint64_t forced_n1)
{
    // 4 GiB of complex64 per scratch buffer (the radix-stage path has two);
    // FFTSEG_SUB_SAMPLES caps a sub-batch at fewer samples
    uint64_t max_sub = 1ull << 29;
    if (const char *e = getenv("FFTSEG_SUB_SAMPLES"))
        max_sub = std::max<uint64_t>(1, std::min<uint64_t>(max_sub, strtoull(e, nullptr, 10)));
    int st = plan_choose(p, n, batch, dir, forced_variant, forced_split_variants, forced_n1,
                         max_sub);
    if (st != FFT_OK || p->kind == Plan::COPY)
        return st;
    hipError_t e;
    if (p->kind == Plan::SINGLE) {
        if ((e = upload(root_table(n), &p->tw)) != hipSuccess)
            return e == hipErrorOutOfMemory ? set_error(FFT_ERR_OUT_OF_MEMORY, "twiddles")
                                            : hip_error(e, "twiddle upload");
        return set_ok();
    }
    {
        const uint64_t lo = 1ull << p->sh;
        std::vector<c32> tl(lo), th((n + lo - 1) / lo);
        for (uint64_t j = 0; j < lo; ++j)
            tl[j] = root_forward(j, n);
        for (uint64_t j = 0; j < th.size(); ++j)
            th[j] = root_forward(j * lo, n);
        if ((e = upload(tl, &p->tl)) != hipSuccess || (e = upload(th, &p->th)) != hipSuccess)
            return e == hipErrorOutOfMemory ? set_error(FFT_ERR_OUT_OF_MEMORY, "twiddles")
                                            : hip_error(e, "twiddle upload");
    }
    if (p->kind == Plan::FOURSTEP &&
        ((e = upload(root_table(p->n1), &p->tw)) != hipSuccess ||
         (e = upload(root_table(p->n2), &p->tw2)) != hipSuccess))
        return e == hipErrorOutOfMemory ? set_error(FFT_ERR_OUT_OF_MEMORY, "twiddles")
                                        : hip_error(e, "twiddle upload");
    e = hipMalloc(&p->scratch, p->scratch_bytes);
    if (e != hipSuccess) {
        p->scratch = nullptr;
        (void)hipGetLastError();
        return set_error(FFT_ERR_OUT_OF_MEMORY, "scratch of %zu bytes", p->scratch_bytes);
    }
    return set_ok();
}

int plan_build_real(Plan *p, uint64_t n, uint64_t batch, int dir)
{
    p->n = n;
    p->batch = batch;
    p->dir = dir;
    if (hipGetDevice(&p->device) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(FFT_ERR_HIP, "no HIP device available");
    }
    const uint64_t m = n / 2;
    std::vector<c32> hw(m + 1);
    for (uint64_t k = 0; k <= m; ++k)
        hw[k] = root_forward(k, n);
    hipError_t e;
    p->sp = find_aux(m);
    if (p->sp && p->sp->launch_real) {
        // the split fused into the m-point one-pass kernel
        p->kind = Plan::REAL;
        p->grid_mult = p->sp->grid_mult;
        if ((e = upload(root_table(m), &p->tw)) != hipSuccess ||
            (e = upload(hw, &p->tw2)) != hipSuccess)
            return e == hipErrorOutOfMemory ? set_error(FFT_ERR_OUT_OF_MEMORY, "twiddles")
                                            : hip_error(e, "twiddle upload");
        return set_ok();
    }
    // the m-point complex plan over sub-batches, the split as its own pass
    p->sp = nullptr;
    p->kind = Plan::REAL_SPLIT;
    const uint64_t max_sub_samples = 1ull << 28;  // 2 GiB of complex64 in the split buffer
    p->sub_batch = std::max<uint64_t>(1, std::min<uint64_t>(batch, max_sub_samples / m));
    p->inner = new Plan();
    if (plan_build(p->inner, m, p->sub_batch, dir, -1) != FFT_OK)
        return last_status();
    if ((e = upload(hw, &p->tw2)) != hipSuccess)
        return e == hipErrorOutOfMemory ? set_error(FFT_ERR_OUT_OF_MEMORY, "twiddles")
                                        : hip_error(e, "twiddle upload");
    const size_t zb = p->sub_batch * m * sizeof(c32);
    if ((e = hipMalloc(&p->zbuf, zb)) != hipSuccess) {
        p->zbuf = nullptr;
        (void)hipGetLastError();
        return set_error(FFT_ERR_OUT_OF_MEMORY, "split buffer of %zu bytes", zb);
    }
    p->scratch_bytes = zb + p->inner->scratch_bytes;
    return set_ok();
}

int reject_real(const Plan *p, const char *what)
{
    if (p && is_real(p))
        return set_error(FFT_ERR_INVALID_ARG, "%s takes complex plans; real plans run through"
                         " fft_exec_segments", what);
    return FFT_OK;
}

void plan_free(Plan *p)
{
    if (p->used && p->last_stream_valid)
        (void)hipStreamSynchronize(p->last_stream);
    for (void *q : {p->tw, p->tw2, p->tl, p->th, p->scratch, p->zbuf})
        if (q)
            (void)hipFree(q);
    if (p->inner) {
        plan_free(p->inner);
        delete p->inner;
        p->inner = nullptr;
    }
    stream_state_free(p);
    if (p->graph_exec)
        (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    if (p->capture_stream)
        (void)hipStreamDestroy(p->capture_stream);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    p->capture_stream = nullptr;
    p->tw = p->tw2 = p->tl = p->th = p->scratch = p->zbuf = nullptr;
}

// ---------------------------------------------------------------------------
// argument checks before any device work
int check_device_range(const void *ptr, uint64_t bytes, const char *name)
{
    void *base = nullptr;
    size_t size = 0;
    hipError_t e = hipMemGetAddressRange(&base, &size, const_cast<void *>(ptr));
    if (e == hipSuccess && base) {
        const uintptr_t b = (uintptr_t)base, q = (uintptr_t)ptr;
        if (q < b || q - b > size || bytes > size - (q - b))
            return set_error(FFT_ERR_BOUNDS,
                             "%s: %llu bytes from %p exceed its allocation [%p, +%zu)", name,
                             (unsigned long long)bytes, ptr, base, size);
        return FFT_OK;
    }
    (void)hipGetLastError();
    hipPointerAttribute_t attr;
    std::memset(&attr, 0, sizeof(attr));
    e = hipPointerGetAttributes(&attr, ptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(FFT_ERR_INVALID_ARG, "%s (%p) is not device memory", name, ptr);
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return set_error(FFT_ERR_INVALID_ARG, "%s (%p) is not device memory", name, ptr);
    return FFT_OK;
}

int check_io(const void *in, const void *out, uint64_t bytes)
{
    if (!in || !out)
        return set_error(FFT_ERR_INVALID_ARG, "in/out must not be NULL");
    if (((uintptr_t)in & 7u) || ((uintptr_t)out & 7u))
        return set_error(FFT_ERR_ALIGNMENT, "in/out must be 8-byte aligned");
    if (in != out) {
        const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
        if (a < b + bytes && b < a + bytes)
            return set_error(FFT_ERR_OVERLAP, "in and out overlap without being equal");
    }
    int st = check_device_range(in, bytes, "in");
    if (st != FFT_OK)
        return st;
    if (in != out && (st = check_device_range(out, bytes, "out")) != FFT_OK)
        return st;
    return FFT_OK;
}

// ---------------------------------------------------------------------------
// Identity transform (segment length 1) as a streaming copy.  Each
// workgroup moves one tile of 256 x K accesses, all loads issued before the
// stores, non-temporal; 16-byte accesses when both pointers allow them and
// the sample count is even, else 8-byte ones.  The dynamic LDS of each
// launch is not used: it holds residency at 3 workgroups per CU, which
// measured faster (5.8 TB/s) than the 8 the registers allow (5.4 TB/s) or
// a device-to-device hipMemcpyAsync (4.3 TB/s).
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
constexpr unsigned kCopyLds = 48 * 1024;

template <class T, int K>
__global__ void __launch_bounds__(256)
    identity_copy_kernel(const T *__restrict__ in, T *__restrict__ out, uint64_t n)
{
    extern __shared__ float unused_lds[];
    const uint64_t tile = 256ull * K;
    for (uint64_t base = (uint64_t)blockIdx.x * tile; base < n; base += (uint64_t)gridDim.x * tile) {
        T v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint64_t i = base + threadIdx.x + 256ull * k;
            if (i < n)
                v[k] = __builtin_nontemporal_load(in + i);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint64_t i = base + threadIdx.x + 256ull * k;
            if (i < n)
                __builtin_nontemporal_store(v[k], out + i);
        }
    }
    if (n == UINT64_MAX)  // never true: keeps the (unused) allocation referenced
        unused_lds[threadIdx.x] = 0.f;
}

template <class T, int K>
int identity_copy(const void *in, void *out, uint64_t n, hipStream_t s)
{
    const uint64_t tiles = (n + 256ull * K - 1) / (256ull * K);
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(tiles, 0x7fffffffull));
    hipLaunchKernelGGL((identity_copy_kernel<T, K>), dim3(grid), dim3(256), kCopyLds, s,
                       (const T *)in, (T *)out, n);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? FFT_OK : hip_error(e, "identity copy");
}

// enqueue the transform of `batch` segments (arguments already checked)
int plan_enqueue(Plan *p, const void *in, void *out, uint64_t batch, hipStream_t s)
{
    const uint64_t n = p->n;
    const int dir = p->dir;
    switch (p->kind) {
    case Plan::COPY:
        if (in != out) {
            const bool wide = ((((uintptr_t)in | (uintptr_t)out) & 15u) == 0) && !(batch & 1);
            const int st = wide ? identity_copy<f4v, 8>(in, out, batch / 2, s)
                                : identity_copy<f2v, 16>(in, out, batch, s);
            if (st != FFT_OK)
                return st;
        }
        break;
    case Plan::SINGLE: {
        const SinglePassDesc *d = p->sp;
        const uint64_t groups = (batch + d->segs_per_wg - 1) / d->segs_per_wg;
        // an output base inside a 128-byte line: the kernel with rotated
        // lanes puts each wave's stores back on line boundaries
        const uint64_t out_m = ((uintptr_t)out / sizeof(c32)) % kLineSamples;
        if (out_m) {
            int rv = -1;
            const void *rk[2] = {nullptr, nullptr};
            const sp_rotated_launch_fn rl = rotated_launcher(n, &rv, rk);
            if (rl && rv == d->variant) {
                const unsigned grid = grid_for(rk[dir > 0], d->threads * d->segs_per_wg, groups,
                                               p->device, p->grid_mult);
                rl(dir, in, out, p->tw, batch, (int)((kLineSamples - out_m) % kLineSamples),
                   grid, s);
                break;
            }
        }
        const unsigned grid = grid_for(d->kernel[dir > 0], d->threads * d->segs_per_wg,
                                       groups, p->device, p->grid_mult);
        d->launch(dir, in, out, p->tw, batch, grid, s);
        break;
    }
    case Plan::REAL: {
        const SinglePassDesc *d = p->sp;
        const uint64_t groups = (batch + d->segs_per_wg - 1) / d->segs_per_wg;
        const unsigned grid = grid_for(d->kernel_real[dir > 0], d->threads * d->segs_per_wg,
                                       groups, p->device, p->grid_mult);
        d->launch_real(dir, in, out, p->tw, p->tw2, batch, grid, s);
        break;
    }
    case Plan::REAL_SPLIT: {
        const uint64_t m = n / 2;
        for (uint64_t s0 = 0; s0 < batch; s0 += p->sub_batch) {
            const uint64_t sb = std::min(p->sub_batch, batch - s0);
            int st;
            if (dir < 0) {
                // n floats per row in = m complex; m + 1 complex per row out
                if ((st = plan_enqueue(p->inner, (const c32 *)in + s0 * m, p->zbuf, sb, s)) !=
                        FFT_OK ||
                    (st = real_split_enqueue(dir, p->zbuf, (c32 *)out + s0 * (m + 1), p->tw2, m,
                                             sb, s)) != FFT_OK)
                    return st;
            } else {
                if ((st = real_split_enqueue(dir, (const c32 *)in + s0 * (m + 1), p->zbuf,
                                             p->tw2, m, sb, s)) != FFT_OK ||
                    (st = plan_enqueue(p->inner, p->zbuf, (c32 *)out + s0 * m, sb, s)) != FFT_OK)
                    return st;
            }
        }
        break;
    }
    case Plan::FOURSTEP: {
        const ColumnDesc *cd = p->col;
        const RowDesc *rd = p->row;
        // Segments that start inside a 128-byte line (a base pointer off a
        // line boundary): column blocks start at the first line-aligned
        // column and wrap round, Y sits at the input's offset within a
        // line, and row blocks start where the output's lines do, so both
        // passes move whole lines.  The shifted forms exist for each
        // length's default tiles.
        const uint64_t in_m = ((uintptr_t)in / sizeof(c32)) % kLineSamples,
                       out_m = ((uintptr_t)out / sizeof(c32)) % kLineSamples;
        if (in_m || out_m) {
            const ColumnDesc *cs = cd->launch_shifted ? cd : find_column_shifted(p->n1);
            const RowDesc *rs = rd->launch_shifted ? rd : find_row_shifted(p->n2);
            if (cs && rs && p->n2 % (uint64_t)cs->cols == 0 && p->n1 % (uint64_t)rs->rows == 0) {
                const int sa = (int)((kLineSamples - in_m) % kLineSamples);
                const int sb = (int)((kLineSamples - out_m) % kLineSamples);
                c32 *ybuf = (c32 *)p->scratch + in_m;
                for (uint64_t s0 = 0; s0 < batch; s0 += p->sub_batch) {
                    const uint64_t sbat = std::min(p->sub_batch, batch - s0);
                    const uint64_t ta = sbat * (p->n2 / (uint64_t)cs->cols);
                    const uint64_t tb = sbat * (p->n1 / (uint64_t)rs->rows);
                    const unsigned ga = grid_for(cs->kernel_shifted[dir > 0],
                                                 cs->threads * cs->cols, ta, p->device,
                                                 p->grid_mult);
                    const unsigned gb = grid_for(rs->kernel_shifted[dir > 0],
                                                 rs->threads * rs->rows, tb, p->device,
                                                 p->grid_mult);
                    cs->launch_shifted(dir, (const c32 *)in + s0 * n, ybuf, p->tw, p->tl, p->th,
                                       p->sh, (int)p->n2, sbat, sa, ga, s);
                    rs->launch_shifted(dir, ybuf, (c32 *)out + s0 * n, p->tw2, (int)p->n1, sbat,
                                       sb, gb, s);
                }
                break;
            }
        }
        for (uint64_t s0 = 0; s0 < batch; s0 += p->sub_batch) {
            const uint64_t sb = std::min(p->sub_batch, batch - s0);
            const c32 *x = (const c32 *)in + s0 * n;
            c32 *y = (c32 *)out + s0 * n;
            const uint64_t ta = sb * (p->n2 / (uint64_t)cd->cols);
            const uint64_t tb = sb * (p->n1 / (uint64_t)rd->rows);
            const unsigned ga = grid_for(cd->kernel[dir > 0], cd->threads * cd->cols, ta,
                                         p->device, p->grid_mult);
            const unsigned gb = grid_for(rd->kernel[dir > 0], rd->threads * rd->rows, tb,
                                         p->device, p->grid_mult);
            (p->y_blocked ? cd->launch_yblocked : cd->launch)(dir, x, p->scratch, p->tw, p->tl,
                                                              p->th, p->sh, (int)p->n2, sb,
                                                              ga, s);
            (p->y_blocked ? rd->launch_yblocked : rd->launch)(dir, p->scratch, y, p->tw2,
                                                              (int)p->n1, sb, gb, s);
        }
        break;
    }
    case Plan::GENERIC: {
        const int ns = (int)p->radices.size();
        c32 *bufs[2] = {(c32 *)p->scratch, (c32 *)p->scratch + p->sub_batch * n};
        for (uint64_t s0 = 0; s0 < batch; s0 += p->sub_batch) {
            const uint64_t sb = std::min(p->sub_batch, batch - s0);
            const c32 *x = (const c32 *)in + s0 * n;
            c32 *y = (c32 *)out + s0 * n;
            const uint64_t threads_total = sb * n;
            uint64_t l = 1;
            for (int i = 0; i < ns; ++i) {
                const int r = p->radices[i];
                const void *src = i == 0 ? (const void *)x : (const void *)bufs[(i - 1) & 1];
                void *dst = (i == ns - 1 && !(ns == 1 && in == out)) ? (void *)y
                                                                     : (void *)bufs[i & 1];
                const uint64_t work = threads_total / r;
                const unsigned grid =
                    (unsigned)std::min<uint64_t>((work + 255) / 256, 1ull << 20);
                launch_generic_stage(r, dir, src, dst, p->tl, p->th, p->sh, n, l, sb, grid, s);
                l *= (uint64_t)r;
            }
            if (ns == 1 && in == out) {
                hipError_t e = hipMemcpyAsync(y, bufs[0], sb * n * sizeof(c32),
                                              hipMemcpyDeviceToDevice, s);
                if (e != hipSuccess)
                    return hip_error(e, "fallback copy");
            }
        }
        break;
    }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_error(e, "kernel launch");
    p->used = true;
    p->last_stream = s;
    p->last_stream_valid = true;
    return set_ok();
}

int plan_describe(const Plan *p, std::string &js)
{
    char buf[1024];
    auto rad = [](const int *r, int n) {
        std::string s = "[";
        for (int i = 0; i < n; ++i)
            s += (i ? "," : "") + std::to_string(r[i]);
        return s + "]";
    };
    switch (p->kind) {
    case Plan::COPY:
        snprintf(buf, sizeof buf, "{\"kind\":\"copy\",\"n\":%llu,\"batch\":%llu}",
                 (unsigned long long)p->n, (unsigned long long)p->batch);
        break;
    case Plan::SINGLE:
        snprintf(buf, sizeof buf,
                 "{\"kind\":\"single_pass\",\"n\":%llu,\"batch\":%llu,\"direction\":%d,"
                 "\"variant\":%d,\"radices\":%s,\"threads_per_segment\":%d,"
                 "\"segments_per_workgroup\":%d,\"lds_pad_shift\":%d,\"nontemporal\":%d,"
                 "\"lds_bytes\":%d,\"shuffle_exchange\":%d,\"grid_mult\":%d,"
                 "\"scratch_bytes\":0}",
                 (unsigned long long)p->n, (unsigned long long)p->batch, p->dir,
                 p->sp->variant, rad(p->sp->radices, p->sp->nrad).c_str(), p->sp->threads,
                 p->sp->segs_per_wg, p->sp->pad_shift, p->sp->nontemporal,
                 p->sp->lds_bytes, p->sp->shuffle, p->grid_mult);
        break;
    case Plan::FOURSTEP:
        snprintf(buf, sizeof buf,
                 "{\"kind\":\"four_step\",\"n\":%llu,\"batch\":%llu,\"direction\":%d,"
                 "\"n1\":%llu,\"n2\":%llu,\"radices_n1\":%s,\"radices_n2\":%s,"
                 "\"columns_per_workgroup\":%d,\"rows_per_workgroup\":%d,"
                 "\"column_variant\":%d,\"row_variant\":%d,\"grid_mult\":%d,"
                 "\"lds_bytes\":[%d,%d],\"sub_batch\":%llu,\"scratch_bytes\":%zu,"
                 "\"y_blocked\":%d}",
                 (unsigned long long)p->n, (unsigned long long)p->batch, p->dir,
                 (unsigned long long)p->n1, (unsigned long long)p->n2,
                 rad(p->col->radices, p->col->nrad).c_str(),
                 rad(p->row->radices, p->row->nrad).c_str(), p->col->cols, p->row->rows,
                 p->col->variant, p->row->variant, p->grid_mult,
                 p->col->lds_bytes, p->row->lds_bytes, (unsigned long long)p->sub_batch,
                 p->scratch_bytes, (int)p->y_blocked);
        break;
    case Plan::REAL:
        snprintf(buf, sizeof buf,
                 "{\"kind\":\"real\",\"n\":%llu,\"batch\":%llu,\"direction\":%d,"
                 "\"complex_length\":%llu,\"radices\":%s,\"threads_per_segment\":%d,"
                 "\"segments_per_workgroup\":%d,\"grid_mult\":%d,\"scratch_bytes\":0}",
                 (unsigned long long)p->n, (unsigned long long)p->batch, p->dir,
                 (unsigned long long)(p->n / 2), rad(p->sp->radices, p->sp->nrad).c_str(),
                 p->sp->threads, p->sp->segs_per_wg, p->grid_mult);
        break;
    case Plan::REAL_SPLIT: {
        std::string inner;
        plan_describe(p->inner, inner);
        js = "{\"kind\":\"real\",\"n\":" + std::to_string(p->n) +
             ",\"batch\":" + std::to_string(p->batch) + ",\"direction\":" +
             std::to_string(p->dir) + ",\"complex_length\":" + std::to_string(p->n / 2) +
             ",\"separate_split\":1,\"sub_batch\":" + std::to_string(p->sub_batch) +
             ",\"scratch_bytes\":" + std::to_string(p->scratch_bytes) +
             ",\"complex_plan\":" + inner + "}";
        return FFT_OK;
    }
    case Plan::GENERIC:
        snprintf(buf, sizeof buf,
                 "{\"kind\":\"radix_stages\",\"n\":%llu,\"batch\":%llu,\"direction\":%d,"
                 "\"radices\":%s,\"sub_batch\":%llu,\"scratch_bytes\":%zu}",
                 (unsigned long long)p->n, (unsigned long long)p->batch, p->dir,
                 rad(p->radices.data(), (int)p->radices.size()).c_str(),
                 (unsigned long long)p->sub_batch, p->scratch_bytes);
        break;
    }
    js = buf;
    return FFT_OK;
}

int validate_create(uint64_t n, uint64_t batch, int dir)
{
    if (n == 0)
        return set_error(FFT_ERR_INVALID_ARG, "segment_len must be > 0");
    if (batch == 0)
        return set_error(FFT_ERR_INVALID_ARG, "batch must be > 0");
    if (dir != FFT_FORWARD && dir != FFT_INVERSE)
        return set_error(FFT_ERR_INVALID_ARG, "direction must be -1 or +1 (got %d)", dir);
    if (n > (1ull << 24))
        return set_error(FFT_ERR_UNSUPPORTED_LENGTH, "segment_len %llu exceeds 2^24",
                         (unsigned long long)n);
    if (!smooth235(n))
        return set_error(FFT_ERR_UNSUPPORTED_LENGTH,
                         "segment_len %llu has a prime factor other than 2, 3, 5",
                         (unsigned long long)n);
    if (batch > SIZE_MAX / 8 / n)
        return set_error(FFT_ERR_INVALID_ARG, "batch * segment_len * 8 overflows size_t");
    return FFT_OK;
}

int factorize(uint64_t n, int *radices, int max)
{
    if (n == 0)
        return set_error(FFT_ERR_INVALID_ARG, "n must be > 0");
    if (n > (1ull << 24) || !smooth235(n))
        return set_error(FFT_ERR_UNSUPPORTED_LENGTH, "unsupported length %llu",
                         (unsigned long long)n);
    std::vector<int> r;
    int v = tuned_variant(n);
    const SinglePassDesc *d = find_single(n, v < 0 ? 0 : v);
    if (!d)
        d = find_single(n, 0);
    if (d)
        r.assign(d->radices, d->radices + d->nrad);
    else
        r = generic_radices(n);
    if (!radices && max != 0)
        return set_error(FFT_ERR_INVALID_ARG, "radices is NULL");
    for (int i = 0; i < (int)r.size() && i < max; ++i)
        radices[i] = r[i];
    set_ok();
    return (int)r.size();
}

}  // namespace fftseg

// ===========================================================================
// C entry points
using namespace fftseg;

#define FFT_GUARD_BEGIN try {
#define FFT_GUARD_END(ret)                                                         \
    }                                                                              \
    catch (const std::bad_alloc &)                                                 \
    {                                                                              \
        set_error(FFT_ERR_OUT_OF_MEMORY, "host allocation failed");                \
        return ret;                                                                \
    }                                                                              \
    catch (...)                                                                    \
    {                                                                              \
        set_error(FFT_ERR_INVALID_ARG, "internal error");                          \
        return ret;                                                                \
    }

static fft_plan_t create_impl(size_t segment_len, size_t batch, int direction, int variant,
                              int split = -1)
{
    if (validate_create(segment_len, batch, direction) != FFT_OK)
        return nullptr;
    Plan *p = new Plan();
    if (plan_build(p, segment_len, batch, direction, variant, split) != FFT_OK) {
        const int st = last_status();
        std::string msg = last_message();
        plan_free(p);
        delete p;
        set_error(st, "%s", msg.c_str());
        return nullptr;
    }
    return reinterpret_cast<fft_plan_t>(p);
}

extern "C" fft_plan_t fft_plan_create(size_t segment_len, size_t batch, int direction)
{
    FFT_GUARD_BEGIN
    return create_impl(segment_len, batch, direction, -1);
    FFT_GUARD_END(nullptr)
}

extern "C" fft_plan_t fft_plan_create_variant(size_t segment_len, size_t batch,
                                              int direction, int variant)
{
    FFT_GUARD_BEGIN
    if (variant < 0) {
        set_error(FFT_ERR_INVALID_ARG, "variant must be >= 0");
        return nullptr;
    }
    return create_impl(segment_len, batch, direction, variant);
    FFT_GUARD_END(nullptr)
}

extern "C" fft_plan_t fft_plan_create_real(size_t segment_len, size_t batch, int direction)
{
    FFT_GUARD_BEGIN
    if (validate_create(segment_len, batch, direction) != FFT_OK)
        return nullptr;
    if (segment_len < 4 || segment_len % 2) {
        set_error(FFT_ERR_UNSUPPORTED_LENGTH, "real segments need an even length >= 4 (got %zu)",
                  segment_len);
        return nullptr;
    }
    Plan *p = new Plan();
    if (plan_build_real(p, segment_len, batch, direction) != FFT_OK) {
        const int st = last_status();
        std::string msg = last_message();
        plan_free(p);
        delete p;
        set_error(st, "%s", msg.c_str());
        return nullptr;
    }
    return reinterpret_cast<fft_plan_t>(p);
    FFT_GUARD_END(nullptr)
}

extern "C" int fft_split_info(size_t n, size_t *n1, size_t *n2, int *ncol, int *nrow)
{
    FFT_GUARD_BEGIN
    int c = 0, r = 0;
    const ColumnDesc *cd = nullptr;
    const RowDesc *rd = nullptr;
    const bool two = n > 0 && variant_count(n) == 0 && find_split(n, &cd, &rd, 0, 0);
    if (two)
        split_variant_counts(n, &c, &r);
    if (n1)
        *n1 = two ? (size_t)cd->n1 : 0;
    if (n2)
        *n2 = two ? (size_t)rd->n2 : 0;
    if (ncol)
        *ncol = c;
    if (nrow)
        *nrow = r;
    set_ok();
    return two ? 1 : 0;
    FFT_GUARD_END(FFT_ERR_INVALID_ARG)
}

extern "C" fft_plan_t fft_plan_create_split(size_t segment_len, size_t batch, int direction,
                                            int column_variant, int row_variant)
{
    FFT_GUARD_BEGIN
    int c = 0, r = 0;
    if (validate_create(segment_len, batch, direction) != FFT_OK)
        return nullptr;
    if (variant_count(segment_len) != 0 || !split_variant_counts(segment_len, &c, &r)) {
        set_error(FFT_ERR_INVALID_ARG, "length %zu is not a two-pass length", segment_len);
        return nullptr;
    }
    if (column_variant < 0 || column_variant >= c || row_variant < 0 || row_variant >= r) {
        set_error(FFT_ERR_INVALID_ARG, "tile variants (%d, %d) outside [0, %d) x [0, %d)",
                  column_variant, row_variant, c, r);
        return nullptr;
    }
    return create_impl(segment_len, batch, direction, -1, column_variant | (row_variant << 8));
    FFT_GUARD_END(nullptr)
}

extern "C" int fft_variant_count(size_t n)
{
    set_ok();
    return variant_count(n);
}

extern "C" int fft_exec_segments_n(fft_plan_t plan, const void *in, void *out,
                                   size_t batch, void *stream)
{
    FFT_GUARD_BEGIN
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p)
        return set_error(FFT_ERR_INVALID_ARG, "plan is NULL");
    if (batch == 0 || batch > p->batch)
        return set_error(FFT_ERR_INVALID_ARG, "batch %zu outside [1, %llu]", batch,
                         (unsigned long long)p->batch);
    int st;
    if (is_real(p)) {
        // forward: n floats in, n/2+1 complex out; inverse the other way round
        const uint64_t rb = (uint64_t)batch * p->n * sizeof(float);
        const uint64_t cb = (uint64_t)batch * (p->n / 2 + 1) * sizeof(c32);
        const uint64_t ib = p->dir < 0 ? rb : cb, ob = p->dir < 0 ? cb : rb;
        if (!in || !out)
            return set_error(FFT_ERR_INVALID_ARG, "in/out must not be NULL");
        if (((uintptr_t)in & 7u) || ((uintptr_t)out & 7u))
            return set_error(FFT_ERR_ALIGNMENT, "in/out must be 8-byte aligned");
        const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
        if (a < b + ob && b < a + ib)
            return set_error(FFT_ERR_OVERLAP, "real transforms run out of place: in and out"
                             " overlap");
        if ((st = check_device_range(in, ib, "in")) != FFT_OK ||
            (st = check_device_range(out, ob, "out")) != FFT_OK)
            return st;
    } else {
        const uint64_t bytes = (uint64_t)batch * p->n * sizeof(c32);
        st = check_io(in, out, bytes);
        if (st != FFT_OK)
            return st;
    }
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess)
        return hip_error(hipGetLastError(), "hipGetDevice");
    if (cur != p->device && hipSetDevice(p->device) != hipSuccess)
        return hip_error(hipGetLastError(), "hipSetDevice");
    st = plan_enqueue(p, in, out, batch, (hipStream_t)stream);
    if (cur != p->device)
        (void)hipSetDevice(cur);
    return st;
    FFT_GUARD_END(FFT_ERR_INVALID_ARG)
}

extern "C" int fft_exec_segments(fft_plan_t plan, const void *in, void *out, void *stream)
{
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p)
        return set_error(FFT_ERR_INVALID_ARG, "plan is NULL");
    return fft_exec_segments_n(plan, in, out, p->batch, stream);
}

extern "C" int fft_plan_destroy(fft_plan_t plan)
{
    FFT_GUARD_BEGIN
    Plan *p = reinterpret_cast<Plan *>(plan);
    if (!p)
        return set_ok();
    plan_free(p);
    delete p;
    return set_ok();
    FFT_GUARD_END(FFT_ERR_INVALID_ARG)
}

extern "C" int fft_last_status(void) { return last_status(); }
extern "C" const char *fft_last_error(void) { return last_message(); }

extern "C" int fft_plan_factorize(size_t n, int *radices, int max)
{
    FFT_GUARD_BEGIN
    return factorize(n, radices, max);
    FFT_GUARD_END(FFT_ERR_INVALID_ARG)
}

extern "C" int fft_plan_describe(fft_plan_t plan, char *buf, size_t len)
{
    FFT_GUARD_BEGIN
    const Plan *p = reinterpret_cast<const Plan *>(plan);
    if (!p)
        return set_error(FFT_ERR_INVALID_ARG, "plan is NULL");
    std::string js;
    plan_describe(p, js);
    if (buf && len) {
        const size_t k = std::min(len - 1, js.size());
        std::memcpy(buf, js.data(), k);
        buf[k] = 0;
    }
    set_ok();
    return (int)js.size();
    FFT_GUARD_END(FFT_ERR_INVALID_ARG)
}

extern "C" size_t fft_plan_scratch_bytes(fft_plan_t plan)
{
    const Plan *p = reinterpret_cast<const Plan *>(plan);
    if (!p) {
        set_error(FFT_ERR_INVALID_ARG, "plan is NULL");
        return 0;
    }
    set_ok();
    return p->scratch_bytes;
}
