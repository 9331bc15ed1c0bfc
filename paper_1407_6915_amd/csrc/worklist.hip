// Uneven batches in two persistent launches (fft_worklist_*).
//
// The paper batches the fixed-length segments of one block into one plan
// (Sec. III); here segments of different lengths, at arbitrary offsets, go
// through one persistent kernel.  The host compiles the entries into tasks,
// each filling one 256-thread workgroup tile:
//   single pass  up to S whole segments of one length (S = 16 for 256, ...)
//   two pass     one column tile (pass A) or row tile (pass B) of a
//                65536-point segment (256 x 256)
// Workgroups claim tasks (a few at a time) through an atomic cursor in list
// order.  The kernel runs twice: first over every pass-A task and every
// single-pass task (longest first), then over every pass-B task.  The
// kernel boundary orders a segment's second pass after its first, so no
// workgroup waits on another and no device-scope fence is needed (on this
// chip such a release/acquire pair writes back or invalidates a whole XCD's
// L2, which costs far more than the launch).
// 16384-point segments are "wide": their one-pass tile (512 threads, split
// LDS exchanges) does not fit the 256-thread workgroup, so they run in a
// launch of their own between the two, one segment per workgroup tile,
// instead of as two passes of 128 x 128.
// 2^20-point segments leave the work-list kernel altogether: a 1024-point
// column tile that fits its workgroup (256 threads, 35 KB of LDS) holds only
// 4 columns, 32-byte pieces of each line, and ran at a quarter of the plain
// four-step kernels' rate.  Each run of consecutive 2^20-point entries whose
// inputs and outputs advance by one segment goes through a four-step plan of
// that length instead (its 16-column radix-32 tiles, 512 threads, and its
// line-shifted forms for runs that start inside a line).
#include "fftseg.h"
#include "runtime.hpp"
#include "tile.hpp"

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace fftseg {
namespace wl {

enum Kind : uint32_t {
    K256,
    K1000,
    K1024,
    K1536,
    K4096,
    K6000,
    K16384W,
    K65536A,
    K65536B,
    K1M,  // 2^20: through the four-step plan, no tasks
    KCOUNT
};

struct Item {          // one segment
    uint64_t in_off;   // samples from in_base
    uint64_t out_off;  // samples from out_base
    uint64_t y_off;    // two-pass: samples from the scratch base
};

struct Task {
    uint32_t kind;
    uint32_t item;    // single pass: first item; two pass: the segment's item
    uint32_t count;   // single pass: segments in the task (whole tiles of S)
    uint32_t tile;    // two pass: first column/row block
    uint32_t ntiles;  // two pass: blocks in the task
    uint32_t shift;   // two pass: column (pass A) / row (pass B) where block 0 starts
    uint32_t pad[2];
};

struct Tables {      // per kind, device pointers
    const c32 *tw;   // W_M of the tile transform
    const c32 *tl, *th;
    int sh;
    int pad;
};

constexpr int kThreads = 256;

// routine shapes (streamed global access, twiddles reloaded per task and
// read in pairs)
using Sh256 = Shape<256, 16, Radices<16, 16>>;
using P256 = SinglePassPolicy<Sh256, 16, 4, true, 0, false, 1, false, false, false, false, true>;
using Sh1000 = Shape<1000, 100, Radices<10, 10, 10>>;
using P1000 = SinglePassPolicy<Sh1000, 2, 4, true, 0, true>;
using Sh1024 = Shape<1024, 64, Radices<16, 16, 4>>;
using P1024 = SinglePassPolicy<Sh1024, 4, 4, true, 0, false, 1, false, false, false, false, true>;
using Sh1536 = Shape<1536, 96, Radices<16, 16, 6>>;
using P1536 = SinglePassPolicy<Sh1536, 2, 4, true, 0, true, 1, false, false, false, false, true>;
using Sh4096 = Shape<4096, 256, Radices<16, 16, 16>>;
using P4096 = SinglePassPolicy<Sh4096, 1, 4, true, 0, false, 1, false, false, false, false, true>;
using Sh6000 = Shape<6000, 256, Radices<16, 15, 25>>;
// 6000-point tiles exchange the real parts, then the imaginary parts, through
// LDS: half the space (25.5 instead of 51 KB), so the 34.8 KB of the 4096-point
// and two-pass tiles sets the kernel's LDS and 4 workgroups fit a CU instead
// of 3 (4-5 % faster on a mixed list of every kind; lists of 4096-point
// segments alone are about 5 % slower under the tighter register budget)
using P6000 = SinglePassPolicy<Sh6000, 1, 4, true, 0, false, 1, false, false, false, true, true>;
using Sh256c = Shape<256, 16, Radices<16, 16>>;
using PCol256 = ColumnPolicy<Sh256c, 16, 4, true, 0, false, 1, false, false, true, true, true>;
using PRow256 = RowPolicy<Sh256c, 16, 4, true, 0, false, 1, false, false, true, true>;

constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kLdsElems =
    cmax(cmax(cmax(P256::kLdsElems, P1000::kLdsElems), cmax(P1024::kLdsElems, P1536::kLdsElems)),
         cmax(cmax(P4096::kLdsElems, lds_c32<P6000::kLdsElems, P6000::kSplit>()),
              cmax(PCol256::kLdsElems, PRow256::kLdsElems)));

static_assert(4 * (kLdsElems * sizeof(c32) + sizeof(uint32_t)) <= 160 * 1024,
              "four workgroups must fit the 160 KB of LDS of a CU");
static_assert(P256::kThreads <= kThreads && P1000::kThreads <= kThreads &&
                  P1024::kThreads <= kThreads && P1536::kThreads <= kThreads &&
                  P4096::kThreads <= kThreads && P6000::kThreads <= kThreads,
              "single-pass routines must fit the workgroup");
static_assert(PCol256::kThreads == kThreads && PRow256::kThreads == kThreads,
              "two-pass routines use the whole workgroup");

// tasks claimed per atomic on the cursor: 2 was 3 % faster on a mixed list
// than 4 (with one 65536-point block per task, more of a segment's blocks run
// at once) and than 1 (twice the atomics)
constexpr uint32_t kClaim = 2;
// grid of the wide launch: one workgroup per 16384-point segment (its tile
// re-reads its twiddles per segment, so a persistent grid keeps nothing in
// registers; 0 = no cap, as FFTSEG_GRID_MULT=0)
constexpr int kWideGridMult = 0;
// grid of the two work-list launches: 4 x the resident workgroups (the
// extra ones start as the first finish and claim what is left; measured
// 2-3 % faster on the uneven workload than exactly one resident wave)
constexpr int kWorkListGridMult = 4;
// samples per 128-byte cache line
constexpr uint64_t kLine = 16;

// a value the compiler must recompute per loop iteration (see below)
__device__ __forceinline__ int opaque(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// Every loop below passes an opaque copy of the lane index down: the
// routines of all kinds are inlined into one kernel, and lane-derived
// addresses lifted out of the loops would all stay live at once.
template <class Sh, class Pol, int D>
__device__ __forceinline__ void run_single(c32 *lds, const Tables &tb, const Task &t,
                                           const Item *__restrict__ items, const c32 *in,
                                           c32 *out, int tid0)
{
    for (uint32_t first = 0; first < t.count; first += Pol::S) {
        const int tid = opaque(tid0);
        const int slot = tid / Sh::T;
        const bool valid = Pol::active(tid) && first + slot < t.count;
        const Item it = valid ? items[t.item + first + slot] : Item{0, 0, 0};
        single_tile<Sh, Pol, D>(lds, tb.tw, tid, tid, in + it.in_off, out + it.out_off, valid);
    }
}

template <class Sh, class Pol, int D>
__device__ __forceinline__ void run_columns(c32 *lds, const Tables &tb, const Task &t,
                                            const Item *__restrict__ items, const c32 *in,
                                            c32 *ybuf, int tid0, int n2)
{
    // LDS twiddle buffers alternate over the task's tiles; the barrier that
    // ends every task orders the next task's first write after this one's
    // last reads
    const Item it = items[t.item];
    for (uint32_t k = 0; k < t.ntiles; ++k) {
        const int tid = opaque(tid0);
        column_tile<Sh, Pol, D>(lds, tb.tw, tb.tl, tb.th, tb.sh, tid, tid, in + it.in_off,
                                ybuf + it.y_off, (int)((t.tile + k) * Pol::C + t.shift), n2,
                                (int)(k & 1));
    }
}

template <class Sh, class Pol, int D>
__device__ __forceinline__ void run_rows(c32 *lds, const Tables &tb, const Task &t,
                                         const Item *__restrict__ items, const c32 *ybuf,
                                         c32 *out, int tid0, int n1)
{
    const Item it = items[t.item];
    for (uint32_t k = 0; k < t.ntiles; ++k) {
        const int tid = opaque(tid0);
        row_tile<Sh, Pol, D>(lds, tb.tw, tid, tid, ybuf + it.y_off, out + it.out_off,
                             (int)((t.tile + k) * Pol::C + t.shift), n1);
    }
}

template <int D>
// 4 workgroups per CU: 128 VGPRs a lane at most
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
    worklist_kernel(const Task *__restrict__ tasks, uint32_t n_tasks,
                    const Item *__restrict__ items, const Tables *__restrict__ tables,
                    const c32 *in, c32 *out, c32 *ybuf, uint32_t *cursor)
{
    __shared__ c32 lds[kLdsElems];
    __shared__ uint32_t s_task;
    for (;;) {
        // lane index made opaque per task: keeps the compiler from lifting
        // every routine's lane-derived addresses out of the loop (they
        // would all stay live across tasks)
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        if (tid == 0)
            s_task = atomicAdd(cursor, kClaim);
        __syncthreads();
        const uint32_t base = s_task;
        __syncthreads();
        if (base >= n_tasks)
            break;
        const uint32_t end = base + kClaim < n_tasks ? base + kClaim : n_tasks;
        for (uint32_t ti = base; ti < end; ++ti) {
            tid = opaque(tid);
            const Task t = tasks[ti];
            const Tables tb = tables[t.kind];
            switch (t.kind) {
            case K256: run_single<Sh256, P256, D>(lds, tb, t, items, in, out, tid); break;
            case K1000: run_single<Sh1000, P1000, D>(lds, tb, t, items, in, out, tid); break;
            case K1024: run_single<Sh1024, P1024, D>(lds, tb, t, items, in, out, tid); break;
            case K1536: run_single<Sh1536, P1536, D>(lds, tb, t, items, in, out, tid); break;
            case K4096: run_single<Sh4096, P4096, D>(lds, tb, t, items, in, out, tid); break;
            case K6000: run_single<Sh6000, P6000, D>(lds, tb, t, items, in, out, tid); break;
            case K65536A:
                run_columns<Sh256c, PCol256, D>(lds, tb, t, items, in, ybuf, tid, 256);
                break;
            case K65536B:
                run_rows<Sh256c, PRow256, D>(lds, tb, t, items, ybuf, out, tid, 256);
                break;
            default: break;
            }
            __syncthreads();  // LDS and s_task reuse by the next task
        }
    }
}

// The wide tiles: one 16384-point segment per 512-thread workgroup tile,
// items [0, n) of the wide range, grid-stride (every wide tile is the same
// size, so no cursor is needed).
using ShWide = Shape<16384, 512, Radices<16, 32, 32>>;
using PWide =
    SinglePassPolicy<ShWide, 1, 4, true, 0, false, 4, false, false, false, true, true>;

template <int D>
__global__ void __launch_bounds__(PWide::kThreads) __attribute__((amdgpu_waves_per_eu(4)))
    worklist_wide_kernel(const Item *__restrict__ items, uint32_t n, const c32 *__restrict__ tw,
                         const c32 *in, c32 *out)
{
    __shared__ float lds[PWide::kLdsElems];
    using S0 = Stage<ShWide, 0, 1>;
    for (uint32_t g = blockIdx.x; g < n; g += gridDim.x) {
        const int tid = opaque(threadIdx.x);  // as in single_pass_split_kernel
        const Item it = items[g];
        const c32 *x = in + it.in_off;
        const typename PWide::Ctx ctx{out + it.out_off, true};
        c32 v[ShWide::kMaxE];
        st_gather<S0, ShWide>(v, tid, [&](int i) { return gload<true>(x + i); });
        tile_run_split<ShWide, PWide, D, 0, 1>(v, lds, tw, tid, threadIdx.x, ctx);
    }
}

// zero the two launches' cursors (a kernel rather than a memset so the whole
// launch sequence can be captured into a graph)
__global__ void __launch_bounds__(256) clear_kernel(uint32_t *ctl, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        ctl[i] = 0u;
}

// Task sizes: a single-pass task is `group` whole tiles of S segments
// (about 64 KiB of input); a two-pass segment's `tiles` column (row) blocks
// are cut into tasks of `group` blocks.  Fewer, larger tasks keep the
// cursor's atomics off the critical path, but a 65536-point segment's blocks
// go one per task: workgroups that claim neighbouring tasks then transform
// the blocks of one segment side by side, and its 128-byte pieces of each
// 2 KB row or column run reach memory close together in time (8 blocks per
// task, walked by one workgroup in turn, were 3-5 % slower on the whole).
struct LengthInfo {
    uint32_t n;
    bool two_pass;
    bool wide;    // one-pass tile of its own launch (worklist_wide_kernel)
    Kind a, b;    // single pass: a only
    int per_tile; // single pass: segments per tile (S); two pass: blocks per pass
    int group;    // tiles (blocks) per task
    int n1, n2;
    bool planned; // runs through a four-step plan, not the work-list kernel
};

const LengthInfo kLengths[] = {
    {256, false, false, K256, K256, P256::S, 2, 0, 0},
    {1000, false, false, K1000, K1000, P1000::S, 4, 0, 0},
    {1024, false, false, K1024, K1024, P1024::S, 2, 0, 0},
    {1536, false, false, K1536, K1536, P1536::S, 3, 0, 0},
    {4096, false, false, K4096, K4096, P4096::S, 2, 0, 0},
    {6000, false, false, K6000, K6000, P6000::S, 2, 0, 0},
    {16384, false, true, K16384W, K16384W, 1, 1, 0, 0},
    {65536, true, false, K65536A, K65536B, 256 / PCol256::C, 1, 256, 256},
    {1u << 20, true, false, K1M, K1M, 0, 0, 1024, 1024, true},
};

const LengthInfo *length_info(uint32_t n)
{
    for (const LengthInfo &l : kLengths)
        if (l.n == n)
            return &l;
    return nullptr;
}

// Route of a one-pass length: 0 = tiles of the work-list kernel, 1 + k =
// a launch of its own through the k-th indexed one-pass kernel of the
// length (its dense kernel over the listed offsets), at *grid_mult resident
// workgroup waves per CU (0: the candidate's own).  A tuned route wins;
// otherwise every length with an indexed kernel takes candidate 0.
int route_of(uint32_t n, int *grid_mult)
{
    *grid_mult = 0;
    int cnt = 0;
    const SinglePassDesc *t = indexed_table(n, &cnt);
    int g = 0;
    const int r = tuned_wl_route(n, &g);
    if (r == 0 || (r > 0 && r <= cnt && t[r - 1].launch_indexed)) {
        *grid_mult = g;
        return r;
    }
    return cnt > 0 && t[0].launch_indexed ? 1 : 0;
}

// Route of a two-pass length: 0 = column and row tasks of the work-list
// kernel, 1 = the two passes over the listed segments as launches of their
// own (the plan's tiles, indexed).  Tuned, else 0: on the uneven workload
// (65536-point segments packed at unaligned offsets among others) the
// tasks took 12.1 ms and the indexed passes 13.7.
int route_two_pass(uint32_t n, int *grid_mult)
{
    *grid_mult = 0;
    const ColumnDesc *c = nullptr;
    const RowDesc *r = nullptr;
    const bool have = indexed_four_step(n, &c, &r);
    int g = 0;
    const int t = tuned_wl_route(n, &g);
    if (t == 0 || (t == 1 && have)) {
        *grid_mult = g;
        return t;
    }
    return 0;
}

}  // namespace wl

struct WorkList {
    int dir = -1;
    int device = 0;
    // per-kind twiddle tables, built once
    wl::Tables *d_tables = nullptr;
    std::vector<void *> table_mem;
    size_t table_bytes = 0;
    // the current entries
    uint64_t n_items = 0;
    uint64_t max_in = 0, max_out = 0;  // highest sample touched (+1)
    bool in_place_ok = false;          // outputs hit no other entry's input
    uint32_t n_tasks = 0, n_first = 0;  // tasks; of which run in the first launch
    uint32_t n_two_pass = 0;            // two-pass segments
    uint32_t wide_first = 0, n_wide = 0;  // items of the wide launch
    unsigned wide_grid = 1;
    const c32 *wide_tw = nullptr;        // its twiddle table (one of table_mem)
    uint64_t counts[wl::KCOUNT] = {};
    // one-pass lengths routed to indexed launches of their own: each covers
    // items [first, first + count) of the item array
    struct IndexedRun {
        const SinglePassDesc *d;
        uint32_t kind, first, count;
        int grid_mult;  // 0: the candidate's own
        unsigned grid;
        bool operator==(const IndexedRun &o) const
        {
            return d == o.d && kind == o.kind && first == o.first && count == o.count &&
                   grid == o.grid;
        }
    };
    std::vector<IndexedRun> indexed;
    // the two-pass length routed to indexed passes of its own: items
    // [first, first + count), Y at count * (n + 16) samples of d_y
    struct IndexedTwoPass {
        const ColumnDesc *col = nullptr;
        const RowDesc *row = nullptr;
        uint32_t n = 0, first = 0, count = 0;
        int grid_mult = 0;
        unsigned grid_a = 0, grid_b = 0;
        bool operator==(const IndexedTwoPass &o) const
        {
            return col == o.col && row == o.row && n == o.n && first == o.first &&
                   count == o.count && grid_a == o.grid_a && grid_b == o.grid_b;
        }
    } two_pass_idx;
    std::vector<wl::Tables> h_tables;  // host copy of d_tables
    // planned lengths: runs of consecutive entries, and the plan they go
    // through (built for at least the longest run)
    struct PlanRun {
        uint64_t in_off, out_off, count;
    };
    std::vector<PlanRun> plan_runs;
    uint64_t plan_len = 0, plan_max_run = 0;
    Plan *plan = nullptr;
    // false while the entries compiled last lack their device arrays or
    // plan (a reset that failed after replacing them): nothing may run
    bool ready = false;
    uint64_t samples = 0;
    size_t y_bytes = 0;
    unsigned grid = 1;
    // device arrays, grown on demand
    wl::Task *d_tasks = nullptr;
    size_t cap_tasks = 0;
    wl::Item *d_items = nullptr;
    size_t cap_items = 0;
    uint32_t *d_ctl = nullptr;
    size_t cap_ctl = 0;
    c32 *d_y = nullptr;
    size_t cap_y = 0;
    // pinned staging of the task/item upload
    void *h_stage = nullptr;
    size_t cap_stage = 0;
    hipEvent_t stage_done = nullptr;
    // graph replay: the captured launches hold every value of LaunchKey
    // as a fixed argument, so the graph is replayed only while the current
    // entries give the same key
    struct LaunchKey {
        const void *in = nullptr;
        void *out = nullptr;
        uint32_t n_tasks = 0, n_first = 0, wide_first = 0, n_wide = 0;
        unsigned grid = 0, wide_grid = 0;
        const void *tasks = nullptr, *items = nullptr, *ctl = nullptr, *y = nullptr;
        const Plan *plan = nullptr;
        std::vector<PlanRun> runs;
        std::vector<IndexedRun> indexed;
        IndexedTwoPass two_pass_idx;
        bool operator==(const LaunchKey &o) const
        {
            if (!(two_pass_idx == o.two_pass_idx))
                return false;
            if (in != o.in || out != o.out || n_tasks != o.n_tasks || n_first != o.n_first ||
                wide_first != o.wide_first || n_wide != o.n_wide || grid != o.grid ||
                wide_grid != o.wide_grid || tasks != o.tasks || items != o.items ||
                ctl != o.ctl || y != o.y || plan != o.plan || runs.size() != o.runs.size() ||
                !(indexed == o.indexed))
                return false;
            for (size_t i = 0; i < runs.size(); ++i)
                if (runs[i].in_off != o.runs[i].in_off || runs[i].out_off != o.runs[i].out_off ||
                    runs[i].count != o.runs[i].count)
                    return false;
            return true;
        }
    };
    LaunchKey key(const void *in, void *out) const
    {
        LaunchKey k;
        k.in = in;
        k.out = out;
        k.n_tasks = n_tasks;
        k.n_first = n_first;
        k.wide_first = wide_first;
        k.n_wide = n_wide;
        k.grid = grid;
        k.wide_grid = wide_grid;
        k.tasks = d_tasks;
        k.items = d_items;
        k.ctl = d_ctl;
        k.y = d_y;
        k.plan = plan;
        k.runs = plan_runs;
        k.indexed = indexed;
        k.two_pass_idx = two_pass_idx;
        return k;
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    LaunchKey graph_key;
    hipStream_t capture_stream = nullptr;

    void drop_graph()
    {
        if (graph_exec)
            (void)hipGraphExecDestroy(graph_exec);
        if (graph)
            (void)hipGraphDestroy(graph);
        graph_exec = nullptr;
        graph = nullptr;
    }

    ~WorkList()
    {
        drop_graph();
        if (capture_stream)
            (void)hipStreamDestroy(capture_stream);
        if (stage_done)
            (void)hipEventDestroy(stage_done);
        if (h_stage)
            (void)hipHostFree(h_stage);
        for (void *p : {(void *)d_tasks, (void *)d_items, (void *)d_tables, (void *)d_ctl,
                        (void *)d_y})
            if (p)
                (void)hipFree(p);
        for (void *p : table_mem)
            if (p)
                (void)hipFree(p);
        if (plan) {
            plan_free(plan);
            delete plan;
        }
    }
};

namespace {

std::vector<c32> roots(uint64_t n)
{
    std::vector<c32> t(n);
    for (uint64_t m = 0; m < n; ++m)
        t[m] = root_forward(m, n);
    return t;
}

int wl_tables(WorkList *w)
{
    using namespace wl;
    std::vector<Tables> tables(KCOUNT, Tables{nullptr, nullptr, nullptr, 0, 0});
    auto up = [&](const std::vector<c32> &v, const c32 **out) -> int {
        void *d = nullptr;
        hipError_t e = hipMalloc(&d, v.size() * sizeof(c32));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(FFT_ERR_OUT_OF_MEMORY, "twiddle table");
        }
        w->table_mem.push_back(d);
        w->table_bytes += v.size() * sizeof(c32);
        if ((e = hipMemcpy(d, v.data(), v.size() * sizeof(c32), hipMemcpyHostToDevice)) !=
            hipSuccess)
            return hip_error(e, "twiddle upload");
        *out = (const c32 *)d;
        return FFT_OK;
    };
    int st;
    for (const LengthInfo &L : kLengths) {
        if (L.planned)
            continue;  // the plan has its own tables
        if (!L.two_pass) {
            if ((st = up(roots(L.n), &tables[L.a].tw)) != FFT_OK)
                return st;
            if (L.wide)
                w->wide_tw = tables[L.a].tw;
            continue;
        }
        if ((st = up(roots((uint64_t)L.n1), &tables[L.a].tw)) != FFT_OK ||
            (st = up(roots((uint64_t)L.n2), &tables[L.b].tw)) != FFT_OK)
            return st;
        int sh = 0;
        while ((1ull << sh) * (1ull << sh) < L.n)
            ++sh;
        const uint64_t lo = 1ull << sh;
        std::vector<c32> tl(lo), th((L.n + lo - 1) / lo);
        for (uint64_t j = 0; j < lo; ++j)
            tl[j] = root_forward(j, L.n);
        for (uint64_t j = 0; j < th.size(); ++j)
            th[j] = root_forward(j * lo, L.n);
        if ((st = up(tl, &tables[L.a].tl)) != FFT_OK || (st = up(th, &tables[L.a].th)) != FFT_OK)
            return st;
        tables[L.a].sh = sh;
    }
    w->h_tables = tables;
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, tables.size() * sizeof(Tables));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(FFT_ERR_OUT_OF_MEMORY, "table index");
    }
    w->d_tables = (Tables *)d;
    if ((e = hipMemcpy(d, tables.data(), tables.size() * sizeof(Tables),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return hip_error(e, "table index upload");
    return FFT_OK;
}

// host-side checks and task compilation; fills the WorkList's metadata
int wl_compile(WorkList *w, const fft_work_t *items, size_t n, std::vector<wl::Task> &tasks,
               std::vector<wl::Item> &hitems)
{
    using namespace wl;
    constexpr size_t NL = sizeof(kLengths) / sizeof(kLengths[0]);
    std::vector<std::vector<uint32_t>> bucket(NL);
    uint64_t max_in = 0, max_out = 0, samples = 0;
    if (n > 0xffffffffull)
        return set_error(FFT_ERR_INVALID_ARG, "work list too long");
    for (size_t i = 0; i < n; ++i) {
        const LengthInfo *li = length_info(items[i].segment_len);
        if (!li)
            return set_error(FFT_ERR_UNSUPPORTED_LENGTH,
                             "work item %zu: length %u has no work-list routine", i,
                             items[i].segment_len);
        const uint64_t len = items[i].segment_len;
        if (items[i].in_off > (UINT64_MAX >> 4) - len || items[i].out_off > (UINT64_MAX >> 4) - len)
            return set_error(FFT_ERR_INVALID_ARG, "work item %zu: offset out of range", i);
        max_in = std::max<uint64_t>(max_in, items[i].in_off + len);
        max_out = std::max<uint64_t>(max_out, items[i].out_off + len);
        bucket[li - kLengths].push_back((uint32_t)i);
        samples += len;
    }
    // The range checks work on runs: maximal stretches of consecutive
    // entries of one length whose inputs and outputs both advance by that
    // length (a job's segments, typically).  Entries of one run never
    // overlap each other, so checking the runs' extents is the same as
    // checking every entry, at a cost set by the number of runs.
    struct Run {
        uint64_t in0, in1, out0, out1;  // input and output extents [0, 1)
        bool same;                      // in0 == out0: the run is in place
    };
    std::vector<Run> runs;
    for (size_t i = 0; i < n; ++i) {
        const uint64_t len = items[i].segment_len;
        const uint64_t ia = items[i].in_off, oa = items[i].out_off;
        if (i > 0 && items[i - 1].segment_len == len && ia == runs.back().in1 &&
            oa == runs.back().out1) {
            runs.back().in1 += len;
            runs.back().out1 += len;
        } else {
            runs.push_back({ia, ia + len, oa, oa + len, ia == oa});
        }
    }
    const size_t nr = runs.size();
    // outputs must not overlap each other
    {
        std::vector<std::pair<uint64_t, uint64_t>> r(nr);
        for (size_t i = 0; i < nr; ++i)
            r[i] = {runs[i].out0, runs[i].out1};
        std::sort(r.begin(), r.end());
        for (size_t i = 1; i < nr; ++i)
            if (r[i].first < r[i - 1].second)
                return set_error(FFT_ERR_OVERLAP, "two work items write overlapping outputs");
    }
    // with in_base == out_base an output may only coincide with its own
    // input: inputs sorted by start, prefix top-2 of their ends; an output
    // [a, b) meets input j iff start_j < b and end_j > a
    bool in_place_ok = true;
    if (nr) {
        std::vector<size_t> ord(nr);
        for (size_t i = 0; i < nr; ++i)
            ord[i] = i;
        std::sort(ord.begin(), ord.end(),
                  [&](size_t x, size_t y) { return runs[x].in0 < runs[y].in0; });
        std::vector<uint64_t> starts(nr);
        for (size_t k = 0; k < nr; ++k)
            starts[k] = runs[ord[k]].in0;
        std::vector<std::pair<uint64_t, size_t>> best(nr), second(nr);
        std::pair<uint64_t, size_t> b1{0, SIZE_MAX}, b2{0, SIZE_MAX};
        for (size_t k = 0; k < nr; ++k) {
            const size_t j = ord[k];
            const std::pair<uint64_t, size_t> e{runs[j].in1, j};
            if (e.first > b1.first) {
                b2 = b1;
                b1 = e;
            } else if (e.first > b2.first) {
                b2 = e;
            }
            best[k] = b1;
            second[k] = b2;
        }
        for (size_t i = 0; i < nr && in_place_ok; ++i) {
            const uint64_t a = runs[i].out0, b = runs[i].out1;
            const size_t k =
                (size_t)(std::lower_bound(starts.begin(), starts.end(), b) - starts.begin());
            if (k == 0)
                continue;
            const auto &m1 = best[k - 1], &m2 = second[k - 1];
            const bool own_same = runs[i].same;
            if (m1.first > a && !(m1.second == i && own_same))
                in_place_ok = false;
            else if (m1.second == i && own_same && m2.first > a)
                in_place_ok = false;
        }
    }
    // tasks: all pass-A tiles, then single-pass tiles (first launch), then
    // pass-B tiles (second launch); longest lengths first within each group
    tasks.clear();
    hitems.clear();
    hitems.reserve(n);
    std::vector<Task> a_tasks, s_tasks, b_tasks;
    std::vector<Item> wide_items, idx_items, tp_items;
    std::vector<WorkList::IndexedRun> indexed;
    WorkList::IndexedTwoPass tp_idx;
    std::vector<WorkList::PlanRun> plan_runs;
    uint64_t plan_len = 0, plan_max_run = 0;
    uint64_t y_samples = 0;
    uint32_t two_pass = 0;
    uint64_t counts[KCOUNT] = {};
    for (int li = (int)NL - 1; li >= 0; --li) {
        const LengthInfo &L = kLengths[li];
        const auto &b = bucket[li];
        if (L.planned) {
            // bucket entries are in list order: consecutive entries whose
            // input and output both advance by one segment form a run
            for (uint32_t idx : b) {
                const uint64_t ia = items[idx].in_off, oa = items[idx].out_off;
                if (!plan_runs.empty() &&
                    plan_runs.back().in_off + plan_runs.back().count * L.n == ia &&
                    plan_runs.back().out_off + plan_runs.back().count * L.n == oa)
                    ++plan_runs.back().count;
                else
                    plan_runs.push_back({ia, oa, 1});
                plan_max_run = std::max(plan_max_run, plan_runs.back().count);
            }
            if (!b.empty())
                plan_len = L.n;
            counts[L.a] += b.size();
            two_pass += (uint32_t)b.size();
            continue;
        }
        if (L.wide) {
            for (uint32_t idx : b)
                wide_items.push_back({items[idx].in_off, items[idx].out_off, 0});
            counts[L.a] += b.size();
        } else if (int gm = 0, r = route_two_pass(L.n, &gm); L.two_pass && r == 1) {
            if (!b.empty()) {
                indexed_four_step(L.n, &tp_idx.col, &tp_idx.row);
                tp_idx.n = L.n;
                tp_idx.count = (uint32_t)b.size();
                tp_idx.grid_mult = gm;
                for (uint32_t idx : b)
                    tp_items.push_back({items[idx].in_off, items[idx].out_off, 0});
                y_samples = std::max<uint64_t>(y_samples, b.size() * (uint64_t)(L.n + kLine));
                counts[L.a] += b.size();
                two_pass += (uint32_t)b.size();
            }
        } else if (L.two_pass) {
            for (uint32_t idx : b) {
                const uint32_t item = (uint32_t)hitems.size();
                // Segments may start anywhere in a 128-byte line (16
                // samples).  Column blocks then start at the first column
                // whose address is line-aligned, so every block reads and
                // writes whole lines (the last block wraps round to columns
                // 0..shift-1, whose pieces pair up into lines with those of
                // the neighbouring rows); Y gets the input's offset within
                // a line, and the row blocks of pass B start where the
                // output's rows do.
                const uint64_t in_m = items[idx].in_off % kLine,
                               out_m = items[idx].out_off % kLine;
                const uint64_t y_off = (y_samples + kLine - 1) / kLine * kLine + in_m;
                hitems.push_back({items[idx].in_off, items[idx].out_off, y_off});
                y_samples = y_off + L.n;
                const uint32_t sa = (uint32_t)((kLine - in_m) % kLine),
                               sb = (uint32_t)((kLine - out_m) % kLine);
                for (int t = 0; t < L.per_tile; t += L.group) {
                    const uint32_t nt = (uint32_t)std::min(L.group, L.per_tile - t);
                    a_tasks.push_back({(uint32_t)L.a, item, 1, (uint32_t)t, nt, sa, {0, 0}});
                    b_tasks.push_back({(uint32_t)L.b, item, 1, (uint32_t)t, nt, sb, {0, 0}});
                }
                counts[L.a] += 1;
                ++two_pass;
            }
        } else if (int gm = 0, r = route_of(L.n, &gm); r > 0 && !b.empty()) {
            int cnt = 0;
            const SinglePassDesc *d = indexed_table(L.n, &cnt) + (r - 1);
            indexed.push_back({d, (uint32_t)L.a, (uint32_t)idx_items.size(), (uint32_t)b.size(),
                               gm, 0});
            for (uint32_t idx : b)
                idx_items.push_back({items[idx].in_off, items[idx].out_off, 0});
            counts[L.a] += b.size();
        } else {
            const size_t per_task = (size_t)L.per_tile * (size_t)L.group;
            for (size_t k = 0; k < b.size(); k += per_task) {
                const uint32_t first = (uint32_t)hitems.size();
                const uint32_t cnt = (uint32_t)std::min<size_t>(per_task, b.size() - k);
                for (uint32_t j = 0; j < cnt; ++j)
                    hitems.push_back({items[b[k + j]].in_off, items[b[k + j]].out_off, 0});
                s_tasks.push_back({(uint32_t)L.a, first, cnt, 0, 0, 0, {0, 0}});
                counts[L.a] += cnt;
            }
        }
    }
    // the wide launch's items follow the task items, the indexed launches'
    // items follow those
    const uint32_t wide_first = (uint32_t)hitems.size();
    hitems.insert(hitems.end(), wide_items.begin(), wide_items.end());
    for (auto &r : indexed)
        r.first += (uint32_t)hitems.size();
    hitems.insert(hitems.end(), idx_items.begin(), idx_items.end());
    tp_idx.first = (uint32_t)hitems.size();
    hitems.insert(hitems.end(), tp_items.begin(), tp_items.end());
    tasks.reserve(a_tasks.size() + s_tasks.size() + b_tasks.size());
    tasks.insert(tasks.end(), a_tasks.begin(), a_tasks.end());
    tasks.insert(tasks.end(), s_tasks.begin(), s_tasks.end());
    tasks.insert(tasks.end(), b_tasks.begin(), b_tasks.end());
    if (tasks.size() > 0xffffffffull)
        return set_error(FFT_ERR_INVALID_ARG, "work list too long");
    w->n_items = n;
    w->max_in = max_in;
    w->max_out = max_out;
    w->samples = samples;
    w->in_place_ok = in_place_ok;
    w->n_tasks = (uint32_t)tasks.size();
    w->n_first = (uint32_t)(a_tasks.size() + s_tasks.size());
    w->n_two_pass = two_pass;
    w->wide_first = wide_first;
    w->n_wide = (uint32_t)wide_items.size();
    w->indexed.swap(indexed);
    w->two_pass_idx = tp_idx;
    w->plan_runs.swap(plan_runs);
    w->plan_len = plan_len;
    w->plan_max_run = plan_max_run;
    w->y_bytes = y_samples * sizeof(c32);
    std::memcpy(w->counts, counts, sizeof(counts));
    return FFT_OK;
}

template <class T>
int grow(T **ptr, size_t *cap, size_t need, const char *what)
{
    if (need <= *cap)
        return FFT_OK;
    const size_t want = std::max(need, *cap * 2);
    if (*ptr)
        (void)hipFree(*ptr);
    *ptr = nullptr;
    *cap = 0;
    void *d = nullptr;
    if (hipMalloc(&d, want * sizeof(T)) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(FFT_ERR_OUT_OF_MEMORY, "%s (%zu bytes)", what, want * sizeof(T));
    }
    *ptr = (T *)d;
    *cap = want;
    return FFT_OK;
}

// compile and upload new entries; device arrays grow (after a device-wide
// synchronisation) when they are too small; the upload goes through
// pinned staging on `stream`, ordered before later work on that stream
int wl_reset(WorkList *w, const fft_work_t *items, size_t n, hipStream_t s)
{
    using namespace wl;
    std::vector<Task> tasks;
    std::vector<Item> hitems;
    int st = wl_compile(w, items, n, tasks, hitems);
    if (st != FFT_OK)
        return st;  // entries rejected: the previous ones still stand
    w->ready = false;
    const size_t need_ctl = 2;  // one task cursor per launch
    const size_t need_y = w->y_bytes / sizeof(c32);
    if (tasks.size() > w->cap_tasks || hitems.size() > w->cap_items || need_ctl > w->cap_ctl ||
        need_y > w->cap_y) {
        (void)hipDeviceSynchronize();  // old arrays may still be in use
        w->drop_graph();
        if ((st = grow(&w->d_tasks, &w->cap_tasks, std::max<size_t>(tasks.size(), 1), "tasks")) !=
                FFT_OK ||
            (st = grow(&w->d_items, &w->cap_items, std::max<size_t>(hitems.size(), 1), "items")) !=
                FFT_OK ||
            (st = grow(&w->d_ctl, &w->cap_ctl, need_ctl, "cursors")) != FFT_OK ||
            (st = grow(&w->d_y, &w->cap_y, std::max<size_t>(need_y, 1), "two-pass scratch")) !=
                FFT_OK)
            return st;
    }
    if (w->plan_len && (!w->plan || w->plan->n != w->plan_len ||
                        w->plan->batch < w->plan_max_run)) {
        // a plan for at least the longest run (at least twice the old one,
        // so that growing runs rebuild it rarely); its scratch may be in use
        const uint64_t batch =
            std::max<uint64_t>(w->plan_max_run,
                               w->plan && w->plan->n == w->plan_len ? 2 * w->plan->batch : 1);
        (void)hipDeviceSynchronize();
        w->drop_graph();
        if (w->plan) {
            plan_free(w->plan);
            delete w->plan;
            w->plan = nullptr;
        }
        Plan *p = new Plan();
        if ((st = plan_build(p, w->plan_len, batch, w->dir, -1)) != FFT_OK) {
            plan_free(p);
            delete p;
            return st;
        }
        w->plan = p;
    }
    const size_t tb = tasks.size() * sizeof(Task), ib = hitems.size() * sizeof(Item);
    hipError_t e;
    if (!w->stage_done && (e = hipEventCreateWithFlags(&w->stage_done, hipEventDisableTiming)) !=
                              hipSuccess)
        return hip_error(e, "hipEventCreate");
    // the previous upload must have left the staging buffer
    if ((e = hipEventSynchronize(w->stage_done)) != hipSuccess)
        return hip_error(e, "hipEventSynchronize");
    if (tb + ib > w->cap_stage) {
        if (w->h_stage)
            (void)hipHostFree(w->h_stage);
        w->h_stage = nullptr;
        w->cap_stage = 0;
        const size_t want = std::max(tb + ib, w->cap_stage * 2);
        if (hipHostMalloc(&w->h_stage, want, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            w->h_stage = nullptr;
            return set_error(FFT_ERR_OUT_OF_MEMORY, "pinned staging of %zu bytes", want);
        }
        w->cap_stage = want;
    }
    std::memcpy(w->h_stage, tasks.data(), tb);
    std::memcpy((char *)w->h_stage + tb, hitems.data(), ib);
    if (tb && (e = hipMemcpyAsync(w->d_tasks, w->h_stage, tb, hipMemcpyHostToDevice, s)) !=
                  hipSuccess)
        return hip_error(e, "task upload");
    if (ib && (e = hipMemcpyAsync(w->d_items, (char *)w->h_stage + tb, ib,
                                  hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_error(e, "item upload");
    if ((e = hipEventRecord(w->stage_done, s)) != hipSuccess)
        return hip_error(e, "hipEventRecord");
    const void *k = w->dir < 0 ? (const void *)&worklist_kernel<-1> : (const void *)&worklist_kernel<1>;
    const unsigned g = grid_for(k, kThreads, std::max<uint64_t>(1, w->n_tasks), w->device,
                                kWorkListGridMult);
    const void *kw = w->dir < 0 ? (const void *)&worklist_wide_kernel<-1>
                                : (const void *)&worklist_wide_kernel<1>;
    const unsigned gw = grid_for(kw, PWide::kThreads, std::max<uint64_t>(1, w->n_wide), w->device,
                                 kWideGridMult);
    w->grid = g;
    w->wide_grid = gw;
    if (WorkList::IndexedTwoPass &t = w->two_pass_idx; t.count) {
        const uint64_t n1 = (uint64_t)t.col->n1, n2 = (uint64_t)t.row->n2;
        const int gm = t.grid_mult > 0 ? t.grid_mult : two_pass_grid_mult(n1);
        t.grid_a = grid_for(t.col->kernel_indexed[w->dir > 0], t.col->threads * t.col->cols,
                            t.count * (n2 / (uint64_t)t.col->cols), w->device, gm);
        t.grid_b = grid_for(t.row->kernel_indexed[w->dir > 0], t.row->threads * t.row->rows,
                            t.count * (n1 / (uint64_t)t.row->rows), w->device, gm);
    }
    for (auto &r : w->indexed) {
        const SinglePassDesc *d = r.d;
        const uint64_t groups = (r.count + d->segs_per_wg - 1) / d->segs_per_wg;
        r.grid = grid_for(d->kernel_indexed[w->dir > 0], d->threads * d->segs_per_wg, groups,
                          w->device, r.grid_mult > 0 ? r.grid_mult : d->grid_mult);
    }
    w->ready = true;
    return set_ok();
}

int wl_enqueue(WorkList *w, const void *in, void *out, hipStream_t s)
{
    using namespace wl;
    // planned runs first: they touch only their own ranges and the plan's
    // scratch, so their order against the work-list launches is free
    for (const WorkList::PlanRun &r : w->plan_runs) {
        const int st = plan_enqueue(w->plan, (const c32 *)in + r.in_off,
                                    (c32 *)out + r.out_off, r.count, s);
        if (st != FFT_OK)
            return st;
    }
    // the two-pass length with passes of its own: A, then B
    if (const WorkList::IndexedTwoPass &t = w->two_pass_idx; t.count) {
        const wl::Tables &ta = w->h_tables[wl::K65536A], &tb = w->h_tables[wl::K65536B];
        const uint64_t *offs = reinterpret_cast<const uint64_t *>(w->d_items + t.first);
        t.col->launch_indexed(w->dir, in, w->d_y, ta.tw, ta.tl, ta.th, ta.sh, t.row->n2, offs,
                              t.count, t.grid_a, s);
        t.row->launch_indexed(w->dir, in, w->d_y, out, tb.tw, t.col->n1, offs, t.count,
                              t.grid_b, s);
    }
    // one-pass lengths with launches of their own
    for (const WorkList::IndexedRun &r : w->indexed)
        r.d->launch_indexed(w->dir, in, out, w->h_tables[r.kind].tw,
                            reinterpret_cast<const uint64_t *>(w->d_items + r.first), r.count,
                            r.grid, s);
    if (w->n_tasks == 0 && w->n_wide == 0) {
        hipError_t e = hipGetLastError();
        return e == hipSuccess ? set_ok() : hip_error(e, "indexed launch");
    }
    hipLaunchKernelGGL(clear_kernel, dim3(1), dim3(256), 0, s, w->d_ctl, 2u);
    // launch 0: pass-A and single-pass tasks; then the wide tiles; launch 1:
    // pass-B tasks
    const uint32_t first[2] = {0, w->n_first};
    const uint32_t count[2] = {w->n_first, w->n_tasks - w->n_first};
    for (int l = 0; l < 2; ++l) {
        if (l == 1 && w->n_wide) {
            if (w->dir < 0)
                hipLaunchKernelGGL((worklist_wide_kernel<-1>), dim3(w->wide_grid),
                                   dim3(PWide::kThreads), 0, s, w->d_items + w->wide_first,
                                   w->n_wide, w->wide_tw, (const c32 *)in, (c32 *)out);
            else
                hipLaunchKernelGGL((worklist_wide_kernel<1>), dim3(w->wide_grid),
                                   dim3(PWide::kThreads), 0, s, w->d_items + w->wide_first,
                                   w->n_wide, w->wide_tw, (const c32 *)in, (c32 *)out);
        }
        if (count[l] == 0)
            continue;
        const unsigned grid = std::min<unsigned>(w->grid, (count[l] + kClaim - 1) / kClaim);
        if (w->dir < 0)
            hipLaunchKernelGGL((worklist_kernel<-1>), dim3(grid), dim3(kThreads), 0, s,
                               w->d_tasks + first[l], count[l], w->d_items, w->d_tables,
                               (const c32 *)in, (c32 *)out, w->d_y, w->d_ctl + l);
        else
            hipLaunchKernelGGL((worklist_kernel<1>), dim3(grid), dim3(kThreads), 0, s,
                               w->d_tasks + first[l], count[l], w->d_items, w->d_tables,
                               (const c32 *)in, (c32 *)out, w->d_y, w->d_ctl + l);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_error(e, "work-list launch");
    return set_ok();
}

// device memory the work list holds now: its arrays at their capacities,
// the two-pass scratch, the twiddle tables and the four-step plan's
// scratch and tables
size_t wl_device_bytes(const WorkList *w)
{
    size_t b = w->cap_tasks * sizeof(wl::Task) + w->cap_items * sizeof(wl::Item) +
               w->cap_ctl * sizeof(uint32_t) + w->cap_y * sizeof(c32) + w->table_bytes +
               wl::KCOUNT * sizeof(wl::Tables);
    if (w->plan) {
        const Plan *p = w->plan;
        const uint64_t lo = 1ull << p->sh;
        b += p->scratch_bytes + (p->n1 + p->n2 + lo + (p->n + lo - 1) / lo) * sizeof(c32);
    }
    return b;
}

int wl_check_io(WorkList *w, const void *in, void *out)
{
    if (!in || !out)
        return set_error(FFT_ERR_INVALID_ARG, "in_base/out_base must not be NULL");
    if (((uintptr_t)in & 7u) || ((uintptr_t)out & 7u))
        return set_error(FFT_ERR_ALIGNMENT, "bases must be 8-byte aligned");
    if (!w->ready)
        return set_error(FFT_ERR_INVALID_ARG,
                         "the last reset failed after taking its entries: reset again");
    if (w->n_tasks == 0 && w->n_wide == 0 && w->plan_runs.empty() && w->indexed.empty() &&
        !w->two_pass_idx.count)
        return FFT_OK;
    if (in == out && !w->in_place_ok)
        return set_error(FFT_ERR_OVERLAP,
                         "in_base == out_base but an output range overlaps another entry's input");
    if (in != out) {
        const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
        const uint64_t ai = w->max_in * sizeof(c32), bo = w->max_out * sizeof(c32);
        if (a < b + bo && b < a + ai)
            return set_error(FFT_ERR_OVERLAP, "in and out buffers overlap without being equal");
    }
    int st = check_device_range(in, w->max_in * sizeof(c32), "in_base");
    if (st != FFT_OK)
        return st;
    if (out != in && (st = check_device_range(out, w->max_out * sizeof(c32), "out_base")) != FFT_OK)
        return st;
    return FFT_OK;
}

}  // namespace
}  // namespace fftseg

using namespace fftseg;

extern "C" fft_worklist_t fft_worklist_create(const fft_work_t *items, size_t n, int direction)
{
    try {
        if (!items && n) {
            set_error(FFT_ERR_INVALID_ARG, "items is NULL");
            return nullptr;
        }
        if (direction != FFT_FORWARD && direction != FFT_INVERSE) {
            set_error(FFT_ERR_INVALID_ARG, "direction must be -1 or +1");
            return nullptr;
        }
        WorkList *w = new WorkList();
        w->dir = direction;
        // host-side checks first: nothing touches the device for bad entries
        std::vector<wl::Task> tasks;
        std::vector<wl::Item> hitems;
        int st = wl_compile(w, items, n, tasks, hitems);
        if (st == FFT_OK && hipGetDevice(&w->device) != hipSuccess) {
            (void)hipGetLastError();
            st = set_error(FFT_ERR_HIP, "no HIP device available");
        }
        if (st == FFT_OK)
            st = wl_tables(w);
        if (st == FFT_OK)
            st = wl_reset(w, items, n, nullptr);
        if (st == FFT_OK && hipStreamSynchronize(nullptr) != hipSuccess)
            st = hip_error(hipGetLastError(), "hipStreamSynchronize");
        if (st != FFT_OK) {
            const int code = last_status();
            std::string msg = last_message();
            delete w;
            set_error(code, "%s", msg.c_str());
            return nullptr;
        }
        return reinterpret_cast<fft_worklist_t>(w);
    } catch (...) {
        set_error(FFT_ERR_OUT_OF_MEMORY, "host allocation failed");
        return nullptr;
    }
}

extern "C" int fft_worklist_reset(fft_worklist_t wlh, const fft_work_t *items, size_t n,
                                  void *stream)
{
    try {
        WorkList *w = reinterpret_cast<WorkList *>(wlh);
        if (!w)
            return set_error(FFT_ERR_INVALID_ARG, "work list is NULL");
        if (!items && n)
            return set_error(FFT_ERR_INVALID_ARG, "items is NULL");
        return wl_reset(w, items, n, (hipStream_t)stream);
    } catch (...) {
        return set_error(FFT_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

extern "C" int fft_worklist_exec(fft_worklist_t wlh, const void *in_base, void *out_base,
                                 void *stream)
{
    WorkList *w = reinterpret_cast<WorkList *>(wlh);
    if (!w)
        return set_error(FFT_ERR_INVALID_ARG, "work list is NULL");
    int st = wl_check_io(w, in_base, out_base);
    if (st != FFT_OK)
        return st;
    return wl_enqueue(w, in_base, out_base, (hipStream_t)stream);
}

extern "C" int fft_worklist_exec_graph(fft_worklist_t wlh, const void *in_base, void *out_base,
                                       void *stream)
{
    WorkList *w = reinterpret_cast<WorkList *>(wlh);
    if (!w)
        return set_error(FFT_ERR_INVALID_ARG, "work list is NULL");
    int st = wl_check_io(w, in_base, out_base);
    if (st != FFT_OK)
        return st;
    if (w->n_tasks == 0 && w->n_wide == 0 && w->plan_runs.empty() && w->indexed.empty() &&
        !w->two_pass_idx.count)
        return set_ok();
    hipError_t e;
    WorkList::LaunchKey k = w->key(in_base, out_base);
    if (!w->graph_exec || !(w->graph_key == k)) {
        w->drop_graph();
        if (!w->capture_stream &&
            (e = hipStreamCreateWithFlags(&w->capture_stream, hipStreamNonBlocking)) != hipSuccess)
            return hip_error(e, "hipStreamCreate");
        if ((e = hipStreamBeginCapture(w->capture_stream, hipStreamCaptureModeThreadLocal)) !=
            hipSuccess)
            return hip_error(e, "hipStreamBeginCapture");
        st = wl_enqueue(w, in_base, out_base, w->capture_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(w->capture_stream, &g);
        if (st != FFT_OK) {
            if (g)
                (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess)
            return hip_error(e, "hipStreamEndCapture");
        w->graph = g;
        if ((e = hipGraphInstantiate(&w->graph_exec, g, nullptr, nullptr, 0)) != hipSuccess) {
            w->graph_exec = nullptr;
            return hip_error(e, "hipGraphInstantiate");
        }
        w->graph_key = std::move(k);
    }
    if ((e = hipGraphLaunch(w->graph_exec, (hipStream_t)stream)) != hipSuccess)
        return hip_error(e, "hipGraphLaunch");
    return set_ok();
}

extern "C" int fft_worklist_status(fft_worklist_t wlh, void *stream)
{
    WorkList *w = reinterpret_cast<WorkList *>(wlh);
    if (!w)
        return set_error(FFT_ERR_INVALID_ARG, "work list is NULL");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess)
        return hip_error(e, "hipStreamSynchronize");
    // both launches drain their task lists; every task was claimed iff the
    // cursors passed the list ends
    if (!w->d_ctl || w->n_tasks == 0)
        return set_ok();
    uint32_t cur[2] = {0, 0};
    if ((e = hipMemcpy(cur, w->d_ctl, sizeof(cur), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_error(e, "status read");
    if (cur[0] < w->n_first || cur[1] < w->n_tasks - w->n_first)
        return set_error(FFT_ERR_HIP, "the last run did not claim every task");
    return set_ok();
}

extern "C" int fft_worklist_describe(fft_worklist_t wlh, char *buf, size_t len)
{
    const WorkList *w = reinterpret_cast<const WorkList *>(wlh);
    if (!w)
        return set_error(FFT_ERR_INVALID_ARG, "work list is NULL");
    std::string js = "{\"items\":" + std::to_string(w->n_items) +
                     ",\"tasks\":" + std::to_string(w->n_tasks) +
                     ",\"first_launch_tasks\":" + std::to_string(w->n_first) +
                     ",\"two_pass_segments\":" + std::to_string(w->n_two_pass) +
                     ",\"wide_segments\":" + std::to_string(w->n_wide) +
                     ",\"wide_grid\":" + std::to_string(w->wide_grid) +
                     ",\"plan_runs\":" + std::to_string(w->plan_runs.size()) +
                     ",\"indexed_launches\":" + std::to_string(w->indexed.size()) +
                     ",\"indexed_two_pass_segments\":" + std::to_string(w->two_pass_idx.count) +
                     ",\"samples\":" + std::to_string(w->samples) +
                     ",\"scratch_bytes\":" + std::to_string(w->y_bytes) +
                     ",\"device_bytes\":" + std::to_string(wl_device_bytes(w)) +
                     ",\"in_place_ok\":" + (w->in_place_ok ? "true" : "false") +
                     ",\"grid\":" + std::to_string(w->grid) + ",\"segments_per_length\":{";
    bool first = true;
    for (const wl::LengthInfo &L : wl::kLengths) {
        if (!w->counts[L.a])
            continue;
        js += std::string(first ? "" : ",") + "\"" + std::to_string(L.n) +
              "\":" + std::to_string(w->counts[L.a]);
        first = false;
    }
    js += "},\"indexed\":{";
    first = true;
    for (const WorkList::IndexedRun &r : w->indexed) {
        js += std::string(first ? "" : ",") + "\"" + std::to_string(r.d->n) +
              "\":{\"candidate\":" + std::to_string(r.d->variant) +
              ",\"segments\":" + std::to_string(r.count) + ",\"grid\":" +
              std::to_string(r.grid) + "}";
        first = false;
    }
    js += "}}";
    if (buf && len) {
        const size_t k = std::min(len - 1, js.size());
        std::memcpy(buf, js.data(), k);
        buf[k] = 0;
    }
    set_ok();
    return (int)js.size();
}

extern "C" int fft_worklist_destroy(fft_worklist_t wlh)
{
    WorkList *w = reinterpret_cast<WorkList *>(wlh);
    if (w) {
        (void)hipDeviceSynchronize();
        delete w;
    }
    return set_ok();
}

// ---------------------------------------------------------------------------
// One call per batch: the work lists behind it are kept per (device,
// direction, stream).  Calls on one stream are ordered by the stream, so
// they may share one work list's device arrays and scratch; calls on
// different streams get different work lists.  Kept until
// fft_worklist_cache_clear (never freed by a static destructor: HIP may be
// finalised before it would run).
namespace fftseg {
namespace {
struct CachedList {
    int device;
    int dir;
    void *stream;
    WorkList *w;
};
std::mutex g_cache_mu;
std::vector<CachedList> g_cache;
}  // namespace
}  // namespace fftseg

extern "C" int fft_exec_worklist(const fft_work_t *items, size_t n, int direction,
                                 const void *in_base, void *out_base, void *stream)
{
    try {
        if (!items && n)
            return set_error(FFT_ERR_INVALID_ARG, "items is NULL");
        if (direction != FFT_FORWARD && direction != FFT_INVERSE)
            return set_error(FFT_ERR_INVALID_ARG, "direction must be -1 or +1");
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) {
            (void)hipGetLastError();
            return set_error(FFT_ERR_HIP, "no HIP device available");
        }
        std::lock_guard<std::mutex> lk(g_cache_mu);
        WorkList *w = nullptr;
        for (CachedList &c : g_cache)
            if (c.device == dev && c.dir == direction && c.stream == stream)
                w = c.w;
        int st;
        if (!w) {
            // an empty list first: its tables and arrays, then the entries
            fft_worklist_t h = fft_worklist_create(nullptr, 0, direction);
            if (!h)
                return last_status();
            w = reinterpret_cast<WorkList *>(h);
            g_cache.push_back({dev, direction, stream, w});
        }
        if ((st = wl_reset(w, items, n, (hipStream_t)stream)) != FFT_OK ||
            (st = wl_check_io(w, in_base, out_base)) != FFT_OK)
            return st;
        return wl_enqueue(w, in_base, out_base, (hipStream_t)stream);
    } catch (...) {
        return set_error(FFT_ERR_OUT_OF_MEMORY, "host allocation failed");
    }
}

extern "C" int fft_worklist_cache_clear(void)
{
    std::lock_guard<std::mutex> lk(g_cache_mu);
    if (!g_cache.empty())
        (void)hipDeviceSynchronize();
    for (CachedList &c : g_cache)
        delete c.w;
    g_cache.clear();
    return set_ok();
}

extern "C" int fft_worklist_indexed_count(uint32_t segment_len)
{
    set_ok();
    const wl::LengthInfo *li = wl::length_info(segment_len);
    if (li && li->two_pass && !li->planned) {
        const ColumnDesc *c = nullptr;
        const RowDesc *r = nullptr;
        return indexed_four_step(segment_len, &c, &r) ? 1 : 0;
    }
    if (!li || li->two_pass || li->wide || li->planned)
        return 0;
    int cnt = 0;
    (void)indexed_table(segment_len, &cnt);
    return cnt;
}

extern "C" int fft_worklist_supported(uint32_t segment_len)
{
    set_ok();
    return wl::length_info(segment_len) != nullptr;
}
