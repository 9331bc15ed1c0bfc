// Internal runtime declarations shared by the entry-point sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "radix.hpp"
#include "registry.hpp"

namespace fftseg {

struct Plan {
    enum Kind { COPY, SINGLE, FOURSTEP, GENERIC, REAL, REAL_SPLIT };
    uint64_t n = 0, batch = 0;
    int dir = -1;
    int device = 0;
    Kind kind = COPY;
    const SinglePassDesc *sp = nullptr;
    const ColumnDesc *col = nullptr;
    const RowDesc *row = nullptr;
    uint64_t n1 = 0, n2 = 0;
    std::vector<int> radices;   // fallback path
    void *tw = nullptr;         // W_N (single pass) or W_N1 (four-step) table
    void *tw2 = nullptr;        // W_N2 table (four-step); W_N^k, k <= N/2 (real)
    void *tl = nullptr, *th = nullptr;  // two-level W_N table
    int sh = 0;
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    uint64_t sub_batch = 0;
    bool y_blocked = false;     // FOURSTEP: Y in blocks of 16 columns between the passes
    int grid_mult = 0;          // 0: one workgroup per tile
    bool used = false;
    bool last_stream_valid = false;
    hipStream_t last_stream = nullptr;
    // graph replay state
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    const void *graph_in = nullptr;
    void *graph_out = nullptr;
    hipStream_t capture_stream = nullptr;
    void *stream_state = nullptr;  // pinned host ring of the streaming path
    // REAL_SPLIT: the complex n/2-point plan (batch = sub_batch) and the
    // buffer of its spectra (forward) or inputs (inverse), sub_batch rows
    Plan *inner = nullptr;
    void *zbuf = nullptr;
};

inline bool is_real(const Plan *p) { return p->kind == Plan::REAL || p->kind == Plan::REAL_SPLIT; }

int set_ok();
int set_error(int status, const char *fmt, ...);
int hip_error(hipError_t e, const char *what);
int last_status();
const char *last_message();

c32 root_forward(uint64_t m, uint64_t n);
const SinglePassDesc *find_single(uint64_t n, int variant);
const SinglePassDesc *find_aux(uint64_t n);
// the length's default frame kernel: the first row of n with one
const SinglePassDesc *find_frames(uint64_t n);
int variant_count(uint64_t n);
// n1: the column length to use (0: the planner's balanced choice)
bool find_split(uint64_t n, const ColumnDesc **col, const RowDesc **row, int col_variant,
                int row_variant, uint64_t n1 = 0);
// every column length n1 for which n = n1 * n2 has compiled column and row tiles
std::vector<uint64_t> split_candidates(uint64_t n);
// the column / row tiles of a length that have the shifted (line-aligned,
// wrapping) form, or null
const ColumnDesc *find_column_shifted(uint64_t n1);
const RowDesc *find_row_shifted(uint64_t n2);
// complex samples per 128-byte cache line
constexpr uint64_t kLineSamples = 16;
int split_variant_counts(uint64_t n, int *ncol, int *nrow);
unsigned grid_for(const void *kernel, int threads, uint64_t work_groups, int dev,
                  int grid_mult);

int validate_create(uint64_t n, uint64_t batch, int dir);
// forced_variant: single-pass variant (-1: tuned/default); forced_split_variants:
// column variant | row variant << 8 of a four-step plan (-1: tuned/default)
// forced_n1: column length of a four-step plan (0: tuned/default)
int plan_build(Plan *p, uint64_t n, uint64_t batch, int dir, int forced_variant,
               int forced_split_variants = -1, uint64_t forced_n1 = 0);
// the kernels, split and sub-batch of a plan (host only: no device memory);
// a sub-batch fills at most max_sub_samples samples of each scratch buffer
// (two-pass plans have one, the radix-stage path two)
int plan_choose(Plan *p, uint64_t n, uint64_t batch, int dir, int forced_variant,
                int forced_split_variants, uint64_t forced_n1, uint64_t max_sub_samples);
void plan_free(Plan *p);
int plan_enqueue(Plan *p, const void *in, void *out, uint64_t batch, hipStream_t s);
// real-input plans: length n = 2m through the m-point one-pass kernel, or,
// where m has none, through the m-point complex plan and a separate split pass
int plan_build_real(Plan *p, uint64_t n, uint64_t batch, int dir);
int real_split_enqueue(int dir, const void *in, void *out, const void *hw, uint64_t m,
                       uint64_t batch, hipStream_t s);
// entry points that only take complex segments refuse real plans
int reject_real(const Plan *p, const char *what);
int plan_describe(const Plan *p, std::string &js);
int check_io(const void *in, const void *out, uint64_t bytes);
int check_device_range(const void *ptr, uint64_t bytes, const char *name);

void stream_state_free(Plan *p);

struct TunedChoice {
    uint64_t n;
    int variant;      // single-pass variant, -1 for two-pass and fallback plans
    int grid_mult;
    double us;        // measured time per exec when tuned (0 if loaded without)
    uint64_t batch;
    int col_variant;  // two-pass plans: column and row tile variants
    int row_variant;
    uint64_t n1 = 0;  // two-pass plans: column length of the split (0: the planner's)
    // work lists, one-pass lengths: -1 not tuned, 0 the work-list kernel's
    // tiles, 1 + k the k-th indexed one-pass kernel of the length, at
    // wl_grid resident workgroup waves per CU
    int wl_route = -1;
    int wl_grid = 0;
    double wl_us = 0;  // its measured time per exec
};
// persistent grid of the four-step passes by column length: resident
// workgroup waves per CU
int two_pass_grid_mult(uint64_t n1);
int tuned_variant(uint64_t n);
// the tuned work-list route of length n (-1 if none) and its grid
int tuned_wl_route(uint64_t n, int *grid);
// record a work-list route for n without touching the plan choice
void set_tuned_wl_route(uint64_t n, int route, int grid, double us);
int tuned_grid_mult(uint64_t n, int variant, int fallback);
void tuned_split_variants(uint64_t n, int *col_variant, int *row_variant, uint64_t *n1);
void set_tuned(const TunedChoice &c);
void clear_tuned();
std::vector<TunedChoice> tuned_snapshot();

}  // namespace fftseg
