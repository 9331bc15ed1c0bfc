// fft_exec_segments_noalloc: the batched transform without a plan and
// without any device allocation.
//
// For callers that cannot allocate device memory (code under stream
// capture, serving loops, harnesses that forbid it).  Everything the
// kernels need beyond the caller's in/out buffers -- the twiddle tables and
// the Y buffer between the two passes of long segments -- lives in one
// file-scope device array of fixed size.  Each call recomputes the tables on
// the device (a small kernel, so that a captured call carries them), then
// runs the same kernels fft_exec_segments runs, long segments in
// sub-batches whose Y fits the array.  The array is this GPU's, shared by
// every call on it: calls that overlap in time on one GPU race.
#include "fftseg.h"
#include "runtime.hpp"

#include <cmath>
#include <mutex>

namespace fftseg {
namespace {

// tables: W_N (one pass) or W_N1, W_N2 and the two-level W_N (two passes)
constexpr uint64_t kTableSamples = 1ull << 15;
// Y: 2^24 samples plus two lines: one sub-batch of a two-pass length (up to
// 2^22 points, so at least 4 segments), or the two buffers of the
// radix-stage path (lengths up to 2^23; 2^24 is refused)
constexpr uint64_t kYSamples = (1ull << 24) + 2 * kLineSamples;
constexpr uint64_t kScratchBytes = (kTableSamples + kYSamples) * sizeof(c32);

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// the array's device address, per device (taken once, with that device
// current; the host-side name `scratch` is not a device address)
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

int scratch_ptr(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(FFT_ERR_INVALID_ARG, "device %d outside [0, %d)", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return set_error(FFT_ERR_HIP, "hipGetSymbolAddress(scratch): %s",
                             hipGetErrorString(e));
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return FFT_OK;
}

// exp(-2 pi i m / n) in FP64, the angle folded to the first octant in exact
// integer arithmetic (8 m < 2^28 here), rounded once to float32
__device__ c32 device_root(uint64_t m, uint64_t n)
{
    m %= n;
    const uint64_t m8 = m * 8u;
    const uint64_t o = m8 / n, r = m8 - o * n;
    const uint64_t j = (o + 1) / 2;
    const double quarter_pi = 0.78539816339744830961566084581987572;
    const double x = ((double)((long long)o - 2 * (long long)j) + (double)r / (double)n) *
                     quarter_pi;
    double sx, cx;
    sincos(x, &sx, &cx);
    double c, s;
    switch (j & 3) {
    case 0: c = cx; s = sx; break;
    case 1: c = -sx; s = cx; break;
    case 2: c = -cx; s = -sx; break;
    default: c = sx; s = -cx; break;
    }
    return c32{(float)c, (float)(-s)};
}

// Up to four consecutive tables: table t holds count[t] entries
// W_{mod[t]}^{j * step[t]}, j < count[t].
struct TableSet {
    uint64_t count[4], mod[4], step[4];
};

__global__ void __launch_bounds__(256) static_tables_kernel(c32 *tables, TableSet ts,
                                                            uint64_t total)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * 256) {
        uint64_t j = i;
        int t = 0;
        while (t < 3 && j >= ts.count[t]) {
            j -= ts.count[t];
            ++t;
        }
        tables[i] = device_root(j * ts.step[t], ts.mod[t]);
    }
}

int noalloc_enqueue(uint64_t n, uint64_t batch, int dir, const void *in, void *out,
                    hipStream_t s)
{
    Plan p;  // host-side description only: its pointers go into `scratch`
    int st = plan_choose(&p, n, batch, dir, -1, -1, 0, kYSamples - kLineSamples);
    if (st != FFT_OK)
        return st;
    if (p.kind == Plan::GENERIC)
        p.sub_batch = std::min<uint64_t>(batch, kYSamples / 2 / n);
    if (p.kind != Plan::COPY && p.kind != Plan::SINGLE && p.sub_batch == 0)
        return set_error(FFT_ERR_UNSUPPORTED_LENGTH,
                         "length %llu runs radix stage by stage through two buffers of "
                         "%llu samples; the static scratch holds %llu",
                         (unsigned long long)n, (unsigned long long)n,
                         (unsigned long long)kYSamples);
    TableSet ts{};
    uint64_t total = 0;
    switch (p.kind) {
    case Plan::COPY: break;
    case Plan::SINGLE:
        ts.count[0] = n; ts.mod[0] = n; ts.step[0] = 1;
        break;
    case Plan::FOURSTEP:
    case Plan::GENERIC: {
        const uint64_t lo = 1ull << p.sh;
        ts.count[0] = lo; ts.mod[0] = n; ts.step[0] = 1;                  // tl
        ts.count[1] = (n + lo - 1) / lo; ts.mod[1] = n; ts.step[1] = lo;  // th
        if (p.kind == Plan::FOURSTEP) {
            ts.count[2] = p.n1; ts.mod[2] = p.n1; ts.step[2] = 1;         // W_N1
            ts.count[3] = p.n2; ts.mod[3] = p.n2; ts.step[3] = 1;         // W_N2
        }
        break;
    }
    default:
        return set_error(FFT_ERR_INVALID_ARG, "real plans are not served here");
    }
    for (int t = 0; t < 4; ++t)
        total += ts.count[t];
    if (total > kTableSamples)
        return set_error(FFT_ERR_UNSUPPORTED_LENGTH,
                         "the tables of length %llu (%llu entries) exceed the %llu of static "
                         "scratch", (unsigned long long)n, (unsigned long long)total,
                         (unsigned long long)kTableSamples);
    void *base = nullptr;
    if ((st = scratch_ptr(p.device, &base)) != FFT_OK)
        return st;
    c32 *tables = (c32 *)base;
    c32 *y = tables + kTableSamples;
    if (total) {
        const unsigned grid = (unsigned)std::min<uint64_t>((total + 255) / 256, 1024);
        hipLaunchKernelGGL(static_tables_kernel, dim3(grid), dim3(256), 0, s, tables, ts, total);
    }
    switch (p.kind) {
    case Plan::SINGLE: p.tw = tables; break;
    case Plan::FOURSTEP:
        p.tl = tables;
        p.th = tables + ts.count[0];
        p.tw = tables + ts.count[0] + ts.count[1];
        p.tw2 = tables + ts.count[0] + ts.count[1] + ts.count[2];
        p.scratch = y;
        break;
    case Plan::GENERIC:
        p.tl = tables;
        p.th = tables + ts.count[0];
        p.scratch = y;
        break;
    default: break;
    }
    st = plan_enqueue(&p, in, out, batch, s);
    // nothing of the description is device memory: keep plan_free's hands off
    p.tw = p.tw2 = p.tl = p.th = p.scratch = nullptr;
    return st;
}

}  // namespace
}  // namespace fftseg

using namespace fftseg;

extern "C" int fft_exec_segments_noalloc(size_t segment_len, size_t batch, int direction,
                                         const void *in, void *out, void *stream)
{
    try {
        if (validate_create(segment_len, batch, direction) != FFT_OK)
            return last_status();
        int st = check_io(in, out, (uint64_t)batch * segment_len * sizeof(c32));
        if (st != FFT_OK)
            return st;
        return noalloc_enqueue(segment_len, batch, direction, in, out, (hipStream_t)stream);
    } catch (...) {
        return set_error(FFT_ERR_INVALID_ARG, "internal error");
    }
}
