// Overlapping, optionally windowed segments (fft_exec_frames).
//
// The paper cuts the signal into disjoint segments and names overlapping
// transforms as future work (Sec. VI).  Frame s here starts at sample s*hop
// of the signal (hop < N overlaps consecutive frames) and is multiplied by a
// real window before its transform, i.e. a short-time Fourier transform.
// Lengths with an LDS-resident kernel read the frames directly through a
// strided gather in the kernel's first stage, and two-pass lengths through
// the column loads of their first pass, so the overlapping input is read
// once per frame and nothing is staged; the radix-stage lengths first
// gather the windowed frames into the output buffer and transform it in
// place.
#include <stdlib.h>

#include "fftseg.h"
#include "runtime.hpp"

namespace fftseg {
namespace {

__global__ void __launch_bounds__(256)
    frame_gather_kernel(const c32 *__restrict__ in, c32 *__restrict__ out, uint64_t n,
                        uint64_t frames, uint64_t hop, const float *__restrict__ window)
{
    const uint64_t total = frames * n;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t s = i / n, k = i - s * n;
        c32 v = in[s * hop + k];
        if (window) {
            const float w = window[k];
            v = c32{v.x * w, v.y * w};
        }
        out[i] = v;
    }
}

int frames_enqueue(Plan *p, const c32 *in, c32 *out, uint64_t frames, uint64_t hop,
                   const float *window, hipStream_t s)
{
    const uint64_t n = p->n;
    if (p->kind == Plan::SINGLE) {
        // the plan's own kernel variant when it has a frame form, else the
        // length's default frame kernel (at its own grid, unless the
        // FFTSEG_GRID_MULT override set the plan's)
        const SinglePassDesc *d = p->sp && p->sp->launch_strided ? p->sp : find_frames(n);
        if (d && d->launch_strided) {
            const uint64_t groups = (frames + d->segs_per_wg - 1) / d->segs_per_wg;
            const int gm = d == p->sp || getenv("FFTSEG_GRID_MULT") ? p->grid_mult : d->grid_mult;
            const unsigned grid = grid_for(d->kernel_strided[p->dir > 0],
                                           d->threads * d->segs_per_wg, groups, p->device, gm);
            d->launch_strided(p->dir, in, out, p->tw, frames, hop, n, window, grid, s);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return hip_error(e, "frame kernel launch");
            p->used = true;
            p->last_stream = s;
            p->last_stream_valid = true;
            return set_ok();
        }
    }
    if (p->kind == Plan::FOURSTEP && p->col->launch_frames) {
        // the column pass reads the frames; the row pass as for segments
        const ColumnDesc *cd = p->col;
        const RowDesc *rd = p->row;
        const int dir = p->dir;
        // Y in 16-column blocks where the plan keeps it so and the column
        // tile has the blocked frame form
        const bool yb = p->y_blocked && cd->launch_frames_yblocked;
        for (uint64_t s0 = 0; s0 < frames; s0 += p->sub_batch) {
            const uint64_t sb = std::min(p->sub_batch, frames - s0);
            const uint64_t ta = sb * (p->n2 / (uint64_t)cd->cols);
            const uint64_t tb = sb * (p->n1 / (uint64_t)rd->rows);
            const unsigned ga = grid_for(cd->kernel_frames[dir > 0], cd->threads * cd->cols, ta,
                                         p->device, p->grid_mult);
            const unsigned gb = grid_for(rd->kernel[dir > 0], rd->threads * rd->rows, tb,
                                         p->device, p->grid_mult);
            (yb ? cd->launch_frames_yblocked : cd->launch_frames)(
                dir, in + s0 * hop, p->scratch, p->tw, p->tl, p->th, p->sh, (int)p->n2, sb, hop,
                window, ga, s);
            (yb ? rd->launch_yblocked : rd->launch)(dir, p->scratch, out + s0 * n, p->tw2,
                                                    (int)p->n1, sb, gb, s);
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return hip_error(e, "frame kernel launch");
        p->used = true;
        p->last_stream = s;
        p->last_stream_valid = true;
        return set_ok();
    }
    const uint64_t total = frames * n;
    const unsigned grid = (unsigned)std::min<uint64_t>((total + 255) / 256, 1u << 20);
    hipLaunchKernelGGL(frame_gather_kernel, dim3(grid), dim3(256), 0, s, in, out, n, frames,
                       hop, window);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_error(e, "frame gather launch");
    return plan_enqueue(p, out, out, frames, s);
}

}  // namespace
}  // namespace fftseg

using namespace fftseg;

extern "C" int fft_exec_frames(fft_plan_t plan, const void *in, size_t in_len, void *out,
                               size_t n_frames, size_t hop, const float *window,
                               void *stream)
{
    try {
        Plan *p = reinterpret_cast<Plan *>(plan);
        if (!p)
            return set_error(FFT_ERR_INVALID_ARG, "plan is NULL");
        if (reject_real(p, "fft_exec_frames") != FFT_OK)
            return last_status();
        if (!in || !out)
            return set_error(FFT_ERR_INVALID_ARG, "in/out must not be NULL");
        if (n_frames == 0 || n_frames > p->batch)
            return set_error(FFT_ERR_INVALID_ARG, "n_frames %zu outside [1, %llu]", n_frames,
                             (unsigned long long)p->batch);
        if (hop == 0)
            return set_error(FFT_ERR_INVALID_ARG, "hop must be at least 1");
        if (((uintptr_t)in & 7u) || ((uintptr_t)out & 7u) || ((uintptr_t)window & 3u))
            return set_error(FFT_ERR_ALIGNMENT, "in/out must be 8-byte, window 4-byte aligned");
        const uint64_t n = p->n;
        // samples the frames read: (n_frames - 1) * hop + n, without overflow
        if ((uint64_t)(n_frames - 1) > (UINT64_MAX / 16 - n) / hop)
            return set_error(FFT_ERR_INVALID_ARG, "frame range overflows");
        const uint64_t need = (uint64_t)(n_frames - 1) * hop + n;
        if (need > in_len)
            return set_error(FFT_ERR_BOUNDS, "%zu frames of %llu with hop %zu read %llu samples,"
                             " in holds %zu", n_frames, (unsigned long long)n, hop,
                             (unsigned long long)need, in_len);
        const uint64_t in_bytes = need * sizeof(c32), out_bytes = n_frames * n * sizeof(c32);
        const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
        if (a < b + out_bytes && b < a + in_bytes)
            return set_error(FFT_ERR_OVERLAP, "frames are read from and written to overlapping"
                             " memory");
        int st = check_device_range(in, in_bytes, "in");
        if (st == FFT_OK)
            st = check_device_range(out, out_bytes, "out");
        if (st == FFT_OK && window)
            st = check_device_range(window, n * sizeof(float), "window");
        if (st != FFT_OK)
            return st;
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess)
            return hip_error(hipGetLastError(), "hipGetDevice");
        if (cur != p->device && hipSetDevice(p->device) != hipSuccess)
            return hip_error(hipGetLastError(), "hipSetDevice");
        st = frames_enqueue(p, (const c32 *)in, (c32 *)out, n_frames, hop, window,
                            (hipStream_t)stream);
        if (cur != p->device)
            (void)hipSetDevice(cur);
        return st;
    } catch (const std::bad_alloc &) {
        return set_error(FFT_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return set_error(FFT_ERR_INVALID_ARG, "internal error");
    }
}
