// Real-input segments whose half length has no one-pass kernel: the N/2-point
// complex transform runs as its own plan (four-step or radix stages) and the
// even/odd split runs as a separate pass over the spectra.  With N = 2M,
// z[m] = x[2m] + i x[2m+1] and Z = DFT_M(z):
//   forward  X[k] = (A + B)/2 - i W_N^k (A - B)/2,  A = Z[k mod M],
//            B = conj Z[(M - k) mod M],  0 <= k <= M  (M + 1 bins per row)
//   inverse  Z[k] = (A + B) + i W_N^{-k} (A - B),  A = X[k], B = conj X[M - k],
//            0 <= k < M, the imaginary parts of X[0] and X[M] dropped; the
//            unnormalised inverse M-point transform of Z is x[2m] + i x[2m+1].
// hw holds W_N^k = exp(-2 pi i k / N), k = 0..M.
#include "runtime.hpp"

#include <algorithm>

namespace fftseg {
namespace {

__global__ void __launch_bounds__(256)
    real_split_forward_kernel(const c32 *__restrict__ z, c32 *__restrict__ x,
                              const c32 *__restrict__ hw, uint64_t m, uint64_t batch)
{
    const uint64_t row = m + 1, total = batch * row;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t seg = i / row, k = i - seg * row;
        const c32 *zs = z + seg * m;
        const c32 a = zs[k == m ? 0 : k];
        const c32 r = zs[k == 0 ? 0 : m - k];
        const c32 e = {0.5f * (a.x + r.x), 0.5f * (a.y - r.y)};  // (A + B) / 2
        const c32 d = {0.5f * (a.x - r.x), 0.5f * (a.y + r.y)};  // (A - B) / 2
        x[i] = cadd(e, cmul(mul_di<-1>(d), hw[k]));
    }
}

__global__ void __launch_bounds__(256)
    real_split_inverse_kernel(const c32 *__restrict__ x, c32 *__restrict__ z,
                              const c32 *__restrict__ hw, uint64_t m, uint64_t batch)
{
    const uint64_t total = batch * m;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t seg = i / m, k = i - seg * m;
        const c32 *xs = x + seg * (m + 1);
        c32 a = xs[k];
        const c32 r = xs[m - k];
        c32 b = {r.x, -r.y};
        if (k == 0) {
            a.y = 0.f;
            b.y = 0.f;
        }
        const c32 d = cmulc(csub(a, b), hw[k]);  // (A - B) W_N^{-k}
        z[i] = cadd(cadd(a, b), mul_di<1>(d));
    }
}

unsigned elementwise_grid(uint64_t total)
{
    return (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((total + 255) / 256, 1u << 20));
}

}  // namespace

int real_split_enqueue(int dir, const void *in, void *out, const void *hw, uint64_t m,
                       uint64_t batch, hipStream_t s)
{
    if (dir < 0)
        hipLaunchKernelGGL(real_split_forward_kernel, dim3(elementwise_grid(batch * (m + 1))),
                           dim3(256), 0, s, (const c32 *)in, (c32 *)out, (const c32 *)hw, m,
                           batch);
    else
        hipLaunchKernelGGL(real_split_inverse_kernel, dim3(elementwise_grid(batch * m)),
                           dim3(256), 0, s, (const c32 *)in, (c32 *)out, (const c32 *)hw, m,
                           batch);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? set_ok() : hip_error(e, "real split launch");
}

}  // namespace fftseg
