// Predicate-filtered indirect write for gfx950: out[idx[i]] = in[i]*in[i].
//
// Every partition runs the whole iteration space; the write index is
// computed unconditionally and the write is kept only when it lands in the
// partition's owner rows [own_lo, own_hi) — the guard the paper's
// predicate-based filtering places around each array write.
#include "k_common.h"
#include "kernels.h"

namespace jk {

namespace {

__global__ void __launch_bounds__(256)
scatter_sq_kernel(const double *__restrict__ in, const int32_t *__restrict__ idx, double *__restrict__ out,
                  int64_t i_lo, int64_t i_hi, int64_t own_lo, int64_t own_hi) {
    const int64_t i = i_lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= i_hi) return;
    const int64_t k = idx[i];
    const double v = in[i] * in[i];
    if (k >= own_lo && k < own_hi) out[k] = v;
}

}  // namespace

hipError_t launch_scatter(const Launch &L, hipStream_t s) {
    const int64_t n = L.hi[0] - L.lo[0];
    if (n <= 0) return hipSuccess;
    const int64_t own_lo = L.own_lo, own_hi = L.own_hi;
    hipLaunchKernelGGL(scatter_sq_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       (const double *)L.a[0].ptr, (const int32_t *)L.a[1].ptr, (double *)L.a[2].ptr, L.lo[0],
                       L.hi[0], own_lo, own_hi);
    return hipGetLastError();
}

}  // namespace jk
