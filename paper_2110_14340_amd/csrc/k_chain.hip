// The statement chain of the paper's predicate-filtering example (Sec.
// "Predicate-Based Filtering", Fig. conv-code) as a loop body for gfx950.
//
// Iteration t takes (i, j, k) = idx[t] and x = xs[t] and runs
//   a[i] = x;  b[i] = a[i];  x = c[j];  a[k] = x;  b[k] = a[k];
// Under filtering every partition runs every iteration against its own
// replicas of a and b, and each statement is guarded by the union of the
// owner ranges of the arrays whose partition-local values it feeds:
//   a[i] = x       when i lies in a's or b's range (b[i] reads it next)
//   b[i] = a[i]    when i lies in b's range
//   x = c[j]       when k lies in a's or b's range, else x = 0 (the read of c
//                  is skipped where nothing kept depends on it)
//   a[k] = x       when k lies in a's or b's range
//   b[k] = a[k]    when k lies in b's range
// The index arithmetic is outside every guard.  Duplicated execution (an
// aliased call: a and b the same array) passes ranges covering everything.
// One lane per iteration; the loads of idx and xs are contiguous.
#include "jacc.h"
#include "k_common.h"
#include "kernels.h"

namespace jk {

namespace {

constexpr int kChainThreads = 256;

__global__ void __launch_bounds__(kChainThreads)
chain_kernel(double *a, double *b, const double *__restrict__ c, const int32_t *__restrict__ idx,
             const double *__restrict__ xs, int64_t t_lo, int64_t t_hi, int64_t n_ab, int64_t n_c, int64_t a_lo,
             int64_t a_hi, int64_t b_lo, int64_t b_hi) {
    const int64_t t = t_lo + (int64_t)blockIdx.x * kChainThreads + threadIdx.x;
    if (t >= t_hi) return;
    const int64_t i = idx[3 * t], j = idx[3 * t + 1], k = idx[3 * t + 2];
    if (i < 0 || i >= n_ab || k < 0 || k >= n_ab || j < 0 || j >= n_c) return;  // skipped iteration
    double x = xs[t];
    const bool ia = i >= a_lo && i < a_hi, ib = i >= b_lo && i < b_hi;
    const bool ka = k >= a_lo && k < a_hi, kb = k >= b_lo && k < b_hi;
    if (ia || ib) a[i] = x;
    if (ib) b[i] = a[i];
    x = (ka || kb) ? c[j] : 0.0;
    if (ka || kb) a[k] = x;
    if (kb) b[k] = a[k];
}

}  // namespace

hipError_t launch_chain(const Launch &L, hipStream_t s) {
    const int64_t n = L.hi[0] - L.lo[0];
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + kChainThreads - 1) / kChainThreads);
    // a, b and c are whole replicas: rows [0, slab_hi)
    const int64_t n_ab = L.a[0].slab_hi < L.a[1].slab_hi ? L.a[0].slab_hi : L.a[1].slab_hi;
    hipLaunchKernelGGL(chain_kernel, dim3(nb), dim3(kChainThreads), 0, s, (double *)L.a[0].ptr, (double *)L.a[1].ptr,
                       (const double *)L.a[2].ptr, (const int32_t *)L.a[3].ptr, (const double *)L.a[4].ptr, L.lo[0],
                       L.hi[0], n_ab, L.a[2].slab_hi, L.own_lo, L.own_hi, L.own2_lo, L.own2_hi);
    return hipGetLastError();
}

}  // namespace jk
