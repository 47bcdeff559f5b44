// CSR sparse matrix-vector product for gfx950.
//
// G lanes cooperate on one row (G = 8 by default for ~16 non-zeros per
// row): lane g of the group adds val[k]*x[col[k]] for k = row_ptr[i] + g,
// + g + G, ... in increasing k, then the group adds its lanes by a fixed
// butterfly.  col/val reads of a group are contiguous; x is gathered.
#include "k_common.h"
#include "kernels.h"

namespace jk {

namespace {

constexpr int kSpmvThreads = 256;

template <int G>
__global__ void __launch_bounds__(kSpmvThreads)
spmv_kernel(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, const double *__restrict__ val,
            const double *__restrict__ x, double *__restrict__ y, int64_t r_lo, int64_t r_hi) {
    const int64_t t = (int64_t)blockIdx.x * kSpmvThreads + threadIdx.x;
    const int64_t i = r_lo + t / G;
    const int g = threadIdx.x & (G - 1);
    double s = 0.0;
    const bool live = i < r_hi;
    if (live) {
        const int32_t kb = rp[i], ke = rp[i + 1];
        for (int32_t k = kb + g; k < ke; k += G) s += val[k] * x[col[k]];
    }
#pragma unroll
    for (int m = 1; m < G; m <<= 1) s += __shfl_xor(s, m, kWave);
    if (live && g == 0) y[i] = s;
}

}  // namespace

hipError_t launch_spmv(const Launch &L, hipStream_t s) {
    const int64_t n = L.hi[0] - L.lo[0];
    if (n <= 0) return hipSuccess;
    const int G = 8;
    const int64_t rows_per_block = kSpmvThreads / G;
    const unsigned nb = (unsigned)((n + rows_per_block - 1) / rows_per_block);
    hipLaunchKernelGGL(spmv_kernel<8>, dim3(nb), dim3(kSpmvThreads), 0, s, (const int32_t *)L.a[0].ptr,
                       (const int32_t *)L.a[1].ptr, (const double *)L.a[2].ptr, (const double *)L.a[3].ptr,
                       (double *)L.a[4].ptr, L.lo[0], L.hi[0]);
    return hipGetLastError();
}

}  // namespace jk
