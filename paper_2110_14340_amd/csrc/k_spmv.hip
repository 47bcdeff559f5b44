// CSR sparse matrix-vector product for gfx950.
//
// G lanes cooperate on one row (G = 4, 8 or 16; 16 by default for ~16
// non-zeros per row: one gather per lane): lane g of the group adds val[k]*x[col[k]] for k = row_ptr[i] + g,
// + g + G, ... in increasing k, then the group adds its lanes by a fixed
// butterfly.  col/val reads of a group are contiguous; x is gathered.
#include "k_common.h"
#include "kernels.h"

namespace jk {

namespace {

constexpr int kSpmvThreads = 256;

template <int G, bool NT>
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
        for (int32_t k = kb + g; k < ke; k += G) {
            // NT: col and val are read once, so they are loaded non-temporally
            // and leave the caches to the gathered x
            const int32_t c = NT ? __builtin_nontemporal_load(&col[k]) : col[k];
            const double v = NT ? __builtin_nontemporal_load(&val[k]) : val[k];
            s += v * x[c];
        }
    }
#pragma unroll
    for (int m = 1; m < G; m <<= 1) s += __shfl_xor(s, m, kWave);
    if (live && g == 0) y[i] = s;
}

}  // namespace

hipError_t launch_spmv(const Launch &L, hipStream_t s) {
    const int64_t n = L.hi[0] - L.lo[0];
    if (n <= 0) return hipSuccess;
    // configuration: tile = lanes per row (4, 8 or 16), order 2 = non-temporal
    // col/val loads
    const int G = L.cfg.tile;
    const bool nt = L.cfg.order == 2;
    const int64_t rows_per_block = kSpmvThreads / G;
    const unsigned nb = (unsigned)((n + rows_per_block - 1) / rows_per_block);
#define SPMV_ARGS                                                                                                  \
    (const int32_t *)L.a[0].ptr, (const int32_t *)L.a[1].ptr, (const double *)L.a[2].ptr, (const double *)L.a[3].ptr, \
        (double *)L.a[4].ptr, L.lo[0], L.hi[0]
#define SPMV_LAUNCH(GG)                                                                                 \
    do {                                                                                                \
        if (nt)                                                                                         \
            hipLaunchKernelGGL((spmv_kernel<GG, true>), dim3(nb), dim3(kSpmvThreads), 0, s, SPMV_ARGS); \
        else                                                                                            \
            hipLaunchKernelGGL((spmv_kernel<GG, false>), dim3(nb), dim3(kSpmvThreads), 0, s, SPMV_ARGS); \
    } while (0)
    switch (G) {
        case 4: SPMV_LAUNCH(4); break;
        case 16: SPMV_LAUNCH(16); break;
        default: SPMV_LAUNCH(8); break;
    }
#undef SPMV_LAUNCH
#undef SPMV_ARGS
    return hipGetLastError();
}

}  // namespace jk
