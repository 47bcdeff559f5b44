// Reduction loop body (sum / sum of squares), per-partition finaliser and
// the cross-partition combine, for gfx950.
//
// Order of additions (fixed for a given configuration and partition): each
// lane keeps 8 running sums over a grid-stride walk, adds them pairwise,
// the wave adds its lanes by a butterfly, the workgroup adds its waves in
// order, the finaliser adds workgroup partials with a fixed tree, and the
// combine adds the partitions' results in partition order (the paper filters
// a reduction by the range of the outer iterator on each device and then
// combines the per-device values, Sec. "Predicate-Based Filtering").
#include "k_common.h"
#include "kernels.h"

namespace jk {

namespace {

constexpr int kSumThreads = 256;
constexpr int kSumUnroll = 8;
constexpr int kSumMaxBlocks = 2048;

template <bool SQ>
__global__ void __launch_bounds__(kSumThreads)
sum_kernel(const double *__restrict__ x, int64_t begin, int64_t n, double *__restrict__ wg_partials) {
    __shared__ double sh[kSumThreads / kWave];
    const int64_t chunk = (int64_t)kSumThreads * kSumUnroll;
    const int64_t stride = chunk * gridDim.x;
    double a[kSumUnroll];
#pragma unroll
    for (int u = 0; u < kSumUnroll; ++u) a[u] = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * chunk; base < n; base += stride) {
        double v[kSumUnroll];
#pragma unroll
        for (int u = 0; u < kSumUnroll; ++u) {
            const int64_t e = base + threadIdx.x + (int64_t)u * kSumThreads;
            v[u] = e < n ? x[begin + e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kSumUnroll; ++u) a[u] += SQ ? v[u] * v[u] : v[u];
    }
    const double t = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    const double s = block_sum(t, sh);
    if (threadIdx.x == 0) wg_partials[blockIdx.x] = s;
}

// The partitions of one SUM loop in one launch: partition q's workgroups
// [wg_begin, wg_begin + nb) run exactly the grid-stride walk its own launch
// of nb workgroups would, so every partial has the same bits.
struct SumPart {
    const double *x;
    int64_t begin, n;  // the partition's elements x[begin .. begin + n)
    int64_t wg_begin, nb;
    double *partials;  // its nb workgroup partials
};
struct SumParts {
    SumPart p[kMaxPack];
    int32_t n;
};
typedef const __attribute__((address_space(4))) SumPart ConstSumPart;

template <bool SQ>
__global__ void __launch_bounds__(kSumThreads) sum_parts_kernel(SumParts sp) {
    __shared__ double sh[kSumThreads / kWave];
    ConstSumPart *cp = (ConstSumPart *)&sp.p[0];
    const int64_t b = blockIdx.x;
    int q = 0;
    for (int k = 1; k < sp.n; ++k)
        if (cp[k].wg_begin <= b) q = k;
    const double *x = cp[q].x;
    double *partials = cp[q].partials;
    const int64_t begin = cp[q].begin, n = cp[q].n, nb = cp[q].nb, local = b - cp[q].wg_begin;
    const int64_t chunk = (int64_t)kSumThreads * kSumUnroll;
    const int64_t stride = chunk * nb;
    double a[kSumUnroll];
#pragma unroll
    for (int u = 0; u < kSumUnroll; ++u) a[u] = 0.0;
    for (int64_t base = local * chunk; base < n; base += stride) {
        double v[kSumUnroll];
#pragma unroll
        for (int u = 0; u < kSumUnroll; ++u) {
            const int64_t e = base + threadIdx.x + (int64_t)u * kSumThreads;
            v[u] = e < n ? x[begin + e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kSumUnroll; ++u) a[u] += SQ ? v[u] * v[u] : v[u];
    }
    const double t = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    const double s = block_sum(t, sh);
    if (threadIdx.x == 0) partials[local] = s;
}

// out = ordered sum of p[0..n): thread t keeps 8 running sums, sum u taking
// p[t + (8j+u)*1024] for j = 0, 1, ... (eight independent loads in flight
// per step instead of one dependent chain), adds them pairwise, then the
// workgroup sum.
constexpr int kFinThreads = 1024;
constexpr int kFinUnroll = 8;

__device__ __forceinline__ void finalise_block(const double *__restrict__ p, int64_t n, double *__restrict__ out,
                                               double *sh) {
    double a[kFinUnroll];
#pragma unroll
    for (int u = 0; u < kFinUnroll; ++u) a[u] = 0.0;
    for (int64_t base = threadIdx.x; base < n; base += (int64_t)kFinThreads * kFinUnroll) {
        double v[kFinUnroll];
#pragma unroll
        for (int u = 0; u < kFinUnroll; ++u) {
            const int64_t i = base + (int64_t)u * kFinThreads;
            v[u] = i < n ? p[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kFinUnroll; ++u) a[u] += v[u];
    }
    const double t = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    const double s = block_sum(t, sh);
    if (threadIdx.x == 0) *out = s;
}

__global__ void __launch_bounds__(kFinThreads)
finalise_kernel(const double *__restrict__ p, int64_t n, double *__restrict__ out) {
    __shared__ double sh[kFinThreads / kWave];
    finalise_block(p, n, out, sh);
}

// Workgroup k finalises segment k (the same additions as finalise_kernel).
__global__ void __launch_bounds__(kFinThreads) finalise_many_kernel(const double *__restrict__ base, Segments seg) {
    __shared__ double sh[kFinThreads / kWave];
    const int k = blockIdx.x;
    finalise_block(base + seg.off[k], seg.n[k], seg.out[k], sh);
}

__global__ void combine_kernel(const double *__restrict__ partials, CombineList list, double *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < list.n; ++k) s += partials[list.idx[k]];
        *out = s;
    }
}

}  // namespace

int64_t sum_workgroups(const Launch &L) {
    const int64_t n = (L.hi[0] - L.lo[0]) * L.a[0].row_elems;
    int64_t nb = (n + (int64_t)kSumThreads * kSumUnroll - 1) / ((int64_t)kSumThreads * kSumUnroll);
    if (nb > kSumMaxBlocks) nb = kSumMaxBlocks;
    return nb < 1 ? 1 : nb;
}

hipError_t launch_sum(const Launch &L, hipStream_t s) {
    const int64_t n = (L.hi[0] - L.lo[0]) * L.a[0].row_elems;
    const int64_t begin = L.lo[0] * L.a[0].row_elems;
    const int64_t nb = sum_workgroups(L);
    const double *x = (const double *)L.a[0].ptr;
    if (L.scalars[0] != 0.0)
        hipLaunchKernelGGL(sum_kernel<true>, dim3((unsigned)nb), dim3(kSumThreads), 0, s, x, begin, n, L.wg_partials);
    else
        hipLaunchKernelGGL(sum_kernel<false>, dim3((unsigned)nb), dim3(kSumThreads), 0, s, x, begin, n, L.wg_partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalise(L.wg_partials, nb, L.part_out, s);
}

hipError_t launch_sum_parts(const Launch *L, int n, double *wg_partials, int64_t wg_capacity, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (n > kMaxPack) return hipErrorInvalidValue;
    SumParts sp{};
    Segments seg{};
    int64_t wg = 0;
    for (int k = 0; k < n; ++k) {
        const Launch &Lk = L[k];
        const int64_t nb = sum_workgroups(Lk);
        SumPart &d = sp.p[sp.n++];
        d.x = (const double *)Lk.a[0].ptr;
        d.begin = Lk.lo[0] * Lk.a[0].row_elems;
        d.n = (Lk.hi[0] - Lk.lo[0]) * Lk.a[0].row_elems;
        d.wg_begin = wg;
        d.nb = nb;
        d.partials = wg_partials + wg;
        seg.off[seg.count] = wg;
        seg.n[seg.count] = nb;
        seg.out[seg.count] = Lk.part_out;
        ++seg.count;
        wg += nb;
    }
    if (wg > wg_capacity) return hipErrorInvalidValue;
    if (L[0].scalars[0] != 0.0)
        hipLaunchKernelGGL(sum_parts_kernel<true>, dim3((unsigned)wg), dim3(kSumThreads), 0, s, sp);
    else
        hipLaunchKernelGGL(sum_parts_kernel<false>, dim3((unsigned)wg), dim3(kSumThreads), 0, s, sp);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_finalise_many(wg_partials, seg, s);
}

hipError_t launch_finalise(const double *partials, int64_t n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(finalise_kernel, dim3(1), dim3(kFinThreads), 0, s, partials, n, out);
    return hipGetLastError();
}

hipError_t launch_finalise_many(const double *base, const Segments &seg, hipStream_t s) {
    if (seg.count <= 0) return hipSuccess;
    if (seg.count > kMaxPack) return hipErrorInvalidValue;
    hipLaunchKernelGGL(finalise_many_kernel, dim3((unsigned)seg.count), dim3(kFinThreads), 0, s, base, seg);
    return hipGetLastError();
}

hipError_t launch_combine(const double *partials, const CombineList &list, double *out, hipStream_t s) {
    hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(64), 0, s, partials, list, out);
    return hipGetLastError();
}

}  // namespace jk
