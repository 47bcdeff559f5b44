// CSR sparse matrix-vector product for gfx950: the plain row-parallel form
// and a column-banded form for x vectors larger than an XCD's L2.
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

// ---------------------------------------------------------------------------
// Column-banded form.  The columns are cut into B = 8*S bands of width W; a
// partition's entries are copied once into band-major order (all of band 0's
// entries row by row, then band 1's, ...), keeping their order inside each
// row and band.  Workgroup b of the banded launch runs on XCD b mod 8 and
// handles only the S bands of that XCD, one after the other, so the x values
// an XCD gathers at any time (one band, ncols/B doubles) stay in its L2
// instead of crossing the fabric once per gathered double.  Each row's band
// sums go to a partial array; a second kernel adds them in band order.
// ---------------------------------------------------------------------------
constexpr int kBandThreads = 256;
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;  // elements per thread in a scan block

// cnt[b*n + r] = entries of row r0 + r whose column lies in band b
__global__ void band_count_kernel(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int64_t r0,
                                  int64_t n, int64_t W, int B, int32_t *__restrict__ cnt) {
    const int64_t r = (int64_t)blockIdx.x * kBandThreads + threadIdx.x;
    if (r >= n) return;
    const int32_t kb = rp[r0 + r], ke = rp[r0 + r + 1];
    for (int b = 0; b < B; ++b) {
        int32_t c = 0;
        for (int32_t k = kb; k < ke; ++k) c += (col[k] / W == b) ? 1 : 0;
        cnt[(int64_t)b * n + r] = c;
    }
}

// exclusive scan of v[0, len) in blocks of kScanThreads*kScanPer: out gets
// each element's offset inside its block, sums[blk] the block total
__global__ void __launch_bounds__(kScanThreads)
scan_blocks_kernel(const int32_t *__restrict__ v, int64_t len, int32_t *__restrict__ out, int32_t *__restrict__ sums) {
    __shared__ int32_t sh[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanThreads * kScanPer + (int64_t)threadIdx.x * kScanPer;
    int32_t loc[kScanPer];
    int32_t t = 0;
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
        loc[u] = t;
        t += base + u < len ? v[base + u] : 0;
    }
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {  // inclusive scan of the thread totals
        const int32_t add = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    const int32_t before = threadIdx.x > 0 ? sh[threadIdx.x - 1] : 0;
#pragma unroll
    for (int u = 0; u < kScanPer; ++u)
        if (base + u < len) out[base + u] = before + loc[u];
    if (threadIdx.x == kScanThreads - 1) sums[blockIdx.x] = sh[kScanThreads - 1];
}

// exclusive scan of the nb block totals in place (one workgroup; nb is at
// most kScanThreads*kScanPer), and the grand total at sums[nb]
__global__ void __launch_bounds__(kScanThreads) scan_sums_kernel(int32_t *__restrict__ sums, int64_t nb) {
    __shared__ int32_t sh[kScanThreads];
    const int64_t base = (int64_t)threadIdx.x * kScanPer;
    int32_t loc[kScanPer];
    int32_t t = 0;
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
        loc[u] = t;
        t += base + u < nb ? sums[base + u] : 0;
    }
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const int32_t add = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    const int32_t before = threadIdx.x > 0 ? sh[threadIdx.x - 1] : 0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kScanPer; ++u)
        if (base + u < nb) sums[base + u] = before + loc[u];
    if (threadIdx.x == kScanThreads - 1) sums[nb] = sh[kScanThreads - 1];
}

__global__ void scan_add_kernel(int32_t *__restrict__ out, int64_t len, const int32_t *__restrict__ sums) {
    const int64_t i = (int64_t)blockIdx.x * kBandThreads + threadIdx.x;
    if (i < len) out[i] += sums[i / ((int64_t)kScanThreads * kScanPer)];
    if (i == len) out[len] = sums[(len + (int64_t)kScanThreads * kScanPer - 1) / ((int64_t)kScanThreads * kScanPer)];
}

// copies row r's entries into band-major order at the offsets bptr gives
__global__ void band_fill_kernel(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                 const double *__restrict__ val, int64_t r0, int64_t n, int64_t W, int B,
                                 const int32_t *__restrict__ bptr, int32_t *__restrict__ bcol,
                                 double *__restrict__ bval) {
    const int64_t r = (int64_t)blockIdx.x * kBandThreads + threadIdx.x;
    if (r >= n) return;
    const int32_t kb = rp[r0 + r], ke = rp[r0 + r + 1];
    for (int b = 0; b < B; ++b) {
        int32_t pos = bptr[(int64_t)b * n + r];
        for (int32_t k = kb; k < ke; ++k) {
            const int32_t c = col[k];
            if (c / W == b) {
                bcol[pos] = c;
                bval[pos] = val[k];
                ++pos;
            }
        }
    }
}

// partial[b*n + r] = sum over row r's entries of band b (G lanes per row,
// entries k, k+G, ... per lane, then a fixed butterfly); `wg` is the
// workgroup's index within the partition's launch (a multiple of 8 from
// the grid's start, so wg & 7 is still the XCD it runs on)
template <int G>
__device__ __forceinline__ void band_block(const int32_t *__restrict__ bptr, const int32_t *__restrict__ bcol,
                                           const double *__restrict__ bval, const double *__restrict__ x,
                                           double *__restrict__ part, int64_t n, int S, int64_t chunks, int64_t wg) {
    const int xcd = (int)(wg & 7);
    const int64_t t = wg >> 3;
    const int pass = (int)(t / chunks);
    const int64_t chunk = t % chunks;
    const int band = xcd * S + pass;
    const int64_t r = chunk * (kBandThreads / G) + threadIdx.x / G;
    const int g = threadIdx.x & (G - 1);
    double s = 0.0;
    if (r < n) {
        const int32_t kb = bptr[(int64_t)band * n + r], ke = bptr[(int64_t)band * n + r + 1];
        for (int32_t k = kb + g; k < ke; k += G)
            s += __builtin_nontemporal_load(&bval[k]) * x[__builtin_nontemporal_load(&bcol[k])];
    }
#pragma unroll
    for (int m = 1; m < G; m <<= 1) s += __shfl_xor(s, m, kWave);
    if (r < n && g == 0) part[(int64_t)band * n + r] = s;
}

template <int G>
__global__ void __launch_bounds__(kBandThreads)
spmv_band_kernel(const int32_t *__restrict__ bptr, const int32_t *__restrict__ bcol, const double *__restrict__ bval,
                 const double *__restrict__ x, double *__restrict__ part, int64_t n, int S, int64_t chunks) {
    band_block<G>(bptr, bcol, bval, x, part, n, S, chunks, blockIdx.x);
}

// The partitions of one banded product in one launch: partition q's
// workgroups [wg_begin, wg_begin + 8*S*chunks) and, for the combine,
// [comb_begin, comb_begin + ceil(n / kBandThreads)).  Descriptors are read
// through the constant address space (their pointers are then known to be
// global).
struct SpmvPart {
    const int32_t *bptr, *bcol;
    const double *bval, *x;
    double *part, *y;
    int64_t n, r0, chunks, wg_begin, comb_begin;
};
struct SpmvParts {
    SpmvPart p[kMaxPack];
    int32_t n;
};
typedef const __attribute__((address_space(4))) SpmvPart ConstSpmvPart;

template <int G>
__global__ void __launch_bounds__(kBandThreads) spmv_band_parts_kernel(SpmvParts sp, int S) {
    ConstSpmvPart *cp = (ConstSpmvPart *)&sp.p[0];
    const int64_t b = blockIdx.x;
    int q = 0;
    for (int k = 1; k < sp.n; ++k)
        if (cp[k].wg_begin <= b) q = k;
    band_block<G>(cp[q].bptr, cp[q].bcol, cp[q].bval, cp[q].x, cp[q].part, cp[q].n, S, cp[q].chunks,
                  b - cp[q].wg_begin);
}

__global__ void band_combine_parts_kernel(SpmvParts sp, int B) {
    ConstSpmvPart *cp = (ConstSpmvPart *)&sp.p[0];
    const int64_t b = blockIdx.x;
    int q = 0;
    for (int k = 1; k < sp.n; ++k)
        if (cp[k].comb_begin <= b) q = k;
    const double *part = cp[q].part;
    double *y = cp[q].y;
    const int64_t n = cp[q].n, r = (b - cp[q].comb_begin) * kBandThreads + threadIdx.x;
    if (r >= n) return;
    double s = 0.0;
    for (int k = 0; k < B; ++k) s += part[(int64_t)k * n + r];
    y[cp[q].r0 + r] = s;
}

// One lane per row and band, R rows per lane (rows r, r + blockDim, ...):
// the band offsets, the first two entries and their x values of all R rows
// are loaded before any is used, so each lane keeps 2R gathers in flight;
// entries beyond the second follow in increasing k (the same additions, in
// the same order, as one lane walking the row).
template <int R>
__global__ void __launch_bounds__(kBandThreads)
spmv_band_rows_kernel(const int32_t *__restrict__ bptr, const int32_t *__restrict__ bcol,
                      const double *__restrict__ bval, const double *__restrict__ x, double *__restrict__ part,
                      int64_t n, int S, int64_t chunks) {
    const int64_t wg = blockIdx.x;
    const int xcd = (int)(wg & 7);
    const int64_t t = wg >> 3;
    const int pass = (int)(t / chunks);
    const int64_t chunk = t % chunks;
    const int64_t band_base = (int64_t)(xcd * S + pass) * n;
    int64_t r[R];
    int32_t kb[R], ke[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
        r[u] = chunk * (kBandThreads * R) + u * kBandThreads + threadIdx.x;
        kb[u] = ke[u] = 0;
        if (r[u] < n) {
            kb[u] = bptr[band_base + r[u]];
            ke[u] = bptr[band_base + r[u] + 1];
        }
    }
    int32_t c0[R], c1[R];
    double v0[R], v1[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
        c0[u] = c1[u] = -1;
        v0[u] = v1[u] = 0.0;
        if (kb[u] < ke[u]) {
            c0[u] = __builtin_nontemporal_load(&bcol[kb[u]]);
            v0[u] = __builtin_nontemporal_load(&bval[kb[u]]);
        }
        if (kb[u] + 1 < ke[u]) {
            c1[u] = __builtin_nontemporal_load(&bcol[kb[u] + 1]);
            v1[u] = __builtin_nontemporal_load(&bval[kb[u] + 1]);
        }
    }
    double x0[R], x1[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
        x0[u] = c0[u] >= 0 ? x[c0[u]] : 0.0;
        x1[u] = c1[u] >= 0 ? x[c1[u]] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
        double s = 0.0;
        if (c0[u] >= 0) s += v0[u] * x0[u];
        if (c1[u] >= 0) s += v1[u] * x1[u];
        for (int32_t k = kb[u] + 2; k < ke[u]; ++k)
            s += __builtin_nontemporal_load(&bval[k]) * x[__builtin_nontemporal_load(&bcol[k])];
        if (r[u] < n) part[band_base + r[u]] = s;
    }
}

// y[r0 + r] = partial[0][r] + partial[1][r] + ... in band order
__global__ void band_combine_kernel(const double *__restrict__ part, int64_t n, int B, double *__restrict__ y,
                                    int64_t r0) {
    const int64_t r = (int64_t)blockIdx.x * kBandThreads + threadIdx.x;
    if (r >= n) return;
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += part[(int64_t)b * n + r];
    y[r0 + r] = s;
}

}  // namespace

int64_t band_width(int64_t ncols, int bands) { return (ncols + bands - 1) / bands; }

int64_t band_scan_blocks(int64_t len) { return (len + (int64_t)kScanThreads * kScanPer - 1) / ((int64_t)kScanThreads * kScanPer); }

hipError_t build_bands(const Launch &L, const BandBufs &bb, hipStream_t s) {
    const int64_t r0 = L.lo[0], n = L.hi[0] - L.lo[0];
    if (n <= 0) return hipSuccess;
    const int B = bb.bands;
    const int64_t W = band_width(bb.ncols, B);
    const int64_t len = (int64_t)B * n;
    const int64_t nb = band_scan_blocks(len);
    if (nb > (int64_t)kScanThreads * kScanPer) return hipErrorInvalidValue;
    const unsigned rows_grid = (unsigned)((n + kBandThreads - 1) / kBandThreads);
    const int32_t *rp = (const int32_t *)L.a[0].ptr, *col = (const int32_t *)L.a[1].ptr;
    const double *val = (const double *)L.a[2].ptr;
    int32_t *cnt = (int32_t *)bb.part;  // the partials are free until the product runs
    hipLaunchKernelGGL(band_count_kernel, dim3(rows_grid), dim3(kBandThreads), 0, s, rp, col, r0, n, W, B, cnt);
    hipLaunchKernelGGL(scan_blocks_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, cnt, len, bb.bptr, bb.sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(kScanThreads), 0, s, bb.sums, nb);
    hipLaunchKernelGGL(scan_add_kernel, dim3((unsigned)((len + kBandThreads) / kBandThreads)), dim3(kBandThreads), 0, s,
                       bb.bptr, len, bb.sums);
    hipLaunchKernelGGL(band_fill_kernel, dim3(rows_grid), dim3(kBandThreads), 0, s, rp, col, val, r0, n, W, B, bb.bptr,
                       bb.bcol, bb.bval);
    return hipGetLastError();
}

hipError_t launch_spmv_banded(const Launch &L, const BandBufs &bb, hipStream_t s) {
    const int64_t r0 = L.lo[0], n = L.hi[0] - L.lo[0];
    if (n <= 0) return hipSuccess;
    const int G = L.cfg.tile;
    const int S = bb.bands / 8;
    const double *x = (const double *)L.a[3].ptr;
    if (G == 1 && (L.cfg.rows == 2 || L.cfg.rows == 4)) {  // several rows per lane
        const int R = L.cfg.rows;
        const int64_t chunks = (n + (int64_t)kBandThreads * R - 1) / ((int64_t)kBandThreads * R);
        const unsigned grid = (unsigned)(8 * (int64_t)S * chunks);
        if (R == 2)
            hipLaunchKernelGGL((spmv_band_rows_kernel<2>), dim3(grid), dim3(kBandThreads), 0, s, bb.bptr, bb.bcol,
                               bb.bval, x, bb.part, n, S, chunks);
        else
            hipLaunchKernelGGL((spmv_band_rows_kernel<4>), dim3(grid), dim3(kBandThreads), 0, s, bb.bptr, bb.bcol,
                               bb.bval, x, bb.part, n, S, chunks);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(band_combine_kernel, dim3((unsigned)((n + kBandThreads - 1) / kBandThreads)),
                           dim3(kBandThreads), 0, s, bb.part, n, bb.bands, (double *)L.a[4].ptr, r0);
        return hipGetLastError();
    }
    const int64_t chunks = (n + kBandThreads / G - 1) / (kBandThreads / G);
    const unsigned grid = (unsigned)(8 * (int64_t)S * chunks);
#define SPMV_BAND(GG)                                                                                           \
    hipLaunchKernelGGL((spmv_band_kernel<GG>), dim3(grid), dim3(kBandThreads), 0, s, bb.bptr, bb.bcol, bb.bval, x, \
                       bb.part, n, S, chunks)
    switch (G) {  // a row's band holds about nnz/bands entries: few lanes per row
        case 1: SPMV_BAND(1); break;
        case 2: SPMV_BAND(2); break;
        case 4: SPMV_BAND(4); break;
        case 16: SPMV_BAND(16); break;
        default: SPMV_BAND(8); break;
    }
#undef SPMV_BAND
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(band_combine_kernel, dim3((unsigned)((n + kBandThreads - 1) / kBandThreads)), dim3(kBandThreads),
                       0, s, bb.part, n, bb.bands, (double *)L.a[4].ptr, r0);
    return hipGetLastError();
}

hipError_t launch_spmv_banded_parts(const Launch *L, const BandBufs *bb, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (n > kMaxPack) return hipErrorInvalidValue;
    const int G = L[0].cfg.tile;
    const int S = bb[0].bands / 8;
    if (G != 1 && G != 2 && G != 4 && G != 8 && G != 16) return hipErrorInvalidValue;
    SpmvParts sp{};
    int64_t wg = 0, comb = 0;
    for (int k = 0; k < n; ++k) {
        const int64_t rows = L[k].hi[0] - L[k].lo[0];
        if (rows <= 0) continue;
        if (bb[k].bands != bb[0].bands) return hipErrorInvalidValue;
        SpmvPart &d = sp.p[sp.n++];
        d.bptr = bb[k].bptr;
        d.bcol = bb[k].bcol;
        d.bval = bb[k].bval;
        d.x = (const double *)L[k].a[3].ptr;
        d.part = bb[k].part;
        d.y = (double *)L[k].a[4].ptr;
        d.n = rows;
        d.r0 = L[k].lo[0];
        d.chunks = (rows + kBandThreads / G - 1) / (kBandThreads / G);
        d.wg_begin = wg;
        d.comb_begin = comb;
        wg += 8 * (int64_t)S * d.chunks;
        comb += (rows + kBandThreads - 1) / kBandThreads;
    }
    if (sp.n == 0) return hipSuccess;
    if (wg > (int64_t)INT32_MAX) return hipErrorInvalidValue;
#define SPMV_BAND_PARTS(GG) \
    hipLaunchKernelGGL((spmv_band_parts_kernel<GG>), dim3((unsigned)wg), dim3(kBandThreads), 0, s, sp, S)
    switch (G) {
        case 1: SPMV_BAND_PARTS(1); break;
        case 2: SPMV_BAND_PARTS(2); break;
        case 4: SPMV_BAND_PARTS(4); break;
        case 16: SPMV_BAND_PARTS(16); break;
        default: SPMV_BAND_PARTS(8); break;
    }
#undef SPMV_BAND_PARTS
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(band_combine_parts_kernel, dim3((unsigned)comb), dim3(kBandThreads), 0, s, sp, bb[0].bands);
    return hipGetLastError();
}

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
