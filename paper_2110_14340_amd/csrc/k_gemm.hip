// Dense FP64 contraction C = A*B on the gfx950 matrix cores
// (v_mfma_f64_16x16x4f64).
//
// Workgroup: 256 threads (4 waves) computing a 128x128 tile of C; each wave
// owns a 64x64 sub-tile as 4x4 MFMA blocks of 16x16 (64 FP64 accumulators
// per lane).  The k dimension is walked in slabs of 16 or 32 in increasing
// order (no split-k, so every element's accumulation order is the same for
// every partition count and slab depth), staged through LDS: the next
// slab's global loads are in flight in registers while the current slab
// feeds the matrix cores.
//
// MFMA operand layout (16x16x4, FP64, wave64): lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; accumulator element r of lane l is D[4*r + l/16][l%16]
// (rows interleave across the four 16-lane groups).
#include "k_common.h"
#include "kernels.h"

namespace jk {

namespace {

constexpr int BM = 128, BN = 128;
constexpr int kGemmThreads = 256;
constexpr int SB = BN + 16;  // LDS row stride of B (doubles)

typedef double d4 __attribute__((ext_vector_type(4)));

// Tile of workgroup b: the 8 XCDs take consecutive workgroup ids in turn, so
// XCD x is given the x-th contiguous eighth of the tiles; inside it, tiles
// are walked in groups of 8 tile-rows (column by column), so the
// workgroups resident on one XCD share few A row-panels and B column-panels
// and most panel reads hit that XCD's L2.
__device__ __forceinline__ void gemm_tile(int64_t tiles_m, int64_t tiles_n, int64_t *ti, int64_t *tj) {
    const int64_t b = blockIdx.x, n = gridDim.x;
    const int64_t t = (n & 7) == 0 ? (b & 7) * (n >> 3) + (b >> 3) : b;
    constexpr int64_t G = 8;
    const int64_t group = t / (G * tiles_n);
    const int64_t first = group * G;
    const int64_t rows = tiles_m - first < G ? tiles_m - first : G;
    const int64_t in_group = t - group * G * tiles_n;
    *ti = first + in_group % rows;
    *tj = in_group / rows;
}

// BK = 16: two LDS buffers, one barrier per k-slab.  BK = 32: one LDS
// buffer (the register staging holds the next slab), two barriers per slab
// of twice the work, so the next slab's loads have longer to arrive.
// WN = waves along N: 2 (256 threads, 64x64 per wave) or 4 (512 threads,
// 64x32 per wave: half the accumulators per lane, twice the waves).
// (the 512-thread form asks for four waves per SIMD, i.e. at most 128
// registers, so that two of its workgroups fit on a compute unit)
template <int BK, int WN>
__global__ void __launch_bounds__(kGemmThreads * WN / 2, (WN == 4 && BK == 16) ? 4 : 1)
gemm_kernel(const double *__restrict__ A, const double *__restrict__ B, double *__restrict__ C, int64_t m_lo,
            int64_t m_hi, int64_t N, int64_t L, int64_t lda, int64_t ldb, int64_t ldc, int64_t n_lo, int64_t n_hi,
            int64_t tiles_m, int64_t tiles_n) {
    constexpr int NT = kGemmThreads * WN / 2;  // threads
    constexpr int JT = 4 * 2 / WN;             // 16-column MFMA blocks per wave
    constexpr int NBUF = BK == 16 ? 2 : 1;
    constexpr int SA = BK + 2;           // LDS row stride of A (doubles): conflict-free fragment reads
    constexpr int U = 64 * BK / NT;      // double pairs per thread per operand and slab
    constexpr int KP = BK / 2;           // A: k pairs per row
    __shared__ __align__(16) double As[NBUF][BM * SA];
    __shared__ __align__(16) double Bs[NBUF][BK * SB];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    int64_t ti, tj;
    gemm_tile(tiles_m, tiles_n, &ti, &tj);
    const int64_t row0 = m_lo + ti * BM;
    const int64_t col0 = n_lo + tj * BN;
    const bool full_mn = row0 + BM <= m_hi && col0 + BN <= n_hi && (lda & 1) == 0 && (ldb & 1) == 0;

    // global -> register staging: the A tile (128 x BK) and the B tile
    // (BK x 128) are 64*BK double pairs each, U per thread (16-byte loads for
    // full tiles)
    dvec2 ra[U], rb[U];
    auto load_tiles = [&](int64_t k0) {
        const bool full = full_mn && k0 + BK <= L;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = tid + u * NT;
            const int r = idx / KP, kp = (idx % KP) * 2;    // A: row, k pair
            const int kr = idx >> 6, cp = (idx & 63) * 2;   // B: k, column pair
            if (full) {
                ra[u] = *reinterpret_cast<const dvec2 *>(A + (row0 + r) * lda + k0 + kp);
                rb[u] = *reinterpret_cast<const dvec2 *>(B + (k0 + kr) * ldb + col0 + cp);
            } else {
                const int64_t gi = row0 + r, gk = k0 + kp;
                ra[u].x = (gi < m_hi && gk < L) ? A[gi * lda + gk] : 0.0;
                ra[u].y = (gi < m_hi && gk + 1 < L) ? A[gi * lda + gk + 1] : 0.0;
                const int64_t gkb = k0 + kr, gj = col0 + cp;
                rb[u].x = (gkb < L && gj < n_hi) ? B[gkb * ldb + gj] : 0.0;
                rb[u].y = (gkb < L && gj + 1 < n_hi) ? B[gkb * ldb + gj + 1] : 0.0;
            }
        }
    };
    auto store_tiles = [&](int buf) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = tid + u * NT;
            const int r = idx / KP, kp = (idx % KP) * 2;
            *reinterpret_cast<dvec2 *>(&As[buf][r * SA + kp]) = ra[u];
            const int kr = idx >> 6, cp = (idx & 63) * 2;
            *reinterpret_cast<dvec2 *>(&Bs[buf][kr * SB + cp]) = rb[u];
        }
    };

    d4 acc[4][JT];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < JT; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    const int nk = (int)((L + BK - 1) / BK);
    load_tiles(0);
    store_tiles(0);
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = NBUF == 2 ? (kt & 1) : 0;
        if (kt + 1 < nk) load_tiles((int64_t)(kt + 1) * BK);
        const double *as = As[buf];
        const double *bs = Bs[buf];
#pragma unroll
        for (int kk = 0; kk < BK / 4; ++kk) {
            double a[4], b[JT];
            const int kq = kk * 4 + (lane >> 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = as[(wm * 64 + i * 16 + (lane & 15)) * SA + kq];
#pragma unroll
            for (int j = 0; j < JT; ++j) b[j] = bs[kq * SB + wn * (16 * JT) + j * 16 + (lane & 15)];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < JT; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (kt + 1 < nk) {
            if (NBUF == 1) __syncthreads();  // every wave is done reading the single buffer
            store_tiles(NBUF == 2 ? (buf ^ 1) : 0);
        }
        __syncthreads();
    }
    // write back: acc[i][j][r] -> C[row0 + wm*64 + i*16 + 4*r + lane/16][col0 + wn*16*JT + j*16 + lane%16]
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t gi = row0 + wm * 64 + i * 16 + 4 * r + (lane >> 4);
            if (gi >= m_hi) continue;
#pragma unroll
            for (int j = 0; j < JT; ++j) {
                const int64_t gj = col0 + wn * (16 * JT) + j * 16 + (lane & 15);
                if (gj < n_hi) C[gi * ldc + gj] = acc[i][j][r];
            }
        }
}

}  // namespace

hipError_t launch_gemm(const Launch &L, hipStream_t s) {
    // arguments: A (M x Lk), B (Lk x N), C (M x N); iteration box rows
    // [lo0, hi0) of C, columns [lo1, hi1)
    const int64_t m = L.hi[0] - L.lo[0], n = L.hi[1] - L.lo[1];
    if (m <= 0 || n <= 0) return hipSuccess;
    const int64_t Lk = L.a[0].row_elems;
    const int64_t N = L.a[2].row_elems;
    const int64_t tiles_m = (m + BM - 1) / BM, tiles_n = (n + BN - 1) / BN;
    // configuration fields: `tile` = k-slab depth (16 or 32), `bx` = threads
    // (256: 4 waves of 64x64, 512: 8 waves of 64x32)
    const dim3 grid((unsigned)(tiles_m * tiles_n));
#define GEMM_ARGS                                                                                                 \
    (const double *)L.a[0].ptr, (const double *)L.a[1].ptr, (double *)L.a[2].ptr, L.lo[0], L.hi[0], N, Lk, Lk, \
        L.a[1].row_elems, N, L.lo[1], L.hi[1], tiles_m, tiles_n
    const bool wide = L.cfg.bx == 512;
    if (L.cfg.tile == 16) {
        if (wide)
            hipLaunchKernelGGL((gemm_kernel<16, 4>), grid, dim3(512), 0, s, GEMM_ARGS);
        else
            hipLaunchKernelGGL((gemm_kernel<16, 2>), grid, dim3(256), 0, s, GEMM_ARGS);
    } else {
        if (wide)
            hipLaunchKernelGGL((gemm_kernel<32, 4>), grid, dim3(512), 0, s, GEMM_ARGS);
        else
            hipLaunchKernelGGL((gemm_kernel<32, 2>), grid, dim3(256), 0, s, GEMM_ARGS);
    }
#undef GEMM_ARGS
    return hipGetLastError();
}

}  // namespace jk
