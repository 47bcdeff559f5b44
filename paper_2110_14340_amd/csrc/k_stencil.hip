// Stencil loop bodies for gfx950: Jacobi-2D 5-point and heat-3D 7-point.
//
// Both stream the array once from HBM: each lane owns VEC consecutive
// elements of the contiguous (innermost) dimension and marches through
// `tile` rows (2-D) or planes (3-D) of the outer dimension, keeping the
// previous, current and next row/plane in registers, so every element of
// the marched dimension is loaded once per lane column.  Horizontal
// neighbours come from the adjacent lanes by cross-lane shuffles; only the
// two edge lanes of a wave fetch one extra element each (a cache hit).
// Loads for the next U rows are issued before the current U rows are
// computed so each lane keeps several 16-byte loads in flight.
//
// Arithmetic (with floating-point contraction disabled at build time):
//   Jacobi: out = 0.25 * ((up + down) + (left + right))
//   Heat:   lap = ((xm + xp) + (ym + yp)) + (zm + zp) - 6.0*u ;  out = u + alpha*lap
// which is the operation order of the CPU oracle, so results are bit-exact.
#include "k_common.h"
#include "kernels.h"

namespace jk {

namespace {

constexpr int kU = 4;  // rows loaded ahead of the rows being computed

// ---------------------------------------------------------------------------
// Jacobi-2D
// ---------------------------------------------------------------------------
// One ring entry: VEC own values plus, for the two edge lanes of the wave,
// the element just left (lane 0) or right (lane 63) of the wave's span.
template <int VEC>
struct Row {
    double v[VEC];
    double edge;
};

template <int VEC>
__device__ __forceinline__ void load_row(const double *__restrict__ in, int64_t row, int64_t nx, int64_t j,
                                         bool inb, int lane, bool need_l, bool need_r, Row<VEC> &r) {
    const double *p = in + row * nx + j;
    if (inb) {
        load_vec<VEC>(p, r.v);
    } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) r.v[v] = 0.0;
    }
    r.edge = 0.0;
    if (lane == 0 && need_l) r.edge = p[-1];
    if (lane == kWave - 1 && need_r) r.edge = p[VEC];
}

template <int VEC>
__global__ void __launch_bounds__(1024)
jacobi2d_kernel(const double *__restrict__ in, double *__restrict__ out, int64_t nx, int64_t r_lo, int64_t r_hi,
                int64_t c_lo, int64_t c_hi, int64_t col0, int tile) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t j = col0 + ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
    const int64_t i0 = r_lo + ((int64_t)blockIdx.y * blockDim.y + threadIdx.y) * tile;
    if (i0 >= r_hi) return;  // uniform across the wave (one threadIdx.y per wave)
    const int64_t i1 = i0 + tile < r_hi ? i0 + tile : r_hi;

    const bool inb = j < c_hi + 1 && j < nx;  // lane holds columns needed by the box
    bool comp[VEC];
    bool all = true;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        comp[v] = (j + v >= c_lo) && (j + v < c_hi);
        all = all && comp[v];
    }
    // the wave's edge lanes need one more element when they compute the
    // element next to the wave's span
    const bool need_l = comp[0];
    const bool need_r = comp[VEC - 1];

    Row<VEC> r[kU + 2];
#pragma unroll
    for (int k = 0; k < kU + 2; ++k) {
        const int64_t row = i0 - 1 + k;
        if (row <= i1) load_row<VEC>(in, row, nx, j, inb, lane, need_l, need_r, r[k]);
    }
    for (int64_t i = i0; i < i1; i += kU) {
        Row<VEC> nxt[kU];
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            const int64_t row = i + kU + 1 + k;
            if (row <= i1) load_row<VEC>(in, row, nx, j, inb, lane, need_l, need_r, nxt[k]);
        }
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            const int64_t row = i + k;
            if (row < i1) {
                const Row<VEC> &up = r[k], &mid = r[k + 1], &dn = r[k + 2];
                double left[VEC], right[VEC];
                // left of v[0] is the previous lane's last value; right of
                // v[VEC-1] is the next lane's first value
                double lprev = __shfl_up(mid.v[VEC - 1], 1, kWave);
                double rnext = __shfl_down(mid.v[0], 1, kWave);
                if (lane == 0) lprev = mid.edge;
                if (lane == kWave - 1) rnext = mid.edge;
                left[0] = lprev;
                right[VEC - 1] = rnext;
#pragma unroll
                for (int v = 1; v < VEC; ++v) left[v] = mid.v[v - 1];
#pragma unroll
                for (int v = 0; v < VEC - 1; ++v) right[v] = mid.v[v + 1];
                double o[VEC];
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const double vert = up.v[v] + dn.v[v];
                    const double horz = left[v] + right[v];
                    o[v] = 0.25 * (vert + horz);
                }
                double *q = out + row * nx + j;
                if (all) {
                    store_vec<VEC>(q, o);
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v)
                        if (comp[v]) q[v] = o[v];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) r[k] = r[kU + k];
#pragma unroll
        for (int k = 0; k < kU; ++k) r[2 + k] = nxt[k];
    }
}

// ---------------------------------------------------------------------------
// Heat-3D (+ optional residual)
// ---------------------------------------------------------------------------
template <int VEC>
struct Col {
    double v[VEC];
    double edge;
};

template <int VEC>
__device__ __forceinline__ void load_col(const double *__restrict__ in, int64_t z, int64_t y, int64_t ny,
                                         int64_t nx, int64_t x, bool inb, int lane, bool need_l, bool need_r,
                                         Col<VEC> &c) {
    const double *p = in + (z * ny + y) * nx + x;
    if (inb) {
        load_vec<VEC>(p, c.v);
    } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) c.v[v] = 0.0;
    }
    c.edge = 0.0;
    if (lane == 0 && need_l) c.edge = p[-1];
    if (lane == kWave - 1 && need_r) c.edge = p[VEC];
}

template <int VEC, bool RES>
__global__ void __launch_bounds__(1024)
heat3d_kernel(const double *__restrict__ in, double *__restrict__ out, int64_t ny, int64_t nx, int64_t z_lo,
              int64_t z_hi, int64_t y_lo, int64_t y_hi, int64_t x_lo, int64_t x_hi, int64_t col0, int tile,
              double alpha, double *__restrict__ wg_partials) {
    __shared__ double sh[16];
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t x = col0 + ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
    const int64_t y = y_lo + (int64_t)blockIdx.y * blockDim.y + threadIdx.y;
    const int64_t z0 = z_lo + (int64_t)blockIdx.z * tile;
    const int64_t z1 = z0 + tile < z_hi ? z0 + tile : z_hi;
    double acc = 0.0;
    // y is uniform per wave; a wave outside the box does no memory access
    // but must still take part in the workgroup reduction
    if (y < y_hi && z0 < z1) {
        const bool inb = x < x_hi + 1 && x < nx;
        bool comp[VEC];
        bool all = true;
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            comp[v] = (x + v >= x_lo) && (x + v < x_hi);
            all = all && comp[v];
        }
        const bool need_l = comp[0];
        const bool need_r = comp[VEC - 1];
        const int64_t plane = ny * nx;

        Col<VEC> r[kU + 2];
#pragma unroll
        for (int k = 0; k < kU + 2; ++k) {
            const int64_t z = z0 - 1 + k;
            if (z <= z1) load_col<VEC>(in, z, y, ny, nx, x, inb, lane, need_l, need_r, r[k]);
        }
        for (int64_t zb = z0; zb < z1; zb += kU) {
            Col<VEC> nxt[kU];
#pragma unroll
            for (int k = 0; k < kU; ++k) {
                const int64_t z = zb + kU + 1 + k;
                if (z <= z1) load_col<VEC>(in, z, y, ny, nx, x, inb, lane, need_l, need_r, nxt[k]);
            }
#pragma unroll
            for (int k = 0; k < kU; ++k) {
                const int64_t z = zb + k;
                if (z < z1) {
                    const Col<VEC> &zm = r[k], &c = r[k + 1], &zp = r[k + 2];
                    // y neighbours of this plane (rows of the same plane, cache hits)
                    double ym[VEC], yp[VEC];
                    const double *pc = in + (z * ny + y) * nx + x;
                    if (inb) {
                        load_vec<VEC>(pc - nx, ym);
                        load_vec<VEC>(pc + nx, yp);
                    } else {
#pragma unroll
                        for (int v = 0; v < VEC; ++v) ym[v] = yp[v] = 0.0;
                    }
                    double lprev = __shfl_up(c.v[VEC - 1], 1, kWave);
                    double rnext = __shfl_down(c.v[0], 1, kWave);
                    if (lane == 0) lprev = c.edge;
                    if (lane == kWave - 1) rnext = c.edge;
                    double xm[VEC], xp[VEC];
                    xm[0] = lprev;
                    xp[VEC - 1] = rnext;
#pragma unroll
                    for (int v = 1; v < VEC; ++v) xm[v] = c.v[v - 1];
#pragma unroll
                    for (int v = 0; v < VEC - 1; ++v) xp[v] = c.v[v + 1];
                    double o[VEC];
#pragma unroll
                    for (int v = 0; v < VEC; ++v) {
                        const double px = xm[v] + xp[v];
                        const double py = ym[v] + yp[v];
                        const double pz = zm.v[v] + zp.v[v];
                        const double lap = ((px + py) + pz) - 6.0 * c.v[v];
                        o[v] = c.v[v] + alpha * lap;
                        if (RES && comp[v]) {
                            const double d = o[v] - c.v[v];
                            acc += d * d;
                        }
                    }
                    double *q = out + (z * ny + y) * nx + x;
                    if (all) {
                        store_vec<VEC>(q, o);
                    } else {
#pragma unroll
                        for (int v = 0; v < VEC; ++v)
                            if (comp[v]) q[v] = o[v];
                    }
                    (void)plane;
                }
            }
#pragma unroll
            for (int k = 0; k < 2; ++k) r[k] = r[kU + k];
#pragma unroll
            for (int k = 0; k < kU; ++k) r[2 + k] = nxt[k];
        }
    }
    if (RES) {
        const double s = block_sum(acc, sh);
        if (threadIdx.x == 0 && threadIdx.y == 0) {
            const int64_t b = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
            wg_partials[b] = s;
        }
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

hipError_t launch_jacobi2d(const Launch &L, hipStream_t s) {
    const Cfg &c = L.cfg;
    const int64_t nx = L.ext[1];
    const int64_t col0 = c.vec == 2 ? (L.lo[1] & ~(int64_t)1) : L.lo[1];
    const int64_t ncols = L.hi[1] - col0;
    const int64_t nrows = L.hi[0] - L.lo[0];
    if (nrows <= 0 || ncols <= 0) return hipSuccess;
    dim3 block(c.bx, c.by);
    dim3 grid((unsigned)cdiv(ncols, (int64_t)c.bx * c.vec), (unsigned)cdiv(nrows, (int64_t)c.by * c.tile));
    const double *in = (const double *)L.a[0].ptr;
    double *out = (double *)L.a[1].ptr;
    if (c.vec == 2)
        hipLaunchKernelGGL(jacobi2d_kernel<2>, grid, block, 0, s, in, out, nx, L.lo[0], L.hi[0], L.lo[1], L.hi[1],
                           col0, c.tile);
    else
        hipLaunchKernelGGL(jacobi2d_kernel<1>, grid, block, 0, s, in, out, nx, L.lo[0], L.hi[0], L.lo[1], L.hi[1],
                           col0, c.tile);
    return hipGetLastError();
}

static dim3 heat_grid(const Launch &L, int64_t col0) {
    const Cfg &c = L.cfg;
    const int64_t ncols = L.hi[2] - col0;
    return dim3((unsigned)cdiv(ncols, (int64_t)c.bx * c.vec), (unsigned)cdiv(L.hi[1] - L.lo[1], c.by),
                (unsigned)cdiv(L.hi[0] - L.lo[0], c.tile));
}

int64_t heat3d_workgroups(const Launch &L) {
    const int64_t col0 = L.cfg.vec == 2 ? (L.lo[2] & ~(int64_t)1) : L.lo[2];
    dim3 g = heat_grid(L, col0);
    return (int64_t)g.x * g.y * g.z;
}

hipError_t launch_heat3d(const Launch &L, hipStream_t s) {
    const Cfg &c = L.cfg;
    const int64_t ny = L.ext[1], nx = L.ext[2];
    const int64_t col0 = c.vec == 2 ? (L.lo[2] & ~(int64_t)1) : L.lo[2];
    if (L.hi[0] <= L.lo[0] || L.hi[1] <= L.lo[1] || L.hi[2] <= L.lo[2]) return hipSuccess;
    dim3 block(c.bx, c.by);
    dim3 grid = heat_grid(L, col0);
    const double *in = (const double *)L.a[0].ptr;
    double *out = (double *)L.a[1].ptr;
    const double alpha = L.scalars[0];
    const bool res = L.wg_partials != nullptr;
#define HEAT_ARGS in, out, ny, nx, L.lo[0], L.hi[0], L.lo[1], L.hi[1], L.lo[2], L.hi[2], col0, c.tile, alpha, L.wg_partials
    if (c.vec == 2) {
        if (res) hipLaunchKernelGGL((heat3d_kernel<2, true>), grid, block, 0, s, HEAT_ARGS);
        else hipLaunchKernelGGL((heat3d_kernel<2, false>), grid, block, 0, s, HEAT_ARGS);
    } else {
        if (res) hipLaunchKernelGGL((heat3d_kernel<1, true>), grid, block, 0, s, HEAT_ARGS);
        else hipLaunchKernelGGL((heat3d_kernel<1, false>), grid, block, 0, s, HEAT_ARGS);
    }
#undef HEAT_ARGS
    return hipGetLastError();
}

}  // namespace jk
