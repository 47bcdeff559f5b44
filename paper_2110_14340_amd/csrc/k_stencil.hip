// Stencil loop bodies for gfx950: Jacobi-2D 5-point and heat-3D 7-point,
// and the persistent kernel that runs many small sweeps in one launch.
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
// A tile is the work of one workgroup; the regular kernels map blockIdx to
// tiles, the persistent kernel walks a task table's tiles with a fixed
// grid.  Both call the same tile functions, so results are bit-identical.
//
// Arithmetic (floating-point contraction disabled at build time):
//   Jacobi: out = 0.25 * ((up + down) + (left + right))
//   Heat:   lap = ((xm + xp) + (ym + yp)) + (zm + zp) - 6.0*u ;  out = u + alpha*lap
// which is the operation order of the CPU oracle, so results are bit-exact.
#include "jacc.h"
#include "k_common.h"
#include "kernels.h"

namespace jk {

namespace {

constexpr int kU = 4;  // rows loaded ahead of the rows being computed

// One ring entry: VEC own values plus, for the two edge lanes of the wave,
// the element just left (lane 0) or right (lane 63) of the wave's span.
template <int VEC>
struct Row {
    double v[VEC];
    double edge;
};

template <int VEC>
__device__ __forceinline__ void load_row(const double *__restrict__ p, bool inb, int lane, bool need_l, bool need_r,
                                         Row<VEC> &r) {
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

// Left/right neighbours of the VEC values of `mid` (cross-lane shuffles; the
// edge lanes use the element they loaded beside the wave's span).
template <int VEC>
__device__ __forceinline__ void horizontal(const Row<VEC> &mid, int lane, double (&left)[VEC], double (&right)[VEC]) {
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
}

// Output stores (the box's own rows and every mirror) go through a
// global-address-space pointer: a pointer read from a descriptor table or
// picked by a loop index is otherwise generic, and stored through with flat
// operations, which count against the counter the cross-lane shuffles wait
// on.  Full-vector stores are non-temporal: a sweep's output is not read
// again in the same launch.
template <int VEC>
__device__ __forceinline__ void store_nt(double *p, const double (&o)[VEC]) {
    typedef __attribute__((address_space(1))) double GDouble;
    typedef __attribute__((address_space(1))) dvec2 GDvec2;
    GDouble *q = (GDouble *)p;
    if constexpr (VEC == 2) {
        dvec2 t;
        t.x = o[0];
        t.y = o[1];
        __builtin_nontemporal_store(t, (GDvec2 *)q);
    } else {
        __builtin_nontemporal_store(o[0], q);
    }
}

template <int VEC>
__device__ __forceinline__ void store_masked(double *p, const double (&o)[VEC], bool all, const bool (&comp)[VEC]) {
    if (all) {
        store_nt<VEC>(p, o);
    } else {
        typedef __attribute__((address_space(1))) double GDouble;
        GDouble *q = (GDouble *)p;
#pragma unroll
        for (int v = 0; v < VEC; ++v)
            if (comp[v]) q[v] = o[v];
    }
}

// Mirror handling of a kernel (MM): 0 the launch writes no mirrors (the
// code is left out), 1 a loop over mirrors passed as kernel arguments, 3
// the same loop over column mirrors (ColMirrors: an array split along dim
// 1, where the lanes holding a column another slab keeps store that
// element there too), 4 the column mirrors of a descriptor, unrolled, 2
// the two mirrors of a descriptor read from memory, unrolled (a loop index
// into a descriptor held in registers puts the whole descriptor in scratch
// memory: 40 % slower).  The forms schedule differently: without the loop
// the compiler keeps more loads in flight in more registers (the Jacobi
// tile 100 registers and four waves per SIMD, against 80 and six with the
// loop), which measured 2 % faster on 8192^2 sweeps but 7 % slower on heat
// 512^3 and 20-40 % slower on batches of small grids; so only large Jacobi
// launches without mirrors take form 0.
//
// Stores an output row (or plane) `r` at offset `off` from its row start,
// and again into every mirror holding row r (uniform test per row); with
// column mirrors (MM 3 and 4) each computed element of columns col ..
// col+VEC-1 that a holder keeps goes to that holder's slab as well.
template <int VEC, int MM, typename MT = Mirrors>
__device__ __forceinline__ void store_out(double *out, int64_t off, int64_t r, int64_t col, const MT &mir,
                                          const double (&o)[VEC], bool all, const bool (&comp)[VEC]) {
    store_masked<VEC>(out + off, o, all, comp);
    if constexpr (MM == 3 || MM == 4) {
        typedef __attribute__((address_space(1))) double GDouble;
        constexpr int kN = MM == 4 ? 2 : 0;  // 4: unrolled over the descriptor's two entries
        auto one = [&](const ColMirror &m) {
#pragma unroll
            for (int v = 0; v < VEC; ++v)
                if (comp[v] && col + v >= m.lo && col + v < m.hi) *(GDouble *)(m.ptr + r * m.pitch + col + v) = o[v];
        };
        if constexpr (kN == 2) {
#pragma unroll
            for (int k = 0; k < 2; ++k)
                if (k < mir.n) one(mir.m[k]);
        } else {
            for (int k = 0; k < mir.n; ++k) one(mir.m[k]);
        }
    } else if constexpr (MM == 1) {
        for (int k = 0; k < mir.n; ++k)
            if (r >= mir.m[k].lo && r < mir.m[k].hi) store_masked<VEC>(mir.m[k].ptr + off, o, all, comp);
    } else if constexpr (MM == 2) {
#pragma unroll
        for (int k = 0; k < 2; ++k)
            if (k < mir.n && r >= mir.m[k].lo && r < mir.m[k].hi)
                store_masked<VEC>(mir.m[k].ptr + off, o, all, comp);
    }
}

// March direction of the wave's tile q: with march == 2 odd tiles run toward
// lower rows, so the two rows a pair of neighbouring tiles share are read by
// both at about the same time (both at their start or both at their end)
// and the second read hits in L2.  The stencils are symmetric in the marched
// dimension and the vertical pair sum is commutative, so the direction never
// changes a result bit.
__device__ __forceinline__ int64_t march_dir(int march, int64_t q) { return (march == 2 && (q & 1)) ? -1 : 1; }

// ---------------------------------------------------------------------------
// Jacobi-2D tile: lanes [tx] of row-group [ty] of workgroup tile (bxi, byi)
// ---------------------------------------------------------------------------
template <int VEC, int MM, typename MT = Mirrors>
__device__ __forceinline__ void jacobi_tile(const double *__restrict__ in, double *__restrict__ out, int64_t nx,
                                            int64_t pitch, int64_t r_lo, int64_t r_hi, int64_t c_lo, int64_t c_hi,
                                            int64_t col0, int tile, int march, const MT &mir, int64_t bxi,
                                            int64_t byi, int tx, int ty, int bdx, int bdy,
                                            int64_t own_lo = INT64_MIN, int64_t own_hi = INT64_MAX) {
    const int lane = tx & (kWave - 1);
    const int64_t j = col0 + (bxi * bdx + tx) * VEC;
    const int64_t q = byi * bdy + ty;
    const int64_t i0 = r_lo + q * tile;
    if (i0 >= r_hi) return;  // uniform across the wave (one ty per wave)
    const int64_t i1 = i0 + tile < r_hi ? i0 + tile : r_hi;
    const int64_t n = i1 - i0;
    const int64_t d = march_dir(march, q);
    const int64_t a = d > 0 ? i0 : i1 - 1;  // first row computed
    const bool inb = j < c_hi + 1 && j < nx;  // lane holds columns the box needs
    bool comp[VEC];
    bool all = true;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        comp[v] = (j + v >= c_lo) && (j + v < c_hi);
        all = all && comp[v];
    }
    const bool need_l = comp[0];
    const bool need_r = comp[VEC - 1];

    // ring entry k holds row a + (k-1)*d; loads k = 0 .. n+1
    Row<VEC> r[kU + 2];
#pragma unroll
    for (int k = 0; k < kU + 2; ++k)
        if (k <= n + 1) load_row<VEC>(in + (a + (k - 1) * d) * pitch + j, inb, lane, need_l, need_r, r[k]);
    for (int64_t m = 0; m < n; m += kU) {
        Row<VEC> nxt[kU];
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            const int64_t idx = m + kU + 2 + k;
            if (idx <= n + 1) load_row<VEC>(in + (a + (idx - 1) * d) * pitch + j, inb, lane, need_l, need_r, nxt[k]);
        }
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            if (m + k < n) {
                const int64_t row = a + (m + k) * d;
                const Row<VEC> &prev = r[k], &mid = r[k + 1], &next = r[k + 2];
                double left[VEC], right[VEC];
                horizontal<VEC>(mid, lane, left, right);
                double o[VEC];
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const double vert = prev.v[v] + next.v[v];
                    const double horz = left[v] + right[v];
                    o[v] = 0.25 * (vert + horz);
                }
                // write guard of a filtered loop (every partition computes the
                // whole box and keeps its owner rows); uniform per row
                if (row >= own_lo && row < own_hi) store_out<VEC, MM, MT>(out, row * pitch + j, row, j, mir, o, all, comp);
            }
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) r[k] = r[kU + k];
#pragma unroll
        for (int k = 0; k < kU; ++k) r[2 + k] = nxt[k];
    }
}

// Tile of a 1-D grid's workgroup: row-major (order 1), or XCD-aware (order
// 2): workgroup b runs on XCD b mod 8, and XCD x takes the x-th contiguous
// eighth of the tiles in row-major order.
__device__ __forceinline__ int64_t tile_of(int order) {
    const int64_t b = blockIdx.x, n = gridDim.x;
    if (order == 2 && (n & 7) == 0) return (b & 7) * (n >> 3) + (b >> 3);
    return b;
}

template <int VEC, int MM>
__global__ void __launch_bounds__(1024)
jacobi2d_kernel(const double *__restrict__ in, double *__restrict__ out, int64_t nx, int64_t pitch, int64_t r_lo,
                int64_t r_hi, int64_t c_lo, int64_t c_hi, int64_t col0, int tile, int march, Mirrors mir, int64_t gx,
                int order, int64_t own_lo, int64_t own_hi) {
    const int64_t t = tile_of(order);
    jacobi_tile<VEC, MM>(in, out, nx, pitch, r_lo, r_hi, c_lo, c_hi, col0, tile, march, mir, t % gx, t / gx, threadIdx.x,
                     threadIdx.y, blockDim.x, blockDim.y, own_lo, own_hi);
}

// The same sweep over a column slab of an array split along dim 1 whose
// written columns other slabs keep (column mirrors).
template <int VEC>
__global__ void __launch_bounds__(1024)
jacobi2d_cols_kernel(const double *__restrict__ in, double *__restrict__ out, int64_t nx, int64_t pitch, int64_t r_lo,
                     int64_t r_hi, int64_t c_lo, int64_t c_hi, int64_t col0, int tile, int march, ColMirrors mir,
                     int64_t gx, int order) {
    const int64_t t = tile_of(order);
    jacobi_tile<VEC, 3, ColMirrors>(in, out, nx, pitch, r_lo, r_hi, c_lo, c_hi, col0, tile, march, mir, t % gx, t / gx,
                                    threadIdx.x, threadIdx.y, blockDim.x, blockDim.y);
}

// ---------------------------------------------------------------------------
// Heat-3D tile: row y = y_lo + byi*bdy + ty, planes [z_lo + bzi*tile, +tile)
// Returns this lane's sum of (u'-u)^2 when RES.
// ---------------------------------------------------------------------------
template <int VEC, bool RES, int MM>
__device__ __forceinline__ double heat_tile(const double *__restrict__ in, double *__restrict__ out, int64_t ny,
                                            int64_t nx, int64_t z_lo, int64_t z_hi, int64_t y_lo, int64_t y_hi,
                                            int64_t x_lo, int64_t x_hi, int64_t col0, int tile, int march, double alpha,
                                            const Mirrors &mir, int64_t bxi, int64_t byi, int64_t bzi, int tx,
                                            int ty, int bdx, int bdy, int64_t own_lo = INT64_MIN,
                                            int64_t own_hi = INT64_MAX) {
    const int lane = tx & (kWave - 1);
    const int64_t x = col0 + (bxi * bdx + tx) * VEC;
    const int64_t y = y_lo + byi * bdy + ty;
    const int64_t z0 = z_lo + bzi * tile;
    const int64_t z1 = z0 + tile < z_hi ? z0 + tile : z_hi;
    double acc = 0.0;
    if (y >= y_hi || z0 >= z1) return acc;  // uniform across the wave
    const int64_t n = z1 - z0;
    const int64_t d = march_dir(march, bzi);
    const int64_t a = d > 0 ? z0 : z1 - 1;  // first plane computed
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
    const double *base = in + y * nx + x;

    // ring entry k holds plane a + (k-1)*d; loads k = 0 .. n+1
    Row<VEC> r[kU + 2];
#pragma unroll
    for (int k = 0; k < kU + 2; ++k)
        if (k <= n + 1) load_row<VEC>(base + (a + (k - 1) * d) * plane, inb, lane, need_l, need_r, r[k]);
    for (int64_t m = 0; m < n; m += kU) {
        Row<VEC> nxt[kU];
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            const int64_t idx = m + kU + 2 + k;
            if (idx <= n + 1) load_row<VEC>(base + (a + (idx - 1) * d) * plane, inb, lane, need_l, need_r, nxt[k]);
        }
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            if (m + k < n) {
                const int64_t z = a + (m + k) * d;
                const bool keep = z >= own_lo && z < own_hi;  // write guard of a filtered loop
                const Row<VEC> &zprev = r[k], &c = r[k + 1], &znext = r[k + 2];
                // y neighbours: rows of the same plane (cache hits)
                double ym[VEC], yp[VEC];
                const double *pc = base + z * plane;
                if (inb) {
                    load_vec<VEC>(pc - nx, ym);
                    load_vec<VEC>(pc + nx, yp);
                } else {
#pragma unroll
                    for (int v = 0; v < VEC; ++v) ym[v] = yp[v] = 0.0;
                }
                double xm[VEC], xp[VEC];
                horizontal<VEC>(c, lane, xm, xp);
                double o[VEC];
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const double px = xm[v] + xp[v];
                    const double py = ym[v] + yp[v];
                    const double pz = zprev.v[v] + znext.v[v];
                    const double lap = ((px + py) + pz) - 6.0 * c.v[v];
                    o[v] = c.v[v] + alpha * lap;
                    if (RES && comp[v] && keep) {
                        const double dd = o[v] - c.v[v];
                        acc += dd * dd;
                    }
                }
                if (keep) store_out<VEC, MM>(out, z * plane + y * nx + x, z, x, mir, o, all, comp);
            }
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) r[k] = r[kU + k];
#pragma unroll
        for (int k = 0; k < kU; ++k) r[2 + k] = nxt[k];
    }
    return acc;
}

// ---------------------------------------------------------------------------
// Heat-3D tile with R rows per wave: the wave's lanes own VEC columns of R
// consecutive rows y = yb .. yb+R-1 and march through the planes of the
// tile.  The y neighbours of the inner rows are the lane's own registers;
// only the rows yb-1 and yb+R are loaded beside them, so a plane of R
// output rows costs R+2 row loads instead of 3R.  Rows past the box's last
// row are clamped to the boundary row y_hi (in bounds, never stored).
// Three planes are held per row; the z sums are formed first, which frees
// the oldest plane, and its registers then receive the loads of the plane
// after next while the rest of the current plane is computed.
// ---------------------------------------------------------------------------
template <int VEC, int R>
struct Planes {
    double v[R + 2][VEC];  // v[k]: row min(yb + k - 1, y_hi)
    double edge[R];        // beside the wave's span, rows 1..R (edge lanes only)
};

template <int VEC, int R>
__device__ __forceinline__ void load_plane(const double *__restrict__ p, int64_t nx, int64_t yb, int64_t y_hi, int rr,
                                           bool inb, int lane, bool need_l, bool need_r, Planes<VEC, R> &P) {
#pragma unroll
    for (int k = 0; k < R + 2; ++k) {
        const int64_t y = yb + k - 1 < y_hi ? yb + k - 1 : y_hi;
        const double *q = p + y * nx;
        if (inb) {
            load_vec<VEC>(q, P.v[k]);
        } else {
#pragma unroll
            for (int v = 0; v < VEC; ++v) P.v[k][v] = 0.0;
        }
        if (k >= 1 && k <= R) {
            P.edge[k - 1] = 0.0;
            if (k - 1 < rr) {
                if (lane == 0 && need_l) P.edge[k - 1] = q[-1];
                if (lane == kWave - 1 && need_r) P.edge[k - 1] = q[VEC];
            }
        }
    }
}

template <int VEC, int R, bool RES, int MM>
__device__ __forceinline__ double heat_rows_tile(const double *__restrict__ in, double *__restrict__ out, int64_t ny,
                                                 int64_t nx, int64_t z_lo, int64_t z_hi, int64_t y_lo, int64_t y_hi,
                                                 int64_t x_lo, int64_t x_hi, int64_t col0, int tile, int march,
                                                 double alpha, const Mirrors &mir, int64_t bxi, int64_t byi,
                                                 int64_t bzi, int tx, int ty, int bdx, int bdy, int64_t own_lo,
                                                 int64_t own_hi) {
    const int lane = tx & (kWave - 1);
    const int64_t x = col0 + (bxi * bdx + tx) * VEC;
    const int64_t yb = y_lo + (byi * bdy + ty) * R;
    const int64_t z0 = z_lo + bzi * tile;
    const int64_t z1 = z0 + tile < z_hi ? z0 + tile : z_hi;
    double acc = 0.0;
    if (yb >= y_hi || z0 >= z1) return acc;  // uniform across the wave
    const int rr = (int)(y_hi - yb < R ? y_hi - yb : R);
    const int64_t n = z1 - z0;
    const int64_t d = march_dir(march, bzi);
    const int64_t a = d > 0 ? z0 : z1 - 1;  // first plane computed
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
    const double *col = in + x;

    // plane k (k = 0 .. n+1) is a + (k-1)*d
    auto load = [&](int64_t k, Planes<VEC, R> &P) {
        load_plane<VEC, R>(col + (a + (k - 1) * d) * plane, nx, yb, y_hi, rr, inb, lane, need_l, need_r, P);
    };
    // computes plane m from A (plane m-1), B (m), C (m+1), then refills A
    // with plane m+2 (index k = m+3) when there is one
    auto step = [&](Planes<VEC, R> &A, const Planes<VEC, R> &B, const Planes<VEC, R> &C, int64_t m) {
        double pz[R][VEC];
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int v = 0; v < VEC; ++v) pz[i][v] = A.v[i + 1][v] + C.v[i + 1][v];
        if (m + 3 <= n + 1) load(m + 3, A);
        const int64_t z = a + m * d;
        const bool keep = z >= own_lo && z < own_hi;  // write guard of a filtered loop
#pragma unroll
        for (int i = 0; i < R; ++i) {
            if (i < rr) {
                Row<VEC> c;
#pragma unroll
                for (int v = 0; v < VEC; ++v) c.v[v] = B.v[i + 1][v];
                c.edge = B.edge[i];
                double xm[VEC], xp[VEC];
                horizontal<VEC>(c, lane, xm, xp);
                double o[VEC];
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    const double px = xm[v] + xp[v];
                    const double py = B.v[i][v] + B.v[i + 2][v];
                    const double lap = ((px + py) + pz[i][v]) - 6.0 * c.v[v];
                    o[v] = c.v[v] + alpha * lap;
                    if (RES && comp[v] && keep) {
                        const double dd = o[v] - c.v[v];
                        acc += dd * dd;
                    }
                }
                if (keep) store_out<VEC, MM>(out, z * plane + (yb + i) * nx + x, z, x, mir, o, all, comp);
            }
        }
    };
    Planes<VEC, R> P0, P1, P2;
    load(0, P0);
    load(1, P1);
    load(2, P2);
    for (int64_t m = 0; m < n; m += 3) {
        step(P0, P1, P2, m);
        if (m + 1 < n) step(P1, P2, P0, m + 1);
        if (m + 2 < n) step(P2, P0, P1, m + 2);
    }
    return acc;
}

// Heat tile coordinates of tile t.  Orders 1 and 2: x fastest, then y, then
// z.  Order 3 (t taken XCD-aware as in order 2): y-blocks of 8 tile rows
// walked through all z tiles before the next y-block, so the workgroups
// resident on one XCD at a time form a compact (x, 8 y, few z) brick and
// both the y-halo rows and the z-halo planes they share meet in its L2.
constexpr int64_t kHeatYBlock = 8;
__device__ __forceinline__ void heat_coords(int64_t t, int64_t gx, int64_t gy, int64_t gz, int order, int64_t &bxi,
                                            int64_t &byi, int64_t &bzi) {
    bxi = t % gx;
    const int64_t r = t / gx;
    if (order != 3) {
        byi = r % gy;
        bzi = r / gy;
        return;
    }
    const int64_t full = gy / kHeatYBlock;  // complete y-blocks
    if (r < full * kHeatYBlock * gz) {
        const int64_t blk = r / (kHeatYBlock * gz), q = r % (kHeatYBlock * gz);
        bzi = q / kHeatYBlock;
        byi = blk * kHeatYBlock + q % kHeatYBlock;
    } else {
        const int64_t r2 = r - full * kHeatYBlock * gz, rem = gy - full * kHeatYBlock;
        bzi = r2 / rem;
        byi = full * kHeatYBlock + r2 % rem;
    }
}

template <int VEC, int R, bool RES, int MM>
__global__ void __launch_bounds__(R == 1 ? 1024 : 256)
heat3d_kernel(const double *__restrict__ in, double *__restrict__ out, int64_t ny, int64_t nx, int64_t z_lo,
              int64_t z_hi, int64_t y_lo, int64_t y_hi, int64_t x_lo, int64_t x_hi, int64_t col0, int tile,
              int march, double alpha, double *__restrict__ wg_partials, Mirrors mir, int64_t gx, int64_t gy,
              int order, int64_t own_lo, int64_t own_hi) {
    __shared__ double sh[16];
    const int64_t t = tile_of(order == 3 ? 2 : order);
    const int64_t gz = (int64_t)gridDim.x / (gx * gy);
    int64_t bxi, byi, bzi;
    heat_coords(t, gx, gy, gz, order, bxi, byi, bzi);
    double acc;
    if constexpr (R == 1)
        acc = heat_tile<VEC, RES, MM>(in, out, ny, nx, z_lo, z_hi, y_lo, y_hi, x_lo, x_hi, col0, tile, march, alpha, mir,
                                  bxi, byi, bzi, threadIdx.x, threadIdx.y, blockDim.x, blockDim.y, own_lo, own_hi);
    else
        acc = heat_rows_tile<VEC, R, RES, MM>(in, out, ny, nx, z_lo, z_hi, y_lo, y_hi, x_lo, x_hi, col0, tile, march,
                                          alpha, mir, bxi, byi, bzi, threadIdx.x, threadIdx.y, blockDim.x,
                                          blockDim.y, own_lo, own_hi);
    if (RES) {
        const double s = block_sum(acc, sh);
        if (threadIdx.x == 0 && threadIdx.y == 0) wg_partials[t] = s;  // partials in tile order
    }
}

// ---------------------------------------------------------------------------
// Persistent kernel: one launch runs the tiles of every task of a group
// (workgroup b takes tiles b, b + grid, b + 2*grid, ...; the grid normally
// has one workgroup per tile).  JONLY: a group of Jacobi tasks only; without
// the heat bodies the kernel needs fewer registers, so more workgroups are
// resident at once.
// ---------------------------------------------------------------------------
// One tile (local index `local`) of task T.
template <bool JONLY>
__device__ __forceinline__ void persistent_tile(const PTask &T, int64_t local) {
    const int64_t bxi = local % T.gx;
    const int64_t rest = local / T.gx;
    const double *in = T.in;
    double *out = T.out;
    const Mirrors mir = T.mir;
    if (JONLY || T.kind == JACC_LOOP_JACOBI2D) {
        if (T.vec == 2)
            jacobi_tile<2, 2>(in, out, T.e1, T.e1, T.lo[0], T.hi[0], T.lo[1], T.hi[1], T.col0, T.tile, T.march, mir, bxi,
                           rest, threadIdx.x, 0, kPersistentThreads, 1);
        else
            jacobi_tile<1, 2>(in, out, T.e1, T.e1, T.lo[0], T.hi[0], T.lo[1], T.hi[1], T.col0, T.tile, T.march, mir, bxi,
                           rest, threadIdx.x, 0, kPersistentThreads, 1);
    } else if constexpr (!JONLY) {
        const int64_t byi = rest % T.gy, bzi = rest / T.gy;
        if (T.vec == 2)
            (void)heat_tile<2, false, 2>(in, out, T.e1, T.e2, T.lo[0], T.hi[0], T.lo[1], T.hi[1], T.lo[2], T.hi[2],
                                      T.col0, T.tile, T.march, T.alpha, mir, bxi, byi, bzi, threadIdx.x, 0,
                                      kPersistentThreads, 1);
        else
            (void)heat_tile<1, false, 2>(in, out, T.e1, T.e2, T.lo[0], T.hi[0], T.lo[1], T.hi[1], T.lo[2], T.hi[2],
                                      T.col0, T.tile, T.march, T.alpha, mir, bxi, byi, bzi, threadIdx.x, 0,
                                      kPersistentThreads, 1);
    }
}

// Workgroup b runs tile b of the concatenated tile list of all tasks (the
// task found by a binary search over the tasks' first tiles); with fewer
// workgroups than tiles it would take tiles b, b + grid, ... .
// The task table is read through the constant address space: the data
// pointers loaded from it are then known to address global memory (as
// kernel arguments are), so the tile bodies use global loads and stores.
// Read as generic pointers they would become flat operations, which also
// count against the counter the cross-lane shuffles wait on, so every
// shuffle would wait for all the loads in flight.
typedef const __attribute__((address_space(4))) PTask ConstTask;

// Field-by-field copy (the implicit copy constructor takes a generic
// reference).
__device__ __forceinline__ PTask load_task(ConstTask *p) {
    PTask T;
    T.kind = p->kind;
    T.vec = p->vec;
    T.tile = p->tile;
    T.march = p->march;
    T.in = p->in;
    T.out = p->out;
    T.e1 = p->e1;
    T.e2 = p->e2;
    for (int d = 0; d < 3; ++d) {
        T.lo[d] = p->lo[d];
        T.hi[d] = p->hi[d];
    }
    T.col0 = p->col0;
    T.alpha = p->alpha;
    T.gx = p->gx;
    T.gy = p->gy;
    T.gz = p->gz;
    T.ntiles = p->ntiles;
    T.tile_begin = p->tile_begin;
    T.mir.n = p->mir.n;
    for (int k = 0; k < 2; ++k) {
        T.mir.m[k].ptr = p->mir.m[k].ptr;
        T.mir.m[k].lo = p->mir.m[k].lo;
        T.mir.m[k].hi = p->mir.m[k].hi;
    }
    return T;
}

template <bool JONLY>
__global__ void __launch_bounds__(kPersistentThreads)
persistent_kernel(const PTask *__restrict__ tasks, int ntasks, int64_t total) {
    ConstTask *ct = (ConstTask *)tasks;
    for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
        int lo = 0, hi = ntasks - 1;  // last task whose first tile is <= t
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (ct[mid].tile_begin <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        const PTask T = load_task(ct + lo);
        persistent_tile<JONLY>(T, t - T.tile_begin);
    }
}

// ---------------------------------------------------------------------------
// Packed partitions: the K partitions of one eager stencil loop in one
// launch.  Partition q's tiles take workgroups [begin, begin + span) of the
// grid (begin and span multiples of 8, so workgroup b still runs on XCD
// b mod 8 and the XCD-aware orders map tiles within the partition as a
// launch of its own would); workgroups past its tile count return at once.
// The descriptors are read through the constant address space, so their
// pointers are known to address global memory.
// ---------------------------------------------------------------------------
struct PartDesc {
    const double *in;
    double *out;
    int64_t lo0, hi0;     // the partition's iterations along dim 0
    int64_t tiles, begin;  // its tile count and first workgroup
    int64_t partial_off;   // its first workgroup partial (heat residual)
    Mirrors mir;
};
struct PartPack {
    PartDesc p[kMaxPack];
    int32_t n;
};
typedef const __attribute__((address_space(4))) PartDesc ConstPart;

__device__ __forceinline__ PartDesc load_part(ConstPart *p) {
    PartDesc d;
    d.in = p->in;
    d.out = p->out;
    d.lo0 = p->lo0;
    d.hi0 = p->hi0;
    d.tiles = p->tiles;
    d.begin = p->begin;
    d.partial_off = p->partial_off;
    d.mir.n = p->mir.n;
    for (int k = 0; k < 2; ++k) {
        d.mir.m[k].ptr = p->mir.m[k].ptr;
        d.mir.m[k].lo = p->mir.m[k].lo;
        d.mir.m[k].hi = p->mir.m[k].hi;
    }
    return d;
}

// The partition of this workgroup and its tile within the partition (-1:
// a padding workgroup).
__device__ __forceinline__ int64_t part_tile(const PartPack &pk, int order, PartDesc &d) {
    ConstPart *cp = (ConstPart *)&pk.p[0];
    const int64_t b = blockIdx.x;
    int q = 0;
    for (int k = 1; k < pk.n; ++k)
        if (cp[k].begin <= b) q = k;
    d = load_part(cp + q);
    const int64_t span = (q + 1 < pk.n ? cp[q + 1].begin : (int64_t)gridDim.x) - d.begin;
    const int64_t local = b - d.begin;
    const int64_t t = order >= 2 ? (local & 7) * (span >> 3) + (local >> 3) : local;
    return t < d.tiles ? t : -1;
}

template <int VEC, int MM>
__global__ void __launch_bounds__(1024)
jacobi2d_parts_kernel(PartPack pk, int64_t nx, int64_t c_lo, int64_t c_hi, int64_t col0, int tile, int march,
                      int64_t gx, int order) {
    PartDesc d;
    const int64_t t = part_tile(pk, order, d);
    if (t < 0) return;
    jacobi_tile<VEC, MM>(d.in, d.out, nx, nx, d.lo0, d.hi0, c_lo, c_hi, col0, tile, march, d.mir, t % gx, t / gx,
                     threadIdx.x, threadIdx.y, blockDim.x, blockDim.y);
}

// Packed partitions of a JACOBI2D loop over arrays split along dim 1: each
// partition has its own columns, slab pitch and column mirrors.
struct ColPartDesc {
    const double *in;
    double *out;
    int64_t tiles, begin;              // its tile count and first workgroup
    int64_t c_lo, c_hi, col0, pitch;  // its columns, first lane column, slab row pitch
    int64_t gx;                        // tiles per row of tiles
    ColMirrors mir;
};
struct ColPartPack {
    ColPartDesc p[kMaxPack];
    int32_t n;
};
typedef const __attribute__((address_space(4))) ColPartDesc ConstColPart;

__device__ __forceinline__ ColPartDesc load_colpart(ConstColPart *p) {
    ColPartDesc d;
    d.in = p->in;
    d.out = p->out;
    d.tiles = p->tiles;
    d.begin = p->begin;
    d.c_lo = p->c_lo;
    d.c_hi = p->c_hi;
    d.col0 = p->col0;
    d.pitch = p->pitch;
    d.gx = p->gx;
    d.mir.n = p->mir.n;
    for (int k = 0; k < 2; ++k) {
        d.mir.m[k].ptr = p->mir.m[k].ptr;
        d.mir.m[k].lo = p->mir.m[k].lo;
        d.mir.m[k].hi = p->mir.m[k].hi;
        d.mir.m[k].pitch = p->mir.m[k].pitch;
    }
    return d;
}

template <int VEC>
__global__ void __launch_bounds__(1024)
jacobi2d_colparts_kernel(ColPartPack pk, int64_t nx, int64_t r_lo, int64_t r_hi, int tile, int march, int order) {
    ConstColPart *cp = (ConstColPart *)&pk.p[0];
    const int64_t b = blockIdx.x;
    int q = 0;
    for (int k = 1; k < pk.n; ++k)
        if (cp[k].begin <= b) q = k;
    const ColPartDesc d = load_colpart(cp + q);
    const int64_t span = (q + 1 < pk.n ? cp[q + 1].begin : (int64_t)gridDim.x) - d.begin;
    const int64_t local = b - d.begin;
    const int64_t t = order >= 2 ? (local & 7) * (span >> 3) + (local >> 3) : local;
    if (t >= d.tiles) return;
    jacobi_tile<VEC, 4, ColMirrors>(d.in, d.out, nx, d.pitch, r_lo, r_hi, d.c_lo, d.c_hi, d.col0, tile, march, d.mir,
                                    t % d.gx, t / d.gx, threadIdx.x, threadIdx.y, blockDim.x, blockDim.y);
}

template <int VEC, int R, bool RES, int MM>
__global__ void __launch_bounds__(R == 1 ? 1024 : 256)
heat3d_parts_kernel(PartPack pk, int64_t ny, int64_t nx, int64_t y_lo, int64_t y_hi, int64_t x_lo, int64_t x_hi,
                    int64_t col0, int tile, int march, double alpha, double *__restrict__ wg_partials, int64_t gx,
                    int64_t gy, int order) {
    __shared__ double sh[16];
    PartDesc d;
    const int64_t t = part_tile(pk, order == 3 ? 2 : order, d);
    if (t < 0) return;  // the whole workgroup: no barrier is left waiting
    const int64_t gz = d.tiles / (gx * gy);
    int64_t bxi, byi, bzi;
    heat_coords(t, gx, gy, gz, order, bxi, byi, bzi);
    double acc;
    if constexpr (R == 1)
        acc = heat_tile<VEC, RES, MM>(d.in, d.out, ny, nx, d.lo0, d.hi0, y_lo, y_hi, x_lo, x_hi, col0, tile, march, alpha,
                                  d.mir, bxi, byi, bzi, threadIdx.x, threadIdx.y, blockDim.x, blockDim.y);
    else
        acc = heat_rows_tile<VEC, R, RES, MM>(d.in, d.out, ny, nx, d.lo0, d.hi0, y_lo, y_hi, x_lo, x_hi, col0, tile,
                                          march, alpha, d.mir, bxi, byi, bzi, threadIdx.x, threadIdx.y, blockDim.x,
                                          blockDim.y, INT64_MIN, INT64_MAX);
    if (RES) {
        const double sum = block_sum(acc, sh);
        if (threadIdx.x == 0 && threadIdx.y == 0) wg_partials[d.partial_off + t] = sum;  // in tile order
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

static int64_t col_start(int64_t lo, int vec) { return vec == 2 ? (lo & ~(int64_t)1) : lo; }

hipError_t launch_jacobi2d(const Launch &L, hipStream_t s) {
    const Cfg &c = L.cfg;
    const int64_t nx = L.ext[1];
    const int64_t col0 = col_start(L.lo[1], c.vec);
    const int64_t ncols = L.hi[1] - col0;
    const int64_t nrows = L.hi[0] - L.lo[0];
    if (nrows <= 0 || L.hi[1] <= L.lo[1]) return hipSuccess;
    dim3 block(c.bx, c.by);
    const int64_t gx = cdiv(ncols, (int64_t)c.bx * c.vec), gy = cdiv(nrows, (int64_t)c.by * c.tile);
    dim3 grid((unsigned)(gx * gy));
    const double *in = (const double *)L.a[0].ptr;
    double *out = (double *)L.a[1].ptr;
    // elements between vertically adjacent values: the row length, or the
    // slab width of arrays partitioned along columns (both arguments alike)
    const int64_t pitch = L.a[0].row_elems;
    if (L.a[1].row_elems != pitch) return hipErrorInvalidValue;
    const bool filtered = L.own_hi > L.own_lo;  // FILTERED output: keep the owner rows only
    const int64_t own_lo = filtered ? L.own_lo : INT64_MIN, own_hi = filtered ? L.own_hi : INT64_MAX;
#define JACOBI_LAUNCH(V, M)                                                                                   \
    hipLaunchKernelGGL((jacobi2d_kernel<V, M>), grid, block, 0, s, in, out, nx, pitch, L.lo[0], L.hi[0], L.lo[1], \
                       L.hi[1], col0, c.tile, c.march, L.mir, gx, c.order, own_lo, own_hi)
    if (L.cmir.n > 0) {  // column mirrors: an array split along dim 1
#define JCOLS_LAUNCH(V)                                                                                           \
    hipLaunchKernelGGL((jacobi2d_cols_kernel<V>), grid, block, 0, s, in, out, nx, pitch, L.lo[0], L.hi[0], L.lo[1], \
                       L.hi[1], col0, c.tile, c.march, L.cmir, gx, c.order)
        if (c.vec == 2)
            JCOLS_LAUNCH(2);
        else
            JCOLS_LAUNCH(1);
#undef JCOLS_LAUNCH
        return hipGetLastError();
    }
    // the mirror-free form for launches of at least 2^22 cells without mirrors
    const bool lean = L.mir.n == 0 && nrows * (L.hi[1] - L.lo[1]) >= ((int64_t)1 << 22);
    if (c.vec == 2) {
        if (lean)
            JACOBI_LAUNCH(2, 0);
        else
            JACOBI_LAUNCH(2, 1);
    } else {
        if (lean)
            JACOBI_LAUNCH(1, 0);
        else
            JACOBI_LAUNCH(1, 1);
    }
#undef JACOBI_LAUNCH
    return hipGetLastError();
}

static dim3 heat_grid(const Launch &L, int64_t col0) {
    const Cfg &c = L.cfg;
    const int64_t ncols = L.hi[2] - col0;
    return dim3((unsigned)cdiv(ncols, (int64_t)c.bx * c.vec), (unsigned)cdiv(L.hi[1] - L.lo[1], (int64_t)c.by * c.rows),
                (unsigned)cdiv(L.hi[0] - L.lo[0], c.tile));
}

static bool heat_empty(const Launch &L) {
    return L.hi[0] <= L.lo[0] || L.hi[1] <= L.lo[1] || L.hi[2] <= L.lo[2];
}

int64_t heat3d_workgroups(const Launch &L) {
    if (heat_empty(L)) return 0;
    dim3 g = heat_grid(L, col_start(L.lo[2], L.cfg.vec));
    return (int64_t)g.x * g.y * g.z;
}

hipError_t launch_heat3d(const Launch &L, hipStream_t s) {
    const Cfg &c = L.cfg;
    const int64_t ny = L.ext[1], nx = L.ext[2];
    const int64_t col0 = col_start(L.lo[2], c.vec);
    if (heat_empty(L)) return hipSuccess;
    dim3 block(c.bx, c.by);
    const dim3 g3 = heat_grid(L, col0);
    const int64_t gx = g3.x, gy = g3.y;
    dim3 grid((unsigned)((int64_t)g3.x * g3.y * g3.z));
    const double *in = (const double *)L.a[0].ptr;
    double *out = (double *)L.a[1].ptr;
    const double alpha = L.scalars[0];
    const bool res = L.wg_partials != nullptr;
    const bool filtered = L.own_hi > L.own_lo;  // FILTERED output: keep the owner planes only
    const int64_t own_lo = filtered ? L.own_lo : INT64_MIN, own_hi = filtered ? L.own_hi : INT64_MAX;
#define HEAT_ARGS                                                                                                    \
    in, out, ny, nx, L.lo[0], L.hi[0], L.lo[1], L.hi[1], L.lo[2], L.hi[2], col0, c.tile, c.march, alpha,             \
        L.wg_partials, L.mir, gx, gy, c.order, own_lo, own_hi
#define HEAT_LAUNCH(V, R)                                                                    \
    do {                                                                                     \
        if (res)                                                                             \
            hipLaunchKernelGGL((heat3d_kernel<V, R, true, 1>), grid, block, 0, s, HEAT_ARGS);  \
        else                                                                                 \
            hipLaunchKernelGGL((heat3d_kernel<V, R, false, 1>), grid, block, 0, s, HEAT_ARGS); \
    } while (0)
    if (c.vec == 2) {
        switch (c.rows) {
            case 1: HEAT_LAUNCH(2, 1); break;
            case 2: HEAT_LAUNCH(2, 2); break;
            case 4: HEAT_LAUNCH(2, 4); break;
            default: HEAT_LAUNCH(2, 8); break;
        }
    } else {
        switch (c.rows) {
            case 1: HEAT_LAUNCH(1, 1); break;
            case 2: HEAT_LAUNCH(1, 2); break;
            case 4: HEAT_LAUNCH(1, 4); break;
            default: HEAT_LAUNCH(1, 8); break;
        }
    }
#undef HEAT_LAUNCH
#undef HEAT_ARGS
    return hipGetLastError();
}

int64_t parts_partials(const Launch *L, int n) {
    int64_t total = 0;
    for (int k = 0; k < n; ++k) total += heat3d_workgroups(L[k]);
    return total;
}

// The partitions of a JACOBI2D loop over arrays split along dim 1 in one
// launch: every partition has its own columns, pitch and column mirrors.
static hipError_t launch_col_parts(const Launch *L, int n, hipStream_t s) {
    const Launch &L0 = L[0];
    const Cfg &c = L0.cfg;
    const bool xcd = c.order == 2;
    ColPartPack pk{};
    int64_t begin = 0;
    for (int k = 0; k < n; ++k) {
        const Launch &Lk = L[k];
        if (Lk.a[1].row_elems != Lk.a[0].row_elems || Lk.lo[0] != L0.lo[0] || Lk.hi[0] != L0.hi[0])
            return hipErrorInvalidValue;
        if (Lk.hi[0] <= Lk.lo[0] || Lk.hi[1] <= Lk.lo[1]) continue;
        const int64_t col0 = col_start(Lk.lo[1], c.vec);
        const int64_t gx = cdiv(Lk.hi[1] - col0, (int64_t)c.bx * c.vec);
        const int64_t tiles = gx * cdiv(Lk.hi[0] - Lk.lo[0], (int64_t)c.by * c.tile);
        ColPartDesc &d = pk.p[pk.n++];
        d.in = (const double *)Lk.a[0].ptr;
        d.out = (double *)Lk.a[1].ptr;
        d.tiles = tiles;
        d.begin = begin;
        d.c_lo = Lk.lo[1];
        d.c_hi = Lk.hi[1];
        d.col0 = col0;
        d.pitch = Lk.a[0].row_elems;
        d.gx = gx;
        d.mir = Lk.cmir;
        begin += xcd ? (tiles + 7) / 8 * 8 : tiles;
    }
    if (pk.n == 0) return hipSuccess;
    if (begin > (int64_t)INT32_MAX) return hipErrorInvalidValue;
    const dim3 grid((unsigned)begin), block(c.bx, c.by);
    if (c.vec == 2)
        hipLaunchKernelGGL((jacobi2d_colparts_kernel<2>), grid, block, 0, s, pk, L0.ext[1], L0.lo[0], L0.hi[0], c.tile,
                           c.march, c.order);
    else
        hipLaunchKernelGGL((jacobi2d_colparts_kernel<1>), grid, block, 0, s, pk, L0.ext[1], L0.lo[0], L0.hi[0], c.tile,
                           c.march, c.order);
    return hipGetLastError();
}

hipError_t launch_parts(const Launch *L, int n, double *wg_partials, int64_t wg_capacity, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (n > kMaxPack) return hipErrorInvalidValue;
    const Launch &L0 = L[0];
    if (L0.kind == JACC_LOOP_SUM) return launch_sum_parts(L, n, wg_partials, wg_capacity, s);
    const Cfg &c = L0.cfg;
    const bool heat = L0.kind == JACC_LOOP_HEAT3D;
    if (!heat && L0.kind != JACC_LOOP_JACOBI2D) return hipErrorInvalidValue;
    if (!heat && L0.part_dim == 1) return launch_col_parts(L, n, s);  // column slabs
    const bool res = heat && L0.part_out != nullptr;
    const bool xcd = heat ? c.order >= 2 : c.order == 2;
    const int64_t col0 = col_start(L0.lo[heat ? 2 : 1], c.vec);
    int64_t gx, gy = 1;
    if (heat) {
        const dim3 g3 = heat_grid(L0, col0);
        gx = g3.x;
        gy = g3.y;
    } else {
        gx = cdiv(L0.hi[1] - col0, (int64_t)c.bx * c.vec);
    }
    PartPack pk{};
    Segments seg{};
    int64_t begin = 0, partial = 0;
    for (int k = 0; k < n; ++k) {
        const Launch &Lk = L[k];
        int64_t tiles = 0;
        if (heat)
            tiles = heat_empty(Lk) ? 0 : heat3d_workgroups(Lk);
        else if (Lk.hi[0] > Lk.lo[0] && Lk.hi[1] > Lk.lo[1])
            tiles = gx * cdiv(Lk.hi[0] - Lk.lo[0], (int64_t)c.by * c.tile);
        if (res) {  // every reducing partition gets its sum, 0 when it has no tiles
            seg.off[seg.count] = partial;
            seg.n[seg.count] = tiles;
            seg.out[seg.count] = Lk.part_out;
            ++seg.count;
        }
        if (tiles == 0) continue;
        PartDesc &d = pk.p[pk.n++];
        d.in = (const double *)Lk.a[0].ptr;
        d.out = (double *)Lk.a[1].ptr;
        d.lo0 = Lk.lo[0];
        d.hi0 = Lk.hi[0];
        d.tiles = tiles;
        d.begin = begin;
        d.partial_off = partial;
        d.mir = Lk.mir;
        begin += xcd ? (tiles + 7) / 8 * 8 : tiles;
        if (res) partial += tiles;
    }
    if (partial > wg_capacity || begin > (int64_t)INT32_MAX) return hipErrorInvalidValue;
    if (pk.n > 0) {
        const dim3 grid((unsigned)begin), block(c.bx, c.by);
        if (!heat) {
#define JPARTS_LAUNCH(V, M)                                                                                   \
    hipLaunchKernelGGL((jacobi2d_parts_kernel<V, M>), grid, block, 0, s, pk, L0.ext[1], L0.lo[1], L0.hi[1], col0, \
                       c.tile, c.march, gx, c.order)
            if (c.vec == 2)
                JPARTS_LAUNCH(2, 2);
            else
                JPARTS_LAUNCH(1, 2);
#undef JPARTS_LAUNCH
        } else {
#define PARTS_ARGS                                                                                                \
    pk, L0.ext[1], L0.ext[2], L0.lo[1], L0.hi[1], L0.lo[2], L0.hi[2], col0, c.tile, c.march, L0.scalars[0], \
        wg_partials, gx, gy, c.order
#define PARTS_LAUNCH(V, R)                                                                             \
    do {                                                                                               \
        if (res)                                                                                       \
            hipLaunchKernelGGL((heat3d_parts_kernel<V, R, true, 2>), grid, block, 0, s, PARTS_ARGS);  \
        else                                                                                           \
            hipLaunchKernelGGL((heat3d_parts_kernel<V, R, false, 2>), grid, block, 0, s, PARTS_ARGS); \
    } while (0)
            if (c.vec == 2) {
                switch (c.rows) {
                    case 1: PARTS_LAUNCH(2, 1); break;
                    case 2: PARTS_LAUNCH(2, 2); break;
                    case 4: PARTS_LAUNCH(2, 4); break;
                    default: PARTS_LAUNCH(2, 8); break;
                }
            } else {
                switch (c.rows) {
                    case 1: PARTS_LAUNCH(1, 1); break;
                    case 2: PARTS_LAUNCH(1, 2); break;
                    case 4: PARTS_LAUNCH(1, 4); break;
                    default: PARTS_LAUNCH(1, 8); break;
                }
            }
#undef PARTS_LAUNCH
#undef PARTS_ARGS
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return res ? launch_finalise_many(wg_partials, seg, s) : hipSuccess;
}

bool make_task(const Launch &L, PTask *t) {
    *t = PTask{};
    t->kind = L.kind;
    t->vec = L.cfg.vec;
    t->tile = L.cfg.tile;
    t->march = L.cfg.march;
    t->in = (const double *)L.a[0].ptr;
    t->out = (double *)L.a[1].ptr;
    t->mir = L.mir;
    for (int d = 0; d < 3; ++d) {
        t->lo[d] = L.lo[d];
        t->hi[d] = L.hi[d];
    }
    const int64_t w = (int64_t)kPersistentThreads * t->vec;
    if (L.kind == JACC_LOOP_JACOBI2D) {
        t->e1 = L.ext[1];
        t->col0 = col_start(L.lo[1], t->vec);
        if (L.hi[0] <= L.lo[0] || L.hi[1] <= L.lo[1]) return true;
        t->gx = cdiv(L.hi[1] - t->col0, w);
        t->gy = cdiv(L.hi[0] - L.lo[0], t->tile);
        t->gz = 1;
    } else if (L.kind == JACC_LOOP_HEAT3D) {
        t->e1 = L.ext[1];
        t->e2 = L.ext[2];
        t->alpha = L.scalars[0];
        t->col0 = col_start(L.lo[2], t->vec);
        if (heat_empty(L)) return true;
        t->gx = cdiv(L.hi[2] - t->col0, w);
        t->gy = L.hi[1] - L.lo[1];
        t->gz = cdiv(L.hi[0] - L.lo[0], t->tile);
    } else {
        return false;
    }
    t->ntiles = t->gx * t->gy * t->gz;
    return true;
}

// One workgroup per tile (measured: 2.5-5 % faster on 8192^2 steps than a
// resident-sized grid walking static rounds of tiles), up to the largest
// one-dimensional grid; beyond it workgroups take further tiles in strides
// of the grid.
int64_t persistent_grid(int64_t tiles, bool /*jacobi_only*/) {
    const int64_t max_grid = (int64_t)INT32_MAX;
    return tiles < max_grid ? tiles : max_grid;
}

hipError_t launch_persistent(const PTask *tasks, int ntasks, int64_t tiles, int64_t grid, bool jacobi_only,
                             hipStream_t s) {
    if (ntasks <= 0 || tiles <= 0 || grid <= 0) return hipSuccess;
    if (jacobi_only)
        hipLaunchKernelGGL(persistent_kernel<true>, dim3((unsigned)grid), dim3(kPersistentThreads), 0, s, tasks, ntasks,
                           tiles);
    else
        hipLaunchKernelGGL(persistent_kernel<false>, dim3((unsigned)grid), dim3(kPersistentThreads), 0, s, tasks,
                           ntasks, tiles);
    return hipGetLastError();
}

}  // namespace jk
