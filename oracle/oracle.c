/*
 * CPU oracle for the partitioned loop-nest runtime.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link,
 * load or call this file: only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no code, header, table or
 * helper with the HIP library.
 *
 * Every routine is the plain sequential definition of the loop nest it names,
 * in IEEE binary64, built with -O2 -ffp-contract=off (no FMA contraction, no
 * fast-math), so each floating-point operation is exactly the one written.
 *
 * Paper: Matsumura, Garcia De Gonzalo, Pena, "JACC: An OpenACC Runtime
 * Framework with Kernel-Level and Multi-GPU Parallelization" (HiPC 2021,
 * arXiv 2110.14340).  The paper's method distributes a loop nest over devices
 * by dividing the range of each updated array along its parallel dimension
 * equally among devices (Sec. "Division of Multidimensional Arrays"), guards
 * every array write with that device's range (Sec. "Predicate-Based
 * Filtering") and sends the updated data to every other device after each
 * kernel (same section).  The partitioned drivers below follow exactly that
 * simplest scheme: equal owner blocks, write filter by owner block, eager
 * refresh of every replica of every updated row.
 *
 * The paper gives no formula for the loop bodies; the operators used here are
 * the readings recorded in the design notes (Jacobi 5-point average with
 * pairwise sums, explicit 7-point heat step u + alpha*lap).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Compensated summation (Neumaier's improvement of Kahan summation).        */
/* ------------------------------------------------------------------------ */
typedef struct { double s, c; } neum_t;

static void neum_add(neum_t *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double neum_value(const neum_t *a) { return a->s + a->c; }

/* Equal division of the parallel dimension (Sec. "Division of
 * Multidimensional Arrays"): block p of an extent E split K ways is
 * [floor(p*E/K), floor((p+1)*E/K)). */
static int64_t block_lo(int64_t E, int K, int p) { return (int64_t)((__int128)p * E / K); }

/* ------------------------------------------------------------------------ */
/* Jacobi-2D, 5-point average.                                               */
/*   out[i][j] = 0.25 * ((in[i-1][j] + in[i+1][j]) + (in[i][j-1] + in[i][j+1]))
 * over the half-open box [r_lo, r_hi) x [c_lo, c_hi); cells outside the box
 * are not written.  Row-major, ny rows of nx doubles.                        */
/* ------------------------------------------------------------------------ */
void oracle_jacobi2d_sweep(const double *in, double *out, int64_t ny, int64_t nx,
                           int64_t r_lo, int64_t r_hi, int64_t c_lo, int64_t c_hi)
{
    (void)ny;
    for (int64_t i = r_lo; i < r_hi; ++i)
        for (int64_t j = c_lo; j < c_hi; ++j) {
            double vert = in[(i - 1) * nx + j] + in[(i + 1) * nx + j];
            double horz = in[i * nx + (j - 1)] + in[i * nx + (j + 1)];
            out[i * nx + j] = 0.25 * (vert + horz);
        }
}

/* T ping-pong steps over the interior [1, ny-1) x [1, nx-1).  Both buffers
 * must hold the same initial data (so the never-written boundary agrees).
 * Returns 0 when the final state is in a, 1 when it is in b. */
int oracle_jacobi2d(double *a, double *b, int64_t ny, int64_t nx, int64_t steps)
{
    double *src = a, *dst = b;
    for (int64_t t = 0; t < steps; ++t) {
        oracle_jacobi2d_sweep(src, dst, ny, nx, 1, ny - 1, 1, nx - 1);
        double *tmp = src; src = dst; dst = tmp;
    }
    return src == a ? 0 : 1;
}

/* Exact T-step values on the window [r0,r1) x [c0,c1) of a Jacobi run started
 * from u0, computed only over the window's domain of dependence: after s of T
 * steps, only cells within distance T-s of the window can still influence it.
 * Result written row-major into out ((r1-r0) x (c1-c0)). */
int oracle_jacobi2d_window(const double *u0, int64_t ny, int64_t nx, int64_t steps,
                           int64_t r0, int64_t r1, int64_t c0, int64_t c1, double *out)
{
    int64_t R0 = r0 - steps - 1, R1 = r1 + steps + 1, C0 = c0 - steps - 1, C1 = c1 + steps + 1;
    if (R0 < 0) R0 = 0;
    if (C0 < 0) C0 = 0;
    if (R1 > ny) R1 = ny;
    if (C1 > nx) C1 = nx;
    int64_t h = R1 - R0, w = C1 - C0;
    double *a = malloc((size_t)(h * w) * sizeof(double));
    double *b = malloc((size_t)(h * w) * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
    for (int64_t i = 0; i < h; ++i) {
        memcpy(a + i * w, u0 + (R0 + i) * nx + C0, (size_t)w * sizeof(double));
        memcpy(b + i * w, u0 + (R0 + i) * nx + C0, (size_t)w * sizeof(double));
    }
    double *src = a, *dst = b;
    for (int64_t s = 0; s < steps; ++s) {
        int64_t e = steps - 1 - s; /* cells still needed after this step */
        int64_t lo_r = r0 - e, hi_r = r1 + e, lo_c = c0 - e, hi_c = c1 + e;
        if (lo_r < 1) lo_r = 1;
        if (lo_c < 1) lo_c = 1;
        if (hi_r > ny - 1) hi_r = ny - 1;
        if (hi_c > nx - 1) hi_c = nx - 1;
        for (int64_t i = lo_r; i < hi_r; ++i)
            for (int64_t j = lo_c; j < hi_c; ++j) {
                int64_t li = i - R0, lj = j - C0;
                double vert = src[(li - 1) * w + lj] + src[(li + 1) * w + lj];
                double horz = src[li * w + lj - 1] + src[li * w + lj + 1];
                dst[li * w + lj] = 0.25 * (vert + horz);
            }
        double *tmp = src; src = dst; dst = tmp;
    }
    for (int64_t i = r0; i < r1; ++i)
        memcpy(out + (i - r0) * (c1 - c0), src + (i - R0) * w + (c0 - C0),
               (size_t)(c1 - c0) * sizeof(double));
    free(a);
    free(b);
    return 0;
}

/* K-way partitioned Jacobi run (the paper's scheme on K devices, simulated
 * with K private slab arrays).  Partition p owns rows B_p; its slab holds
 * B_p plus one row on each side (clipped to the grid), in two ping-pong
 * copies.  Each step every partition updates only the interior rows it owns
 * (write filter by owner range) reading its own slab; then every row held by
 * more than one slab is refreshed in every non-owner slab from its owner
 * (eager broadcast of updated data).  Finally the owner rows are gathered
 * back into grid.  The result must equal oracle_jacobi2d bit for bit. */
int oracle_jacobi2d_partitioned(double *grid, int64_t ny, int64_t nx, int64_t steps, int K)
{
    if (K < 1 || K > ny) return -1;
    double **sa = calloc((size_t)K, sizeof(double *));
    double **sb = calloc((size_t)K, sizeof(double *));
    int64_t *slo = calloc((size_t)K, sizeof(int64_t));
    int64_t *shi = calloc((size_t)K, sizeof(int64_t));
    int rc = 0;
    for (int p = 0; p < K; ++p) {
        int64_t lo = block_lo(ny, K, p) - 1, hi = block_lo(ny, K, p + 1) + 1;
        if (lo < 0) lo = 0;
        if (hi > ny) hi = ny;
        slo[p] = lo;
        shi[p] = hi;
        size_t bytes = (size_t)((hi - lo) * nx) * sizeof(double);
        sa[p] = malloc(bytes ? bytes : 1);
        sb[p] = malloc(bytes ? bytes : 1);
        if (!sa[p] || !sb[p]) { rc = -1; goto done; }
        memcpy(sa[p], grid + lo * nx, bytes);
        memcpy(sb[p], grid + lo * nx, bytes);
    }
    for (int64_t t = 0; t < steps; ++t) {
        for (int p = 0; p < K; ++p) {
            int64_t lo = block_lo(ny, K, p), hi = block_lo(ny, K, p + 1);
            if (lo < 1) lo = 1;
            if (hi > ny - 1) hi = ny - 1;
            const double *in = sa[p];
            double *out = sb[p];
            for (int64_t i = lo; i < hi; ++i) {
                int64_t li = i - slo[p];
                for (int64_t j = 1; j < nx - 1; ++j) {
                    double vert = in[(li - 1) * nx + j] + in[(li + 1) * nx + j];
                    double horz = in[li * nx + j - 1] + in[li * nx + j + 1];
                    out[li * nx + j] = 0.25 * (vert + horz);
                }
            }
        }
        /* refresh every replica from the owner's freshly written slab */
        for (int p = 0; p < K; ++p)
            for (int64_t r = slo[p]; r < shi[p]; ++r) {
                int q = 0;
                while (q + 1 < K && block_lo(ny, K, q + 1) <= r) ++q;
                if (q == p) continue;
                memcpy(sb[p] + (r - slo[p]) * nx, sb[q] + (r - slo[q]) * nx,
                       (size_t)nx * sizeof(double));
            }
        for (int p = 0; p < K; ++p) { double *tmp = sa[p]; sa[p] = sb[p]; sb[p] = tmp; }
    }
    for (int p = 0; p < K; ++p) {
        int64_t lo = block_lo(ny, K, p), hi = block_lo(ny, K, p + 1);
        if (hi > lo)
            memcpy(grid + lo * nx, sa[p] + (lo - slo[p]) * nx, (size_t)((hi - lo) * nx) * sizeof(double));
    }
done:
    for (int p = 0; p < K; ++p) { free(sa[p]); free(sb[p]); }
    free(sa); free(sb); free(slo); free(shi);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Heat-3D, explicit 7-point step.                                           */
/*   lap = (((u[x-1]+u[x+1]) + (u[y-1]+u[y+1])) + (u[z-1]+u[z+1])) - 6.0*u
 *   u'  = u + alpha*lap
 * over [z_lo,z_hi) x [y_lo,y_hi) x [x_lo,x_hi); array u[z][y][x].
 * When res != NULL, *res receives the compensated sum over the box of
 * (u' - u)^2, the difference taken between the stored values.              */
/* ------------------------------------------------------------------------ */
static double heat_cell(const double *in, int64_t ny, int64_t nx, int64_t z, int64_t y, int64_t x,
                        double alpha)
{
    int64_t c = (z * ny + y) * nx + x;
    double px = in[c - 1] + in[c + 1];
    double py = in[c - nx] + in[c + nx];
    double pz = in[c - ny * nx] + in[c + ny * nx];
    double lap = ((px + py) + pz) - 6.0 * in[c];
    return in[c] + alpha * lap;
}

void oracle_heat3d_sweep(const double *in, double *out, int64_t nz, int64_t ny, int64_t nx,
                         int64_t z_lo, int64_t z_hi, int64_t y_lo, int64_t y_hi,
                         int64_t x_lo, int64_t x_hi, double alpha, double *res)
{
    (void)nz;
    neum_t acc = {0.0, 0.0};
    for (int64_t z = z_lo; z < z_hi; ++z)
        for (int64_t y = y_lo; y < y_hi; ++y)
            for (int64_t x = x_lo; x < x_hi; ++x) {
                int64_t c = (z * ny + y) * nx + x;
                double v = heat_cell(in, ny, nx, z, y, x, alpha);
                out[c] = v;
                double d = v - in[c];
                neum_add(&acc, d * d);
            }
    if (res) *res = neum_value(&acc);
}

/* T ping-pong steps over the interior; residuals[t] (if not NULL) receives
 * the residual of step t.  Returns 0 when the result is in a, 1 if in b. */
int oracle_heat3d(double *a, double *b, int64_t nz, int64_t ny, int64_t nx, int64_t steps,
                  double alpha, double *residuals)
{
    double *src = a, *dst = b;
    for (int64_t t = 0; t < steps; ++t) {
        oracle_heat3d_sweep(src, dst, nz, ny, nx, 1, nz - 1, 1, ny - 1, 1, nx - 1, alpha,
                            residuals ? residuals + t : NULL);
        double *tmp = src; src = dst; dst = tmp;
    }
    return src == a ? 0 : 1;
}

/* Exact T-step field on the window [z0,z1) x [y0,y1) x [x0,x1), computed only
 * over the window's domain of dependence (as oracle_jacobi2d_window). */
int oracle_heat3d_window(const double *u0, int64_t nz, int64_t ny, int64_t nx, int64_t steps,
                         double alpha, int64_t z0, int64_t z1, int64_t y0, int64_t y1,
                         int64_t x0, int64_t x1, double *out)
{
    int64_t Z0 = z0 - steps - 1, Z1 = z1 + steps + 1;
    int64_t Y0 = y0 - steps - 1, Y1 = y1 + steps + 1;
    int64_t X0 = x0 - steps - 1, X1 = x1 + steps + 1;
    if (Z0 < 0) Z0 = 0;
    if (Y0 < 0) Y0 = 0;
    if (X0 < 0) X0 = 0;
    if (Z1 > nz) Z1 = nz;
    if (Y1 > ny) Y1 = ny;
    if (X1 > nx) X1 = nx;
    int64_t d = Z1 - Z0, h = Y1 - Y0, w = X1 - X0;
    size_t cells = (size_t)(d * h * w);
    double *a = malloc(cells * sizeof(double));
    double *b = malloc(cells * sizeof(double));
    if (!a || !b) { free(a); free(b); return -1; }
    for (int64_t z = 0; z < d; ++z)
        for (int64_t y = 0; y < h; ++y) {
            const double *row = u0 + ((Z0 + z) * ny + (Y0 + y)) * nx + X0;
            memcpy(a + (z * h + y) * w, row, (size_t)w * sizeof(double));
            memcpy(b + (z * h + y) * w, row, (size_t)w * sizeof(double));
        }
    double *src = a, *dst = b;
    for (int64_t s = 0; s < steps; ++s) {
        int64_t e = steps - 1 - s;
        int64_t lz = z0 - e, hz = z1 + e, ly = y0 - e, hy = y1 + e, lx = x0 - e, hx = x1 + e;
        if (lz < 1) lz = 1;
        if (ly < 1) ly = 1;
        if (lx < 1) lx = 1;
        if (hz > nz - 1) hz = nz - 1;
        if (hy > ny - 1) hy = ny - 1;
        if (hx > nx - 1) hx = nx - 1;
        for (int64_t z = lz; z < hz; ++z)
            for (int64_t y = ly; y < hy; ++y)
                for (int64_t x = lx; x < hx; ++x)
                    dst[((z - Z0) * h + (y - Y0)) * w + (x - X0)] =
                        heat_cell(src, h, w, z - Z0, y - Y0, x - X0, alpha);
        double *tmp = src; src = dst; dst = tmp;
    }
    for (int64_t z = z0; z < z1; ++z)
        for (int64_t y = y0; y < y1; ++y)
            memcpy(out + ((z - z0) * (y1 - y0) + (y - y0)) * (x1 - x0),
                   src + ((z - Z0) * h + (y - Y0)) * w + (x0 - X0), (size_t)(x1 - x0) * sizeof(double));
    free(a);
    free(b);
    return 0;
}

/* K-way partitioned heat run over z-plane slabs (same scheme as the
 * partitioned Jacobi oracle, planes instead of rows).  The residual of each
 * step is reduced per partition over the planes it owns, then the K partial
 * sums are added in partition order: the paper filters a reduction by the
 * range of the outermost parallel iterator and combines the per-device
 * results (Sec. "Predicate-Based Filtering", reduction paragraph). */
int oracle_heat3d_partitioned(double *grid, int64_t nz, int64_t ny, int64_t nx, int64_t steps,
                              double alpha, int K, double *residuals)
{
    if (K < 1 || K > nz) return -1;
    int64_t plane = ny * nx;
    double **sa = calloc((size_t)K, sizeof(double *));
    double **sb = calloc((size_t)K, sizeof(double *));
    int64_t *slo = calloc((size_t)K, sizeof(int64_t));
    int64_t *shi = calloc((size_t)K, sizeof(int64_t));
    double *part = calloc((size_t)K, sizeof(double));
    int rc = 0;
    for (int p = 0; p < K; ++p) {
        int64_t lo = block_lo(nz, K, p) - 1, hi = block_lo(nz, K, p + 1) + 1;
        if (lo < 0) lo = 0;
        if (hi > nz) hi = nz;
        slo[p] = lo;
        shi[p] = hi;
        size_t bytes = (size_t)((hi - lo) * plane) * sizeof(double);
        sa[p] = malloc(bytes ? bytes : 1);
        sb[p] = malloc(bytes ? bytes : 1);
        if (!sa[p] || !sb[p]) { rc = -1; goto done; }
        memcpy(sa[p], grid + lo * plane, bytes);
        memcpy(sb[p], grid + lo * plane, bytes);
    }
    for (int64_t t = 0; t < steps; ++t) {
        for (int p = 0; p < K; ++p) {
            int64_t lo = block_lo(nz, K, p), hi = block_lo(nz, K, p + 1);
            if (lo < 1) lo = 1;
            if (hi > nz - 1) hi = nz - 1;
            neum_t acc = {0.0, 0.0};
            const double *in = sa[p];
            double *out = sb[p];
            for (int64_t z = lo; z < hi; ++z)
                for (int64_t y = 1; y < ny - 1; ++y)
                    for (int64_t x = 1; x < nx - 1; ++x) {
                        int64_t c = ((z - slo[p]) * ny + y) * nx + x;
                        double v = heat_cell(in, ny, nx, z - slo[p], y, x, alpha);
                        out[c] = v;
                        double dd = v - in[c];
                        neum_add(&acc, dd * dd);
                    }
            part[p] = neum_value(&acc);
        }
        if (residuals) {
            double r = 0.0;
            for (int p = 0; p < K; ++p) r += part[p];
            residuals[t] = r;
        }
        for (int p = 0; p < K; ++p)
            for (int64_t r = slo[p]; r < shi[p]; ++r) {
                int q = 0;
                while (q + 1 < K && block_lo(nz, K, q + 1) <= r) ++q;
                if (q == p) continue;
                memcpy(sb[p] + (r - slo[p]) * plane, sb[q] + (r - slo[q]) * plane,
                       (size_t)plane * sizeof(double));
            }
        for (int p = 0; p < K; ++p) { double *tmp = sa[p]; sa[p] = sb[p]; sb[p] = tmp; }
    }
    for (int p = 0; p < K; ++p) {
        int64_t lo = block_lo(nz, K, p), hi = block_lo(nz, K, p + 1);
        if (hi > lo)
            memcpy(grid + lo * plane, sa[p] + (lo - slo[p]) * plane,
                   (size_t)((hi - lo) * plane) * sizeof(double));
    }
done:
    for (int p = 0; p < K; ++p) { free(sa[p]); free(sb[p]); }
    free(sa); free(sb); free(slo); free(shi); free(part);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Sum reduction: s = sum x[i] (squares != 0: sum x[i]^2), compensated.      */
/* ------------------------------------------------------------------------ */
double oracle_sum(const double *x, int64_t n, int squares)
{
    neum_t acc = {0.0, 0.0};
    for (int64_t i = 0; i < n; ++i) neum_add(&acc, squares ? x[i] * x[i] : x[i]);
    return neum_value(&acc);
}

/* Partitioned sum: each of K owner blocks of [0,n) is reduced on its own,
 * then the K partial sums are added in partition order. */
double oracle_sum_partitioned(const double *x, int64_t n, int K, int squares)
{
    double total = 0.0;
    for (int p = 0; p < K; ++p) {
        int64_t lo = block_lo(n, K, p), hi = block_lo(n, K, p + 1);
        total += oracle_sum(x + lo, hi - lo, squares);
    }
    return total;
}

/* ------------------------------------------------------------------------ */
/* Dense contraction C = A * B, A: M x L, B: L x N, C: M x N, row-major.     */
/* Plain i-k-j triple loop, k ascending, C starting from zero.               */
/* ------------------------------------------------------------------------ */
void oracle_gemm(const double *A, const double *B, double *C, int64_t M, int64_t N, int64_t L)
{
    for (int64_t i = 0; i < M; ++i) {
        double *c = C + i * N;
        for (int64_t j = 0; j < N; ++j) c[j] = 0.0;
        for (int64_t k = 0; k < L; ++k) {
            double a = A[i * L + k];
            const double *b = B + k * N;
            for (int64_t j = 0; j < N; ++j) c[j] += a * b[j];
        }
    }
}

/* One row block [i0, i1) of C only (for sampled checks at full size). */
void oracle_gemm_rows(const double *A, const double *B, double *C, int64_t N, int64_t L,
                      int64_t i0, int64_t i1)
{
    for (int64_t i = i0; i < i1; ++i) {
        double *c = C + (i - i0) * N;
        for (int64_t j = 0; j < N; ++j) c[j] = 0.0;
        for (int64_t k = 0; k < L; ++k) {
            double a = A[i * L + k];
            const double *b = B + k * N;
            for (int64_t j = 0; j < N; ++j) c[j] += a * b[j];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* CSR sparse matrix-vector product, k ascending within each row.           */
/*   y[i] = sum_{k=rp[i]}^{rp[i+1]-1} val[k] * x[col[k]]                     */
/* ------------------------------------------------------------------------ */
void oracle_spmv_csr(const int32_t *rp, const int32_t *col, const double *val, const double *x,
                     double *y, int64_t row_lo, int64_t row_hi)
{
    for (int64_t i = row_lo; i < row_hi; ++i) {
        double s = 0.0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) s += val[k] * x[col[k]];
        y[i] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* Statement chain of the paper's predicate-filtering example (Sec.          */
/* "Predicate-Based Filtering", Fig. conv-code).  Iteration t, in order,      */
/* with (i, j, k) = idx[3t..3t+2] and x = xs[t]:                              */
/*   a[i] = x;  b[i] = a[i];  x = c[j];  a[k] = x;  b[k] = a[k];             */
/* An iteration whose i or k lies outside [0, min(na, nb)) or whose j lies   */
/* outside [0, nc) is skipped.  a and b may be the same array.               */
/* ------------------------------------------------------------------------ */
void oracle_pred_chain(double *a, int64_t na, double *b, int64_t nb, const double *c, int64_t nc,
                       const int32_t *idx, const double *xs, int64_t lo, int64_t hi)
{
    int64_t nab = na < nb ? na : nb;
    for (int64_t t = lo; t < hi; ++t) {
        int64_t i = idx[3 * t], j = idx[3 * t + 1], k = idx[3 * t + 2];
        if (i < 0 || i >= nab || k < 0 || k >= nab || j < 0 || j >= nc) continue;
        double x = xs[t];
        a[i] = x;
        b[i] = a[i];
        x = c[j];
        a[k] = x;
        b[k] = a[k];
    }
}

/* The same chain run the paper's way on K devices: every device holds its
 * own copies of a and b and runs every iteration, each statement guarded as
 * in the example by the owner ranges (equal division) of the arrays whose
 * local values it feeds; afterwards each device's owner rows are what the
 * others receive, so the result is the owner rows gathered.  Returns 0, or
 * -1 on a bad K or a failed allocation. */
int oracle_pred_chain_partitioned(double *a, int64_t na, double *b, int64_t nb, const double *c, int64_t nc,
                                  const int32_t *idx, const double *xs, int64_t lo, int64_t hi, int K)
{
    if (K < 1 || K > na || K > nb) return -1;
    int64_t nab = na < nb ? na : nb;
    double *ra = malloc((size_t)na * sizeof(double)), *rb = malloc((size_t)nb * sizeof(double));
    double *out_a = malloc((size_t)na * sizeof(double)), *out_b = malloc((size_t)nb * sizeof(double));
    if (!ra || !rb || !out_a || !out_b) {
        free(ra);
        free(rb);
        free(out_a);
        free(out_b);
        return -1;
    }
    for (int p = 0; p < K; ++p) {
        int64_t alo = block_lo(na, K, p), ahi = block_lo(na, K, p + 1);
        int64_t blo = block_lo(nb, K, p), bhi = block_lo(nb, K, p + 1);
        memcpy(ra, a, (size_t)na * sizeof(double)); /* device p's replicas */
        memcpy(rb, b, (size_t)nb * sizeof(double));
        for (int64_t t = lo; t < hi; ++t) {
            int64_t i = idx[3 * t], j = idx[3 * t + 1], k = idx[3 * t + 2];
            if (i < 0 || i >= nab || k < 0 || k >= nab || j < 0 || j >= nc) continue;
            int i_a = alo <= i && i < ahi, i_b = blo <= i && i < bhi;
            int k_a = alo <= k && k < ahi, k_b = blo <= k && k < bhi;
            double x = xs[t];
            if (i_a || i_b) ra[i] = x;
            if (i_b) rb[i] = ra[i];
            x = (k_a || k_b) ? c[j] : 0.0;
            if (k_a || k_b) ra[k] = x;
            if (k_b) rb[k] = ra[k];
        }
        memcpy(out_a + alo, ra + alo, (size_t)(ahi - alo) * sizeof(double));
        memcpy(out_b + blo, rb + blo, (size_t)(bhi - blo) * sizeof(double));
    }
    memcpy(a, out_a, (size_t)na * sizeof(double));
    memcpy(b, out_b, (size_t)nb * sizeof(double));
    free(ra);
    free(rb);
    free(out_a);
    free(out_b);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Indirect write: out[idx[i]] = in[i]*in[i] for i in [lo, hi) (distinct     */
/* indices; an index outside [0, n_out) is skipped).                         */
/* ------------------------------------------------------------------------ */
void oracle_scatter_sq(const double *in, const int32_t *idx, double *out, int64_t n_out, int64_t lo, int64_t hi)
{
    for (int64_t i = lo; i < hi; ++i) {
        int64_t k = idx[i];
        if (k >= 0 && k < n_out) out[k] = in[i] * in[i];
    }
}

/* K-way partitioned version with the paper's write filter: every partition
 * runs all iterations and keeps the writes whose target lies in its owner
 * block, into a private copy of that block; the blocks are then gathered. */
int oracle_scatter_sq_partitioned(const double *in, const int32_t *idx, double *out, int64_t n_out, int64_t lo,
                                  int64_t hi, int K)
{
    if (K < 1 || K > n_out) return -1;
    for (int p = 0; p < K; ++p) {
        int64_t b0 = block_lo(n_out, K, p), b1 = block_lo(n_out, K, p + 1);
        double *mine = malloc((size_t)(b1 - b0 + 1) * sizeof(double));
        if (!mine) return -1;
        memcpy(mine, out + b0, (size_t)(b1 - b0) * sizeof(double));
        for (int64_t i = lo; i < hi; ++i) {
            int64_t k = idx[i];
            double v = in[i] * in[i];
            if (b0 <= k && k < b1) mine[k - b0] = v;
        }
        memcpy(out + b0, mine, (size_t)(b1 - b0) * sizeof(double));
        free(mine);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Multi-threaded forms of the full-grid runs, for full-size references and  */
/* the all-core CPU timing.  Threads split the rows (planes) of each sweep;  */
/* every element is computed by the same expression as in the sequential     */
/* routine and no element's arithmetic depends on which thread runs it, so   */
/* the fields are bit-identical to oracle_jacobi2d / oracle_heat3d /         */
/* oracle_gemm.  nthreads <= 0 takes the OpenMP default.                     */
/* ------------------------------------------------------------------------ */
static int team(int nthreads) { return nthreads > 0 ? nthreads : omp_get_max_threads(); }

/* Threads a multi-threaded routine uses for a given request. */
int oracle_threads(int nthreads) { return team(nthreads); }

int oracle_jacobi2d_mt(double *a, double *b, int64_t ny, int64_t nx, int64_t steps, int nthreads)
{
    double *src = a, *dst = b;
    for (int64_t t = 0; t < steps; ++t) {
#pragma omp parallel for schedule(static) num_threads(team(nthreads))
        for (int64_t i = 1; i < ny - 1; ++i)
            oracle_jacobi2d_sweep(src, dst, ny, nx, i, i + 1, 1, nx - 1);
        double *tmp = src; src = dst; dst = tmp;
    }
    return src == a ? 0 : 1;
}

/* The residual of a step is formed per plane (a compensated sum over the
 * plane's interior cells in x-fastest order), and the plane sums are then
 * added in plane order with compensation.  The field is bit-identical to
 * oracle_heat3d; the residual is another correctly compensated summation
 * order of the same terms (within a few units in the last place of it). */
int oracle_heat3d_mt(double *a, double *b, int64_t nz, int64_t ny, int64_t nx, int64_t steps,
                     double alpha, double *residuals, int nthreads)
{
    double *plane_sum = malloc((size_t)(nz > 0 ? nz : 1) * sizeof(double));
    if (!plane_sum) return -1;
    double *src = a, *dst = b;
    for (int64_t t = 0; t < steps; ++t) {
#pragma omp parallel for schedule(static) num_threads(team(nthreads))
        for (int64_t z = 1; z < nz - 1; ++z)
            oracle_heat3d_sweep(src, dst, nz, ny, nx, z, z + 1, 1, ny - 1, 1, nx - 1, alpha, &plane_sum[z]);
        if (residuals) {
            neum_t acc = {0.0, 0.0};
            for (int64_t z = 1; z < nz - 1; ++z) neum_add(&acc, plane_sum[z]);
            residuals[t] = neum_value(&acc);
        }
        double *tmp = src; src = dst; dst = tmp;
    }
    free(plane_sum);
    return src == a ? 0 : 1;
}

void oracle_gemm_mt(const double *A, const double *B, double *C, int64_t M, int64_t N, int64_t L, int nthreads)
{
#pragma omp parallel for schedule(dynamic, 8) num_threads(team(nthreads))
    for (int64_t i = 0; i < M; ++i) oracle_gemm_rows(A, B, C + i * N, N, L, i, i + 1);
}

void oracle_spmv_csr_mt(const int32_t *rp, const int32_t *col, const double *val, const double *x, double *y,
                        int64_t row_lo, int64_t row_hi, int nthreads)
{
#pragma omp parallel for schedule(static, 4096) num_threads(team(nthreads))
    for (int64_t i = row_lo; i < row_hi; ++i) oracle_spmv_csr(rp, col, val, x, y, i, i + 1);
}
