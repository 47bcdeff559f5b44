// Internal interface between the runtime (runtime.cpp) and the HIP loop
// bodies (k_*.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jk {

// One argument as a kernel sees it: `ptr` is the device address of global
// row 0 of the array *as if* the slab started there (slab pointer minus
// slab_lo rows), so kernels index with global row numbers; only rows
// [slab_lo, slab_hi) may be touched.  For a 2-D array partitioned along
// dim 1 the slab holds columns [slab_lo, slab_hi) of every row, `ptr` is
// the slab pointer minus slab_lo elements, and element (i, j) sits at
// ptr + i*row_elems + j.
struct Arg {
    const void *ptr;       // biased pointer (see above)
    int64_t slab_lo, slab_hi;
    int64_t row_elems;     // elements per row of dim 0 (the slab's width when split along dim 1)
};

struct Cfg {
    int bx, by, tile, vec, persistent, order, march, rows;
};

// Write-through targets of a stencil launch: rows [lo, hi) of dim 0 that the
// launch writes are also stored at `ptr` (biased like Arg::ptr), which is
// another partition's slab holding those rows as halo.
struct Mirror {
    double *ptr;
    int64_t lo, hi;
};
struct Mirrors {
    Mirror m[2];
    int n;
};
// Column mirrors (a 2-D array split along dim 1): [lo, hi) are the columns
// the holder slab keeps, pitch its row length in elements, and ptr is biased
// so that ptr[row * pitch + column] is global (row, column).
struct ColMirror {
    double *ptr;
    int64_t lo, hi, pitch;
};
struct ColMirrors {
    ColMirror m[2];
    int n;
};

// One partition's launch of one loop nest.
struct Launch {
    int kind;
    int ndim;
    int64_t lo[3], hi[3];       // iteration box (dim 0 already clipped to the partition)
    int64_t ext[4];             // extents of the first argument's array
    Arg a[6];
    int nargs;
    double scalars[4];
    Cfg cfg;
    int part_dim;     // the dimension the arrays are split along (0, or 1 for 2-D column slabs)
    Mirrors mir;      // stencil kinds only
    ColMirrors cmir;  // JACOBI2D on arrays split along dim 1 (mir is then empty)
    int64_t own_lo, own_hi;    // owner rows of a FILTERED output (writes elsewhere are dropped)
    int64_t own2_lo, own2_hi;  // owner rows of a second FILTERED output (PRED_CHAIN's b)
    // reductions: workgroup partials go to `wg_partials` (capacity
    // `wg_capacity` doubles); the finaliser writes their ordered sum to
    // `part_out`.  Both null when the loop reduces nothing.
    double *wg_partials;
    int64_t wg_capacity;
    double *part_out;
    int64_t part_rows;  // iterations along dim 0 of the largest partition (for defaults)
};

// Launches the loop body (and, for reductions, the per-partition
// finaliser) on `s`.  Returns hipErrorInvalidValue for a configuration the
// body does not support; the runtime validates shapes before calling.
hipError_t launch_loop(const Launch &L, hipStream_t s);

// Checks a configuration for a loop without launching; returns 0 if legal.
int check_config(const Launch &L);

// Fills in defaults for zero fields of a configuration.
Cfg default_config(int kind, const Launch &L, Cfg c);

// Reduction combine: out[0] = sum of partials[idx[k]] for k = 0..n-1 in
// that order (idx lists the reducing partitions in partition order; each
// partition's finaliser writes partials[p]).
struct CombineList {
    int n;
    int idx[64];
};
hipError_t launch_combine(const double *partials, const CombineList &list, double *out, hipStream_t s);

// One loop of a persistent task group: a stencil sweep cut into tiles of
// 256 threads (256*vec columns x `tile` rows, or x 1 row x `tile` planes).
struct PTask {
    int32_t kind;  // JACC_LOOP_JACOBI2D or JACC_LOOP_HEAT3D
    int32_t vec, tile, march;
    const double *in;
    double *out;
    int64_t e1, e2;  // extents of dims 1 and 2 (2-D: e1 = row length)
    int64_t lo[3], hi[3];
    int64_t col0;
    double alpha;
    int64_t gx, gy, gz;
    int64_t ntiles, tile_begin;
    Mirrors mir;
};
constexpr int kPersistentThreads = 256;

// Builds the task record of a launch (false if the kind cannot run inside
// the persistent kernel).
bool make_task(const Launch &L, PTask *t);

// Workgroups of a persistent launch over `tiles` tiles (one per tile).
int64_t persistent_grid(int64_t tiles, bool jacobi_only);

// Launches the persistent kernel with `grid` workgroups over `ntasks` device
// task records whose tiles total `tiles` (jacobi_only: every task is a
// Jacobi sweep, which selects the variant without the heat bodies).
hipError_t launch_persistent(const PTask *tasks, int ntasks, int64_t tiles, int64_t grid, bool jacobi_only,
                             hipStream_t s);

// The partitions of one eager stencil (or SUM) loop in one launch ("packed"): the
// launches of its partitions (the same kind, configuration and box apart
// from the dim-0 range, pointers, mirrors and reduction target), at most
// kMaxPack.  Each partition's tiles take a run of workgroups starting at a
// multiple of 8, so the XCD-aware tile orders hold within it.  With a
// residual, partition p's workgroup partials go to wg_partials + (its first
// tile among all partitions') and one finaliser launch writes every
// partition's ordered sum to its part_out.  Returns hipErrorInvalidValue
// for more than kMaxPack launches or more than wg_capacity partials.
constexpr int kMaxPack = 16;
hipError_t launch_parts(const Launch *L, int n, double *wg_partials, int64_t wg_capacity, hipStream_t s);
// Workgroup partials a packed heat launch with a residual writes.
int64_t parts_partials(const Launch *L, int n);

// out[k] = ordered sum of base[off[k] .. off[k] + n[k]) for k < count, each
// in the finaliser's order (one workgroup per segment).
struct Segments {
    int64_t off[kMaxPack], n[kMaxPack];
    double *out[kMaxPack];
    int32_t count;
};
hipError_t launch_finalise_many(const double *base, const Segments &seg, hipStream_t s);
// The partitions of one SUM loop in one launch, then their finalisers (the
// same bits as a launch per partition).
hipError_t launch_sum_parts(const Launch *L, int n, double *wg_partials, int64_t wg_capacity, hipStream_t s);

// Number of workgroups the loop's reduction writes partials for (for
// sizing; <= wg_capacity is required).
int64_t reduction_workgroups(const Launch &L);

// ---- per-kind launchers (k_*.hip) -----------------------------------------
hipError_t launch_jacobi2d(const Launch &L, hipStream_t s);
hipError_t launch_heat3d(const Launch &L, hipStream_t s);
int64_t heat3d_workgroups(const Launch &L);
hipError_t launch_sum(const Launch &L, hipStream_t s);
int64_t sum_workgroups(const Launch &L);
hipError_t launch_finalise(const double *partials, int64_t n, double *out, hipStream_t s);
hipError_t launch_gemm(const Launch &L, hipStream_t s);
hipError_t launch_spmv(const Launch &L, hipStream_t s);

// Column-banded SpMV of one partition (rows L.lo[0]..L.hi[0]): device
// buffers of its band-major copy.  bands = 8*S; bptr holds bands*n + 1
// offsets, sums band_scan_blocks(bands*n) + 1 scan totals, bcol/bval the
// partition's entries, part bands*n doubles (also the counts' scratch during
// the build).
struct BandBufs {
    int bands;
    int64_t ncols;
    int32_t *bptr, *sums, *bcol;
    double *bval, *part;
};
int64_t band_width(int64_t ncols, int bands);
int64_t band_scan_blocks(int64_t len);
hipError_t build_bands(const Launch &L, const BandBufs &bb, hipStream_t s);
hipError_t launch_spmv_banded(const Launch &L, const BandBufs &bb, hipStream_t s);
// The banded products of n partitions (their band-major copies bb[k], the
// same band count) in one launch, then one combine launch (the same bits as
// a launch per partition).
hipError_t launch_spmv_banded_parts(const Launch *L, const BandBufs *bb, int n, hipStream_t s);
hipError_t launch_scatter(const Launch &L, hipStream_t s);
hipError_t launch_chain(const Launch &L, hipStream_t s);

// Fills `height` lines of `width_bytes` bytes, `pitch_bytes` apart from
// `base`, with 0xFF bytes (k_fill.hip; all three multiples of 4).
hipError_t launch_poison(void *base, size_t pitch_bytes, size_t width_bytes, int64_t height, hipStream_t s);

// ---- learned cost model (k_mlp.hip) ----------------------------------------
constexpr int kMlpHidden = 64;
constexpr int kMlpMaxFeatures = 16;

// Device buffers of one model: parameters, Adam moments, gradient, feature
// scaler, and per-sample scratch for `cap` samples.
struct MlpBufs {
    int F = 0, cap = 0;
    float *params = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *mu = nullptr, *sd = nullptr;
    float *xs = nullptr, *h1 = nullptr, *h2 = nullptr, *h3 = nullptr, *yhat = nullptr, *g = nullptr;
    float *d1 = nullptr, *d2 = nullptr, *d3 = nullptr, *sqerr = nullptr;
    float *loss = nullptr;  // loss of each training step
    int64_t loss_at = 0;    // index written by the next backward pass
};
int mlp_nparams(int F);
size_t mlp_lds_bytes(int F);
// Forward pass of n samples (rows idx[b] of X, or row b when idx is null);
// keep = store the activations for a backward pass.
hipError_t mlp_forward(const MlpBufs &B, const float *X, const int *idx, int n, float *yhat, bool keep,
                       hipStream_t s);
// Deltas, parameter gradient (B.grad) and mean squared error (B.loss[loss_at])
// of the last kept forward pass.
hipError_t mlp_backward(const MlpBufs &B, const float *y, const int *idx, int n, hipStream_t s);
// One Adam step (t is 1-based).
hipError_t mlp_adam(const MlpBufs &B, int t, float lr, hipStream_t s);

}  // namespace jk
