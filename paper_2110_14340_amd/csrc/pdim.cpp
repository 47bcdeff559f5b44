// Choice of the parallel dimension of an updated array (Sec. "Division of
// Multidimensional Arrays"): the dimension indexed by the most parallel loop
// iterators, among those the one indexed by the fewest sequential iterators,
// and among equal candidates the leftmost for row-major (C) arrays or the
// rightmost for column-major (Fortran) arrays.  A dimension indexed by no
// parallel iterator is never chosen; when no dimension is, the loop cannot
// be divided without duplicating its computation.
//
// Host-only; the runtime itself partitions dimension 0 of every array.
#include "jacc.h"

extern "C" int jacc_parallel_dim(int ndim, const int *parallel_iters, const int *sequential_iters, int column_major,
                                 int *dim) {
    if (!dim || ndim < 1 || ndim > 16 || !parallel_iters || !sequential_iters) return JACC_ERR_INVALID;
    for (int d = 0; d < ndim; ++d)
        if (parallel_iters[d] < 0 || sequential_iters[d] < 0) return JACC_ERR_INVALID;
    int best = -1;
    for (int k = 0; k < ndim; ++k) {
        const int d = column_major ? ndim - 1 - k : k;  // candidates in preference order
        if (parallel_iters[d] == 0) continue;
        if (best < 0 || parallel_iters[d] > parallel_iters[best] ||
            (parallel_iters[d] == parallel_iters[best] && sequential_iters[d] < sequential_iters[best]))
            best = d;
    }
    *dim = best;
    return JACC_OK;
}
