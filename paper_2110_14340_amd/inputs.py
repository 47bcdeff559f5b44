"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.  This module draws random numbers only: it holds none of the loop
nests' arithmetic.  Every generator uses numpy's PCG64 (default_rng(seed)).

Workload shapes stand in for the paper's application inputs (Table "bench":
CloverLeaf's 2-D double-buffered halo stencils, Himeno/BT/LU/SP 3-D halo
stencils, CG's irregular reads, NPB apps with tens of kernels).
"""
import numpy as np


def rng(seed):
    return np.random.default_rng(seed)


def jacobi_grid(ny, nx, seed):
    """Interior uniform[0,1); boundary ring 0."""
    g = np.zeros((ny, nx), dtype=np.float64)
    if ny > 2 and nx > 2:
        g[1:-1, 1:-1] = rng(seed).random((ny - 2, nx - 2))
    return g


def heat_field(nz, ny, nx, seed):
    """Every cell, faces included, uniform[0,1)."""
    return rng(seed).random((nz, ny, nx))


def uniform(shape, seed, lo=0.0, hi=1.0):
    r = rng(seed).random(shape)
    return lo + (hi - lo) * r if (lo, hi) != (0.0, 1.0) else r


def int_valued(shape, seed, lo, hi):
    """Integer values in [lo, hi], stored as FP64."""
    return rng(seed).integers(lo, hi + 1, size=shape).astype(np.float64)


def gemm_inputs(M, N, L, seed, integer=False):
    """A (M x L), B (L x N): uniform[-1,1), or integers in [-8, 8]."""
    r = rng(seed)
    if integer:
        A = r.integers(-8, 9, size=(M, L)).astype(np.float64)
        B = r.integers(-8, 9, size=(L, N)).astype(np.float64)
    else:
        A = r.random((M, L)) * 2.0 - 1.0
        B = r.random((L, N)) * 2.0 - 1.0
    return A, B


def csr_matrix(nrows, ncols, draws_per_row, seed, integer_values=False):
    """Random CSR matrix: draws_per_row column indices per row drawn
    uniformly with replacement, sorted, duplicates dropped; values N(0,1)
    (or integers in [-4, 4]); plus x uniform[-1,1) of length ncols.
    Returns (row_ptr int32, col int32, val f64, x f64)."""
    r = rng(seed)
    cols = r.integers(0, ncols, size=(nrows, draws_per_row), dtype=np.int64)
    cols.sort(axis=1)
    keep = np.ones_like(cols, dtype=bool)
    keep[:, 1:] = cols[:, 1:] != cols[:, :-1]
    counts = keep.sum(axis=1)
    rp = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    col = cols[keep].astype(np.int32)
    nnz = col.size
    if integer_values:
        val = r.integers(-4, 5, size=nnz).astype(np.float64)
    else:
        val = r.standard_normal(nnz)
    x = r.random(ncols) * 2.0 - 1.0
    return rp.astype(np.int32), col, val, x


def log_uniform_int(r, lo, hi, size):
    """Integers drawn log-uniformly in [lo, hi]."""
    v = np.exp(r.uniform(np.log(lo), np.log(hi + 1), size=size))
    return np.clip(np.floor(v).astype(np.int64), lo, hi)


def batch_shapes(seed, n2d=128, n3d=128, side2d=(64, 4096), side3d=(32, 512)):
    """Shapes of a batch of independent stencil sweeps: n2d 2-D grids with
    each side log-uniform in side2d and n3d 3-D grids with sides log-uniform
    in side3d.  Returns a list of tuples (2-D first, then 3-D)."""
    r = rng(seed)
    s2 = log_uniform_int(r, side2d[0], side2d[1], (n2d, 2))
    s3 = log_uniform_int(r, side3d[0], side3d[1], (n3d, 3))
    return [tuple(int(v) for v in s) for s in s2] + [tuple(int(v) for v in s) for s in s3]


def mlp_init(F, seed, H=64):
    """He-uniform initial weights of the cost-model network (FP64 arrays;
    cast to FP32 for the GPU), zero biases except b4."""
    r = rng(seed)

    def he(fan_out, fan_in):
        lim = np.sqrt(6.0 / fan_in)
        return r.uniform(-lim, lim, size=(fan_out, fan_in))

    return {"W1": he(H, F), "b1": np.zeros(H), "W2": he(H, H), "b2": np.zeros(H),
            "W3": he(H, H), "b3": np.zeros(H), "w4": he(1, H)[0] * 0.5, "b4": np.zeros(1)}


def pred_chain_inputs(na, nb, nc, T, seed, skipped=0):
    """Inputs of the filtering example's statement chain: a (na), b (nb), c
    (nc) and xs (T) uniform[0,1); idx (T x 3 int32) with i and k 2T distinct
    indices drawn without replacement from [0, min(na, nb)) (so no element is
    touched by two iterations) and j uniform over [0, nc).  The first
    `skipped` iterations get an out-of-range index (i, j or k in turn)."""
    r = rng(seed)
    nab = min(na, nb)
    assert 2 * T <= nab
    ik = r.permutation(nab)[:2 * T]
    idx = np.empty((T, 3), dtype=np.int32)
    idx[:, 0] = ik[:T]
    idx[:, 1] = r.integers(0, nc, size=T)
    idx[:, 2] = ik[T:]
    for t in range(min(skipped, T)):
        col = t % 3
        idx[t, col] = (nab if col != 1 else nc) + t if t % 2 == 0 else -1 - t
    return r.random(na), r.random(nb), r.random(nc), idx, r.random(T)
