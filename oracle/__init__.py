"""CPU oracle of the partitioned loop-nest runtime — TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library or its Python
binding, and neither imports the other.

Paper: JACC, an OpenACC runtime framework with kernel-level and multi-GPU
parallelization (Matsumura, Garcia De Gonzalo, Pena; HiPC 2021, arXiv
2110.14340).

Contents
--------
* C library (``oracle.c``, loaded here through ctypes): plain sequential FP64
  definitions of the loop nests — Jacobi-2D 5-point sweep and T-step run,
  heat-3D 7-point step with its residual, sum reduction, dense contraction,
  CSR SpMV — and K-way partitioned runs of the stencils that follow the
  paper's own scheme (equal division of the parallel dimension, writes
  filtered by owner range, eager refresh of every replica after each kernel;
  Sec. "Predicate-Based Filtering", Sec. "Division of Multidimensional
  Arrays").
* ``exact``: exact-rational brute force on tiny grids (fractions.Fraction).
* ``plan``: brute-force set model of owner blocks, slabs, iteration
  sub-ranges, access ranges and the copies a lazy coherence scheme needs.
* ``mlp``: FP64 numpy reference of the cost-model network, loss, gradients
  and Adam step.
* ``tuner``: the autotuner's selection rule and regret definition.

Parity status per function is listed in each module's header; every
function here is pinned by tests in ``tests/test_oracle_*.py``.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64


def lib():
    """Load liboracle.so, building it first if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.oracle_jacobi2d_sweep.argtypes = [_f64p, _f64p, _i64, _i64, _i64, _i64, _i64, _i64]
        L.oracle_jacobi2d_sweep.restype = None
        L.oracle_jacobi2d.argtypes = [_f64p, _f64p, _i64, _i64, _i64]
        L.oracle_jacobi2d.restype = ctypes.c_int
        L.oracle_jacobi2d_window.argtypes = [_f64p, _i64, _i64, _i64, _i64, _i64, _i64, _i64, _f64p]
        L.oracle_jacobi2d_window.restype = ctypes.c_int
        L.oracle_jacobi2d_partitioned.argtypes = [_f64p, _i64, _i64, _i64, ctypes.c_int]
        L.oracle_jacobi2d_partitioned.restype = ctypes.c_int
        L.oracle_heat3d_sweep.argtypes = [_f64p, _f64p, _i64, _i64, _i64, _i64, _i64, _i64, _i64,
                                          _i64, _i64, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
        L.oracle_heat3d_sweep.restype = None
        L.oracle_heat3d.argtypes = [_f64p, _f64p, _i64, _i64, _i64, _i64, ctypes.c_double, _f64p]
        L.oracle_heat3d.restype = ctypes.c_int
        L.oracle_heat3d_window.argtypes = [_f64p, _i64, _i64, _i64, _i64, ctypes.c_double, _i64, _i64,
                                           _i64, _i64, _i64, _i64, _f64p]
        L.oracle_heat3d_window.restype = ctypes.c_int
        L.oracle_heat3d_partitioned.argtypes = [_f64p, _i64, _i64, _i64, _i64, ctypes.c_double,
                                                ctypes.c_int, _f64p]
        L.oracle_heat3d_partitioned.restype = ctypes.c_int
        L.oracle_sum.argtypes = [_f64p, _i64, ctypes.c_int]
        L.oracle_sum.restype = ctypes.c_double
        L.oracle_sum_partitioned.argtypes = [_f64p, _i64, ctypes.c_int, ctypes.c_int]
        L.oracle_sum_partitioned.restype = ctypes.c_double
        L.oracle_gemm.argtypes = [_f64p, _f64p, _f64p, _i64, _i64, _i64]
        L.oracle_gemm.restype = None
        L.oracle_gemm_rows.argtypes = [_f64p, _f64p, _f64p, _i64, _i64, _i64, _i64]
        L.oracle_gemm_rows.restype = None
        L.oracle_spmv_csr.argtypes = [_i32p, _i32p, _f64p, _f64p, _f64p, _i64, _i64]
        L.oracle_spmv_csr.restype = None
        L.oracle_scatter_sq.argtypes = [_f64p, _i32p, _f64p, _i64, _i64, _i64]
        L.oracle_scatter_sq.restype = None
        L.oracle_scatter_sq_partitioned.argtypes = [_f64p, _i32p, _f64p, _i64, _i64, _i64, ctypes.c_int]
        L.oracle_scatter_sq_partitioned.restype = ctypes.c_int
        L.oracle_pred_chain.argtypes = [_f64p, _i64, _f64p, _i64, _f64p, _i64, _i32p, _f64p, _i64, _i64]
        L.oracle_pred_chain.restype = None
        L.oracle_pred_chain_partitioned.argtypes = [_f64p, _i64, _f64p, _i64, _f64p, _i64, _i32p, _f64p, _i64, _i64,
                                                    ctypes.c_int]
        L.oracle_pred_chain_partitioned.restype = ctypes.c_int
        L.oracle_threads.argtypes = [ctypes.c_int]
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_jacobi2d_mt.argtypes = [_f64p, _f64p, _i64, _i64, _i64, ctypes.c_int]
        L.oracle_jacobi2d_mt.restype = ctypes.c_int
        L.oracle_heat3d_mt.argtypes = [_f64p, _f64p, _i64, _i64, _i64, _i64, ctypes.c_double, _f64p,
                                       ctypes.c_int]
        L.oracle_heat3d_mt.restype = ctypes.c_int
        L.oracle_gemm_mt.argtypes = [_f64p, _f64p, _f64p, _i64, _i64, _i64, ctypes.c_int]
        L.oracle_gemm_mt.restype = None
        L.oracle_spmv_csr_mt.argtypes = [_i32p, _i32p, _f64p, _f64p, _f64p, _i64, _i64, ctypes.c_int]
        L.oracle_spmv_csr_mt.restype = None
        _lib = L
    return _lib


def _c(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


# --------------------------------------------------------------------------
# Jacobi-2D 5-point average
# --------------------------------------------------------------------------
def jacobi2d_sweep(u_in, u_out, bounds=None):
    """One sweep from u_in into u_out (in place on u_out) over bounds
    ((r_lo, r_hi), (c_lo, c_hi)); default the interior."""
    ny, nx = u_in.shape
    (r0, r1), (c0, c1) = bounds if bounds is not None else ((1, ny - 1), (1, nx - 1))
    assert u_in.flags.c_contiguous and u_out.flags.c_contiguous
    lib().oracle_jacobi2d_sweep(u_in, u_out, ny, nx, r0, r1, c0, c1)
    return u_out


def jacobi2d(u0, steps):
    """T ping-pong steps from u0 (boundary held); returns the final grid."""
    a = _c(u0).copy()
    b = a.copy()
    which = lib().oracle_jacobi2d(a, b, a.shape[0], a.shape[1], steps)
    return a if which == 0 else b


def jacobi2d_window(u0, steps, rows, cols):
    """Final values of a T-step run on the window rows x cols (half-open
    pairs), computed over the window's domain of dependence only."""
    u0 = _c(u0)
    (r0, r1), (c0, c1) = rows, cols
    out = np.empty((r1 - r0, c1 - c0), dtype=np.float64)
    rc = lib().oracle_jacobi2d_window(u0, u0.shape[0], u0.shape[1], steps, r0, r1, c0, c1, out)
    assert rc == 0
    return out


def jacobi2d_partitioned(u0, steps, K):
    """K-way partitioned run with private slabs and eager replica refresh."""
    g = _c(u0).copy()
    rc = lib().oracle_jacobi2d_partitioned(g, g.shape[0], g.shape[1], steps, K)
    assert rc == 0
    return g


# --------------------------------------------------------------------------
# Heat-3D 7-point explicit step + residual
# --------------------------------------------------------------------------
def heat3d_sweep(u_in, u_out, alpha, bounds=None):
    """One step from u_in into u_out over bounds (3 half-open pairs, default
    the interior); returns the compensated residual sum over the box."""
    nz, ny, nx = u_in.shape
    (z0, z1), (y0, y1), (x0, x1) = bounds if bounds is not None else ((1, nz - 1), (1, ny - 1), (1, nx - 1))
    r = ctypes.c_double(0.0)
    lib().oracle_heat3d_sweep(u_in, u_out, nz, ny, nx, z0, z1, y0, y1, x0, x1, alpha, ctypes.byref(r))
    return r.value


def heat3d(u0, steps, alpha):
    """T steps; returns (final field, residuals[T])."""
    a = _c(u0).copy()
    b = a.copy()
    res = np.zeros(max(steps, 1), dtype=np.float64)
    which = lib().oracle_heat3d(a, b, *a.shape, steps, alpha, res)
    return (a if which == 0 else b), res[:steps]


def heat3d_window(u0, steps, alpha, zs, ys, xs):
    u0 = _c(u0)
    out = np.empty((zs[1] - zs[0], ys[1] - ys[0], xs[1] - xs[0]), dtype=np.float64)
    rc = lib().oracle_heat3d_window(u0, *u0.shape, steps, alpha, zs[0], zs[1], ys[0], ys[1],
                                    xs[0], xs[1], out)
    assert rc == 0
    return out


def heat3d_partitioned(u0, steps, alpha, K):
    """K-way partitioned run over z-plane slabs; returns (field, residuals)."""
    g = _c(u0).copy()
    res = np.zeros(max(steps, 1), dtype=np.float64)
    rc = lib().oracle_heat3d_partitioned(g, *g.shape, steps, alpha, K, res)
    assert rc == 0
    return g, res[:steps]


# --------------------------------------------------------------------------
# Sum, contraction, SpMV
# --------------------------------------------------------------------------
def sum_(x, squares=False):
    x = _c(x).reshape(-1)
    return lib().oracle_sum(x, x.size, int(bool(squares)))


def sum_partitioned(x, K, squares=False):
    x = _c(x).reshape(-1)
    return lib().oracle_sum_partitioned(x, x.size, K, int(bool(squares)))


def gemm(A, B):
    A = _c(A)
    B = _c(B)
    M, L = A.shape
    L2, N = B.shape
    assert L == L2
    C = np.empty((M, N), dtype=np.float64)
    lib().oracle_gemm(A, B, C, M, N, L)
    return C


def gemm_rows(A, B, i0, i1):
    """Rows [i0, i1) of A*B."""
    A = _c(A)
    B = _c(B)
    C = np.empty((i1 - i0, B.shape[1]), dtype=np.float64)
    lib().oracle_gemm_rows(A, B, C, B.shape[1], A.shape[1], i0, i1)
    return C


def spmv_csr(rp, col, val, x, rows=None):
    rp = _c(rp, np.int32)
    col = _c(col, np.int32)
    val = _c(val)
    x = _c(x)
    n = rp.size - 1
    lo, hi = rows if rows is not None else (0, n)
    y = np.zeros(n, dtype=np.float64)
    lib().oracle_spmv_csr(rp, col, val, x, y, lo, hi)
    return y


# --------------------------------------------------------------------------
# Indirect write (predicate-filtered on partitions)
# --------------------------------------------------------------------------
def scatter_sq(inp, idx, out, rows=None):
    """out[idx[i]] = in[i]^2 for i in rows (default all); returns a new array."""
    inp = _c(inp)
    idx = _c(idx, np.int32)
    o = _c(out).copy()
    lo, hi = rows if rows is not None else (0, inp.size)
    lib().oracle_scatter_sq(inp, idx, o, o.size, lo, hi)
    return o


def scatter_sq_partitioned(inp, idx, out, K, rows=None):
    inp = _c(inp)
    idx = _c(idx, np.int32)
    o = _c(out).copy()
    lo, hi = rows if rows is not None else (0, inp.size)
    assert lib().oracle_scatter_sq_partitioned(inp, idx, o, o.size, lo, hi, K) == 0
    return o


# --------------------------------------------------------------------------
# Statement chain of the paper's predicate-filtering example (Sec.
# "Predicate-Based Filtering", Fig. conv-code)
# --------------------------------------------------------------------------
def pred_chain(a, b, c, idx, xs, rows=None):
    """Plain sequential chain; returns new (a, b).  `b is a` runs the aliased
    form (one array written through both names) and returns it twice."""
    idx = _c(idx, np.int32).reshape(-1, 3)
    c, xs = _c(c), _c(xs)
    lo, hi = rows if rows is not None else (0, xs.size)
    ra = _c(a).copy()
    rb = ra if b is a else _c(b).copy()
    lib().oracle_pred_chain(ra, ra.size, rb, rb.size, c, c.size, idx, xs, lo, hi)
    return ra, rb


def pred_chain_partitioned(a, b, c, idx, xs, K, rows=None):
    """The chain on K replicas with the example's guards, owner rows
    gathered; returns new (a, b)."""
    idx = _c(idx, np.int32).reshape(-1, 3)
    c, xs = _c(c), _c(xs)
    lo, hi = rows if rows is not None else (0, xs.size)
    ra, rb = _c(a).copy(), _c(b).copy()
    assert lib().oracle_pred_chain_partitioned(ra, ra.size, rb, rb.size, c, c.size, idx, xs, lo, hi, K) == 0
    return ra, rb


# --------------------------------------------------------------------------
# Multi-threaded full-grid forms (same per-element arithmetic; fields and
# products bit-identical to the sequential routines, the heat residual a
# per-plane compensated order of the same terms).  threads <= 0: the OpenMP
# default (OMP_NUM_THREADS, else every core).
# --------------------------------------------------------------------------
def threads(requested=0):
    """Threads the multi-threaded routines run with for a request."""
    return lib().oracle_threads(int(requested))


def jacobi2d_mt(u0, steps, threads=0):
    a = _c(u0).copy()
    b = a.copy()
    which = lib().oracle_jacobi2d_mt(a, b, a.shape[0], a.shape[1], steps, int(threads))
    return a if which == 0 else b


def heat3d_mt(u0, steps, alpha, threads=0):
    a = _c(u0).copy()
    b = a.copy()
    res = np.zeros(max(steps, 1), dtype=np.float64)
    which = lib().oracle_heat3d_mt(a, b, *a.shape, steps, alpha, res, int(threads))
    assert which >= 0
    return (a if which == 0 else b), res[:steps]


def gemm_mt(A, B, threads=0):
    A = _c(A)
    B = _c(B)
    M, L = A.shape
    L2, N = B.shape
    assert L == L2
    C = np.empty((M, N), dtype=np.float64)
    lib().oracle_gemm_mt(A, B, C, M, N, L, int(threads))
    return C


def spmv_csr_mt(rp, col, val, x, threads=0):
    rp = _c(rp, np.int32)
    col = _c(col, np.int32)
    val = _c(val)
    x = _c(x)
    n = rp.size - 1
    y = np.zeros(n, dtype=np.float64)
    lib().oracle_spmv_csr_mt(rp, col, val, x, y, 0, n, int(threads))
    return y
