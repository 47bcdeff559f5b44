"""GPU parity of the reduction, contraction and SpMV loop bodies against the
CPU oracle, at the stated tolerances (sum: 1e-13 relative to the sum of
magnitudes; GEMM: 1e-12 * ||A||_F ||B||_F in Frobenius norm, exact for
integer-valued inputs; SpMV: 1e-13 relative to each row's sum of
magnitudes)."""
import math

import numpy as np
import pytest

import oracle
from paper_2110_14340_amd import inputs, jacc
from gpu_util import context, say

pytestmark = pytest.mark.gpu


# ------------------------------------------------------------------ sum
@pytest.mark.parametrize("n,K", [(1, 1), (1000, 1), (1000, 3), (123_457, 4), (2_000_003, 8), (2_000_003, 16),
                                 (123_457, 20)])
def test_sum_small(n, K):
    say(f"sum n={n} K={K}")
    x = inputs.uniform(n, seed=n, lo=-1.0, hi=1.0)
    ref = oracle.sum_(x)
    mag = float(np.abs(x).sum())
    with context(K) as c:
        c.enter(x)
        s = c.sum(x)
        sq = c.sum(x, squares=True)
    assert abs(s - ref) <= 1e-13 * mag
    assert abs(sq - oracle.sum_(x, squares=True)) <= 1e-13 * float((x * x).sum())


def test_sum_512_cubed_k1_k4():
    say("sum 512^3 K=1,4")
    x = inputs.uniform((512, 512, 512), seed=7)
    ref = oracle.sum_(x)
    for K in (1, 4):
        with context(K) as c:
            c.enter(x)
            s = c.sum(x)
        assert abs(s - ref) <= 1e-13 * ref


@pytest.mark.parametrize("n,K", [(2_000_003, 3), (1 << 24, 8), (5_000_000, 16)])
def test_sum_packed_partitions_equal_a_launch_per_partition(n, K):
    """One launch over all partitions (the default) and a launch per
    partition on its own stream add in the same order: the sums are
    bit-identical, and within the oracle's bound."""
    say(f"sum packed vs per-partition n={n} K={K}")
    x = inputs.uniform(n, seed=n + K, lo=-1.0, hi=1.0)
    got = []
    for flags in (0, jacc.INIT_NO_PACK):
        with context(K, flags) as c:
            c.enter(x)
            got.append((c.sum(x), c.sum(x, squares=True)))
    assert got[0] == got[1]
    assert abs(got[0][0] - oracle.sum_(x)) <= 1e-13 * float(np.abs(x).sum())


def test_sum_integer_exact_and_deferred_slots():
    say("sum integer exact")
    x = (np.arange(1 << 20) % 1024).astype(np.float64)
    with context(2) as c:
        c.enter(x)
        c.sum(x, slot=5, sync=False)
        c.sum(x, squares=True, slot=6, sync=False)
        vals = c.reductions(5, 2)
    assert vals[0] == (1 << 10) * (1023 * 1024 // 2)
    assert vals[1] == (1 << 10) * sum(i * i for i in range(1024))


# ------------------------------------------------------------------ GEMM
def _gemm_dev(A, B, K, slab=0, threads=0, whole=True):
    C = np.zeros((A.shape[0], B.shape[1]))
    with context(K) as c:
        c.enter(A)
        c.enter(B, whole=whole)
        c.enter(C, clause=jacc.CREATE)
        c.gemm(A, B, C, cfg=jacc.config(tile=slab, bx=threads) if (slab or threads) else None)
        c.exit(C, jacc.COPYOUT)
    return C


@pytest.mark.parametrize("M,N,L,K", [(64, 64, 16, 1), (200, 150, 130, 1), (200, 150, 130, 3),
                                     (129, 257, 33, 2), (1, 5, 7, 1), (300, 17, 1000, 4)])
def test_gemm_small_frobenius_and_integer_exact(M, N, L, K):
    say(f"gemm {M}x{N}x{L} K={K}")
    A, B = inputs.gemm_inputs(M, N, L, seed=3)
    ref = oracle.gemm(A, B)
    Ai, Bi = inputs.gemm_inputs(M, N, L, seed=4, integer=True)
    for slab, threads in ((16, 256), (32, 256), (16, 512), (32, 512)):
        C = _gemm_dev(A, B, K, slab, threads)
        assert np.linalg.norm(C - ref) <= 1e-12 * np.linalg.norm(A) * np.linalg.norm(B)
        assert np.array_equal(_gemm_dev(Ai, Bi, K, slab, threads), oracle.gemm(Ai, Bi))


def test_gemm_4096_full_frobenius_and_integer_exact():
    """C = A*B at 4096^3 against the oracle over every element of C:
    Frobenius-norm bound for uniform inputs, exact equality for
    integer-valued inputs (whose products and sums are all exact)."""
    n = 4096
    A, B = inputs.gemm_inputs(n, n, n, seed=3)
    say(f"oracle: gemm 4096^3 on {oracle.threads()} host threads")
    ref = oracle.gemm_mt(A, B)
    bound = 1e-12 * np.linalg.norm(A) * np.linalg.norm(B)
    C1 = _gemm_dev(A, B, 1)
    say(f"  K=1 Frobenius error {np.linalg.norm(C1 - ref):.3e} (bound {bound:.3e})")
    assert np.linalg.norm(C1 - ref) <= bound
    C4 = _gemm_dev(A, B, 4)
    assert np.array_equal(C1, C4)  # no split-k: partitioning never changes an element's sum order
    assert np.linalg.norm(C4 - ref) <= bound
    assert np.array_equal(C1, _gemm_dev(A, B, 1, 32))  # nor does the k-slab depth
    assert np.array_equal(C1, _gemm_dev(A, B, 1, 16, 256))  # nor the workgroup size
    del C1, C4, ref
    Ai, Bi = inputs.gemm_inputs(n, n, n, seed=5, integer=True)
    say("  integer-valued inputs")
    ref_i = oracle.gemm_mt(Ai, Bi)
    assert np.array_equal(_gemm_dev(Ai, Bi, 4), ref_i)


# ------------------------------------------------------------------ SpMV
def _spmv_dev(rp, col, val, x, K, cfg=None, whole=True):
    y = np.zeros(rp.size - 1)
    with context(K) as c:
        c.enter(rp, halo=(1, 1))
        c.enter(col, whole=whole)
        c.enter(val, whole=whole)
        c.enter(x, whole=whole)
        c.enter(y, clause=jacc.CREATE)
        c.spmv(rp, col, val, x, y, cfg=cfg)
        c.exit(y, jacc.COPYOUT)
    return y


def _row_bound(rp, col, val, x):
    absx = np.abs(val * x[col])
    cs = np.concatenate([[0.0], np.cumsum(absx)])
    return cs[rp[1:]] - cs[rp[:-1]]


@pytest.mark.parametrize("n,K", [(1, 1), (100, 1), (1000, 3), (5000, 4), (5000, 16), (5000, 20)])
def test_spmv_small(n, K):
    say(f"spmv n={n} K={K}")
    rp, col, val, x = inputs.csr_matrix(n, n, 16, seed=8)
    ref = oracle.spmv_csr(rp, col, val, x)
    y = _spmv_dev(rp, col, val, x, K)
    assert np.all(np.abs(y - ref) <= 1e-13 * _row_bound(rp, col, val, x))
    rpi, coli, vali, _ = inputs.csr_matrix(n, n, 16, seed=9, integer_values=True)
    xi = inputs.int_valued(n, seed=10, lo=-10, hi=10)
    ref_i = oracle.spmv_csr(rpi, coli, vali, xi)
    assert np.array_equal(_spmv_dev(rpi, coli, vali, xi, K), ref_i)
    # lanes per row; order 2: non-temporal col/val loads; order 4: column bands (by per XCD)
    for lanes, order, by, rows in ((4, 1, 0, 0), (16, 1, 0, 0), (8, 2, 0, 0), (4, 2, 0, 0), (16, 4, 1, 0), (8, 4, 2, 0),
                                   (4, 4, 8, 0), (1, 4, 1, 0), (2, 4, 2, 0), (1, 4, 1, 2), (1, 4, 2, 4)):
        cfg = jacc.config(tile=lanes, order=order, by=by, rows=rows)
        assert np.all(np.abs(_spmv_dev(rp, col, val, x, K, cfg) - ref) <= 1e-13 * _row_bound(rp, col, val, x))
        assert np.array_equal(_spmv_dev(rpi, coli, vali, xi, K, cfg), ref_i)


@pytest.mark.parametrize("n,K,draws", [(3000, 1, 40), (20000, 3, 70)])
def test_spmv_rows_longer_than_the_lane_group(n, K, draws):
    """Rows of up to `draws` entries: every lane of a row group adds several
    terms in increasing k."""
    say(f"spmv n={n} K={K} up to {draws} entries per row")
    rp, col, val, x = inputs.csr_matrix(n, n, draws, seed=11)
    ref = oracle.spmv_csr(rp, col, val, x)
    bound = 1e-13 * _row_bound(rp, col, val, x)
    for lanes, order, by, rows in ((4, 2, 0, 0), (8, 1, 0, 0), (16, 2, 0, 0), (16, 4, 1, 0), (8, 4, 4, 0), (1, 4, 1, 0),
                                   (2, 4, 2, 0), (1, 4, 1, 4), (1, 4, 2, 2)):
        y = _spmv_dev(rp, col, val, x, K, jacc.config(tile=lanes, order=order, by=by, rows=rows))
        assert np.all(np.abs(y - ref) <= bound)


def test_banded_spmv_rebuilds_after_the_matrix_changes():
    """The banded copy is built at the first product and reused; new values
    (update to the device) and a new row_ptr/col (re-entered arrays) give
    products of the new matrix."""
    say("banded spmv reuse and rebuild")
    n = 30000
    rp, col, val, x = inputs.csr_matrix(n, n, 16, seed=12)
    cfg = jacc.config(tile=16, order=4, by=2)
    y = np.zeros(n)
    with context(3) as c:
        for arr in (col, val, x):
            c.enter(arr, whole=True)
        c.enter(rp, halo=(1, 1))
        c.enter(y, clause=jacc.CREATE)
        for step in range(3):
            if step == 2:
                val[:] = -2.0 * val
                c.update(val, jacc.UPDATE_DEVICE)
            c.spmv(rp, col, val, x, y, cfg=cfg)
            c.update(y, jacc.UPDATE_HOST)
            ref = oracle.spmv_csr(rp, col, val, x)
            assert np.all(np.abs(y - ref) <= 1e-13 * _row_bound(rp, col, val, x)), step
        c.exit(y)


def test_spmv_2_22_rows_k1_k4_every_row():
    say("spmv 2^22 rows K=1,4, every row against the oracle")
    n = 1 << 22
    rp, col, val, x = inputs.csr_matrix(n, n, 16, seed=4)
    ref = oracle.spmv_csr_mt(rp, col, val, x)
    bound = 1e-13 * _row_bound(rp, col, val, x)
    y1 = _spmv_dev(rp, col, val, x, 1)
    y4 = _spmv_dev(rp, col, val, x, 4)
    assert np.array_equal(y1, y4)  # each row's sum order is fixed by the lanes-per-row layout
    bad = np.flatnonzero(np.abs(y4 - ref) > bound)
    assert bad.size == 0, f"{bad.size} rows outside the bound, first {bad[:5]}"
    for by in (1, 2):
        say(f"  column-banded form, {8 * by} bands, K=1 and 4")
        cfg = jacc.config(tile=16, order=4, by=by)
        b1 = _spmv_dev(rp, col, val, x, 1, cfg)
        assert np.array_equal(_spmv_dev(rp, col, val, x, 4, cfg), b1)  # band boundaries do not depend on K
        bad = np.flatnonzero(np.abs(b1 - ref) > bound)
        assert bad.size == 0, f"{bad.size} banded rows outside the bound, first {bad[:5]}"
    say("  col, val and x as one shared read-only copy, K=4 (default and banded forms)")
    assert np.array_equal(_spmv_dev(rp, col, val, x, 4, whole=jacc.SHARED), y4)
    assert np.array_equal(_spmv_dev(rp, col, val, x, 4, cfg, whole=jacc.SHARED), b1)  # b1: the last banded form


# ------------------------------------------------------------------ predicate-filtered scatter
@pytest.mark.parametrize("n,K", [(1000, 1), (1000, 3), (100_003, 4), (1 << 22, 8)])
def test_filtered_scatter_matches_oracle(n, K):
    say(f"scatter n={n} K={K}")
    x = inputs.uniform(n, seed=n % 97, lo=-2, hi=2)
    idx = np.random.default_rng(n % 89).permutation(n).astype(np.int32)
    out = inputs.uniform(n, seed=5)
    ref = oracle.scatter_sq(x, idx, out)
    o = out.copy()
    with context(K) as c:
        c.enter(x, whole=True)
        c.enter(idx, whole=True)
        c.enter(o)
        c.scatter_sq(x, idx, o)
        c.exit(o)
    assert np.array_equal(o, ref)


@pytest.mark.parametrize("M,N,L,K", [(200, 150, 130, 3), (300, 17, 1000, 4)])
def test_gemm_shared_b_equals_replicated(M, N, L, K):
    """B as one shared read-only copy gives the same bits as a replica per
    partition."""
    say(f"gemm shared B {M}x{N}x{L} K={K}")
    A, B = inputs.gemm_inputs(M, N, L, seed=M + K)
    assert np.array_equal(_gemm_dev(A, B, K, whole=jacc.SHARED), _gemm_dev(A, B, K))
