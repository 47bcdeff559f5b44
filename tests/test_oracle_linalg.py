"""Pins of the sum, contraction and SpMV oracles: closed forms, exactly
rounded sums (math.fsum), integer-valued cases where every order of
summation gives the exact result (checked against numpy's integer matmul),
identity and permutation matrices, and dense brute force on small sizes."""
import math

import numpy as np
import pytest

import oracle
from paper_2110_14340_amd import inputs

U = 2.0 ** -53


# ------------------------------------------------------------------ sum
def test_sum_integer_closed_form():
    n = 1 << 20
    x = (np.arange(n) % 1024).astype(np.float64)
    # sum over 1024 full periods of 0..1023
    assert oracle.sum_(x) == (n // 1024) * (1023 * 1024 // 2)


def test_sum_of_squares_integer_closed_form():
    n = 3000
    x = np.arange(n, dtype=np.float64)
    assert oracle.sum_(x, squares=True) == (n - 1) * n * (2 * n - 1) // 6


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_sum_within_two_ulps_of_exactly_rounded(seed):
    x = inputs.uniform(200_001, seed=seed, lo=-1.0, hi=1.0)
    ref = math.fsum(x.tolist())
    s = oracle.sum_(x)
    # Neumaier: |s - S| <= 2u|S| + O(n u^2) sum|x|
    assert abs(s - ref) <= 2 * U * abs(ref) + 4 * x.size * U * U * np.abs(x).sum()


def test_sum_squares_against_fsum_of_rounded_squares():
    x = inputs.uniform(100_003, seed=5)
    sq = (x * x).tolist()
    ref = math.fsum(sq)
    assert abs(oracle.sum_(x, squares=True) - ref) <= 3 * U * ref


@pytest.mark.parametrize("K", [1, 2, 3, 4, 7, 8])
def test_sum_partitioned_within_tolerance(K):
    x = inputs.uniform(123_457, seed=9)
    ref = math.fsum(x.tolist())
    assert abs(oracle.sum_partitioned(x, K) - ref) <= 1e-13 * abs(ref)


def test_sum_empty_is_zero():
    assert oracle.sum_(np.zeros(0)) == 0.0


# ------------------------------------------------------------------ GEMM
@pytest.mark.parametrize("shape", [(64, 48, 80), (1, 7, 3), (33, 17, 65)])
def test_gemm_integer_exact_against_integer_matmul(shape):
    M, N, L = shape
    A, B = inputs.gemm_inputs(M, N, L, seed=3, integer=True)
    ref = A.astype(np.int64) @ B.astype(np.int64)
    assert np.array_equal(oracle.gemm(A, B), ref.astype(np.float64))


def test_gemm_identity_left_gives_B():
    A = np.eye(37)
    _, B = inputs.gemm_inputs(37, 29, 37, seed=4)
    assert np.array_equal(oracle.gemm(A, B), B)


def test_gemm_random_brute_force_fsum():
    M, N, L = 9, 11, 13
    A, B = inputs.gemm_inputs(M, N, L, seed=5)
    C = oracle.gemm(A, B)
    for i in range(M):
        for j in range(N):
            terms = [A[i, k] * B[k, j] for k in range(L)]
            ref = math.fsum(terms)
            # sequential summation: |err| <= (L-1) u sum|terms| (+ product rounding)
            assert abs(C[i, j] - ref) <= (L + 1) * U * math.fsum(abs(t) for t in terms)


def test_gemm_rows_matches_full():
    A, B = inputs.gemm_inputs(20, 12, 15, seed=6)
    full = oracle.gemm(A, B)
    assert np.array_equal(oracle.gemm_rows(A, B, 5, 13), full[5:13])


# ------------------------------------------------------------------ SpMV
def test_spmv_identity_returns_x():
    n = 100
    rp = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    val = np.ones(n)
    x = inputs.uniform(n, seed=1, lo=-1, hi=1)
    assert np.array_equal(oracle.spmv_csr(rp, col, val, x), x)


def test_spmv_permutation():
    n = 57
    perm = np.random.default_rng(2).permutation(n).astype(np.int32)
    rp = np.arange(n + 1, dtype=np.int32)
    x = inputs.uniform(n, seed=3)
    y = oracle.spmv_csr(rp, perm, np.ones(n), x)
    assert np.array_equal(y, x[perm])


def test_spmv_integer_dense_brute_force():
    n = 64
    rp, col, val, _ = inputs.csr_matrix(n, n, 16, seed=4, integer_values=True)
    x = inputs.int_valued(n, seed=5, lo=-10, hi=10)
    dense = np.zeros((n, n), dtype=np.int64)
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            dense[i, col[k]] += int(val[k])
    ref = dense @ x.astype(np.int64)
    assert np.array_equal(oracle.spmv_csr(rp, col, val, x), ref.astype(np.float64))


def test_spmv_random_within_bound_and_empty_rows():
    n = 200
    rp, col, val, x = inputs.csr_matrix(n, 300, 5, seed=6)
    # make rows 10..19 empty
    counts = np.diff(rp).astype(np.int64)
    keep = np.ones(col.size, dtype=bool)
    for i in range(10, 20):
        keep[rp[i]:rp[i + 1]] = False
    counts[10:20] = 0
    rp2 = np.zeros(n + 1, dtype=np.int32)
    rp2[1:] = np.cumsum(counts)
    col2, val2 = col[keep], val[keep]
    y = oracle.spmv_csr(rp2, col2, val2, x)
    assert np.all(y[10:20] == 0.0)
    for i in range(n):
        terms = [val2[k] * x[col2[k]] for k in range(rp2[i], rp2[i + 1])]
        ref = math.fsum(terms)
        assert abs(y[i] - ref) <= (len(terms) + 1) * U * math.fsum(abs(t) for t in terms)


def test_csr_generator_structure():
    rp, col, val, x = inputs.csr_matrix(1000, 5000, 16, seed=7)
    assert rp[0] == 0 and rp[-1] == col.size == val.size
    for i in range(1000):
        c = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0) and 1 <= c.size <= 16
    assert x.size == 5000 and np.all((x >= -1) & (x < 1))


# ------------------------------------------------------------------ scatter
def test_scatter_permutation_against_numpy_fancy_indexing():
    n = 1000
    x = inputs.uniform(n, seed=11, lo=-2, hi=2)
    perm = np.random.default_rng(12).permutation(n).astype(np.int32)
    out = np.full(n, -7.0)
    ref = out.copy()
    ref[perm] = x * x
    assert np.array_equal(oracle.scatter_sq(x, perm, out), ref)


def test_scatter_partial_range_and_out_of_range_indices_skipped():
    x = np.arange(10, dtype=np.float64)
    idx = np.array([3, -1, 11, 0, 9, 4, 5, 6, 7, 8], dtype=np.int32)
    out = np.zeros(10)
    got = oracle.scatter_sq(x, idx, out, rows=(0, 5))
    expect = np.zeros(10)
    expect[3], expect[0], expect[9] = 0.0, 9.0, 16.0
    assert np.array_equal(got, expect)


@pytest.mark.parametrize("K", [1, 2, 3, 5, 8])
def test_scatter_filtered_partitions_equal_plain(K):
    n = 257
    x = inputs.uniform(n, seed=13)
    idx = np.random.default_rng(14).permutation(n).astype(np.int32)
    out = inputs.uniform(n, seed=15)
    assert np.array_equal(oracle.scatter_sq_partitioned(x, idx, out, K), oracle.scatter_sq(x, idx, out))


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_gemm_multithreaded_bit_identical_and_integer_exact(threads):
    A, B = inputs.gemm_inputs(70, 45, 33, seed=7)
    assert np.array_equal(oracle.gemm_mt(A, B, threads), oracle.gemm(A, B))
    Ai, Bi = inputs.gemm_inputs(41, 29, 57, seed=8, integer=True)
    ref = Ai.astype(np.int64) @ Bi.astype(np.int64)
    assert np.array_equal(oracle.gemm_mt(Ai, Bi, threads), ref.astype(np.float64))


@pytest.mark.parametrize("threads", [1, 5])
def test_spmv_multithreaded_bit_identical(threads):
    rp, col, val, x = inputs.csr_matrix(9000, 9000, 16, seed=12)
    assert np.array_equal(oracle.spmv_csr_mt(rp, col, val, x, threads), oracle.spmv_csr(rp, col, val, x))
