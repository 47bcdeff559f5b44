"""Pins of the stencil oracles against facts fixed by the mathematics:
exact fixed points, the discrete maximum principle, symmetry, exact-rational
brute force on tiny grids, and equality of the partitioned and windowed runs
with the plain run.  None of these retypes the oracle's own formula."""
import numpy as np
import pytest

import oracle
from oracle import exact
from paper_2110_14340_amd import inputs

U = 2.0 ** -53  # unit roundoff of binary64


# ------------------------------------------------------------------ Jacobi
@pytest.mark.parametrize("c", [0.1, 1.0e300, -3.7, 0.0, 2.0 ** -1060])
def test_jacobi_constant_field_is_fixed_point(c):
    g = np.full((13, 17), c)
    out = oracle.jacobi2d(g, 9)
    assert np.array_equal(out, g)


def test_jacobi_integer_linear_field_is_fixed_point():
    i, j = np.meshgrid(np.arange(40), np.arange(33), indexing="ij")
    g = (12345.0 * i - 777.0 * j + 2.0 ** 40).astype(np.float64)
    assert np.abs(g).max() < 2.0 ** 50
    out = oracle.jacobi2d(g, 11)
    assert np.array_equal(out, g)


def test_jacobi_maximum_principle_and_boundary_held():
    g = inputs.jacobi_grid(31, 27, seed=3)
    g[0, :] = 0.5
    out = oracle.jacobi2d(g, 25)
    assert out.min() >= g.min() and out.max() <= g.max()
    assert np.array_equal(out[0], g[0]) and np.array_equal(out[-1], g[-1])
    assert np.array_equal(out[:, 0], g[:, 0]) and np.array_equal(out[:, -1], g[:, -1])


def test_jacobi_transpose_and_reflection_bit_exact():
    g = inputs.jacobi_grid(29, 23, seed=4)
    out = oracle.jacobi2d(g, 13)
    assert np.array_equal(oracle.jacobi2d(np.ascontiguousarray(g.T), 13), out.T)
    assert np.array_equal(oracle.jacobi2d(np.ascontiguousarray(g[::-1]), 13), out[::-1])
    assert np.array_equal(oracle.jacobi2d(np.ascontiguousarray(g[:, ::-1]), 13), out[:, ::-1])


@pytest.mark.parametrize("steps", [1, 2, 7, 20])
def test_jacobi_brute_force_8x8_exact(steps):
    # integer data < 2^10: every FP64 intermediate is a dyadic rational with
    # fewer than 53 significant bits for T <= 20, so FP64 equals exact.
    g = inputs.int_valued((8, 8), seed=10 + steps, lo=0, hi=1023)
    ref = exact.jacobi2d(g.tolist(), steps)
    out = oracle.jacobi2d(g, steps)
    for i in range(8):
        for j in range(8):
            assert out[i, j] == ref[i][j], (i, j)


def test_jacobi_brute_force_uniform_within_rounding_bound():
    g = inputs.jacobi_grid(8, 8, seed=5)
    T = 5
    ref = exact.jacobi2d(g.tolist(), T)
    out = oracle.jacobi2d(g, T)
    # each step rounds three sums and one product of a convex average; errors
    # do not amplify through a convex average: |err| <= 4*T*u*max|u0|
    bound = 4 * T * U * np.abs(g).max()
    for i in range(8):
        for j in range(8):
            assert abs(out[i, j] - float(ref[i][j])) <= bound


def test_jacobi_single_sweep_respects_bounds():
    g = inputs.jacobi_grid(12, 10, seed=6)
    out = g.copy()
    oracle.jacobi2d_sweep(g, out, ((3, 7), (2, 5)))
    full = g.copy()
    oracle.jacobi2d_sweep(g, full)
    mask = np.zeros_like(g, dtype=bool)
    mask[3:7, 2:5] = True
    assert np.array_equal(out[mask], full[mask])
    assert np.array_equal(out[~mask], g[~mask])


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5, 7, 8])
def test_jacobi_partitioned_equals_plain(K):
    g = inputs.jacobi_grid(37, 29, seed=7)
    assert np.array_equal(oracle.jacobi2d_partitioned(g, 9, K), oracle.jacobi2d(g, 9))


def test_jacobi_partitioned_one_row_per_partition():
    g = inputs.jacobi_grid(8, 9, seed=8)
    assert np.array_equal(oracle.jacobi2d_partitioned(g, 5, 8), oracle.jacobi2d(g, 5))


@pytest.mark.parametrize("win", [((0, 5), (0, 4)), ((10, 21), (7, 30)), ((38, 40), (35, 41)), ((0, 40), (0, 41))])
def test_jacobi_window_equals_full_run(win):
    g = inputs.jacobi_grid(40, 41, seed=9)
    T = 6
    full = oracle.jacobi2d(g, T)
    (r0, r1), (c0, c1) = win
    assert np.array_equal(oracle.jacobi2d_window(g, T, (r0, r1), (c0, c1)), full[r0:r1, c0:c1])


# ------------------------------------------------------------------ Heat
@pytest.mark.parametrize("c", [0.3, 7.0, -1.0e200])
def test_heat_constant_field_is_fixed_point(c):
    g = np.full((9, 8, 10), c)
    out, res = oracle.heat3d(g, 4, 0.1)
    assert np.array_equal(out, g)
    assert np.all(res == 0.0)


def test_heat_integer_linear_field_is_fixed_point():
    z, y, x = np.meshgrid(np.arange(11), np.arange(9), np.arange(12), indexing="ij")
    g = (1000.0 * z - 37.0 * y + 5.0 * x + 2.0 ** 30).astype(np.float64)
    out, res = oracle.heat3d(g, 5, 0.1)
    assert np.array_equal(out, g)
    assert np.all(res == 0.0)


@pytest.mark.parametrize("steps", [1, 3, 8])
def test_heat_brute_force_8cubed_exact_dyadic_alpha(steps):
    g = inputs.int_valued((8, 8, 8), seed=20 + steps, lo=0, hi=1023)
    ref, ref_res = exact.heat3d(g.tolist(), steps, 0.125)
    out, res = oracle.heat3d(g, steps, 0.125)
    for z in range(8):
        for y in range(8):
            for x in range(8):
                assert out[z, y, x] == ref[z][y][x]
    # residual terms (u'-u)^2 at step index t carry denominators 2^(6(t+1))
    # on top of magnitudes below 2^28, so they are exact up to t = 3; after
    # that the compensated sum is within 6u of the exact value.
    for t in range(steps):
        if t <= 3:
            assert res[t] == ref_res[t]
        else:
            assert abs(res[t] - float(ref_res[t])) <= 6 * U * float(ref_res[t])


def test_heat_brute_force_alpha_point_one_within_bound():
    g = inputs.heat_field(8, 8, 8, seed=2)
    T = 4
    ref, _ = exact.heat3d(g.tolist(), T, 0.1)
    out, _ = oracle.heat3d(g, T, 0.1)
    # per step: the pair sums, the subtraction of 6u, the product by alpha and
    # the final addition each round once (|values| <= 6); the scheme is a
    # convex average (1 - 6*alpha >= 0), so errors do not amplify.
    bound = 8 * T * U * 6.0
    err = max(abs(out[z, y, x] - float(ref[z][y][x])) for z in range(8) for y in range(8) for x in range(8))
    assert err <= bound


def test_heat_residual_matches_exact_sum_of_stored_differences():
    g = inputs.heat_field(7, 9, 8, seed=11)
    nxt = g.copy()
    r = oracle.heat3d_sweep(g, nxt, 0.1)
    ex = exact.residual_of_stored(g, nxt)
    # terms are fl(fl(d)^2) (relative error <= 3u each); compensated sum
    # adds at most 2u relative for non-negative terms
    assert abs(r - float(ex)) <= 6 * U * float(ex)


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5, 7])
def test_heat_partitioned_equals_plain(K):
    g = inputs.heat_field(19, 7, 9, seed=12)
    ref, ref_res = oracle.heat3d(g, 5, 0.1)
    out, res = oracle.heat3d_partitioned(g, 5, 0.1, K)
    assert np.array_equal(out, ref)
    assert np.all(np.abs(res - ref_res) <= 1e-13 * ref_res)


@pytest.mark.parametrize("win", [((0, 3), (0, 4), (0, 5)), ((4, 9), (2, 6), (3, 10)), ((0, 12), (0, 10), (0, 11))])
def test_heat_window_equals_full_run(win):
    g = inputs.heat_field(12, 10, 11, seed=13)
    T = 3
    full, _ = oracle.heat3d(g, T, 0.1)
    zs, ys, xs = win
    assert np.array_equal(oracle.heat3d_window(g, T, 0.1, zs, ys, xs),
                          full[zs[0]:zs[1], ys[0]:ys[1], xs[0]:xs[1]])


# ------------------------------------------------------------------ multi-threaded forms
@pytest.mark.parametrize("threads", [1, 3, 8])
def test_jacobi_multithreaded_bit_identical_to_sequential(threads):
    u0 = inputs.jacobi_grid(203, 131, seed=14)
    assert np.array_equal(oracle.jacobi2d_mt(u0, 9, threads), oracle.jacobi2d(u0, 9))


@pytest.mark.parametrize("threads", [1, 4, 7])
def test_heat_multithreaded_field_identical_and_residual_exact_within_bound(threads):
    g = inputs.heat_field(11, 9, 13, seed=15)
    ref, _ = oracle.heat3d(g, 3, 0.1)
    out, res = oracle.heat3d_mt(g, 3, 0.1, threads)
    assert np.array_equal(out, ref)
    # the residual of the last step against the exact rational sum of the
    # squared differences of the stored fields (per-plane compensated sums,
    # then compensated over planes: terms within 3u, sums within 2u each)
    prev, _ = oracle.heat3d(g, 2, 0.1)
    ex = exact.residual_of_stored(prev, out)
    assert abs(res[-1] - float(ex)) <= 8 * U * float(ex)


def test_oracle_threads_reports_the_request():
    assert oracle.threads(3) == 3
    assert oracle.threads(0) >= 1
