"""GPU parity of the stencil loop bodies and of their K-partitioned runs
against the CPU oracle (bit-exact: floating-point contraction is off on
both sides and the operation order is the same)."""
import numpy as np
import pytest

import oracle
from paper_2110_14340_amd import inputs, jacc
from gpu_util import context, run_heat, run_jacobi, say

pytestmark = pytest.mark.gpu


def _cfg(bx, by, tile, vec, order=0, march=0, rows=0):
    return jacc.config(bx=bx, by=by, tile=tile, vec=vec, order=order, march=march, rows=rows)


# ------------------------------------------------------------------ Jacobi
@pytest.mark.parametrize("K", [1, 4])
def test_jacobi_512_100_steps_bit_exact(K):
    say(f"jacobi 512^2 T=100 K={K}")
    u0 = inputs.jacobi_grid(512, 512, seed=0)
    ref = oracle.jacobi2d(u0, 100)
    out = run_jacobi(u0, 100, K)
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("shape,K,cfg", [
    ((37, 29), 1, None), ((37, 29), 3, None), ((130, 67), 5, _cfg(64, 2, 3, 1)),
    ((200, 258), 7, _cfg(128, 1, 5, 2)), ((64, 1030), 2, _cfg(64, 4, 1, 2)),
    ((9, 9), 7, _cfg(64, 1, 1, 1)), ((300, 130), 4, _cfg(256, 4, 64, 2)),
    ((131, 258), 3, _cfg(128, 2, 5, 2, march=2)), ((77, 67), 1, _cfg(64, 1, 4, 1, order=2, march=2)),
    ((1030, 1026), 4, _cfg(256, 1, 32, 2, order=2, march=2)), ((5, 130), 2, _cfg(64, 1, 3, 2, march=2)),
    ((1030, 66), 16, None), ((1030, 66), 20, None), ((200, 130), 64, _cfg(64, 1, 2, 2)),
])
def test_jacobi_ragged_shapes_partitions_configs(shape, K, cfg):
    say(f"jacobi ragged {shape} K={K}")
    u0 = inputs.jacobi_grid(*shape, seed=11)
    u0[0, :] = 0.75  # a nonzero boundary row must be held, not overwritten
    T = 6
    ref = oracle.jacobi2d(u0, T)
    out = run_jacobi(u0, T, K, cfg=cfg)
    assert np.array_equal(out, ref)


def test_jacobi_constant_and_linear_fields_exact_on_device():
    say("jacobi fixed points")
    c = np.full((66, 70), 0.3)
    assert np.array_equal(run_jacobi(c, 5, 3), c)
    i, j = np.meshgrid(np.arange(66), np.arange(70), indexing="ij")
    lin = (4096.0 * i - 3.0 * j + 7.0).astype(np.float64)
    assert np.array_equal(run_jacobi(lin, 5, 2), lin)


def assert_same(out, ref):
    if not np.array_equal(out, ref):
        bad = np.argwhere(out != ref)
        raise AssertionError(f"{len(bad)} cells differ, first at {tuple(bad[0])}")


@pytest.fixture(scope="module")
def jacobi_8192():
    """Input and the oracle's full 1000-step result (multi-threaded form,
    bit-identical to the sequential oracle)."""
    u0 = inputs.jacobi_grid(8192, 8192, seed=1)
    say(f"oracle: jacobi 8192^2 T=1000 on {oracle.threads()} host threads")
    return u0, oracle.jacobi2d_mt(u0, 1000)


@pytest.mark.parametrize("K,flags", [(1, 0), (2, 0), (4, 0), (8, 0), (8, jacc.INIT_LAZY), (4, jacc.INIT_LAZY),
                                     (8, jacc.INIT_SPLIT), (8, jacc.INIT_NO_PACK), (2, jacc.INIT_NO_PACK)])
def test_jacobi_8192_1000_steps_full_oracle(jacobi_8192, K, flags):
    u0, ref = jacobi_8192
    say(f"jacobi 8192^2 T=1000 K={K} flags={flags} against the full oracle run")
    assert_same(run_jacobi(u0, 1000, K, ctx_flags=flags), ref)


@pytest.mark.parametrize("K,flags", [(4, jacc.INIT_LAZY), (4, jacc.INIT_SPLIT), (3, jacc.INIT_LAZY | jacc.INIT_SPLIT),
                                     (4, jacc.INIT_EAGER), (3, jacc.INIT_EAGER | jacc.INIT_SPLIT)])
def test_jacobi_512_100_steps_coherence_modes(K, flags):
    say(f"jacobi 512^2 T=100 K={K} flags={flags}")
    u0 = inputs.jacobi_grid(512, 512, seed=0)
    assert_same(run_jacobi(u0, 100, K, ctx_flags=flags), oracle.jacobi2d(u0, 100))


@pytest.mark.parametrize("shape,K,cfg", [
    ((37, 29), 3, None), ((130, 67), 5, _cfg(64, 2, 3, 1)), ((200, 258), 7, _cfg(128, 1, 5, 2)),
    ((9, 9), 7, _cfg(64, 1, 1, 1)), ((5, 130), 2, _cfg(64, 1, 3, 2, march=2)), ((1030, 1026), 8, None),
])
def test_jacobi_lazy_pull_ragged(shape, K, cfg):
    """Halo rows pulled by device-to-device copies before each read (the
    copy exchange) instead of written through by the producing kernel."""
    say(f"jacobi lazy {shape} K={K}")
    u0 = inputs.jacobi_grid(*shape, seed=17)
    assert_same(run_jacobi(u0, 7, K, cfg=cfg, ctx_flags=jacc.INIT_LAZY), oracle.jacobi2d(u0, 7))


# ------------------------------------------------------------------ Heat
def _rel_close(a, b, tol=1e-13):
    return np.all(np.abs(a - b) <= tol * np.abs(b))


@pytest.mark.parametrize("shape,K,cfg", [
    ((34, 29, 40), 1, None), ((34, 29, 40), 4, None), ((19, 17, 67), 3, _cfg(64, 2, 3, 1)),
    ((40, 12, 130), 2, _cfg(64, 1, 7, 2)), ((10, 70, 66), 4, _cfg(128, 4, 1, 2)),
    ((41, 13, 130), 3, _cfg(64, 2, 5, 2, march=2)), ((23, 9, 67), 1, _cfg(64, 1, 4, 1, order=2, march=2)),
    ((21, 19, 130), 2, _cfg(64, 2, 4, 2, rows=2)), ((17, 30, 66), 3, _cfg(64, 4, 7, 2, march=2, rows=4)),
    ((13, 21, 131), 1, _cfg(128, 2, 3, 1, rows=8)), ((33, 11, 258), 4, _cfg(128, 1, 16, 2, order=2, rows=8)),
    ((9, 3, 64), 2, _cfg(64, 1, 2, 2, rows=4)), ((12, 37, 70), 2, _cfg(256, 1, 5, 2, march=2, rows=2)),
    ((30, 75, 130), 2, _cfg(64, 2, 3, 2, order=3, march=2, rows=4)), ((19, 9, 66), 1, _cfg(128, 1, 4, 1, order=3)),
    ((26, 140, 258), 3, _cfg(128, 2, 8, 2, order=3, rows=4)),
    ((40, 9, 66), 16, None), ((44, 9, 66), 20, None),
])
def test_heat_small_bit_exact_and_residual(shape, K, cfg):
    say(f"heat {shape} K={K}")
    u0 = inputs.heat_field(*shape, seed=2)
    T = 5
    ref, ref_res = oracle.heat3d(u0, T, 0.1)
    out, res = run_heat(u0, T, 0.1, K, cfg=cfg)
    assert np.array_equal(out, ref)
    assert _rel_close(res, ref_res)


@pytest.fixture(scope="module")
def heat_512():
    u0 = inputs.heat_field(512, 512, 512, seed=2)
    say(f"oracle: heat 512^3 T=100 on {oracle.threads()} host threads")
    ref, ref_res = oracle.heat3d_mt(u0, 100, 0.1)
    return u0, ref, ref_res


@pytest.mark.parametrize("K,flags", [(4, 0), (1, 0), (4, jacc.INIT_LAZY), (4, jacc.INIT_NO_PACK)])
def test_heat_512_100_steps_full_oracle(heat_512, K, flags):
    """The whole 512^3 field after 100 steps equal to the oracle's, and every
    one of the 100 per-step residuals within 1e-13 relative."""
    u0, ref, ref_res = heat_512
    say(f"heat 512^3 T=100 K={K} flags={flags} against the full oracle run")
    out, res = run_heat(u0, 100, 0.1, K, ctx_flags=flags)
    assert_same(out, ref)
    assert res.shape == (100,)
    assert _rel_close(res, ref_res), f"max rel err {np.max(np.abs(res - ref_res) / ref_res):.3e}"
    assert np.all(np.diff(res) <= 0)  # the explicit scheme is a contraction


@pytest.mark.parametrize("shape,K,cfg", [
    ((34, 29, 40), 4, None), ((19, 17, 67), 3, _cfg(64, 2, 3, 1)), ((21, 19, 130), 2, _cfg(64, 2, 4, 2, rows=2)),
    ((26, 140, 258), 3, _cfg(128, 2, 8, 2, order=3, rows=4)),
])
def test_heat_lazy_pull_ragged(shape, K, cfg):
    say(f"heat lazy {shape} K={K}")
    u0 = inputs.heat_field(*shape, seed=18)
    ref, ref_res = oracle.heat3d(u0, 5, 0.1)
    out, res = run_heat(u0, 5, 0.1, K, cfg=cfg, ctx_flags=jacc.INIT_LAZY)
    assert_same(out, ref)
    assert _rel_close(res, ref_res)


# ------------------------------------------------------------------ degenerate launches
def test_empty_iteration_ranges_change_nothing():
    say("empty iteration ranges (Jacobi rows, heat planes, sum)")
    from gpu_util import context
    u = inputs.jacobi_grid(40, 66, seed=5)
    v = np.full_like(u, -3.0)
    h = inputs.heat_field(12, 10, 34, seed=6)
    g = np.full_like(h, -5.0)
    with context(4) as c:
        for arr in (u, v, h, g):
            c.enter(arr, halo=(1, 1))
        jargs = [(u, jacc.READ, -1, 1, 0), (v, jacc.WRITE, 0, 0, 0)]
        c.loop(jacc.JACOBI2D, jacc.bounds((7, 7), (1, 65)), jargs)
        c.loop(jacc.JACOBI2D, jacc.bounds((1, 39), (5, 5)), jargs)
        hargs = [(h, jacc.READ, -1, 1, 0), (g, jacc.WRITE, 0, 0, 0)]
        c.loop(jacc.HEAT3D, jacc.bounds((1, 11), (4, 4), (1, 33)), hargs, scalars=(0.1,), slot=3)
        assert c.reductions(3, 1)[0] == 0.0
        assert c.sum(u, rows=(9, 9)) == 0.0
        c.exit(v)
        c.exit(g)
    assert np.all(v == -3.0) and np.all(g == -5.0)


def test_more_partitions_than_interior_rows():
    say("jacobi 5x70 with K=5 (partitions without interior rows)")
    u0 = inputs.jacobi_grid(5, 70, seed=8)
    assert np.array_equal(run_jacobi(u0, 4, 5), oracle.jacobi2d(u0, 4))


@pytest.mark.parametrize("shape,K,steps", [((512, 512), 4, 100), ((1030, 258), 8, 7), ((40, 66), 3, 5)])
def test_jacobi_split_mode_bit_exact(shape, K, steps):
    say(f"jacobi split mode {shape} K={K} T={steps}")
    u0 = inputs.jacobi_grid(*shape, seed=12)
    assert np.array_equal(run_jacobi(u0, steps, K, ctx_flags=jacc.INIT_SPLIT), oracle.jacobi2d(u0, steps))


@pytest.mark.parametrize("shape,K", [((64, 130), 1), ((131, 258), 3), ((1030, 514), 4)])
def test_filtered_jacobi_equals_hoisted_form(shape, K):
    """Predicate-filtered form (every partition sweeps the whole box from a
    whole replica and keeps its owner rows) against the hoisted form and the
    oracle, then a hoisted sweep that reads the filtered output's halo rows."""
    say(f"filtered jacobi {shape} K={K}")
    from gpu_util import context
    u0 = inputs.jacobi_grid(*shape, seed=21)
    ny, nx = shape
    a = u0.copy()
    b = u0.copy()
    d = u0.copy()
    with context(K) as c:
        c.enter(a, whole=True)
        c.enter(b, halo=(1, 1))
        c.enter(d, halo=(1, 1))
        c.loop(jacc.JACOBI2D, jacc.bounds((1, ny - 1), (1, nx - 1)),
               [(a, jacc.READ, -1, 1, 0), (b, jacc.WRITE | jacc.FILTERED, 0, 0, 0)])
        c.jacobi2d(b, d)
        c.exit(d)
        c.exit(b)
    one = u0.copy()
    oracle.jacobi2d_sweep(u0, one)
    assert np.array_equal(b, one)
    assert np.array_equal(b, run_jacobi(u0, 1, K))
    assert np.array_equal(d, oracle.jacobi2d(u0, 2))


# ------------------------------------------------------------------ arrays split along columns
@pytest.mark.parametrize("shape,K,flags,cfg,T", [
    ((37, 29), 1, 0, None, 6), ((37, 29), 3, 0, None, 6), ((130, 67), 5, 0, _cfg(64, 2, 3, 1), 6),
    ((200, 258), 7, jacc.INIT_EAGER, None, 5), ((9, 40), 8, 0, _cfg(64, 1, 1, 1), 4),
    ((66, 1030), 8, jacc.INIT_LAZY, _cfg(128, 2, 5, 1, march=2), 5), ((1030, 130), 2, 0, _cfg(256, 1, 32, 1, order=2), 4),
    ((512, 512), 4, 0, None, 100), ((131, 258), 3, 0, _cfg(64, 1, 3, 2, march=2), 5),
    ((70, 1030), 7, jacc.INIT_LAZY, _cfg(128, 2, 5, 2), 4), ((33, 514), 5, jacc.INIT_EAGER, _cfg(256, 1, 4, 2), 4),
    ((130, 67), 5, jacc.INIT_NO_PACK, _cfg(64, 2, 3, 1), 6), ((131, 258), 3, jacc.INIT_NO_PACK, _cfg(64, 1, 3, 2), 5),
    ((512, 512), 4, jacc.INIT_NO_PACK, None, 40), ((40, 9), 4, 0, _cfg(64, 1, 2, 1), 5),
    ((40, 1030), 16, 0, None, 4), ((40, 1030), 20, 0, None, 4),
])
def test_jacobi_column_split_bit_exact(shape, K, flags, cfg, T):
    """Arrays split into column blocks with one halo column on each side
    (stored from an even column with an even pitch, so two-double lanes stay
    aligned): by default the kernel writes the columns the neighbouring
    slabs keep (column mirrors) in one packed launch (NO_PACK: a launch per
    partition); under lazy or eager coherence halo columns move as strided
    2-D copies (pulled, or sent after each sweep); every sweep is
    bit-identical to the oracle's, with one or two doubles per lane."""
    say(f"jacobi column split {shape} K={K} flags={flags} T={T}")
    u0 = inputs.jacobi_grid(*shape, seed=17)
    u0[:, 0] = 0.5  # a nonzero boundary column must be held
    assert_same(run_jacobi(u0, T, K, cfg=cfg, ctx_flags=flags, part_dim=1), oracle.jacobi2d(u0, T))


def test_jacobi_column_split_chosen_dimension_and_column_updates():
    """The dimension chooser's pick for a sweep whose parallel iterator
    indexes columns (the inner loop sequential over rows) is dimension 1;
    arrays entered split that way step bit-exactly, and update ranges are
    column ranges: a host edit of columns [20, 30) pushed with
    update(DEVICE) reaches the next sweep, and update(HOST) of columns
    [0, 40) gathers them from their partitions."""
    say("jacobi column split with the chosen dimension and column updates")
    dim = jacc.parallel_dim([0, 1], [1, 0])
    assert dim == 1
    K = 4
    u0 = inputs.jacobi_grid(48, 96, seed=23)
    a = u0.copy()
    b = u0.copy()
    from gpu_util import context
    with context(K, 0) as c:
        c.enter(a, halo=(1, 1), part_dim=dim)
        c.enter(b, halo=(1, 1), part_dim=dim)
        c.jacobi2d(a, b)
        c.jacobi2d(b, a)
        c.update(a, jacc.UPDATE_HOST, 0, 40)
        c.wait()
        ref = oracle.jacobi2d(u0, 2)
        assert_same(a[:, :40], ref[:, :40])
        a[1:-1, 20:30] = 1.25  # interior rows: the boundary rows of b keep their first values
        ref[1:-1, 20:30] = 1.25
        c.update(a, jacc.UPDATE_DEVICE, 20, 30)
        c.jacobi2d(a, b)
        c.exit(a, jacc.DELETE)
        c.exit(b, jacc.COPYOUT)
    assert_same(b, oracle.jacobi2d(ref, 1))


@pytest.mark.parametrize("shape,K,flags", [((34, 29, 66), 3, 0), ((40, 12, 130), 4, jacc.INIT_LAZY),
                                           ((66, 18, 67), 8, jacc.INIT_EAGER)])
def test_heat_packed_partitions_bit_exact(shape, K, flags):
    """Heat steps without a residual in the task kernel's launch shape: the
    K partitions run as the tasks of one launch per step (mirror stores,
    pulls or eager copies around it), bit-identical to the oracle."""
    say(f"heat packed {shape} K={K} flags={flags}")
    u0 = inputs.heat_field(*shape, seed=41)
    cfg = jacc.config(bx=256, by=1, rows=1, order=1, vec=2 if shape[-1] % 2 == 0 else 1)
    a, b = u0.copy(), u0.copy()
    with context(K, flags) as c:
        c.enter(a, halo=(1, 1))
        c.enter(b, halo=(1, 1))
        src, dst = a, b
        for _ in range(5):
            c.heat3d(src, dst, 0.1, cfg=cfg)
            src, dst = dst, src
        c.exit(a, jacc.COPYOUT)
        c.exit(b, jacc.COPYOUT)
    assert np.array_equal(src, oracle.heat3d(u0, 5, 0.1)[0])


@pytest.mark.parametrize("shape,K", [((66, 40, 130), 3), ((130, 34, 66), 4), ((40, 20, 258), 8)])
def test_heat_residuals_packed_equal_a_launch_per_partition(shape, K):
    """Fields and every residual bit-identical between one launch over all
    partitions (the default) and a launch per partition on its own stream."""
    say(f"heat residual packed vs per-partition {shape} K={K}")
    u0 = inputs.heat_field(*shape, seed=43)
    packed = run_heat(u0, 6, 0.1, K)
    per_part = run_heat(u0, 6, 0.1, K, ctx_flags=jacc.INIT_NO_PACK)
    assert np.array_equal(packed[0], per_part[0]) and np.array_equal(packed[1], per_part[1])
    ref, ref_res = oracle.heat3d(u0, 6, 0.1)
    assert np.array_equal(packed[0], ref) and _rel_close(packed[1], ref_res)
