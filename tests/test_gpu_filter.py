"""GPU parity of predicate-based filtering (Sec. "Predicate-Based Filtering"):
the statement chain of the paper's example (Fig. conv-code) on K replicas
under lazy coherence, the paper's eager broadcast, and duplicated execution
of an aliased call; a whole-array read afterwards (pulls of owner blocks);
and the filtered form of every stencil kind against its hoisted form."""
import numpy as np
import pytest

import oracle
from paper_2110_14340_amd import inputs, jacc
from gpu_util import context, run_heat, say

pytestmark = pytest.mark.gpu

MODES = {"lazy": 0, "eager": jacc.INIT_EAGER}


@pytest.mark.parametrize("K", [1, 2, 3, 4, 8])
@pytest.mark.parametrize("mode", ["lazy", "eager"])
def test_pred_chain_equals_oracle(K, mode):
    say(f"pred chain K={K} {mode}")
    a0, b0, c, idx, xs = inputs.pred_chain_inputs(200_003, 150_001, 5_000, 60_000, seed=K, skipped=11)
    ref_a, ref_b = oracle.pred_chain(a0, b0, c, idx, xs)
    # second call: other iterations over the arrays the first one left
    _, _, c2, idx2, xs2 = inputs.pred_chain_inputs(200_003, 150_001, 5_000, 40_000, seed=100 + K)
    ref_a, ref_b = oracle.pred_chain(ref_a, ref_b, c2, idx2, xs2)
    a, b = a0.copy(), b0.copy()
    with context(K, MODES[mode]) as ctx:
        ctx.enter(a, whole=True)
        ctx.enter(b, whole=True)
        for arr in (c, idx, xs, c2, idx2, xs2):
            ctx.enter(arr, whole=True)
        ctx.pred_chain(a, b, c, idx, xs)
        ctx.pred_chain(a, b, c2, idx2, xs2)
        s = ctx.sum(a, sync=True)  # partition 0 sums every row of a: the owner blocks it lacks are pulled
        ctx.exit(b)
        ctx.exit(a)
    assert np.array_equal(a, ref_a)
    assert np.array_equal(b, ref_b)
    want = oracle.sum_(ref_a)
    assert abs(s - want) <= 1e-13 * np.abs(ref_a).sum()


def _device_f64(ptr, n):
    """Host copy of n doubles at a device address (a view through the
    device-array interface, copied by torch)."""
    import torch

    class View:
        __cuda_array_interface__ = {"shape": (n,), "typestr": "<f8", "data": (ptr, False), "version": 2}

    return torch.as_tensor(View(), device="cuda").cpu().numpy().copy()


@pytest.mark.parametrize("K", [1, 3, 4])
def test_aliased_pred_chain_runs_duplicated(K):
    """a passed as b: every partition computes the whole chain on its own
    replica, unfiltered, and nothing moves afterwards; every replica then
    holds the oracle's aliased result."""
    say(f"aliased pred chain K={K}")
    a0, _, c, idx, xs = inputs.pred_chain_inputs(100_000, 100_000, 777, 30_000, seed=7 + K, skipped=5)
    ref, _ = oracle.pred_chain(a0, a0, c, idx, xs)
    a = a0.copy()
    with context(K, 0) as ctx:
        ctx.enter(a, whole=True)
        for arr in (c, idx, xs):
            ctx.enter(arr, whole=True)
        ctx.pred_chain(a, a, c, idx, xs)
        ctx.wait()
        for p in range(K):
            dev, lo, hi = ctx.slab(a, p)
            assert (lo, hi) == (0, a.size)
            assert np.array_equal(_device_f64(dev, a.size), ref), f"replica {p}"
        ctx.exit(a)
    assert np.array_equal(a, ref)


@pytest.mark.parametrize("shape,K", [((40, 37, 66), 1), ((67, 33, 130), 3), ((130, 64, 258), 4)])
def test_filtered_heat_equals_hoisted_form(shape, K):
    """Filtered heat step: every partition sweeps the whole box from a whole
    replica of the input and keeps its owner planes (and sums its residual
    over them only); the field equals the hoisted form's bit for bit and the
    oracle's, the residual is within 1e-13 of the oracle's."""
    say(f"filtered heat {shape} K={K}")
    u0 = inputs.heat_field(*shape, seed=31)
    nz, ny, nx = shape
    a, b = u0.copy(), u0.copy()
    with context(K) as ctx:
        ctx.enter(a, whole=True)
        ctx.enter(b, halo=(1, 1))
        ctx.loop(jacc.HEAT3D, jacc.bounds((1, nz - 1), (1, ny - 1), (1, nx - 1)),
                 [(a, jacc.READ, -1, 1, 0), (b, jacc.WRITE | jacc.FILTERED, 0, 0, 0)], scalars=(0.1,), slot=0)
        res = ctx.reductions(0, 1)[0]
        ctx.exit(b)
        ctx.exit(a, jacc.DELETE)
    ref = u0.copy()
    ref_res = oracle.heat3d_sweep(u0, ref, 0.1)
    assert np.array_equal(b, ref)
    hoisted, _ = run_heat(u0, 1, 0.1, K)
    assert np.array_equal(b, hoisted)
    assert abs(res - ref_res) <= 1e-13 * ref_res


@pytest.mark.parametrize("shape,K", [((67, 33, 130), 3), ((40, 37, 66), 4)])
def test_heat_under_eager_coherence(shape, K):
    """The paper's coherence (every written row sent to every slab holding it
    after each step, no mirror stores): five heat steps with residuals
    against the oracle."""
    say(f"heat {shape} K={K} eager")
    u0 = inputs.heat_field(*shape, seed=41)
    got, res = run_heat(u0, 5, 0.1, K, ctx_flags=jacc.INIT_EAGER)
    ref, ref_res = oracle.heat3d(u0, 5, 0.1)
    assert np.array_equal(got, ref)
    assert np.all(np.abs(res - ref_res) <= 1e-13 * ref_res)
