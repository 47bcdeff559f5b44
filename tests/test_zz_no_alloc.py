"""Allocation-free heat step (jacc_heat3d_noalloc) against the context path.

The no-alloc step must compute what a one-partition HEAT3D loop with a
reduction computes through jacc_parallel_loop: the same field bits and the
same residual (bit-equal here, and within the 1e-13 relative bound against
the CPU oracle).  Two calls in a row, the second on a smaller grid, so the
second reads its workgroup partials from a scratch array the first left
dirty.
"""
import numpy as np
import pytest

import oracle
from paper_2110_14340_amd import inputs, jacc
from gpu_util import context, say

pytestmark = pytest.mark.gpu


def context_step(u0, alpha):
    """One heat step through the context path (K=1, residual into slot 0)."""
    a = u0.copy()
    b = u0.copy()
    with context(1) as c:
        c.enter(a, halo=(1, 1))
        c.enter(b, halo=(1, 1))
        c.heat3d(a, b, alpha, slot=0)
        res = c.reductions(0, 1)[0]
        c.exit(b, jacc.COPYOUT)
        c.exit(a, jacc.DELETE)
    return b, res


def test_noalloc_heat_step_equals_the_context_loop_twice_smaller_second():
    import torch
    torch.cuda.set_device(0)
    alpha = 0.1
    res_dev = torch.full((1,), -1.0, dtype=torch.float64, device="cuda:0")
    for shape, seed in (((130, 72, 258), 21), ((34, 19, 66), 22)):
        say(f"no-alloc heat step {shape} seed {seed}")
        u0 = inputs.heat_field(*shape, seed=seed)
        want_field, want_res = context_step(u0, alpha)
        d_in = torch.from_numpy(u0).to("cuda:0")
        d_out = d_in.clone()
        jacc.heat3d_noalloc(d_in, d_out, alpha, residual=res_dev)
        torch.cuda.synchronize()
        got_field = d_out.cpu().numpy()
        got_res = float(res_dev.cpu()[0])
        assert np.array_equal(got_field, want_field), "field differs from the context loop"
        assert got_res == want_res, f"residual {got_res!r} != context loop {want_res!r}"
        ref_field = u0.copy()
        ref_res = oracle.heat3d_sweep(u0, ref_field, alpha)
        assert np.array_equal(got_field, ref_field), "field differs from the oracle"
        assert abs(got_res - ref_res) <= 1e-13 * ref_res


def test_noalloc_heat_step_without_residual_and_on_a_side_stream():
    import torch
    torch.cuda.set_device(0)
    u0 = inputs.heat_field(18, 40, 33, seed=23)  # odd row length: one double per lane
    want_field, _ = context_step(u0, 0.1)
    d_in = torch.from_numpy(u0).to("cuda:0")
    d_out = d_in.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())  # the copies above ran on the current stream
    with torch.cuda.stream(s):
        jacc.heat3d_noalloc(d_in, d_out, 0.1, residual=None, stream=s)
    s.synchronize()
    assert np.array_equal(d_out.cpu().numpy(), want_field)
