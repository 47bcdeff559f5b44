"""Helpers for the GPU parity tests: open a runtime context on cuda:0 with
PyTorch streams and allocator, run loop sequences through the C ABI."""
import sys

import numpy as np

from paper_2110_14340_amd import jacc


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def context(K, flags=0):
    return jacc.Context(K, streams="torch", allocator="torch", flags=flags)


def run_jacobi(u0, steps, K, cfg=None, ctx_flags=0, part_dim=0):
    """T ping-pong Jacobi sweeps on the device with K partitions (row blocks,
    or column blocks with part_dim=1); returns the final grid (gathered to
    the host)."""
    a = np.ascontiguousarray(u0, dtype=np.float64).copy()
    b = a.copy()
    with context(K, ctx_flags) as c:
        c.enter(a, halo=(1, 1), part_dim=part_dim)
        c.enter(b, halo=(1, 1), part_dim=part_dim)
        src, dst = a, b
        for _ in range(steps):
            c.jacobi2d(src, dst, cfg=cfg)
            src, dst = dst, src
        c.exit(b, jacc.COPYOUT)
        c.exit(a, jacc.COPYOUT)
    return src


def run_heat(u0, steps, alpha, K, cfg=None, ctx_flags=0):
    """T heat steps with the fused residual into slots 0..T-1; returns
    (final field, residuals)."""
    a = np.ascontiguousarray(u0, dtype=np.float64).copy()
    b = a.copy()
    with context(K, ctx_flags) as c:
        c.enter(a, halo=(1, 1))
        c.enter(b, halo=(1, 1))
        src, dst = a, b
        for t in range(steps):
            c.heat3d(src, dst, alpha, slot=t, cfg=cfg)
            src, dst = dst, src
        res = c.reductions(0, steps)
        c.exit(b, jacc.COPYOUT)
        c.exit(a, jacc.COPYOUT)
    return src, res
