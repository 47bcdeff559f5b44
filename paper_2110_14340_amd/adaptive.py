"""Jacobi sweeps whose execution mode is chosen step by step by the adaptive
duplicate-vs-partition policy (Sec. "Adaptive Utilization", Eq. 1-3).

Two contexts hold the grid: one with a single partition (duplicate mode:
the whole loop in one launch, no exchange) and one with n partitions.  Each
step runs in the context the policy names and is timed with HIP events
(one timed execution, no repetition); the policy then sees that time.  In
partitioned mode the halo rows are written through by the producing
kernels, so the exchange time is inside the kernel time and 0 is passed as
the separate exchange time.  When the mode changes, the current grid is
gathered from the old context and scattered into the new one.
"""
import numpy as np

from . import jacc


def jacobi_adaptive(u0, steps, n, peak_bytes_per_s=153e9, cfg=None):
    """Returns (final grid, modes after each step, seconds of each step)."""
    a = np.ascontiguousarray(u0, dtype=np.float64).copy()
    b = a.copy()
    ny, nx = a.shape
    write_bytes = 8.0 * (ny - 2) * (nx - 2)
    ctxs = {jacc.ADAPT_DUPLICATE: jacc.Context(1), jacc.ADAPT_PARTITION: jacc.Context(n)}
    policy = jacc.Adaptive(n, peak_bytes_per_s)
    modes, times = [], []
    try:
        for c in ctxs.values():
            c.enter(a, halo=(1, 1))
            c.enter(b, halo=(1, 1))
        mode = jacc.ADAPT_DUPLICATE
        holder = ctxs[jacc.ADAPT_DUPLICATE]
        bnds = jacc.bounds((1, ny - 1), (1, nx - 1))
        src, dst = a, b
        for _ in range(steps):
            ctx = ctxs[jacc.ADAPT_PARTITION if mode == jacc.ADAPT_PARTITION else jacc.ADAPT_DUPLICATE]
            if ctx is not holder:
                holder.update(src, jacc.UPDATE_HOST)
                ctx.update(src, jacc.UPDATE_DEVICE)
                holder = ctx
            args = [(src, jacc.READ, -1, 1, 0), (dst, jacc.WRITE, 0, 0, 0)]
            ms = ctx.time_loop(jacc.JACOBI2D, bnds, args, cfg=cfg, warmup=0, reps=1)
            t = float(ms[0]) * 1e-3
            mode = policy.observe(t, 0.0, write_bytes)
            modes.append(mode)
            times.append(t)
            src, dst = dst, src
        holder.update(src, jacc.UPDATE_HOST)
        return src.copy(), modes, times
    finally:
        policy.close()
        for c in ctxs.values():
            c.close()
