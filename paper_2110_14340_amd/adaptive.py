"""Jacobi sweeps whose execution mode is chosen step by step by the adaptive
duplicate-vs-partition policy (Sec. "Adaptive Utilization", Eq. 1-3).

Two contexts hold the grid: one with a single partition (duplicate mode:
the whole loop in one launch, no exchange) and one with n partitions.  Each
step runs in the context the policy names and is timed once
(jacc_time_loop_parts): in duplicate mode the policy sees the kernel time;
in partitioned mode it sees the kernel time of one partition (the longest)
as t_kernel and the rest of the step as t_comm.  The partitioned context
pulls halo rows by device-to-device copies before each partition's kernel
(lazy coherence), so t_comm holds the exchange and the cross-stream waits.
When the mode changes, the current grid is gathered from the old context and
scattered into the new one.
"""
import numpy as np

from . import jacc


def jacobi_adaptive(u0, steps, n, peak_bytes_per_s=153e9, cfg=None, lazy=True):
    """Returns (final grid, modes after each step, (t_kernel, t_comm) of each step)."""
    a = np.ascontiguousarray(u0, dtype=np.float64).copy()
    b = a.copy()
    ny, nx = a.shape
    write_bytes = 8.0 * (ny - 2) * (nx - 2)
    ctxs = {jacc.ADAPT_DUPLICATE: jacc.Context(1),
            jacc.ADAPT_PARTITION: jacc.Context(n, flags=jacc.INIT_LAZY if lazy else 0)}
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
            partitioned = mode == jacc.ADAPT_PARTITION
            ctx = ctxs[jacc.ADAPT_PARTITION if partitioned else jacc.ADAPT_DUPLICATE]
            if ctx is not holder:
                holder.update(src, jacc.UPDATE_HOST)
                ctx.update(src, jacc.UPDATE_DEVICE)
                holder = ctx
            args = [(src, jacc.READ, -1, 1, 0), (dst, jacc.WRITE, 0, 0, 0)]
            step_ms, ker_ms = ctx.time_loop_parts(jacc.JACOBI2D, bnds, args, cfg=cfg)
            t_k = float(np.max(ker_ms)) * 1e-3
            t_c = max(0.0, float(step_ms) * 1e-3 - t_k) if partitioned else 0.0
            mode = policy.observe(t_k, t_c, write_bytes)
            modes.append(mode)
            times.append((t_k, t_c))
            src, dst = dst, src
        holder.update(src, jacc.UPDATE_HOST)
        return src.copy(), modes, times
    finally:
        policy.close()
        for c in ctxs.values():
            c.close()
