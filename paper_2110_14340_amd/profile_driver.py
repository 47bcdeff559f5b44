"""Workload driver for rocprofv3 counter and trace runs.

Runs a fixed number of launches of one loop body at its benchmark size,
plus a plain device-to-device copy of known size (1 GiB read + 1 GiB
written) that calibrates the HBM byte counters:

  rocprofv3 --pmc FETCH_SIZE -d <dir> -- python3 -m paper_2110_14340_amd.profile_driver jacobi
  rocprofv3 --pmc WRITE_SIZE -d <dir> -- python3 -m paper_2110_14340_amd.profile_driver jacobi
  rocprofv3 --kernel-trace --stats -d <dir> -- python3 -m paper_2110_14340_amd.profile_driver jacobi

Workloads: jacobi (8192^2), heat (512^3 with the residual), sum (512^3),
gemm (4096^3), spmv (2^22 rows), jacobi_k4 (8192^2 on 4 partitions with
roctx ranges around the runtime's host phases, for --marker-trace).
"""
import sys

import numpy as np


def main(which="jacobi", launches=20, cfg=None):
    import torch
    from . import inputs, jacc
    x = torch.empty(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
    y = torch.empty_like(x)
    x.fill_(1.0)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    if which == "jacobi":
        n = 8192
        u0 = inputs.jacobi_grid(n, n, seed=1)
        a, b = u0.copy(), u0.copy()
        with jacc.Context(1) as c:
            c.enter(a, halo=(1, 1))
            c.enter(b, halo=(1, 1))
            for t in range(launches):
                c.jacobi2d(a, b) if t % 2 == 0 else c.jacobi2d(b, a)
            c.wait()
    elif which == "jacobi_k4":
        n = 8192
        u0 = inputs.jacobi_grid(n, n, seed=1)
        a, b = u0.copy(), u0.copy()
        with jacc.Context(4, flags=jacc.INIT_MARKERS) as c:
            c.enter(a, halo=(1, 1))
            c.enter(b, halo=(1, 1))
            for t in range(launches):
                c.jacobi2d(a, b) if t % 2 == 0 else c.jacobi2d(b, a)
            c.wait()
            c.update(a, jacc.UPDATE_HOST)
    elif which == "heat":
        n = 512
        u0 = inputs.heat_field(n, n, n, seed=2)
        a, b = u0.copy(), u0.copy()
        with jacc.Context(1) as c:
            c.enter(a, halo=(1, 1))
            c.enter(b, halo=(1, 1))
            for t in range(launches):
                (c.heat3d(a, b, 0.1, slot=t, cfg=cfg) if t % 2 == 0 else c.heat3d(b, a, 0.1, slot=t, cfg=cfg))
            c.wait()
    elif which == "gemm":
        A, B = inputs.gemm_inputs(4096, 4096, 4096, seed=3)
        C = np.zeros((4096, 4096))
        with jacc.Context(1) as c:
            c.enter(A)
            c.enter(B, whole=True)
            c.enter(C, clause=jacc.CREATE)
            for _ in range(max(1, launches // 4)):
                c.gemm(A, B, C)
            c.wait()
    elif which == "sum":
        xs = inputs.uniform((512, 512, 512), seed=7)
        with jacc.Context(1) as c:
            c.enter(xs)
            for t in range(launches):
                c.sum(xs, slot=t, sync=False)
            c.wait()
    elif which == "spmv":
        nr = 1 << 22
        rp, col, val, xv = inputs.csr_matrix(nr, nr, 16, seed=4)
        yv = np.zeros(nr)
        with jacc.Context(1) as c:
            c.enter(rp, halo=(1, 1))
            c.enter(col, whole=True)
            c.enter(val, whole=True)
            c.enter(xv, whole=True)
            c.enter(yv, clause=jacc.CREATE)
            for _ in range(launches):
                c.spmv(rp, col, val, xv, yv, cfg=cfg)
            c.wait()
    for _ in range(3):  # the calibration copies, last
        y.copy_(x)
    torch.cuda.synchronize()
    print("profile driver done:", which, flush=True)


if __name__ == "__main__":
    # optional launch configuration after the workload name:
    # bx by tile order march rows (heat only)
    cfg = None
    if len(sys.argv) > 2:
        from . import jacc
        bx, by, tile, order, march, rows = (int(v) for v in sys.argv[2:8])
        cfg = jacc.config(bx=bx, by=by, tile=tile, order=order, march=march, rows=rows)
    main(*(sys.argv[1:2] or ["jacobi"]), cfg=cfg)
