#!/usr/bin/env python3
"""Benchmark of the K-partitioned loop-nest runtime on one MI355X.

Workload (the headline): Jacobi-2D 5-point FP64 on an 8192 x 8192 grid,
`--steps` iterations (default 1000), the grid split into K row-block
partitions held as separate device buffers, with the 1-row halo exchange
planned by the runtime each step.  One "step" is one full sweep of the
partitioned hot path: planning, cross-stream waits, halo copies or halo
write-through and the K partitions' tiles (by default one packed launch for
all K; a launch per partition on its own stream is measured beside it).
Inputs are resident in HBM before the timed region starts (data_enter
happens before it).

Printed: ONE JSON line.  `value` is the K=8 run's algorithmic throughput
(16 bytes per interior cell per step: one 8-byte read and one 8-byte write
at perfect reuse) in GB/s; per-K results and the K-partition overhead are
listed beside it.  `roofline` describes the Jacobi kernel timed with HIP
events on its own stream over the K=1 timed region (single kernel over the
whole grid); `cpu_baseline` times the CPU oracle on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


COUNTERS = os.path.join(ROOT, "profiles", "jacobi2d_counters.json")
# the loop body and the default launch configuration both decide the counted traffic
STENCIL_SOURCES = [os.path.join(ROOT, "paper_2110_14340_amd", "csrc", f) for f in ("k_stencil.hip", "k_common.h", "dispatch.cpp")]


def counted_traffic():
    """HBM bytes per Jacobi launch from the committed FETCH_SIZE/WRITE_SIZE
    counter record, or None when the kernel sources changed since then."""
    import hashlib
    try:
        with open(COUNTERS) as f:
            rec = json.load(f)
        h = hashlib.sha1(b"".join(open(p, "rb").read() for p in STENCIL_SOURCES)).hexdigest()
    except OSError:
        return None
    return int(rec["traffic_bytes_per_launch"]) if rec.get("source_sha1") == h else None


def run_jacobi(ctx_mod, torch, u0, K, steps, warmup, cfg=None, flags=0, part_dim=0):
    """Times `steps` partitioned Jacobi sweeps after `warmup` untimed ones
    (row blocks, or column blocks with part_dim=1).  Returns (seconds,
    stream-0 event seconds)."""
    jacc = ctx_mod
    a = u0.copy()
    b = u0.copy()
    c = jacc.Context(K, flags=flags)
    c.enter(a, halo=(1, 1), part_dim=part_dim)
    c.enter(b, halo=(1, 1), part_dim=part_dim)
    src, dst = a, b
    for _ in range(warmup):
        c.jacobi2d(src, dst, cfg=cfg)
        src, dst = dst, src
    c.wait()
    torch.cuda.synchronize()
    s0 = c.streams[0]
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(s0)
    t0 = time.perf_counter()
    for _ in range(steps):
        c.jacobi2d(src, dst, cfg=cfg)
        src, dst = dst, src
    ev1.record(s0)
    c.wait()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ev_s = ev0.elapsed_time(ev1) / 1e3
    c.exit(a, jacc.DELETE)
    c.exit(b, jacc.DELETE)
    c.close()
    return t1 - t0, ev_s


def run_jacobi_graph(jacc, torch, u0, K, steps, warmup, per_graph=2, persistent=True):
    """The same partitioned sweeps captured once as a graph of `per_graph`
    steps and replayed steps/per_graph times: the K partitions of a step as
    tasks of one persistent launch (halo rows written through by the
    producing tiles), or (persistent=False) as K launches in sequence."""
    a = u0.copy()
    b = u0.copy()
    c = jacc.Context(K)
    c.enter(a, halo=(1, 1))
    c.enter(b, halo=(1, 1))
    cfg = jacc.config(vec=2, persistent=1) if persistent else None
    c.batch_begin()
    for t in range(per_graph):
        (c.jacobi2d(a, b, cfg=cfg) if t % 2 == 0 else c.jacobi2d(b, a, cfg=cfg))
    g = c.batch_end()
    c.batch_launch(g, max(1, warmup // per_graph))
    c.wait()
    torch.cuda.synchronize()
    reps = max(1, steps // per_graph)
    t0 = time.perf_counter()
    c.batch_launch(g, reps)
    c.wait()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c.close()
    return (t1 - t0) * steps / (reps * per_graph)  # scaled to `steps` steps


def cpu_baseline(u0, budget_s=8.0):
    """The CPU oracle on a bounded sample of the same workload: its
    multi-threaded Jacobi form (the same per-element arithmetic, rows split
    over OpenMP threads, bit-identical fields) on all host cores, and beside
    it the plain sequential sweep on one thread."""
    import oracle
    ny, nx = u0.shape
    cells = (ny - 2) * (nx - 2)
    # one thread, sequential sweeps
    out = u0.copy()
    t0 = time.perf_counter()
    oracle.jacobi2d_sweep(u0, out)
    t1 = time.perf_counter() - t0
    n1 = int(max(1, min(200, budget_s / max(t1, 1e-6))))
    a = u0.copy()
    b = u0.copy()
    t0 = time.perf_counter()
    for _ in range(n1):
        oracle.jacobi2d_sweep(a, b)
        a, b = b, a
    dt1 = time.perf_counter() - t0
    # every host core: T sweeps in one call, minus the call's own copies
    cores = oracle.threads()
    t0 = time.perf_counter()
    oracle.jacobi2d_mt(u0, 8, cores)
    probe = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.jacobi2d_mt(u0, 0, cores)
    base = time.perf_counter() - t0
    per = max((probe - base) / 8, 1e-6)
    nm = int(max(2, min(2000, budget_s / per))) // 2 * 2
    t0 = time.perf_counter()
    oracle.jacobi2d_mt(u0, nm, cores)
    dtm = time.perf_counter() - t0 - base
    return {"value": round(16.0 * cells * nm / dtm / 1e9, 3), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"{nm} oracle sweeps of the {ny}x{nx} grid in its multi-threaded form ({cores} OpenMP "
                      f"threads, {dtm:.1f} s; same 16 B/cell algorithmic bytes)",
            "one_thread": {"value": round(16.0 * cells * n1 / dt1 / 1e9, 3), "unit": "GB/s", "cores": 1,
                           "sample": f"{n1} sequential oracle sweeps (1 thread, {dt1:.1f} s)"}}


def extra_workloads(jacc, torch, inputs):
    """Short secondary measurements of the other loop bodies (one GPU): the
    cache-resident Jacobi 512^2 case, heat 512^3 with its residual, sum,
    GEMM and SpMV, each at K=1 and at its partitioned K."""
    out = {}

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    def stencil(u0, K, steps, sweep):
        a, b = u0.copy(), u0.copy()
        c = jacc.Context(K)
        c.enter(a, halo=(1, 1))
        c.enter(b, halo=(1, 1))

        def run():
            for t in range(steps):
                s, d = (a, b) if t % 2 == 0 else (b, a)
                sweep(c, s, d, t)
            c.wait()

        dt = timed(run, 1) / steps
        c.close()
        return dt

    # Jacobi 512^2, T=100: 4 MiB, cache-resident, launch/latency bound
    u0 = inputs.jacobi_grid(512, 512, seed=0)
    for K in (1, 4):
        dt = stencil(u0, K, 100, lambda c, s, d, t: c.jacobi2d(s, d))
        out[f"jacobi2d_512_K{K}"] = {"us_per_step": round(dt * 1e6, 2),
                                     "effective_gbps": round(16 * 510 * 510 / dt / 1e9, 1)}
        # the same 100 steps replayed from a captured two-step graph
        wall = run_jacobi_graph(jacc, torch, u0, K, 100, 20, per_graph=20)
        out[f"jacobi2d_512_K{K}_graph"] = {"us_per_step": round(wall / 100 * 1e6, 2),
                                           "effective_gbps": round(16 * 510 * 510 * 100 / wall / 1e9, 1)}
    # heat 512^3, T=100, residual every step into a device slot
    n = 512
    u0 = inputs.heat_field(n, n, n, seed=2)
    cells = (n - 2) ** 3
    for K in (1, 4):
        dt = stencil(u0, K, 100, lambda c, s, d, t: c.heat3d(s, d, 0.1, slot=t))
        out[f"heat3d_512_K{K}_residual"] = {"gbps": round(16 * cells / dt / 1e9, 1), "ms_per_step": round(dt * 1e3, 4)}
    out["heat3d_k4_overhead"] = round(out["heat3d_512_K1_residual"]["gbps"] / out["heat3d_512_K4_residual"]["gbps"] - 1, 4)
    del u0
    # sum over 512^3 (1 GiB)
    x = inputs.uniform((512, 512, 512), seed=7)
    for K in (1, 4):
        c = jacc.Context(K)
        c.enter(x)
        dt = timed(lambda: c.sum(x), 10)
        out[f"sum_512cubed_K{K}"] = {"gbps": round(x.nbytes / dt / 1e9, 1), "ms": round(dt * 1e3, 4)}

        # the same sums into device slots, read once at the end (no host
        # round trip between them)
        def deferred():
            for i in range(20):
                c.sum(x, slot=i, sync=False)
            c.wait()

        dt = timed(deferred, 3) / 20
        out[f"sum_512cubed_K{K}_slots"] = {"gbps": round(x.nbytes / dt / 1e9, 1), "ms": round(dt * 1e3, 4)}
        c.close()
    del x
    # GEMM 4096^3 FP64 MFMA
    A, B = inputs.gemm_inputs(4096, 4096, 4096, seed=3)
    C = np.zeros((4096, 4096))
    for K, whole, tag in ((1, True, ""), (4, True, ""), (4, jacc.SHARED, "_shared")):
        c = jacc.Context(K)
        c.enter(A)
        c.enter(B, whole=whole)
        c.enter(C, clause=jacc.CREATE)

        # HIP events around back-to-back launches, median of 10
        gargs = [(A, jacc.READ, 0, 0, 0), (B, jacc.READ, 0, 0, 1), (C, jacc.WRITE, 0, 0, 0)]
        dt = float(np.median(c.time_loop(jacc.GEMM, jacc.bounds((0, 4096), (0, 4096)), gargs, warmup=2,
                                          reps=10))) / 1e3
        tf = 2 * 4096 ** 3 / dt / 1e12
        out[f"gemm_4096_K{K}{tag}"] = {"tflops": round(tf, 2), "ms": round(dt * 1e3, 3),
                                  "frac_fp64_peak": round(tf / FP64_MFMA_PEAK_TFLOPS, 3)}
        c.close()
    del A, B, C
    # SpMV 2^22 rows, ~16 nnz/row
    nr = 1 << 22
    rp, col, val, xv = inputs.csr_matrix(nr, nr, 16, seed=4)
    y = np.zeros(nr)
    alg = rp.nbytes + col.nbytes + val.nbytes + xv.nbytes + y.nbytes
    # col, val and x replicated per partition, or one shared read-only copy
    for K, whole, tag in ((1, True, ""), (4, True, ""), (4, jacc.SHARED, "_shared")):
        c = jacc.Context(K)
        c.enter(rp, halo=(1, 1))
        c.enter(col, whole=whole)
        c.enter(val, whole=whole)
        c.enter(xv, whole=whole)
        c.enter(y, clause=jacc.CREATE)

        def sp():
            c.spmv(rp, col, val, xv, y)
            c.wait()

        dt = timed(sp, 10)
        out[f"spmv_2^22_K{K}{tag}"] = {"gbps": round(alg / dt / 1e9, 1), "ms": round(dt * 1e3, 4),
                                       "nnz": int(col.size)}
        c.close()
    del rp, col, val, xv, y
    # 96 independent Jacobi grids (sides 64..1024), 2 sweeps each per pass:
    # eager on 1, 4 and 16 streams (runtime-chosen), and as one graph
    from paper_2110_14340_amd import experiment
    out["independent_loops_ms_per_pass"], _ = experiment.independent_loops()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--k-list", default="1,2,4,8")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the partitions of this "
              "runtime live on a single MI355X and no multi-GPU path is built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2110_14340_amd import inputs, jacc
    jacc.lib()
    n = args.n
    log(f"generating {n}x{n} grid")
    u0 = inputs.jacobi_grid(n, n, seed=1)
    cells = (n - 2) * (n - 2)
    step_bytes = 16.0 * cells
    ks = [int(k) for k in args.k_list.split(",")]
    per_k = {}
    ev_k1 = None
    for K in ks:
        log(f"jacobi K={K}: warmup {args.warmup}, timed {args.steps}")
        wall, ev = run_jacobi(jacc, torch, u0, K, args.steps, args.warmup)
        per_k[K] = {"ms_per_step": round(wall / args.steps * 1e3, 5),
                    "gbps": round(step_bytes * args.steps / wall / 1e9, 1),
                    "event_us_per_step": round(ev / args.steps * 1e6, 2)}
        if K == 1:
            ev_k1 = ev
    # the other issue and coherence modes, at the partitioned K's: a launch
    # per partition on its own stream instead of one packed launch (with
    # 2-4 partitions split into own-block rows first and edge rows after, or
    # unsplit); halo rows pulled by copies before each read (lazy) instead of
    # written through by the producing kernels; split forced at every K
    modes = {}
    for K in ks:
        if K == 1:
            continue
        for name, fl in (("streams", jacc.INIT_NO_PACK), ("lazy_pull", jacc.INIT_LAZY),
                         ("streams_no_split", jacc.INIT_NO_PACK | jacc.INIT_NO_SPLIT), ("split", jacc.INIT_SPLIT)):
            log(f"jacobi K={K} {name}")
            wall, _ = run_jacobi(jacc, torch, u0, K, args.steps, args.warmup, flags=fl)
            modes.setdefault(name, {})[str(K)] = {"ms_per_step": round(wall / args.steps * 1e3, 5),
                                                  "gbps": round(step_bytes * args.steps / wall / 1e9, 1)}
    # the arrays split into column blocks instead (one packed launch per
    # sweep whose tiles write the columns the neighbouring slabs keep)
    for K in ks:
        log(f"jacobi K={K} column blocks")
        wall, _ = run_jacobi(jacc, torch, u0, K, args.steps, args.warmup, part_dim=1)
        modes.setdefault("column_split", {})[str(K)] = {"ms_per_step": round(wall / args.steps * 1e3, 5),
                                                        "gbps": round(step_bytes * args.steps / wall / 1e9, 1)}
    graph, graph_plain = {}, {}
    per_graph = 10 if args.steps >= 10 else 2  # steps per captured graph
    for K in ks:
        log(f"jacobi K={K} as a replayed graph")
        wall = run_jacobi_graph(jacc, torch, u0, K, args.steps, args.warmup, per_graph=per_graph)
        graph[K] = {"ms_per_step": round(wall / args.steps * 1e3, 5),
                    "gbps": round(step_bytes * args.steps / wall / 1e9, 1)}
        wall = run_jacobi_graph(jacc, torch, u0, K, args.steps, args.warmup, per_graph=per_graph, persistent=False)
        graph_plain[K] = {"ms_per_step": round(wall / args.steps * 1e3, 5),
                          "gbps": round(step_bytes * args.steps / wall / 1e9, 1)}
    main_k = max(ks)
    wall_main = per_k[main_k]["ms_per_step"] / 1e3 * args.steps
    value = step_bytes * args.steps / wall_main / 1e9
    result = {
        "metric": "FP64 stencil GB/s (% HBM peak); K-partition overhead; learned vs tuned config",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": per_k[main_k]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"jacobi2d_5pt {n}x{n}, {args.steps} iterations, K={main_k} row-block "
                               f"partitions in separate slabs, 1-row halo exchange per step (mirror stores); "
                               f"the partitions of a step run in one launch (per_k_modes.streams: a launch per "
                               f"partition on K streams)",
                   "grid": [n, n], "K": main_k, "iterations": args.steps, "seed": 1},
        "frac_hbm_peak": round(value / HBM_PEAK_GBS, 4),
        "per_k": {str(k): v for k, v in per_k.items()},
        "per_k_graph_steps_per_graph": per_graph,
        "per_k_graph": {str(k): v for k, v in graph.items()},
        "per_k_graph_plain_launches": {str(k): v for k, v in graph_plain.items()},
        "per_k_modes": modes,
    }
    if 1 in per_k and main_k != 1:
        result["k_overhead"] = round(per_k[main_k]["ms_per_step"] / per_k[1]["ms_per_step"] - 1.0, 4)
    if ev_k1 is not None:
        avg = ev_k1 / args.steps
        ach = step_bytes / avg / 1e9
        result["roofline"] = {"kernel": "jacobi2d_kernel<2> (K=1, whole interior per launch)", "bound": "hbm",
                              "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": counted_traffic(),
                              "avg_launch_us": round(avg * 1e6, 2),
                              "bytes_per_launch": int(step_bytes),
                              "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)"}
    if main_k > 1 and main_k <= 16:
        # the headline K's one packed launch per step (all on stream 0): its
        # average duration from the same HIP events
        avg = per_k[main_k]["event_us_per_step"] / 1e6
        ach = step_bytes / avg / 1e9
        result["roofline_packed"] = {"kernel": f"jacobi2d_parts_kernel<2> ({main_k} partitions, one launch per step)",
                                     "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                                     "avg_launch_us": round(avg * 1e6, 2), "bytes_per_launch": int(step_bytes)}
    if not args.no_extra:
        log("secondary workloads")
        result["extra"] = extra_workloads(jacc, torch, inputs)
    if not args.no_learned:
        log("batched / learned experiment")
        from paper_2110_14340_amd import experiment
        # 96 training shapes (48 2-D, 48 3-D), medians of 3 amortised samples
        result["learned"], _ = experiment.run(log=log, train2d=48, train3d=48, tune_reps=3)
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(u0)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
