"""Batched/learned experiment: hundreds of uneven stencil sweeps in one
captured graph, configured three ways — by the exhaustive autotuner, by the
learned cost model, and by a fixed default configuration — and the graph
time of each (regret of the model against the tuner, gain over the default).

Shapes: 2-D Jacobi sweeps with both sides log-uniform in [64, 4096] and 3-D
heat sweeps with sides log-uniform in [32, 512] (test batch seed 5, data
seed 6); the model is trained only on timings of other shapes (seed 7+).
These stand in for applications with tens to hundreds of kernels of uneven
sizes (the paper's benchmark table).
"""
import os
import tempfile
import time

import numpy as np

from . import inputs, jacc, tuner


def _data(shape, seed):
    return inputs.jacobi_grid(*shape, seed=seed) if len(shape) == 2 else inputs.heat_field(*shape, seed=seed)


def _sweep(ctx, u, v, cfg):
    c = tuner.launch_config(cfg)
    if u.ndim == 2:
        ctx.jacobi2d(u, v, cfg=c)
    else:
        ctx.heat3d(u, v, 0.1, cfg=c)


def graph_time(shapes, datas, configs, reps=10, keep_outputs=False):
    """Enters every loop's arrays with its configuration's K, captures all
    sweeps into one graph, and returns (median ms of `reps` replays, the
    batch's launch counts, outputs or None)."""
    K = max(c["K"] for c in configs)
    ctx = jacc.Context(max(2, K))
    ins, outs = [], []
    try:
        for sh, d, cfg in zip(shapes, datas, configs):
            u = d.copy()
            v = d.copy()
            ctx.enter(u, halo=(1, 1), K=cfg["K"])
            ctx.enter(v, halo=(1, 1), K=cfg["K"])
            ins.append(u)
            outs.append(v)
        ctx.batch_begin()
        for u, v, cfg in zip(ins, outs, configs):
            _sweep(ctx, u, v, cfg)
        g = ctx.batch_end()
        info = ctx.batch_info(g)
        ms = ctx.batch_time(g, warmup=2, reps=reps)
        res = None
        if keep_outputs:
            res = []
            for v in outs:
                ctx.update(v, jacc.UPDATE_HOST)
                res.append(v.copy())
        return float(np.median(ms)), info, res
    finally:
        ctx.close()


def copy_bandwidth(nbytes=1 << 28, reps=5):
    """Device-to-device copy bandwidth (bytes/s, read + write counted once:
    bytes moved per copy), the peak of Eq. 1 on one GPU."""
    import torch
    x = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    y.copy_(x)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        y.copy_(x)
    t1.record()
    t1.synchronize()
    return nbytes * reps / (t0.elapsed_time(t1) * 1e-3)


def eq1_partitions(t_dup_s, write_bytes, n, peak):
    """The partition count Eq. 1 (Sec. "Adaptive Utilization") chooses for a
    loop whose duplicated (one-partition) execution takes t_dup_s: n when
    t_dup > t_dup/n + WriteSize/peak, else 1."""
    return n if t_dup_s > t_dup_s / n + write_bytes / peak else 1


def interleaved_times(shapes, datas, configs_by_name, rounds=3, reps=30):
    """Graph time of each configuration set, measured in `rounds` interleaved
    rounds (A, B, ..., A, B, ...); the minimum of the per-round medians."""
    best = {k: float("inf") for k in configs_by_name}
    for _ in range(rounds):
        for k, cfgs in configs_by_name.items():
            ms, _, _ = graph_time(shapes, datas, cfgs, reps)
            best[k] = min(best[k], ms)
    return best


def run(n2d=128, n3d=128, train2d=64, train3d=64, epochs=300, members=3, tune_reps=5, graph_reps=30, log=print,
        test_shapes=None, train_shapes=None, workdir=None):
    """The batched/learned experiment.  Timing databases and the model file
    go to `workdir` (a fresh temporary directory by default).  Besides the
    exhaustive, learned and default configurations, a fourth set takes the
    partition count from Eq. 1 (duplicate or split over the largest K) and
    the rest of the configuration from the tuner's best candidate at that
    partition count."""
    t_start = time.perf_counter()
    test_shapes = test_shapes or inputs.batch_shapes(5, n2d, n3d)
    train_shapes = train_shapes or inputs.batch_shapes(7, train2d, train3d)
    workdir = workdir or tempfile.mkdtemp(prefix="jacc_learned_")
    train_db = os.path.join(workdir, "train_timings.db")
    test_db = os.path.join(workdir, "test_timings.db")
    model_path = os.path.join(workdir, "cost_model.bin")
    ctx = jacc.Context(max(tuner.KS))
    try:
        # 1. exhaustive timings of the training shapes -> the training database
        t0 = time.perf_counter()
        for li, sh in enumerate(train_shapes):
            tuner.tune(ctx, sh, _data(sh, 1000 + li), db_path=train_db, reps=tune_reps)
            if li % 8 == 7:
                log(f"  tuned {li + 1}/{len(train_shapes)} training shapes")
        t_train_tune = time.perf_counter() - t0
        # 2. the GPU-trained ensemble, from the database, into a model file
        t0 = time.perf_counter()
        rep = tuner.train(ctx, train_db, model_path, members=members, epochs=epochs, seed=9, holdout=5)
        t_fit = time.perf_counter() - t0
        log(f"model: {rep['rows']} timings of {rep['signatures']} shapes ({t_train_tune:.1f} s to tune), "
            f"loss {rep['loss_first']:.4f} -> {rep['loss_last']:.4f} in {epochs} epochs ({t_fit:.1f} s), "
            f"held-out mse {rep['heldout_mse']:.4f}")
        ctx.model_load(model_path)
        # 3. the test batch: exhaustive choice, model choice, default, Eq. 1
        peak = copy_bandwidth()
        nmax = max(tuner.KS)
        exh, mlp, dflt, rule, datas, regret_loop = [], [], [], [], [], []
        t0 = time.perf_counter()
        for li, sh in enumerate(test_shapes):
            d = _data(sh, 6000 + li)
            datas.append(d)
            cands, meds, best = tuner.tune(ctx, sh, d, db_path=test_db, reps=tune_reps)
            exh.append(cands[best])
            pick, pcands, _ = tuner.pick(ctx, sh)
            assert pcands == cands
            mlp.append(pick)
            dflt.append(dict(tuner.DEFAULT_CONFIG))
            regret_loop.append(meds[cands.index(pick)] / meds[best] - 1.0)
            one = [i for i, c in enumerate(cands) if c["K"] == 1]
            t_dup = min(meds[i] for i in one) * 1e-3
            k_rule = eq1_partitions(t_dup, 8.0 * float(np.prod([d - 2 for d in sh])), nmax, peak)
            at_k = [i for i, c in enumerate(cands) if c["K"] == k_rule]
            rule.append(cands[min(at_k, key=lambda i: (meds[i], i))])
            if li % 8 == 7:
                log(f"  tuned {li + 1}/{len(test_shapes)} test shapes")
        t_test_tune = time.perf_counter() - t0
    finally:
        ctx.close()
    log(f"test batch: {len(test_shapes)} loops tuned exhaustively ({t_test_tune:.1f} s)")
    t_exh, info_e, out_e = graph_time(test_shapes, datas, exh, graph_reps, keep_outputs=True)
    t_mlp, info_m, out_m = graph_time(test_shapes, datas, mlp, graph_reps, keep_outputs=True)
    t_def, info_d, out_d = graph_time(test_shapes, datas, dflt, graph_reps, keep_outputs=True)
    t_rule, info_r, out_r = graph_time(test_shapes, datas, rule, graph_reps, keep_outputs=True)
    identical = all(np.array_equal(a, b) and np.array_equal(a, c) and np.array_equal(a, d)
                    for a, b, c, d in zip(out_e, out_m, out_d, out_r))
    cells = sum(float(np.prod([d - 2 for d in sh])) for sh in test_shapes)
    alg_bytes = 16.0 * cells
    ks_used = {"exhaustive": sorted({c["K"] for c in exh}), "learned": sorted({c["K"] for c in mlp}),
               "eq1_rule": sorted({c["K"] for c in rule})}
    result = {
        "loops": len(test_shapes),
        "algorithmic_gb": round(alg_bytes / 1e9, 3),
        "graph_ms": {"exhaustive": round(t_exh, 4), "learned": round(t_mlp, 4), "default": round(t_def, 4),
                     "eq1_rule": round(t_rule, 4)},
        "graph_gbps": {"exhaustive": round(alg_bytes / t_exh / 1e6, 1), "learned": round(alg_bytes / t_mlp / 1e6, 1),
                       "default": round(alg_bytes / t_def / 1e6, 1), "eq1_rule": round(alg_bytes / t_rule / 1e6, 1)},
        "regret_learned_vs_exhaustive": round(t_mlp / t_exh - 1.0, 4),
        "regret_eq1_rule_vs_exhaustive": round(t_rule / t_exh - 1.0, 4),
        "eq1_peak_gbps": round(peak / 1e9, 1),
        "gain_learned_vs_default": round(t_def / t_mlp, 3),
        "mean_per_loop_regret": round(float(np.mean(regret_loop)), 4),
        "median_per_loop_regret": round(float(np.median(regret_loop)), 4),
        "partition_counts_searched": list(tuner.KS),
        "partition_counts_chosen": ks_used,
        "persistent_groups": {"exhaustive": info_e["persistent_groups"], "learned": info_m["persistent_groups"]},
        "outputs_bit_identical_across_configs": bool(identical),
        "train_timings": int(rep["rows"]),
        "train_shapes": len(train_shapes),
        "model_loss_first_last": [round(float(rep["loss_first"]), 5), round(float(rep["loss_last"]), 5)],
        "heldout_mse": round(float(rep["heldout_mse"]), 5),
        "seconds": round(time.perf_counter() - t_start, 1),
    }
    return result, (test_shapes, datas, out_m, {"exhaustive": exh, "learned": mlp, "default": dflt, "eq1_rule": rule})


def independent_loops(n_loops=96, streams=(1, 4, 16), steps=2, seed=11, reps=5, keep_outputs=False):
    """Many independent small Jacobi sweeps issued eagerly, each array held
    whole (one partition), on contexts with 1, 4 and 16 streams: the runtime
    places each loop on a stream by its inputs' last writer or, for
    independent loops, the least recently used stream, and orders dependent
    loops by events (automated asynchronous execution of independent loop
    nests).  The same loop sequence captured as one graph is timed beside
    them, with each loop its own launch and with every loop a task of the
    persistent kernel (the loops of one sweep, independent of each other,
    then share one launch: kernel-level parallelism).  Returns ({variant: ms per pass}, outputs or None); a pass is
    `steps` ping-pong sweeps of every grid (sides log-uniform in [64, 1024])."""
    import torch
    r = inputs.rng(seed)
    shapes = [tuple(int(v) for v in s) for s in inputs.log_uniform_int(r, 64, 1024, (n_loops, 2))]
    out = {}
    outputs = None

    def make(ctx):
        grids = []
        for i, sh in enumerate(shapes):
            a = inputs.jacobi_grid(*sh, seed=seed + i)
            b = a.copy()
            ctx.enter(a, halo=(1, 1), K=1)
            ctx.enter(b, halo=(1, 1), K=1)
            grids.append((a, b))
        return grids

    def one_pass(ctx, grids, cfg=None):
        for t in range(steps):
            for a, b in grids:
                (ctx.jacobi2d(a, b, cfg=cfg) if t % 2 == 0 else ctx.jacobi2d(b, a, cfg=cfg))

    for ns in streams:
        ctx = jacc.Context(ns)
        try:
            grids = make(ctx)
            one_pass(ctx, grids)
            ctx.wait()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                one_pass(ctx, grids)
            ctx.wait()
            torch.cuda.synchronize()
            out[f"eager_{ns}_streams"] = round((time.perf_counter() - t0) / reps * 1e3, 4)
            if keep_outputs and ns == max(streams):
                outputs = []
                for a, b in grids:
                    res = a if steps % 2 == 0 else b
                    ctx.update(res, jacc.UPDATE_HOST)
                    outputs.append(res.copy())
            if ns == max(streams):
                ctx.batch_begin()
                one_pass(ctx, grids)
                g = ctx.batch_end()
                out["graph"] = round(float(np.median(ctx.batch_time(g, warmup=2, reps=reps))), 4)
                # the same pass with every loop a task of the persistent
                # kernel: the independent loops of a sweep share one launch
                ctx.batch_begin()
                one_pass(ctx, grids, jacc.config(persistent=1))
                g = ctx.batch_end()
                out["graph_tasks"] = round(float(np.median(ctx.batch_time(g, warmup=2, reps=reps))), 4)
                out["graph_tasks_launches_per_pass"] = ctx.batch_info(g)["persistent_groups"]
        finally:
            ctx.close()
    return out, (shapes, outputs)
