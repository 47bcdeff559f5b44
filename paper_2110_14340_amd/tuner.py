"""Exhaustive autotuner and learned cost model for batched stencil sweeps.

The paper names aggressive auto-tuning as future work (Sec. "Conclusion");
its adaptive rule (Sec. "Adaptive Utilization") already chooses per kernel
between duplicated and distributed execution from profiled times.  Here the
choice is a launch configuration per loop nest: workgroup shape (bx, by),
rows or planes per lane (tile), doubles per lane (vec), partitions (K) and
persistent execution.  None of these changes the arithmetic of the loop
body, so every choice gives bit-identical results.

* Timing: every candidate is timed the way a batch runs it — as a one-loop
  captured graph on stream 0, replayed and timed with HIP events (median of
  the samples; ties go to the lowest candidate index).
* Timing database: JSON, keyed by GPU architecture, HIP runtime version and
  a hash of the library build, so tuning can resume and stale timings of
  another build are never reused.
* Cost model: the FP32 network of the library (forward, backward and Adam on
  the GPU) trained on log(median time) of the database rows of training
  shapes; it predicts every candidate of a new loop and takes the argmin,
  with the exhaustive tuner as fallback when no model is loaded.
"""
import hashlib
import json
import math
import os

import numpy as np

from . import jacc

DEFAULT_CONFIG = {"bx": 256, "by": 1, "tile": 1, "vec": 1, "K": 1, "persistent": 0, "rows": 1}

BLOCKS = [(64, 1), (128, 1), (256, 1), (512, 1), (64, 4), (128, 2), (256, 2), (256, 4)]
TILES = [1, 4, 16, 64]
VECS = [1, 2]
KS = [1, 2]
PERSISTENT_TILES = [1, 4, 16]
ROWS_3D = [1, 4]  # heat: rows per wave (4 needs workgroups of at most 256 threads)
NFEAT = 13


def candidates(shape):
    """Legal configurations for a stencil sweep over an array of `shape`
    (2-D: Jacobi, 3-D: heat); vec = 2 needs an even innermost extent."""
    even = shape[-1] % 2 == 0
    out = []
    for K in KS:
        if K > shape[0] - 2:
            continue
        for bx, by in BLOCKS:
            for rows in (ROWS_3D if len(shape) == 3 else [1]):
                if rows > 1 and bx * by > 256:
                    continue
                for tile in TILES:
                    for vec in VECS:
                        if vec == 2 and not even:
                            continue
                        out.append({"bx": bx, "by": by, "tile": tile, "vec": vec, "K": K, "persistent": 0,
                                    "rows": rows})
        for tile in PERSISTENT_TILES:
            for vec in VECS:
                if vec == 2 and not even:
                    continue
                out.append({"bx": 256, "by": 1, "tile": tile, "vec": vec, "K": K, "persistent": 1, "rows": 1})
    return out


def config_key(cfg):
    key = f"bx{cfg['bx']}_by{cfg['by']}_t{cfg['tile']}_v{cfg['vec']}_K{cfg['K']}_p{cfg['persistent']}"
    return key + (f"_r{cfg['rows']}" if cfg.get("rows", 1) != 1 else "")


def launch_config(cfg):
    """The library configuration of a candidate (order and march take the
    library's defaults)."""
    return jacc.config(bx=cfg["bx"], by=cfg["by"], tile=cfg["tile"], vec=cfg["vec"], persistent=cfg["persistent"],
                       rows=cfg.get("rows", 1))


def workgroups(shape, cfg):
    """Workgroups one launch of the configuration uses over the interior."""
    if len(shape) == 2:
        rows, cols = shape[0] - 2, shape[1] - 2
        bx, by = (256, 1) if cfg["persistent"] else (cfg["bx"], cfg["by"])
        return math.ceil(cols / (bx * cfg["vec"])) * math.ceil(rows / (by * cfg["tile"]))
    nz, ny, nx = shape[0] - 2, shape[1] - 2, shape[2] - 2
    bx, by = (256, 1) if cfg["persistent"] else (cfg["bx"], cfg["by"])
    return math.ceil(nx / (bx * cfg["vec"])) * math.ceil(ny / (by * cfg.get("rows", 1))) * math.ceil(nz / cfg["tile"])


def features(shape, cfg):
    """The cost model's input: 13 numbers describing the loop and the
    configuration (logs of sizes so that the scale generalises)."""
    dims = list(shape) + [1] * (3 - len(shape))
    cells = float(np.prod([max(1, d - 2) for d in shape]))
    return np.array([
        1.0 if len(shape) == 3 else 0.0,
        math.log2(dims[0]), math.log2(dims[1]), math.log2(max(1, dims[2])),
        math.log2(cells),
        math.log2(cfg["bx"]), math.log2(cfg["by"]), math.log2(cfg["tile"]),
        float(cfg["vec"]), math.log2(cfg["K"]), float(cfg["persistent"]),
        math.log2(workgroups(shape, cfg)), math.log2(cfg.get("rows", 1)),
    ], dtype=np.float64)


def median(samples):
    s = sorted(float(v) for v in samples)
    n = len(s)
    return s[n // 2] if n % 2 else 0.5 * (s[n // 2 - 1] + s[n // 2])


def select(medians):
    """Index of the smallest median, ties to the lowest index."""
    best = 0
    for i, t in enumerate(medians):
        if t < medians[best]:
            best = i
    return best


def build_key():
    with open(jacc.LIB_PATH, "rb") as f:
        h = hashlib.sha1(f.read()).hexdigest()[:12]
    arch, hip = "gfx950", "unknown"
    try:
        import torch
        if torch.cuda.is_available():
            arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        hip = str(torch.version.hip)
    except Exception:
        pass
    return f"{arch}|hip{hip}|{h}"


class TimingDB:
    """Persistent timing database (JSON)."""

    def __init__(self, path=None):
        self.path = path or os.environ.get("JACC_TUNE_DB")
        self.key = build_key()
        self.data = {}
        if self.path and os.path.exists(self.path):
            with open(self.path) as f:
                self.data = json.load(f)
        self.entries = self.data.setdefault(self.key, {})

    @staticmethod
    def signature(shape):
        return "x".join(str(d) for d in shape)

    def get(self, shape, cfg):
        return self.entries.get(self.signature(shape), {}).get(config_key(cfg))

    def put(self, shape, cfg, samples):
        self.entries.setdefault(self.signature(shape), {})[config_key(cfg)] = [float(v) for v in samples]

    def save(self):
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.data, f)
            os.replace(tmp, self.path)


def _loop(ctx, u, v, cfg):
    c = launch_config(cfg)
    if u.ndim == 2:
        ctx.jacobi2d(u, v, cfg=c)
    else:
        ctx.heat3d(u, v, 0.1, cfg=c)


def time_graph(ctx, u, v, cfg, warmup=1, reps=5):
    """HIP-event times (ms) of one sweep u -> v run as a one-loop graph."""
    ctx.batch_begin()
    try:
        _loop(ctx, u, v, cfg)
    finally:
        g = ctx.batch_end()
    try:
        return ctx.batch_time(g, warmup=warmup, reps=reps)
    finally:
        ctx.batch_destroy(g)


def tune(ctx, shape, u0, cands=None, db=None, warmup=1, reps=5):
    """Times every candidate for a sweep over `shape` starting from u0;
    returns (candidates, medians, samples).  Arrays are entered once per K."""
    cands = cands if cands is not None else candidates(shape)
    meds = [None] * len(cands)
    samples = [None] * len(cands)
    byK = {}
    for i, cfg in enumerate(cands):
        if db is not None:
            s = db.get(shape, cfg)
            if s is not None:
                samples[i], meds[i] = s, median(s)
                continue
        byK.setdefault(cfg["K"], []).append(i)
    for K, idx in sorted(byK.items()):
        u = np.ascontiguousarray(u0).copy()
        v = u.copy()
        ctx.enter(u, halo=(1, 1), K=K)
        ctx.enter(v, halo=(1, 1), K=K)
        try:
            for i in idx:
                s = time_graph(ctx, u, v, cands[i], warmup, reps)
                samples[i], meds[i] = list(s), median(s)
                if db is not None:
                    db.put(shape, cands[i], s)
        finally:
            ctx.exit(v, jacc.DELETE)
            ctx.exit(u, jacc.DELETE)
    return cands, meds, samples


class CostModel:
    """Host side of the learned cost model: feature scaling, dataset, and
    the library's GPU network (jacc.Model) for training and inference."""

    def __init__(self, ctx, init_params=None):
        """init_params: one parameter set, or a list of them for an ensemble
        of networks (trained on the same data with different initial weights
        and sample orders; the prediction is their mean)."""
        self.ctx = ctx
        inits = init_params if isinstance(init_params, list) else [init_params]
        self.nets = []
        for p in inits:
            net = jacc.Model(ctx, NFEAT)
            if p is not None:
                net.set_params(p)
            self.nets.append(net)
        self.net = self.nets[0]
        self.mu = np.zeros(NFEAT)
        self.sd = np.ones(NFEAT)
        self.trained = False

    def fit(self, X, y, epochs=300, batch=256, lr=1e-3, seed=0):
        """Trains every member; returns the first member's loss curve."""
        X = np.asarray(X, dtype=np.float64)
        self.mu = X.mean(axis=0)
        sd = X.std(axis=0)
        self.sd = np.where(sd > 0, sd, 1.0)
        curves = []
        for m, net in enumerate(self.nets):
            net.set_scaler(self.mu, self.sd)
            curves.append(net.train(X, np.asarray(y), epochs=epochs, batch=batch, lr=lr, seed=seed + m))
        self.trained = True
        return curves[0]

    def predict(self, X):
        X = np.asarray(X, dtype=np.float64)
        return np.mean([net.predict(X) for net in self.nets], axis=0)

    def pick(self, shape, cands=None):
        """Configuration with the smallest predicted log time (ties to the
        lowest candidate index)."""
        cands = cands if cands is not None else candidates(shape)
        pred = self.predict(np.stack([features(shape, c) for c in cands]))
        return cands[int(np.argmin(pred))], pred

    def close(self):
        for net in self.nets:
            net.close()


def choose(shape, model=None, ctx=None, u0=None, db=None):
    """The configuration for a loop: the model's argmin when a trained model
    is given, else the exhaustive tuner's choice (which needs ctx and u0)."""
    if model is not None and model.trained:
        return model.pick(shape)[0]
    cands, meds, _ = tune(ctx, shape, u0, db=db)
    return cands[select(meds)]
