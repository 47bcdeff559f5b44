"""Autotuner and learned cost model: argument marshalling over the library's
C entry points (jacc_candidates, jacc_features, jacc_tune, jacc_model_train,
jacc_model_load, jacc_model_pick, jacc_choose).

The candidate set, the features, the timing of candidates (captured graphs
of several sweeps on scratch replicas, HIP events), the median and tie rule, the timing
database keyed by device, HIP runtime and library build, the training of the
GPU networks, the model file, the ensemble mean and the argmin all live in
the library (csrc/tune.cpp, csrc/model.cpp, csrc/k_mlp.hip).  What stays here
is the experiment's fixed default configuration and the conversion between
numpy arrays and the C calls.
"""
import os

import numpy as np

from . import jacc

# The fixed configuration the learned choice is compared against: 256
# threads, one row per thread, one double per lane, one partition.
DEFAULT_CONFIG = {"bx": 256, "by": 1, "tile": 1, "vec": 1, "K": 1, "persistent": 0, "rows": 1}
KS = [1, 2, 4, 8]
NFEAT = jacc.NFEATURES


def candidates(shape, ks=KS):
    return jacc.candidates(shape, ks)


def features(shape, cfg):
    return jacc.features(shape, cfg)


def median(samples):
    return jacc.median(samples)


def select(medians):
    """Index of the smallest median, ties to the lowest index."""
    return jacc.argmin(medians)


def config_key(cfg):
    key = f"bx{cfg['bx']}_by{cfg['by']}_t{cfg['tile']}_v{cfg['vec']}_K{cfg['K']}_p{cfg['persistent']}"
    return key + (f"_r{cfg['rows']}" if cfg.get("rows", 1) != 1 else "")


def launch_config(cfg):
    """The library configuration of a candidate (order and march take the
    library's defaults)."""
    return jacc.config(bx=cfg["bx"], by=cfg["by"], tile=cfg["tile"], vec=cfg["vec"], persistent=cfg["persistent"],
                       rows=cfg.get("rows", 1))


def tune(ctx, shape, u0, db_path=None, ks=KS, warmup=1, reps=5):
    """Exhaustive tuning of one sweep over `shape` from data u0 (jacc_tune on
    arrays entered with one partition; the candidates run on the library's
    scratch replicas).  Returns (candidates, medians in ms, chosen index)."""
    u = np.ascontiguousarray(u0, dtype=np.float64).copy()
    v = u.copy()
    ctx.enter(u, halo=(1, 1), K=1)
    ctx.enter(v, halo=(1, 1), K=1)
    try:
        best, cands, med = ctx.tune(u, v, ks=ks, db_path=db_path, warmup=warmup, reps=reps)
    finally:
        ctx.exit(v, jacc.DELETE)
        ctx.exit(u, jacc.DELETE)
    return cands, med, cands.index(best)


def train(ctx, db_path, model_path, members=3, epochs=300, batch=256, lr=1e-3, seed=9, holdout=5):
    """jacc_model_train: the GPU-trained ensemble written to model_path."""
    return ctx.model_train(db_path, model_path, members=members, epochs=epochs, batch=batch, lr=lr, seed=seed,
                           holdout=holdout)


def pick(ctx, shape, ks=KS):
    """The attached model's choice: (candidate, candidates, predictions)."""
    return ctx.model_pick(shape, ks)


def default_db_path():
    return os.environ.get("JACC_TUNE_DB")
