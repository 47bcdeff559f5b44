"""GPU tests of the autotuner and cost-model boundary: the exhaustive choice
follows the selection rule on measured medians, the timing database is
reused, tuning never writes the caller's arrays, a cost model trained on
the GPU from the database is written, loaded and picks the argmin of its
predictions, a loop without a configuration runs the model's pick with
unchanged results, and a corrupt model file falls back to the tuner."""
import numpy as np
import pytest

import oracle
from oracle import tuner as OT
from paper_2110_14340_amd import inputs, jacc, tuner
from gpu_util import context, say

pytestmark = pytest.mark.gpu


def test_tune_selection_rule_database_reuse_and_scratch_replicas(tmp_path):
    say("jacc_tune 130x258, K in {1,2,4}")
    shape = (130, 258)
    u0 = inputs.jacobi_grid(*shape, seed=31)
    db = str(tmp_path / "timings.db")
    u, v = u0.copy(), u0.copy()
    v[1:-1, 1:-1] = -1.0
    before = v.copy()
    with context(4) as c:
        c.enter(u, halo=(1, 1), K=2)
        c.enter(v, halo=(1, 1), K=2)
        best, cands, med = c.tune(u, v, ks=[1, 2, 4], db_path=db, reps=5)
        assert len(cands) == 3 * 70 and med.shape == (len(cands),) and np.all(med > 0)
        assert cands.index(best) == OT.select([[m] for m in med])
        lines = [ln for ln in open(db) if ln[0] not in "#@"]
        assert len(lines) == len(cands)
        best2, _, med2 = c.tune(u, v, ks=[1, 2, 4], db_path=db)  # served from the database
        assert best2 == best and np.array_equal(med2, med)
        c.exit(v)
        c.exit(u)
    assert np.array_equal(v, before)  # candidates ran on scratch replicas


def test_model_trained_from_database_file_pick_and_unconfigured_loop(tmp_path):
    say("cost model: tune 8 shapes, train, load, pick")
    db = str(tmp_path / "train.db")
    path = str(tmp_path / "model.bin")
    shapes = inputs.batch_shapes(40, 5, 3, side2d=(64, 600), side3d=(32, 64))
    with context(8) as c:
        for i, sh in enumerate(shapes):
            data = inputs.jacobi_grid(*sh, seed=i) if len(sh) == 2 else inputs.heat_field(*sh, seed=i)
            tuner.tune(c, sh, data, db_path=db, ks=[1, 2], reps=3)
        rep = c.model_train(db, path, members=2, epochs=60, seed=3, holdout=4)
        say(f"  {rep}")
        assert rep["signatures"] == len(shapes) and rep["loss_last"] < rep["loss_first"]
        assert rep["heldout_mse"] > 0
        c.model_load(path)
        for sh in ((300, 514), (40, 36, 66)):
            best, cands, pred = c.model_pick(sh, [1, 2])
            assert pred.shape == (len(cands),) and np.all(np.isfinite(pred))
            assert cands.index(best) == OT.argmin_predicted(pred)
        # a Jacobi loop with no configuration runs the model's eager pick
        u0 = inputs.jacobi_grid(300, 514, seed=5)
        a, b = u0.copy(), u0.copy()
        c.enter(a, halo=(1, 1), K=2)
        c.enter(b, halo=(1, 1), K=2)
        for t in range(4):
            (c.jacobi2d(a, b) if t % 2 == 0 else c.jacobi2d(b, a))
        c.exit(b)
        c.exit(a)
        assert np.array_equal(a, oracle.jacobi2d(u0, 4))
        # the file loads again in a fresh context and gives the same picks
        with context(2) as c2:
            c2.model_load(path)
            assert c2.model_pick((300, 514), [1, 2])[0] == c.model_pick((300, 514), [1, 2])[0]


def test_corrupt_model_falls_back_to_the_tuner(tmp_path):
    say("jacc_choose with a corrupt model file")
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"JACCCM01" + b"\0" * 64)
    u0 = inputs.jacobi_grid(66, 130, seed=32)
    u, v = u0.copy(), u0.copy()
    with context(2) as c:
        c.enter(u, halo=(1, 1))
        c.enter(v, halo=(1, 1))
        cand, src = c.choose(u, v, model_path=str(bad), ks=[1, 2], db_path=str(tmp_path / "t.db"), reps=3)
        assert src == jacc.CHOICE_TUNER and "model:" in c.last_error()
        assert cand in jacc.candidates((66, 130), [1, 2])
        cand, src = c.choose(u, v, model_path=str(bad), tune=False)
        assert src == jacc.CHOICE_DEFAULT and cand["K"] == 2
