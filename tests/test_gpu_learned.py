"""GPU end-to-end check of the batched/learned path at a small size: the
tuner times every candidate of each loop, the GPU-trained cost model picks a
configuration per loop, and graphs built with the exhaustive, learned and
default configurations produce outputs bit-identical to each other and to
the CPU oracle's single sweeps."""
import numpy as np
import pytest

import oracle
from paper_2110_14340_amd import experiment, inputs
from gpu_util import say

pytestmark = pytest.mark.gpu


def test_small_batched_learned_experiment():
    say("learned experiment, small")
    test_shapes = inputs.batch_shapes(5, 10, 6, side2d=(64, 400), side3d=(32, 64))
    train_shapes = inputs.batch_shapes(7, 6, 4, side2d=(64, 400), side3d=(32, 64))
    res, (shapes, datas, outs, _) = experiment.run(epochs=80, tune_reps=3, graph_reps=5, log=say,
                                                   test_shapes=test_shapes, train_shapes=train_shapes)
    say(str(res))
    assert res["outputs_bit_identical_across_configs"]
    for sh, d, o in zip(shapes, datas, outs):
        ref = d.copy()
        if len(sh) == 2:
            oracle.jacobi2d_sweep(d, ref)
        else:
            oracle.heat3d_sweep(d, ref, 0.1)
        assert np.array_equal(o, ref), sh
    assert res["model_loss_first_last"][1] < res["model_loss_first_last"][0]
    assert np.isfinite(res["regret_learned_vs_exhaustive"])


def test_learned_batch_within_five_percent_of_the_tuner_and_faster_than_default():
    """What the trained network gains.  A fixed seeded batch of 48 uneven
    sweeps (24 2-D with sides log-uniform in [64, 2048], 24 3-D in [32, 256])
    runs as one graph configured three ways; the network was trained on the
    tuner's timings of 96 other shapes of the same laws.  The learned graph
    is within 5 % of the exhaustive tuner's and faster than the fixed default
    configuration (graph times: the minimum over three interleaved rounds of
    the median of 30 replays).  Every output is bit-identical across the
    configurations, including the Eq. 1 rule's."""
    say("learned vs exhaustive vs default, 48-loop batch")
    test_shapes = inputs.batch_shapes(5, 24, 24, side2d=(64, 2048), side3d=(32, 256))
    train_shapes = inputs.batch_shapes(7, 48, 48, side2d=(64, 2048), side3d=(32, 256))
    res, (shapes, datas, _, cfgs) = experiment.run(epochs=300, tune_reps=5, graph_reps=30, log=say,
                                                   test_shapes=test_shapes, train_shapes=train_shapes)
    say(str(res))
    assert res["outputs_bit_identical_across_configs"]
    t = experiment.interleaved_times(shapes, datas, {k: cfgs[k] for k in ("exhaustive", "learned", "default")},
                                     rounds=3, reps=30)
    regret = t["learned"] / t["exhaustive"] - 1.0
    gain = t["default"] / t["learned"]
    say(f"  graph ms {t}; regret {regret:+.4f}, gain over default {gain:.3f}")
    assert regret <= 0.05, f"learned graph {regret:+.2%} slower than the exhaustive tuner's"
    assert gain > 1.0, f"learned graph not faster than the default ({gain:.3f}x)"


def test_full_batch_of_256_sweeps_in_one_graph_equals_oracle():
    """The benchmark's batch (128 2-D + 128 3-D single sweeps, sides
    log-uniform in [64, 4096] and [32, 512]) captured in one graph, small
    loops as persistent tasks and large ones as partitioned launches: every
    output equals its own oracle sweep bit for bit."""
    say("full 256-loop batch in one graph vs oracle")
    from paper_2110_14340_amd import tuner
    shapes = inputs.batch_shapes(5, 128, 128)
    datas = [inputs.jacobi_grid(*sh, seed=6000 + i) if len(sh) == 2 else inputs.heat_field(*sh, seed=6000 + i)
             for i, sh in enumerate(shapes)]
    cfgs = []
    for sh in shapes:
        cells = float(np.prod([d - 2 for d in sh]))
        cfg = dict(tuner.DEFAULT_CONFIG)
        if cells < 2 ** 18:
            cfg.update(persistent=1, tile=4, vec=2 if sh[-1] % 2 == 0 else 1)
        elif len(sh) == 2:
            cfg.update(K=2, tile=8, vec=2 if sh[-1] % 2 == 0 else 1)
        cfgs.append(cfg)
    ms, info, outs = experiment.graph_time(shapes, datas, cfgs, reps=2, keep_outputs=True)
    say(f"  graph {ms:.3f} ms, {info}")
    assert info["persistent_groups"] >= 1
    for sh, d, o in zip(shapes, datas, outs):
        ref = d.copy()
        if len(sh) == 2:
            oracle.jacobi2d_sweep(d, ref)
        else:
            oracle.heat3d_sweep(d, ref, 0.1)
        assert np.array_equal(o, ref), sh
