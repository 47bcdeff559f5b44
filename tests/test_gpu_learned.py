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
    res, (shapes, datas, outs) = experiment.run(epochs=80, tune_reps=3, graph_reps=5, log=say,
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
