"""Automated asynchronous execution of independent loop nests: many whole
(one-partition) Jacobi grids swept eagerly on a 16-stream context give the
oracle's bits, whichever streams the runtime placed them on."""
import numpy as np
import pytest

import oracle
from paper_2110_14340_amd import experiment, inputs

pytestmark = pytest.mark.gpu


def test_independent_loops_on_many_streams_bit_exact():
    print("independent loops: 24 grids, 1/4/16 streams", flush=True)
    seed, steps, reps = 11, 2, 1
    times, (shapes, outs) = experiment.independent_loops(n_loops=24, streams=(1, 4, 16), steps=steps, seed=seed,
                                                         reps=reps, keep_outputs=True)
    assert set(times) == {"eager_1_streams", "eager_4_streams", "eager_16_streams", "graph", "graph_tasks",
                          "graph_tasks_launches_per_pass"}
    # the independent loops of each sweep share one task-kernel launch
    assert times["graph_tasks_launches_per_pass"] == steps
    for i, sh in enumerate(shapes):
        u0 = inputs.jacobi_grid(*sh, seed=seed + i)
        assert np.array_equal(outs[i], oracle.jacobi2d(u0, steps * (1 + reps))), (i, sh)
