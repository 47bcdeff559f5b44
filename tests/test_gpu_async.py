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


def test_packed_sweeps_then_a_partitioned_consumer_on_other_streams():
    """Packed Jacobi sweeps (one launch per sweep on one stream, no event
    recorded after them) followed by a GEMM whose K partitions run on their
    own streams and read the swept rows: each partition's wait records the
    event it needs, so C is the oracle's product of the swept grid."""
    from paper_2110_14340_amd import jacc
    from gpu_util import context, say
    n, K, steps = 320, 4, 5
    say(f"packed sweeps {n}^2 K={K} then a partitioned GEMM")
    u0 = inputs.jacobi_grid(n, n, seed=21)
    B = inputs.uniform((n, 96), seed=22, lo=-1.0, hi=1.0)
    a, b = u0.copy(), u0.copy()
    C = np.zeros((n, 96))
    with context(K) as c:
        c.enter(a, halo=(1, 1))
        c.enter(b, halo=(1, 1))
        c.enter(B, whole=True)
        c.enter(C, clause=jacc.CREATE)
        for t in range(steps):
            (c.jacobi2d(a, b) if t % 2 == 0 else c.jacobi2d(b, a))
        last = b if steps % 2 == 1 else a
        c.gemm(last, B, C)
        c.exit(C, jacc.COPYOUT)
    swept = oracle.jacobi2d(u0, steps)
    ref = oracle.gemm(swept, B)
    assert np.linalg.norm(C - ref) <= 1e-12 * np.linalg.norm(swept) * np.linalg.norm(B)
