"""GPU parity of batched execution: captured single-stream hipGraphs of
partitioned loop sequences, replayed several times with eager work and host
reads between replays, and persistent-kernel task groups of many small
uneven sweeps — every output bit-identical to the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_2110_14340_amd import inputs, jacc
from gpu_util import context, say

pytestmark = pytest.mark.gpu


def test_graph_of_two_jacobi_steps_replayed_with_eager_work_between():
    say("graph replay jacobi 130x98 K=4")
    u0 = inputs.jacobi_grid(130, 98, seed=21)
    a, b = u0.copy(), u0.copy()
    with context(4) as c:
        c.enter(a, halo=(1, 1))
        c.enter(b, halo=(1, 1))
        c.jacobi2d(a, b)
        c.jacobi2d(b, a)
        c.batch_begin()
        c.jacobi2d(a, b)
        c.jacobi2d(b, a)
        g = c.batch_end()          # runs once: 4 steps so far
        assert c.batch_info(g)["replay_safe"]
        steps = 4
        for r in range(4):
            c.batch_launch(g, 1 + r)
            steps += 2 * (1 + r)
            c.update(a, jacc.UPDATE_HOST)
            assert np.array_equal(a, oracle.jacobi2d(u0, steps)), f"replay {r}"
            if r % 2 == 0:         # eager work between replays
                c.jacobi2d(a, b)
                c.jacobi2d(b, a)
                steps += 2
        c.exit(b)
        c.exit(a)
    assert np.array_equal(a, oracle.jacobi2d(u0, steps))


def test_graph_of_heat_steps_with_residual_slots():
    say("graph replay heat 30x20x36 K=2 with residuals")
    u0 = inputs.heat_field(30, 20, 36, seed=22)
    a, b = u0.copy(), u0.copy()
    with context(2) as c:
        c.enter(a, halo=(1, 1))
        c.enter(b, halo=(1, 1))
        c.heat3d(a, b, 0.1, slot=10)   # eager steps first: the captured pair is then a fixed point
        c.heat3d(b, a, 0.1, slot=11)
        c.batch_begin()
        c.heat3d(a, b, 0.1, slot=0)
        c.heat3d(b, a, 0.1, slot=1)
        g = c.batch_end()
        assert c.batch_info(g)["replay_safe"]
        r01 = c.reductions(0, 2)
        c.batch_launch(g, 1)
        r23 = c.reductions(0, 2)
        c.exit(a)
        c.exit(b)
    ref, ref_res = oracle.heat3d(u0, 6, 0.1)
    assert np.array_equal(a, ref)
    assert np.all(np.abs(r01 - ref_res[2:4]) <= 1e-13 * ref_res[2:4])
    assert np.all(np.abs(r23 - ref_res[4:6]) <= 1e-13 * ref_res[4:6])


def _batch_members(seed, n2, n3):
    r = np.random.default_rng(seed)
    shapes = [(int(r.integers(3, 90)), int(r.integers(3, 700))) for _ in range(n2)]
    shapes += [(int(r.integers(3, 20)), int(r.integers(3, 20)), int(r.integers(3, 300))) for _ in range(n3)]
    return shapes


def test_persistent_group_of_uneven_sweeps_bit_exact():
    say("persistent group: 24 uneven 2-D/3-D sweeps")
    shapes = _batch_members(23, 16, 8)
    cfgs = [jacc.config(tile=t, vec=v, persistent=1, march=m) for t in (1, 3, 8) for v in (1, 2) for m in (1, 2)]
    ins, outs, refs = [], [], []
    with context(4) as c:
        for i, sh in enumerate(shapes):
            u = inputs.jacobi_grid(*sh, seed=100 + i) if len(sh) == 2 else inputs.heat_field(*sh, seed=100 + i)
            v = u.copy()
            c.enter(u, halo=(1, 1), K=1)
            c.enter(v, halo=(1, 1), K=1)
            ins.append(u)
            outs.append(v)
            ref = u.copy()
            if len(sh) == 2:
                oracle.jacobi2d_sweep(u, ref)
            else:
                oracle.heat3d_sweep(u, ref, 0.1)
            refs.append(ref)
        c.batch_begin()
        for i, sh in enumerate(shapes):
            cf = cfgs[i % len(cfgs)]
            if cf.vec == 2 and sh[-1] % 2:
                cf = jacc.config(tile=cf.tile, vec=1, persistent=1, march=cf.march)
            if len(sh) == 2:
                c.jacobi2d(ins[i], outs[i], cfg=cf)
            else:
                c.heat3d(ins[i], outs[i], 0.1, cfg=cf)
        g = c.batch_end()
        info = c.batch_info(g)
        assert info["persistent_groups"] == 1 and info["replay_safe"]
        for rep in range(3):
            c.batch_launch(g, 1)
            for i in range(len(shapes)):
                c.update(outs[i], jacc.UPDATE_HOST)
                assert np.array_equal(outs[i], refs[i]), (rep, i, shapes[i])
                outs[i][...] = -1.0   # host copy scribbled between replays
        for i in range(len(shapes)):
            c.exit(outs[i])
            c.exit(ins[i])
    for i in range(len(shapes)):
        assert np.array_equal(outs[i], refs[i])


def test_batch_mixing_persistent_and_partitioned_loops():
    say("batch: persistent small loops + K=2 large loop")
    big = inputs.jacobi_grid(300, 260, seed=31)
    small = [inputs.jacobi_grid(20 + i, 33 + 2 * i, seed=40 + i) for i in range(5)]
    with context(2) as c:
        a, b = big.copy(), big.copy()
        c.enter(a, halo=(1, 1))
        c.enter(b, halo=(1, 1))
        outs = []
        for s in small:
            o = s.copy()
            c.enter(s, halo=(1, 1), K=1)
            c.enter(o, halo=(1, 1), K=1)
            outs.append(o)
        c.jacobi2d(a, b)
        c.jacobi2d(b, a)
        c.batch_begin()
        for s, o in zip(small, outs):
            c.jacobi2d(s, o, cfg=jacc.config(tile=4, vec=1, persistent=1))
        c.jacobi2d(a, b)
        c.jacobi2d(b, a)
        g = c.batch_end()
        assert c.batch_info(g) == {"loops": 7, "persistent_groups": 1, "replay_safe": True}
        c.batch_launch(g, 2)
        for s, o in zip(small, outs):
            c.exit(o)
            c.exit(s)
        c.exit(b)
        c.exit(a)
    assert np.array_equal(a, oracle.jacobi2d(big, 8))
    for s, o in zip(small, outs):
        ref = s.copy()
        oracle.jacobi2d_sweep(s, ref)
        assert np.array_equal(o, ref)


def test_graph_of_partitioned_steps_as_persistent_tasks_k8():
    say("graph: 8 partitions per step as persistent tasks, mirrors, 20 replays")
    u0 = inputs.jacobi_grid(515, 1030, seed=51)
    a, b = u0.copy(), u0.copy()
    cfg = jacc.config(tile=8, vec=2, persistent=1)
    with context(8) as c:
        c.enter(a, halo=(1, 1))
        c.enter(b, halo=(1, 1))
        c.batch_begin()
        c.jacobi2d(a, b, cfg=cfg)
        c.jacobi2d(b, a, cfg=cfg)
        g = c.batch_end()
        assert c.batch_info(g) == {"loops": 2, "persistent_groups": 2, "replay_safe": True}
        c.batch_launch(g, 19)
        c.exit(b)
        c.exit(a)
    assert np.array_equal(a, oracle.jacobi2d(u0, 40))
