"""GPU runs of the debug and configuration aids: NaN poisoning of stale rows
(every run must still equal the oracle bit for bit, so no read skipped its
pull), roctx ranges, and the environment's exhaustive tuning mode."""
import time

import numpy as np
import pytest

import oracle
from paper_2110_14340_amd import inputs, jacc
from gpu_util import context, run_heat, run_jacobi, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,K,flags,part_dim,T", [
    ((512, 512), 4, jacc.INIT_LAZY, 0, 20), ((130, 258), 3, jacc.INIT_LAZY, 1, 9),
    ((300, 130), 8, 0, 1, 7), ((1030, 514), 4, jacc.INIT_SPLIT | jacc.INIT_LAZY, 0, 6),
])
def test_poisoned_jacobi_equals_oracle(shape, K, flags, part_dim, T):
    say(f"poisoned jacobi {shape} K={K} flags={flags} part_dim={part_dim}")
    u0 = inputs.jacobi_grid(*shape, seed=31)
    out = run_jacobi(u0, T, K, ctx_flags=flags | jacc.INIT_POISON, part_dim=part_dim)
    assert np.array_equal(out, oracle.jacobi2d(u0, T))


def test_poisoned_heat_with_residuals_equals_oracle():
    say("poisoned heat 66x40x36 K=4 lazy")
    u0 = inputs.heat_field(66, 40, 36, seed=32)
    T = 6
    out, res = run_heat(u0, T, 0.1, 4, ctx_flags=jacc.INIT_LAZY | jacc.INIT_POISON)
    ref, ref_res = oracle.heat3d(u0, T, 0.1)
    assert np.array_equal(out, ref)
    assert np.all(np.isfinite(res))
    assert np.all(np.abs(res - ref_res) <= 1e-13 * np.abs(ref_res))


def _device_f64(ptr, n):
    """Host copy of n doubles at a device address (a view through the
    device-array interface, copied by torch)."""
    import torch

    class View:
        __cuda_array_interface__ = {"shape": (n,), "typestr": "<f8", "data": (ptr, False), "version": 2}

    return torch.as_tensor(View(), device="cuda").cpu().numpy().copy()


def test_poison_leaves_nan_in_stale_halo_rows_only():
    """The fill itself: after one lazy sweep the halo rows of each
    partition's slab of the output hold NaN and its interior owner rows the
    sweep's values (read back from the slabs), so a read that skipped its
    pull would carry NaN."""
    say("poison fill contents")
    K, n, m = 4, 64, 48
    u0 = inputs.jacobi_grid(n, m, seed=33)
    a, b = u0.copy(), u0.copy()
    ref = oracle.jacobi2d(u0, 1)
    with context(K, jacc.INIT_LAZY | jacc.INIT_POISON) as c:
        c.enter(a, halo=(1, 1))
        c.enter(b, halo=(1, 1))
        c.jacobi2d(a, b)
        c.wait()
        for p in range(K):
            dev, lo, hi = c.slab(b, p)
            slab = _device_f64(dev, (hi - lo) * m).reshape(hi - lo, m)
            blo, bhi = p * n // K, (p + 1) * n // K
            for r in range(lo, hi):
                if blo <= r < bhi:
                    assert np.array_equal(slab[r - lo], ref[r]), (p, r)
                else:
                    assert np.all(np.isnan(slab[r - lo])), (p, r)
        c.exit(a, jacc.DELETE)
        c.exit(b, jacc.COPYOUT)
    assert np.array_equal(b, ref)


def test_markers_do_not_change_results():
    """roctx ranges around the host phases (opened on first use): the run
    is bit-identical to the oracle."""
    say("jacobi K=4 with roctx ranges")
    u0 = inputs.jacobi_grid(258, 130, seed=34)
    assert np.array_equal(run_jacobi(u0, 5, 4, ctx_flags=jacc.INIT_MARKERS), oracle.jacobi2d(u0, 5))


def test_environment_exhaustive_tuning_picks_once_and_runs_exactly(monkeypatch, tmp_path):
    """JACC_TUNE=exhaustive: the first unconfigured call of a loop signature
    times every candidate at the arrays' K (the timing database written to
    JACC_TUNE_DB) and runs the best non-persistent one; later calls reuse
    the pick without tuning; the results equal the oracle."""
    monkeypatch.setenv("JACC_TUNE", "exhaustive")
    db = tmp_path / "tune.db"
    monkeypatch.setenv("JACC_TUNE_DB", str(db))
    say("environment exhaustive tuning, jacobi 258x514 K=2")
    u0 = inputs.jacobi_grid(258, 514, seed=35)
    a, b = u0.copy(), u0.copy()
    with context(2, 0) as c:
        c.enter(a, halo=(1, 1))
        c.enter(b, halo=(1, 1))
        t0 = time.perf_counter()
        c.jacobi2d(a, b)
        c.wait()
        t_first = time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(3):
            c.jacobi2d(b, a)
            c.jacobi2d(a, b)
        c.wait()
        t_next = (time.perf_counter() - t0) / 6
        c.exit(a, jacc.COPYOUT)
        c.exit(b, jacc.COPYOUT)
    say(f"  first call {t_first * 1e3:.1f} ms (tuning), later calls {t_next * 1e3:.3f} ms")
    assert db.exists() and db.stat().st_size > 0
    assert t_next < t_first / 10
    assert np.array_equal(b, oracle.jacobi2d(u0, 7))


def test_timed_loop_records(monkeypatch, tmp_path):
    """JACC_LOG with JACC_LOG_TIMES: each loop that runs on one stream (K=1,
    or packed) carries its device time from events around its work, and the
    derived GB/s is that of the sweep (a 2048^2 Jacobi sweep at K=1 and K=4
    moves 67 MB per step: well above 1 TB/s and below the 8 TB/s peak);
    a GEMM record reports TFLOP/s."""
    import json
    path = tmp_path / "loops.jsonl"
    monkeypatch.setenv("JACC_LOG", str(path))
    monkeypatch.setenv("JACC_LOG_TIMES", "1")
    say("timed loop records")
    u0 = inputs.jacobi_grid(2048, 2048, seed=36)
    for K in (1, 4):
        a, b = u0.copy(), u0.copy()
        with context(K, 0) as c:
            c.enter(a, halo=(1, 1))
            c.enter(b, halo=(1, 1))
            for t in range(6):
                c.jacobi2d(a, b) if t % 2 == 0 else c.jacobi2d(b, a)
            c.wait()
    A, B = inputs.gemm_inputs(512, 512, 512, seed=37)
    C = np.zeros((512, 512))
    with context(2, 0) as c:
        c.enter(A)
        c.enter(B, whole=True)
        c.enter(C, clause=jacc.CREATE)
        c.gemm(A, B, C)
        c.wait()
    recs = [json.loads(line) for line in path.read_text().splitlines()]
    jac = [r for r in recs if r["kind"] == "JACOBI2D"]
    assert len(jac) == 12 and all(r["ms"] is not None and r["ms"] > 0 for r in jac)
    say("  GB/s " + " ".join(f"{r['gbps']:.0f}" for r in jac))
    assert all(1000 < r["gbps"] < 8000 for r in jac[2:6] + jac[8:])
    gemm = [r for r in recs if r["kind"] == "GEMM"]
    assert len(gemm) == 1 and gemm[0]["flop"] == 2 * 512 ** 3 and gemm[0]["ms"] is None  # two streams: untimed
