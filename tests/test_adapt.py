"""The adaptive duplicate-vs-partition switch (Sec. "Adaptive Utilization",
Eq. 1-3): the oracle pinned by hand-computed streams, and the library's
implementation (host code, no GPU) equal to the oracle on random streams."""
import math

import pytest
from hypothesis import given, settings, strategies as st

from oracle import adapt as A
from paper_2110_14340_amd import jacc

PEAK = 153e9  # one xGMI link, bytes per second


def test_switches_on_after_warmup_and_five_eq1_hits():
    # 1 ms kernel writing 64 MiB with n = 8: Eq. 1 is 1e-3 > 1.25e-4 + 4.4e-4
    obs = [(1e-3, 0.0, 64 << 20)] * 7
    assert A.run(obs, 8, PEAK) == [0, 0, 0, 0, 0, 1, 1]


def test_never_switches_when_exchange_dominates():
    # Eq. 1 fails: 1e-4 > 1.25e-5 + 4.4e-4 is false
    assert A.run([(1e-4, 0.0, 64 << 20)] * 20, 8, PEAK) == [0] * 20


def test_single_partition_never_switches():
    # n = 1: t > t + WriteSize/peak never holds
    assert A.run([(5.0, 0.0, 1.0)] * 10, 1, PEAK) == [0] * 10


def test_eq1_hits_are_cumulative_not_consecutive():
    good, bad = (1e-3, 0.0, 64 << 20), (1e-5, 0.0, 64 << 20)
    obs = [good, good, bad, good, bad, good, good, bad, good]
    # warm-up, then hits at observations 2, 4, 6, 7, 9 (1-based)
    assert A.run(obs, 8, PEAK) == [0, 0, 0, 0, 0, 0, 0, 0, 1]


# Dyadic times (units of 2^-13 s, WriteSize 2^20 B) keep every sum exact.
_W = float(1 << 20)
_u = 2.0 ** -13
_DUP = (8 * _u, 0.0, _W)                       # eff_dup * WriteSize = 8u; Eq. 1 holds for n = 4
_SLOW = (4 * _u, 5 * _u, _W)                   # left 9u > 8u (Eq. 3), < n*t_k = 16u: difference +1u
_FAST = (4 * _u, 0.0, _W)                      # left 4u: neither; difference 4u - 8u = -4u
_FASTISH = (4 * _u, 3 * _u, _W)                # left 7u: neither; difference -1u


def test_switches_off_after_five_eq3_violations_with_positive_mean():
    obs = [_DUP] * 6 + [_SLOW, _FASTISH, _SLOW, _SLOW, _FASTISH, _SLOW, _SLOW, _FAST]
    modes = A.run(obs, 4, 1e12)
    assert modes[:6] == [0, 0, 0, 0, 0, 1]
    # five violations at the thirteenth observation; mean (5 - 2)/7 u > 0
    assert modes[6:12] == [1] * 6 and modes[12] == 2
    assert modes[13] == 2  # stays duplicated


def test_five_violations_with_nonpositive_mean_stay_partitioned():
    """The switch-off needs both parts of the rule: five violations of Eq. 3
    occur, but the executions that beat both bounds keep the mean difference
    at or below zero, so the loop stays partitioned until it turns positive."""
    obs = [_DUP] * 6 + [_SLOW, _FAST, _SLOW, _SLOW, _FAST, _SLOW, _SLOW]
    # after them: 5 violations, sum of differences 5u - 8u = -3u
    more = [_SLOW] * 4  # sums -2u, -1u, 0 (not above zero), +1u
    modes = A.run(obs + more, 4, 1e12)
    assert modes[5:13] == [1] * 8
    assert modes[13:16] == [1, 1, 1]
    assert modes[16] == 2


def test_switch_off_through_eq2_alone():
    ws = 1 << 20
    dup = (1e-3, 0.0, ws)
    # left = 2e-4 + 5e-4 = 7e-4 > n*t_k = 4e-4 (Eq. 2) but < eff_dup*ws = 1e-3
    part = (2e-4, 5e-4, ws)
    modes = A.run([dup] * 6 + [part] * 5, 2, 1e12)
    assert modes[5] == 1 and modes[-1] == 2 and modes[-2] == 1


def test_eff_dup_is_mean_of_time_per_byte():
    # five profiled runs with ratios 1, 3, 1, 3, 2 ns/B: eff_dup = 2 ns/B, and
    # all satisfy Eq. 1 (t > t/2 + 1e-6 s) so the fifth switches to PARTITION
    ws = 1e6
    obs = [(9.9, 0, ws)] + [(t, 0, ws) for t in (1e-3, 3e-3, 1e-3, 3e-3, 2e-3)]
    assert A.run(obs, 2, 1e12)[-1] == 1
    # partitioned runs with t_k = 1.5e-3 never violate Eq. 2 (left < 3e-3);
    # Eq. 3's bound is eff_dup * ws = 2e-3
    below = (1.5e-3, 0.5e-3 * (1 - 1e-6), ws)
    above = (1.5e-3, 0.5e-3 * (1 + 1e-6), ws)
    assert A.run(obs + [below] * 10, 2, 1e12)[-1] == 1
    modes = A.run(obs + [above] * 5, 2, 1e12)
    assert modes[-2] == 1 and modes[-1] == 2


def _lib_modes(obs, n, peak):
    a = jacc.Adaptive(n, peak)
    out = [a.observe(*o) for o in obs]
    a.close()
    return out


@settings(max_examples=200, deadline=None)
@given(n=st.integers(1, 8), peak=st.sampled_from([25e9, 153e9, 1e12]),
       obs=st.lists(st.tuples(st.floats(0, 1e-2), st.floats(0, 1e-2), st.floats(1.0, 1e9)), max_size=40))
def test_library_matches_oracle_on_random_streams(n, peak, obs):
    assert _lib_modes(obs, n, peak) == A.run(obs, n, peak)


def test_library_mean_difference_over_partitioned_runs():
    a = jacc.Adaptive(4, 1e12)
    for o in [_DUP] * 6 + [_SLOW, _FAST, _SLOW]:
        a.observe(*o)
    mean, n = a.mean_diff()
    assert n == 3 and mean == (1 - 4 + 1) * _u / 3
    s = a.state()
    assert s["violations"] == 2 and s["eq3"] == 2 and s["eq2"] == 0
    a.close()


def test_library_state_and_errors():
    a = jacc.Adaptive(4, 1e12)
    for _ in range(3):
        a.observe(1e-3, 0.0, 1 << 20)
    s = a.state()
    assert s["mode"] == 0 and s["n_dup"] == 2 and s["eq1"] == 2
    assert math.isclose(s["eff_dup"], 1e-3 / (1 << 20), rel_tol=1e-15)
    assert a.observe(1e-3, 0.0, 0.0, raw=True) == jacc.ERR_INVALID
    assert a.observe(-1.0, 0.0, 1.0, raw=True) == jacc.ERR_INVALID
    assert a.observe(float("nan"), 0.0, 1.0, raw=True) == jacc.ERR_INVALID
    a.close()
    with pytest.raises(jacc.JaccError):
        jacc.Adaptive(0, 1e9)
    with pytest.raises(jacc.JaccError):
        jacc.Adaptive(2, 0.0)
