"""Adaptive duplicate-vs-partition switch — TEST INFRASTRUCTURE ONLY.

Follows Sec. "Adaptive Utilization" (Eq. 1-3) step by step on a list of
observed executions; shares nothing with the library's implementation.

Readings (the paper's text is ambiguous here):
* eff_dup is used as seconds per byte written: Eq. 3 multiplies it by the
  write size to obtain a time, so it is the mean of time/WriteSize over the
  profiled duplicate runs (the warm-up run excluded).
* "five executions" are counted cumulatively (not consecutively).
* the switch-off average is taken over every partitioned execution since
  the switch to partitioned mode, of (t_k + t_c) minus the smaller of the two
  right sides (n * t_k and eff_dup * WriteSize); so runs that beat both
  bounds pull it below zero and can keep the loop partitioned even after
  five violations.  Once switched off the loop stays duplicated.
* t_k is the kernel time of one partition and t_c the rest of the
  partitioned execution (exchange and synchronisation).

Parity pinned by hand-computed streams in tests/test_adapt.py.
"""

DUPLICATE, PARTITION, DUPLICATE_FINAL = 0, 1, 2


def run(observations, n, peak):
    """observations: iterable of (t_kernel, t_comm, write_bytes) in the
    order executed.  Returns the mode chosen after each observation."""
    mode = DUPLICATE
    warmed = False
    ratios = []          # time / WriteSize of profiled duplicate runs
    eq1_hits = 0
    eq2_hits = eq3_hits = 0
    diffs = []           # left - min(right) of every partitioned run
    out = []
    for tk, tc, ws in observations:
        if mode == PARTITION:
            eff_dup = sum(ratios) / len(ratios)
            left = tk + tc
            right2 = tk * n              # Eq. 2
            right3 = eff_dup * ws        # Eq. 3
            if left > right2:
                eq2_hits += 1
            if left > right3:
                eq3_hits += 1
            diffs.append(left - min(right2, right3))
            if (eq2_hits >= 5 or eq3_hits >= 5) and sum(diffs) / len(diffs) > 0:
                mode = DUPLICATE_FINAL
        elif not warmed:
            warmed = True                # warm-up run: not profiled
        elif mode == DUPLICATE:
            ratios.append(tk / ws)
            if tk > tk / n + ws / peak:  # Eq. 1
                eq1_hits += 1
            if eq1_hits >= 5:
                mode = PARTITION
        out.append(mode)
    return out
