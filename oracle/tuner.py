"""Selection rule of the exhaustive autotuner and its regret (test
infrastructure only).

The paper names aggressive auto-tuning as future work (Sec. "Conclusion");
the rule here is the plain definition the runtime's tuner is checked
against: the chosen configuration minimises the median of its timed samples,
ties going to the lowest configuration index.  Regret of a choice is its time
relative to the exhaustive best: (T(chosen) - T(best)) / T(best).
"""
import numpy as np


def median(samples):
    s = sorted(float(v) for v in samples)
    n = len(s)
    if n == 0:
        raise ValueError("no samples")
    return s[n // 2] if n % 2 else 0.5 * (s[n // 2 - 1] + s[n // 2])


def select(samples_per_config):
    """Index of the configuration with the smallest median sample time."""
    best, best_t = None, None
    for i, samples in enumerate(samples_per_config):
        t = median(samples)
        if best_t is None or t < best_t:
            best, best_t = i, t
    return best


def regret(t_chosen, t_best):
    return (float(t_chosen) - float(t_best)) / float(t_best)


def argmin_predicted(pred):
    """Index of the smallest predicted value, ties to the lowest index."""
    pred = np.asarray(pred)
    return int(np.argmin(pred))
